// Device helpers shared by the FP64 and the mixed-precision BBPGD kernels:
// fixed-order wave and workgroup reductions, the step-length / stop rule,
// and the XCD-aware tile map.
#pragma once

#include "rl_internal.hpp"

namespace rl {

// Wave total of a double by DPP lane moves, without the LDS crossbar: two
// quad permutations, the half-row and the row mirror leave every lane of a
// row of 16 holding that row's total (each step adds a lane's value to its
// partner's, and both partners compute the same sum), and the four row totals
// are then combined as (r0 + r1) + (r2 + r3).  Every lane returns the same
// bits.  All 64 lanes must be active.
template <int CTRL>
__device__ __forceinline__ double dpp_f64(double v)
{
    const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, 0xf, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, 0xf, 0xf, false);
    return __hiloint2double(hi, lo);
}

__device__ __forceinline__ double lane_f64(double v, int lane)
{
    return __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(v), lane),
                            __builtin_amdgcn_readlane(__double2loint(v), lane));
}

template <bool MAX>
__device__ __forceinline__ double wave_total(double v)
{
    auto op = [](double a, double b) { return MAX ? fmax(a, b) : a + b; };
    v = op(v, dpp_f64<0xb1>(v));   // quad_perm [1,0,3,2]
    v = op(v, dpp_f64<0x4e>(v));   // quad_perm [2,3,0,1]
    v = op(v, dpp_f64<0x141>(v));  // row_half_mirror
    v = op(v, dpp_f64<0x140>(v));  // row_mirror
    return op(op(lane_f64(v, 0), lane_f64(v, 16)), op(lane_f64(v, 32), lane_f64(v, 48)));
}

// Sums p[0..2] and takes the max of p[3] over the workgroup with one barrier:
// wave totals by DPP, then every thread combines the NW wave totals in wave
// order.  Every thread receives the same result; lds (NW x 4 doubles) is not
// reused afterwards by the callers.
template <int NW>
__device__ __forceinline__ void block_total4(double p[4], double (*lds)[4])
{
    const int wid = threadIdx.x >> 6;
    p[0] = wave_total<false>(p[0]);
    p[1] = wave_total<false>(p[1]);
    p[2] = wave_total<false>(p[2]);
    p[3] = wave_total<true>(p[3]);
    if ((threadIdx.x & 63) == 0) {
        lds[wid][0] = p[0];
        lds[wid][1] = p[1];
        lds[wid][2] = p[2];
        lds[wid][3] = p[3];
    }
    __syncthreads();
    p[0] = lds[0][0];
    p[1] = lds[0][1];
    p[2] = lds[0][2];
    p[3] = lds[0][3];
#pragma unroll
    for (int w = 1; w < NW; ++w) {
        p[0] += lds[w][0];
        p[1] += lds[w][1];
        p[2] += lds[w][2];
        p[3] = fmax(p[3], lds[w][3]);
    }
}

// Workgroup partials of the single-system solvers: `count` slots, kept as two
// arrays of double2, (s.s, s.y) of every slot and then (y.y, residual), so
// that a wave's loads of consecutive slots read whole lines (half as many L2
// requests as four doubles per slot; every rod workgroup reads them all).
__device__ __forceinline__ void partial_put(double *P, int count, int b, const double p[4])
{
    double2 *Q = reinterpret_cast<double2 *>(P);
    Q[b] = make_double2(p[0], p[1]);
    Q[count + b] = make_double2(p[2], p[3]);
}

struct PartFirst {
    double2 u, v, u2, v2;
};

// the thread's slots b and b + NT (clamped: count >= 1 gives in-bounds
// addresses).  The loads are unconditional (see rod_rec_load), so a kernel
// that issues them before its records can reduce them while the records are
// still in flight.
template <int NT>
__device__ __forceinline__ void partials_first_split(const double *__restrict__ P, int count, PartFirst &F)
{
    const double2 *Q = reinterpret_cast<const double2 *>(P);
    const int b = min((int)threadIdx.x, count - 1), b2 = min((int)threadIdx.x + NT, count - 1);
    F.u = Q[b];
    F.v = Q[count + b];
    F.u2 = Q[b2];
    F.v2 = Q[count + b2];
}

// Totals of the `count` slots at `P` (split layout), identical in every
// workgroup: each thread sums its slots in index order, then block_total4.
template <int NW>
__device__ __forceinline__ void sum_partials_split_from(const PartFirst &F, const double *__restrict__ P, int count,
                                                        double p[4], double (*lds)[4])
{
    constexpr int NT = NW * 64;
    const double2 *Q = reinterpret_cast<const double2 *>(P);
    p[0] = p[1] = p[2] = p[3] = 0.0;
    if ((int)threadIdx.x < count) {
        p[0] += F.u.x;
        p[1] += F.u.y;
        p[2] += F.v.x;
        p[3] = fmax(p[3], F.v.y);
    }
    if ((int)threadIdx.x + NT < count) {
        p[0] += F.u2.x;
        p[1] += F.u2.y;
        p[2] += F.v2.x;
        p[3] = fmax(p[3], F.v2.y);
    }
    for (int b = threadIdx.x + 2 * NT; b < count; b += NT) {
        const double2 u = Q[b], v = Q[count + b];
        p[0] += u.x;
        p[1] += u.y;
        p[2] += v.x;
        p[3] = fmax(p[3], v.y);
    }
    block_total4<NW>(p, lds);
}

template <int NW>
__device__ __forceinline__ void sum_partials_split(const double *__restrict__ P, int count, double p[4],
                                                   double (*lds)[4])
{
    PartFirst F;
    partials_first_split<NW * 64>(P, count, F);
    sum_partials_split_from<NW>(F, P, count, p, lds);
}

// Totals of the `count` workgroup partials at `P`, identical in every
// workgroup.  Each thread sums its partials in index order: the first one
// (partials_first, which a kernel may issue early, before it waits on
// anything else), then the rest with kPartChunk loads in flight together.
constexpr int kPartChunk = 2;

// the thread's first partial (clamped: any count >= 1 gives an in-bounds
// address; with count <= 0 nothing is read)
__device__ __forceinline__ void partials_first(const double *__restrict__ P, int count, PartFirst &F)
{
    F.u = F.v = make_double2(0.0, 0.0);
    if (count > 0) {
        const int b = min((int)threadIdx.x, count - 1);
        const double2 *src = reinterpret_cast<const double2 *>(P + 4 * (int64_t)b);
        F.u = src[0];
        F.v = src[1];
    }
}

template <int NW>
__device__ __forceinline__ void sum_partials_from(const PartFirst &F, const double *__restrict__ P, int count,
                                                  double p[4], double (*lds)[4])
{
    constexpr int NT = NW * 64;
    p[0] = p[1] = p[2] = p[3] = 0.0;
    if ((int)threadIdx.x < count) {
        p[0] += F.u.x;
        p[1] += F.u.y;
        p[2] += F.v.x;
        p[3] = fmax(p[3], F.v.y);
    }
    for (int b0 = threadIdx.x + NT; b0 < count; b0 += kPartChunk * NT) {
        double2 u[kPartChunk], v[kPartChunk];
#pragma unroll
        for (int j = 0; j < kPartChunk; ++j) {
            // clamped, so that every load is issued before the first wait
            const int b = min(b0 + j * NT, count - 1);
            const double2 *src = reinterpret_cast<const double2 *>(P + 4 * (int64_t)b);
            u[j] = src[0];
            v[j] = src[1];
        }
#pragma unroll
        for (int j = 0; j < kPartChunk; ++j) {
            if (b0 + j * NT < count) {
                p[0] += u[j].x;
                p[1] += u[j].y;
                p[2] += v[j].x;
                p[3] = fmax(p[3], v[j].y);
            }
        }
    }
    block_total4<NW>(p, lds);
}

template <int NW>
__device__ __forceinline__ void sum_partials(const double *__restrict__ P, int count, double p[4], double (*lds)[4])
{
    PartFirst F;
    partials_first(P, count, F);
    sum_partials_from<NW>(F, P, count, p, lds);
}

// Stop test and step length for iteration k >= 1 from the totals of
// iteration k-1 (s.s, s.y, y.y, residual); status RL_OK / NOT_CONVERGED /
// STAGNATED / ERR_NONFINITE when stopping.
struct Decision {
    double alpha;
    int stop, status;
};

// The state a decision reads, loaded ahead of it (st: the system's state;
// abuf: its two step lengths by iteration parity).
struct DecideIn {
    double tol, amin, amax, aprev;
    long long max_iter;
};

__device__ __forceinline__ DecideIn decide_in(const SolverState *st, const double *abuf, long long k)
{
    return DecideIn{st->tol, st->amin, st->amax, abuf[(k - 1) & 1], st->max_iter};
}

__device__ __forceinline__ Decision decide_from(const DecideIn &in, long long k, const double t[4])
{
    Decision d{0.0, 0, RL_OK};
    const double ss = t[0], sy = t[1], yy = t[2], res = t[3];
    if (!isfinite(ss) || !isfinite(sy) || !isfinite(yy) || !isfinite(res)) {
        d.stop = 1;
        d.status = RL_ERR_NONFINITE;
    } else if (res <= in.tol) {
        d.stop = 1;
        d.status = RL_OK;
    } else if (ss == 0.0) {
        d.stop = 1;
        d.status = RL_STAGNATED;
    } else if (k >= in.max_iter) {
        d.stop = 1;
        d.status = RL_NOT_CONVERGED;
    }
    double al = in.aprev;
    if (sy > 0.0) {
        al = ((k - 1) % 2 == 0) ? ss / sy : sy / yy;
        al = al < in.amin ? in.amin : (al > in.amax ? in.amax : al);
    }
    d.alpha = al;
    return d;
}

__device__ __forceinline__ Decision decide(const SolverState *st, const double *abuf, long long k, const double t[4])
{
    return decide_from(decide_in(st, abuf, k), k, t);
}

// Workgroup -> work-tile map that gives each of the eight XCDs (which take
// workgroups round-robin) a contiguous range of tiles, so that the rods and
// constraints one XCD works on are neighbours in space and share its L2.
__device__ __forceinline__ unsigned xcd_tile(unsigned b, unsigned nblocks)
{
    constexpr unsigned kXcd = 8;
    if (nblocks % kXcd != 0) return b;
    return (b % kXcd) * (nblocks / kXcd) + b / kXcd;
}

// Rounds of a constraint kernel (rw constraints each): XCD x owns the x-th
// eighth of the constraint order and its workgroups sweep it together, band
// after band (workgroup j of the XCD takes round j of each band), so that at
// any moment an XCD works on one stretch of the order.  The partner entries
// that neighbouring workgroups share (the gathered and scattered Q side) are
// then touched while still in that XCD's L2, instead of once per workgroup
// chunk at times far apart.  A workgroup's rounds start at `first`, step by
// `stride` and end before `end`.
struct ConBand {
    int64_t first, stride, end;
};

__device__ __forceinline__ ConBand con_band(unsigned b, unsigned nblocks, int64_t nc, int64_t rw)
{
    constexpr unsigned kXcd = 8;
    if (nblocks % kXcd != 0) return ConBand{(int64_t)b * rw, (int64_t)nblocks * rw, nc};
    const int64_t px = (nc + kXcd - 1) / kXcd, x0 = (int64_t)(b % kXcd) * px;
    return ConBand{x0 + (int64_t)(b / kXcd) * rw, (int64_t)(nblocks / kXcd) * rw, x0 + px < nc ? x0 + px : nc};
}

// ---------------------------------------------------------------------------
// per-rod and per-constraint work of one product (shared by the single and
// the batched solvers)
// ---------------------------------------------------------------------------
template <int MODE>
__device__ __forceinline__ double gamma_prime(double gam, double g, double alpha)
{
    if (MODE == kModeInit) return gam > 0.0 ? gam : 0.0;
    if (MODE == kModeAlpha0) return (gam <= 0.0 && g > 0.0) ? 0.0 : g;
    if (MODE == kModeLoop) {
        const double v = fma(-alpha, g, gam);
        return v > 0.0 ? v : 0.0;
    }
    return gam;
}

// The same step for a bilateral (free) constraint: no projection
// (eq. linearconstraints b: gamma_b may take any sign).
template <int MODE>
__device__ __forceinline__ double gamma_free(double gam, double g, double alpha)
{
    if (MODE == kModeAlpha0) return g;
    if (MODE == kModeLoop) return fma(-alpha, g, gam);
    return gam;
}

// Contact force f = sum +-gamma' e and moment arm sum m = sum +-gamma' s e of
// rod r, split over the LN lanes of the rod and combined by a fixed tree.
// The torque on the rod is dir x m.  A lane takes the records sub,
// sub + LN, ... of each side.  Its first R records of both sides (R rounds)
// are loaded into registers together, before the step-length wait; longer
// lists continue in a loop.  The registers stay live for the
// contact-velocity emission.  Records beyond the rounds are read after the
// wait, read again for the emission (by then often evicted from the L2) and
// hold up their workgroup, so the rounds should cover the rods with more
// contacts than average; each round costs registers and so occupancy.
// Four lanes and three rounds (12 records a side, 4 waves per SIMD) for
// systems with a few constraints per rod (the nematic suspension: 4.7 a side
// on average).  Where the lists are longer (isotropic phi 0.08 with lengths
// up to 1.5: 12 a side on average, where 12 a lane-group re-read 22% of the
// records) the single solves take eight lanes and three rounds (24 a side,
// shorter chains per lane: rod kernel 150.5 -> 127.5 us at 400k rods, FP32
// 94.3 -> 76.6 us), and the batched solve, whose tile tables assume four
// lanes, five rounds (20 a side, 3 waves per SIMD).
constexpr int kRodRounds = 3;
constexpr int kRodRoundsDense = 5;
constexpr int kRodLanesDense = 8;
// dense systems: above 8 constraints per rod
inline bool rod_dense(int64_t n, int64_t nc) { return nc > 8 * n; }

struct RodRec {
    double2 s, g0, g1;  // (gamma, g), (ex, ey), (ez, s)
};

template <int R = kRodRounds>
struct RodLoads {
    int pb, pe, qb, qe;
    int ps, qs;  // general constraint sets: first bilateral record of each side
    RodRec p[R], q[R];  // the first rounds of the P and Q sides
};

// A lane past its rod's list reads a record of zeros instead of branching
// around the loads: unconditional loads let the compiler's wait counts follow
// each load, so work that needs only earlier loads does not wait for these.
// The array is writable (and never written) so that the compiler cannot fold
// the loads of its zeros into branches.
static __device__ double kZeroRecord[4] = {0.0, 0.0, 0.0, 0.0};

__device__ __forceinline__ void rod_rec_load(const double2 *st, const double *geo, int c, int end, RodRec &R)
{
    const bool ok = c < end;
    const double2 *sp = ok ? st + c : reinterpret_cast<const double2 *>(kZeroRecord);
    const double2 *gd = ok ? reinterpret_cast<const double2 *>(geo + 4 * (int64_t)c)
                           : reinterpret_cast<const double2 *>(kZeroRecord);
    R.s = *sp;
    R.g0 = gd[0];
    R.g1 = gd[1];
}

// The arrays come as separate arguments so that a kernel can take them in
// preloaded registers (leading kernel arguments) instead of from the
// argument block.
template <int LN = kRodLanes, int R>
__device__ __forceinline__ void rod_load(const int32_t *pptr, const int32_t *qptr, const double2 *st,
                                         const double2 *stq, const double *geo, const double *qgeo, int64_t r,
                                         bool active, int sub, RodLoads<R> &L)
{
    L.ps = L.qs = 0x7fffffff;
    // an inactive lane reads rod 0's offsets (n >= 1) and keeps an empty list
    const int64_t rr = active ? r : 0;
    const int pb = pptr[rr], pe = pptr[rr + 1], qb = qptr[rr], qe = qptr[rr + 1];
    L.pb = active ? pb + sub : 0;
    L.pe = active ? pe : 0;
    L.qb = active ? qb + sub : 0;
    L.qe = active ? qe : 0;
#pragma unroll
    for (int i = 0; i < R; ++i) {
        rod_rec_load(st, geo, L.pb + i * LN, L.pe, L.p[i]);
        rod_rec_load(stq, qgeo, L.qb + i * LN, L.qe, L.q[i]);
    }
}

template <int R>
__device__ __forceinline__ void rod_load(const SolveArgs &a, int64_t r, bool active, int sub, RodLoads<R> &L)
{
    rod_load(a.pptr, a.qptr, a.st, a.stq, a.geo, a.qgeo, r, active, sub, L);
}

// general constraint sets: a rod's records are unilateral before ps (P side,
// constraint index) and qs (Q side, list position), bilateral from there on
template <int R>
__device__ __forceinline__ void rod_load_split(const SolveArgs &a, int64_t r, bool active, RodLoads<R> &L)
{
    if (active) {
        L.ps = a.psplit[r];
        L.qs = a.qsplit[r];
    }
}

// f += +-gamma' e, m += +-gamma' s e for one incidence record
__device__ __forceinline__ void rod_add(double sign, double gm, double2 g0, double2 g1, double f[3], double m[3])
{
    const double gv = sign * gm, gs = gv * g1.y;
    f[0] += gv * g0.x;
    f[1] += gv * g0.y;
    f[2] += gv * g1.x;
    m[0] += gs * g0.x;
    m[1] += gs * g0.y;
    m[2] += gs * g1.x;
}

template <int MODE, bool BIL>
__device__ __forceinline__ double gamma_of(double gam, double g, double alpha, int c, int split)
{
    if (BIL && c >= split) return gamma_free<MODE>(gam, g, alpha);
    return gamma_prime<MODE>(gam, g, alpha);
}

template <int MODE, bool BIL, int R, int LN>
__device__ __forceinline__ void rod_side(double sign, const double2 *st, const double *geo, int b, int e, int split,
                                         const RodRec *rr, double alpha, double f[3], double m[3])
{
#pragma unroll
    for (int i = 0; i < R; ++i) {
        const int c = b + i * LN;
        if (c >= e) return;
        rod_add(sign, gamma_of<MODE, BIL>(rr[i].s.x, rr[i].s.y, alpha, c, split), rr[i].g0, rr[i].g1, f, m);
    }
    for (int c = b + R * LN; c < e; c += LN) {
        const double2 sg = st[c];
        const double2 *gd = reinterpret_cast<const double2 *>(geo + 4 * (int64_t)c);
        rod_add(sign, gamma_of<MODE, BIL>(sg.x, sg.y, alpha, c, split), gd[0], gd[1], f, m);
    }
}

template <int MODE, bool BIL = false, int LN = kRodLanes, int R>
__device__ __forceinline__ void rod_accumulate(const SolveArgs &a, const RodLoads<R> &L, double alpha, double f[3],
                                               double m[3])
{
    f[0] = f[1] = f[2] = m[0] = m[1] = m[2] = 0.0;
    rod_side<MODE, BIL, R, LN>(1.0, a.st, a.geo, L.pb, L.pe, L.ps, L.p, alpha, f, m);
    rod_side<MODE, BIL, R, LN>(-1.0, a.stq, a.qgeo, L.qb, L.qe, L.qs, L.q, alpha, f, m);
#pragma unroll
    for (int o = 1; o < LN; o <<= 1) {
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            f[d] += __shfl_xor(f[d], o, 64);
            m[d] += __shfl_xor(m[d], o, 64);
        }
    }
}

__device__ __forceinline__ void rod_mob(const SolveArgs &a, int64_t r, bool uni, double &apar, double &aperp,
                                        double &rperp)
{
    if (uni) {
        apar = a.mob.apar;
        aperp = a.mob.aperp;
        rperp = a.mob.rperp;
    } else {
        apar = a.coef[3 * r];
        aperp = a.coef[3 * r + 1];
        rperp = a.coef[3 * r + 2];
    }
}

// The rest of one constraint's update once its rate w = D_c^T (V, W) is
// known (w without q): by mode, the product, the start state, the Cauchy-step
// dot products, the FP64 refresh, or one BBPGD step with its BB dot products
// and natural residual.
template <int MODE>
__device__ __forceinline__ void con_apply(const SolveArgs &a, int64_t c, double w, double q, double2 sg, int qp,
                                          double alpha, double p[4])
{
    if (MODE == kModeApply) {
        a.out[c] = w + q;
    } else if (MODE == kModeInit) {
        w += q;
        const double gp = gamma_prime<kModeInit>(sg.x, 0.0, 0.0);
        a.st[c] = make_double2(gp, w);
        a.stq[qp] = make_double2(gp, w);
        p[2] += w * w;
        p[3] = fmax(p[3], fabs(gp < w ? gp : w));
    } else if (MODE == kModeAlpha0) {
        const double gh = gamma_prime<kModeAlpha0>(sg.x, sg.y, 0.0);
        p[0] += gh * gh;
        p[1] += gh * w;
    } else if (MODE == kModeRefresh) {
        // FP64 gradient of the accumulated iterate; the FP32 correction restarts at 0
        w += q;
        const double gp = gamma_prime<kModeInit>(sg.x, 0.0, 0.0);
        a.st[c] = make_double2(gp, w);
        a.stq[qp] = make_double2(gp, w);
        const float hw = (float)w, bg = -(float)gp;
        a.st32[c] = make_float4(0.0f, hw, bg, hw);
        a.stq32[qp] = make_float4(0.0f, hw, bg, 0.0f);
        p[2] += w * w;
        p[3] = fmax(p[3], fabs(gp < w ? gp : w));
    } else {
        w += q;
        const double gp = gamma_prime<kModeLoop>(sg.x, sg.y, alpha);
        const double sc = gp - sg.x, yc = w - sg.y;
        a.st[c] = make_double2(gp, w);
        a.stq[qp] = make_double2(gp, w);
        p[0] += sc * sc;
        p[1] += sc * yc;
        p[2] += yc * yc;
        p[3] = fmax(p[3], fabs(gp < w ? gp : w));
    }
}

// The same for a general constraint set (FP64): cm >= 0 marks a bilateral
// constraint with compliance cm (its row of Mc has cm added on the diagonal,
// eq. blockdef block F; gamma is not projected and the residual is |w|);
// cm < 0 a unilateral one.  qp < 0: no Q side (a fixed body).
template <int MODE>
__device__ __forceinline__ void con_apply_gen(const SolveArgs &a, int64_t c, double w, double q, double2 sg, int qp,
                                              double cm, double alpha, double p[4])
{
    const bool bil = cm >= 0.0;
    if (MODE == kModeApply) {
        a.out[c] = w + q + (bil ? cm * sg.x : 0.0);
        return;
    }
    if (MODE == kModeAlpha0) {
        const double gh = bil ? sg.y : gamma_prime<kModeAlpha0>(sg.x, sg.y, 0.0);
        p[0] += gh * gh;
        p[1] += gh * (w + (bil ? cm * gh : 0.0));
        return;
    }
    const double gp = MODE == kModeInit ? (bil ? sg.x : gamma_prime<kModeInit>(sg.x, 0.0, 0.0))
                                        : (bil ? gamma_free<kModeLoop>(sg.x, sg.y, alpha)
                                               : gamma_prime<kModeLoop>(sg.x, sg.y, alpha));
    w += q + (bil ? cm * gp : 0.0);
    a.st[c] = make_double2(gp, w);
    if (qp >= 0) a.stq[qp] = make_double2(gp, w);
    const double r = bil ? fabs(w) : fabs(gp < w ? gp : w);
    if (MODE == kModeInit) {
        p[2] += w * w;
    } else {
        const double sc = gp - sg.x, yc = w - sg.y;
        p[0] += sc * sc;
        p[1] += sc * yc;
        p[2] += yc * yc;
    }
    p[3] = fmax(p[3], r);
}

// ---------------------------------------------------------------------------
// contact-velocity form: the rod kernel projects its rod's
// (V, W) onto e at every contact point it takes part in, u = e.(V + s W), so
// the constraint side reads two numbers instead of gathering two rods' six
// and the geometry: w = u_P - u_Q.
// ---------------------------------------------------------------------------
__device__ __forceinline__ double u_along(double2 g0, double2 g1, const double v[3], const double w[3])
{
    const double s = g1.y;
    return g0.x * (v[0] + s * w[0]) + g0.y * (v[1] + s * w[1]) + g1.x * (v[2] + s * w[2]);
}

// The lane's incidences in the same order as rod_accumulate: the first
// rounds are still in registers, later ones are read again (moments after
// the same lane read them).
template <int R, int LN>
__device__ __forceinline__ void emit_side(double *u, const double *geo, int b, int e, const RodRec *rr,
                                          const double v[3], const double w[3])
{
#pragma unroll
    for (int i = 0; i < R; ++i) {
        if (b + i * LN >= e) return;
        u[b + i * LN] = u_along(rr[i].g0, rr[i].g1, v, w);
    }
    for (int c = b + R * LN; c < e; c += LN) {
        const double2 *gd = reinterpret_cast<const double2 *>(geo + 4 * (int64_t)c);
        u[c] = u_along(gd[0], gd[1], v, w);
    }
}

template <int LN = kRodLanes, int R>
__device__ __forceinline__ void rod_emit_u(const SolveArgs &a, const RodLoads<R> &L, const double v[3],
                                           const double w[3])
{
    emit_side<R, LN>(a.uP, a.geo, L.pb, L.pe, L.p, v, w);
    emit_side<R, LN>(a.uQ, a.qgeo, L.qb, L.qe, L.q, v, w);
}

struct ConLoadsU {
    double2 sg;
    double q, up, uq;
    double cm;  // general sets: compliance (bilateral) or -1 (unilateral)
    int qp;
};

// The constraint side's inputs; like rod_load, the arrays may come from
// preloaded kernel arguments.
struct ConIn {
    const int32_t *qpos;
    const double *uP, *qv;
    const double2 *st;
    const double *uQ;
};

template <int MODE>
__device__ __forceinline__ void con_load_u(const ConIn &in, int64_t c, ConLoadsU &L)
{
    L.qp = in.qpos[c];
    L.up = in.uP[c];
    L.q = in.qv[c];
    if (MODE != kModeApply) L.sg = in.st[c];
    L.uq = in.uQ[L.qp];
}

template <int MODE>
__device__ __forceinline__ void con_load_u(const SolveArgs &a, int64_t c, ConLoadsU &L)
{
    con_load_u<MODE>(ConIn{a.qpos, a.uP, a.qv, a.st, a.uQ}, c, L);
}

// general sets: every mode reads the state (the compliance term needs
// gamma), a constraint without a Q side reads no u_Q
__device__ __forceinline__ void con_load_gen(const ConIn &in, const double *cmpv, int64_t c, ConLoadsU &L)
{
    L.qp = in.qpos[c];
    L.up = in.uP[c];
    L.q = in.qv[c];
    L.sg = in.st[c];
    L.cm = cmpv[c];
    L.uq = L.qp >= 0 ? in.uQ[L.qp] : 0.0;
}

template <int MODE>
__device__ __forceinline__ void con_update_u(const SolveArgs &a, int64_t c, const ConLoadsU &L, double alpha,
                                             double p[4])
{
    con_apply<MODE>(a, c, L.up - L.uq, L.q, L.sg, L.qp, alpha, p);
}

template <int MODE>
__device__ __forceinline__ void con_update_gen(const SolveArgs &a, int64_t c, const ConLoadsU &L, double alpha,
                                               double p[4])
{
    con_apply_gen<MODE>(a, c, L.up - L.uq, L.q, L.sg, L.qp, L.cm, alpha, p);
}

}  // namespace rl
