// Device helpers shared by the FP64 and the mixed-precision BBPGD kernels:
// fixed-order wave and workgroup reductions, the step-length / stop rule,
// and the XCD-aware tile map.
#pragma once

#include "rl_internal.hpp"

namespace rl {

__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}
__device__ __forceinline__ double wave_max(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
    return v;
}

// Sums p[0..2] and takes the max of p[3] over the workgroup (fixed tree);
// every thread receives the result.  lds holds NW x 4 doubles plus 4.
template <int NW>
__device__ __forceinline__ void block_reduce4_all(double p[4], double (*lds)[4])
{
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    p[0] = wave_sum(p[0]);
    p[1] = wave_sum(p[1]);
    p[2] = wave_sum(p[2]);
    p[3] = wave_max(p[3]);
    if (lane == 0) {
        lds[wid][0] = p[0];
        lds[wid][1] = p[1];
        lds[wid][2] = p[2];
        lds[wid][3] = p[3];
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < NW; ++w) {
            p[0] += lds[w][0];
            p[1] += lds[w][1];
            p[2] += lds[w][2];
            p[3] = fmax(p[3], lds[w][3]);
        }
        lds[NW][0] = p[0];
        lds[NW][1] = p[1];
        lds[NW][2] = p[2];
        lds[NW][3] = p[3];
    }
    __syncthreads();
    p[0] = lds[NW][0];
    p[1] = lds[NW][1];
    p[2] = lds[NW][2];
    p[3] = lds[NW][3];
    __syncthreads();
}

// Totals of the gcon workgroup partials at `P`, identical in every workgroup.
template <int NW>
__device__ __forceinline__ void sum_partials(const double *__restrict__ P, int gcon, double p[4], double (*lds)[4])
{
    p[0] = p[1] = p[2] = p[3] = 0.0;
    for (int b = threadIdx.x; b < gcon; b += blockDim.x) {
        const double2 *src = reinterpret_cast<const double2 *>(P + 4 * (int64_t)b);
        const double2 u = src[0], v = src[1];
        p[0] += u.x;
        p[1] += u.y;
        p[2] += v.x;
        p[3] = fmax(p[3], v.y);
    }
    block_reduce4_all<NW>(p, lds);
}

// Stop test and step length for iteration k >= 1 from the totals of
// iteration k-1 (s.s, s.y, y.y, residual); status RL_OK / NOT_CONVERGED /
// STAGNATED / ERR_NONFINITE when stopping.
struct Decision {
    double alpha;
    int stop, status;
};

// st: the system's state; abuf: its two step lengths by iteration parity
__device__ __forceinline__ Decision decide(const SolverState *st, const double *abuf, long long k, const double t[4])
{
    Decision d{0.0, 0, RL_OK};
    const double ss = t[0], sy = t[1], yy = t[2], res = t[3];
    if (!isfinite(ss) || !isfinite(sy) || !isfinite(yy) || !isfinite(res)) {
        d.stop = 1;
        d.status = RL_ERR_NONFINITE;
    } else if (res <= st->tol) {
        d.stop = 1;
        d.status = RL_OK;
    } else if (ss == 0.0) {
        d.stop = 1;
        d.status = RL_STAGNATED;
    } else if (k >= st->max_iter) {
        d.stop = 1;
        d.status = RL_NOT_CONVERGED;
    }
    double al = abuf[(k - 1) & 1];
    if (sy > 0.0) {
        al = ((k - 1) % 2 == 0) ? ss / sy : sy / yy;
        al = al < st->amin ? st->amin : (al > st->amax ? st->amax : al);
    }
    d.alpha = al;
    return d;
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

// Contact force f = sum +-gamma' e and moment arm sum m = sum +-gamma' s e of
// rod r, split over the four lanes of the rod and combined by a fixed tree.
// The torque on the rod is dir x m.  The first P-side and the first Q-side
// record of each lane are loaded together (one memory round for almost every
// rod: a lane holds up to four incidences per side in its first round);
// longer lists continue in a loop.
struct RodLoads {
    int pb, pe, qb, qe;
    double2 ps, pg0, pg1;  // first P record: (gamma, g), (ex, ey), (ez, s_i)
    double2 qs, qg0, qg1;  // first Q record: (gamma, g), (ex, ey), (ez, s_j)
};

__device__ __forceinline__ void rod_load(const SolveArgs &a, int64_t r, bool active, int sub, RodLoads &L)
{
    L.pb = L.pe = L.qb = L.qe = 0;
    if (active) {
        L.pb = a.pptr[r] + sub;
        L.pe = a.pptr[r + 1];
        L.qb = a.qptr[r] + sub;
        L.qe = a.qptr[r + 1];
    }
    const double2 z = make_double2(0.0, 0.0);
    L.ps = L.pg0 = L.pg1 = L.qs = L.qg0 = L.qg1 = z;
    if (L.pb < L.pe) {
        const double2 *gd = reinterpret_cast<const double2 *>(a.geo + 4 * (int64_t)L.pb);
        L.ps = a.st[L.pb];
        L.pg0 = gd[0];
        L.pg1 = gd[1];
    }
    if (L.qb < L.qe) {
        const double2 *gd = reinterpret_cast<const double2 *>(a.qgeo + 4 * (int64_t)L.qb);
        L.qs = a.stq[L.qb];
        L.qg0 = gd[0];
        L.qg1 = gd[1];
    }
}

template <int MODE>
__device__ __forceinline__ void rod_accumulate(const SolveArgs &a, const RodLoads &L, double alpha, double f[3],
                                               double m[3])
{
    f[0] = f[1] = f[2] = m[0] = m[1] = m[2] = 0.0;
    if (L.pb < L.pe) {
        const double gm = gamma_prime<MODE>(L.ps.x, L.ps.y, alpha);
        const double gs = gm * L.pg1.y;
        f[0] += gm * L.pg0.x;
        f[1] += gm * L.pg0.y;
        f[2] += gm * L.pg1.x;
        m[0] += gs * L.pg0.x;
        m[1] += gs * L.pg0.y;
        m[2] += gs * L.pg1.x;
        for (int c = L.pb + kRodLanes; c < L.pe; c += kRodLanes) {
            const double2 sg = a.st[c];
            const double2 *gd = reinterpret_cast<const double2 *>(a.geo + 4 * (int64_t)c);
            const double2 g0 = gd[0], g1 = gd[1];
            const double gmc = gamma_prime<MODE>(sg.x, sg.y, alpha);
            const double gsc = gmc * g1.y;
            f[0] += gmc * g0.x;
            f[1] += gmc * g0.y;
            f[2] += gmc * g1.x;
            m[0] += gsc * g0.x;
            m[1] += gsc * g0.y;
            m[2] += gsc * g1.x;
        }
    }
    if (L.qb < L.qe) {
        const double gm = gamma_prime<MODE>(L.qs.x, L.qs.y, alpha);
        const double gs = gm * L.qg1.y;
        f[0] -= gm * L.qg0.x;
        f[1] -= gm * L.qg0.y;
        f[2] -= gm * L.qg1.x;
        m[0] -= gs * L.qg0.x;
        m[1] -= gs * L.qg0.y;
        m[2] -= gs * L.qg1.x;
        for (int k = L.qb + kRodLanes; k < L.qe; k += kRodLanes) {
            const double2 sg = a.stq[k];
            const double2 *gd = reinterpret_cast<const double2 *>(a.qgeo + 4 * (int64_t)k);
            const double2 g0 = gd[0], g1 = gd[1];
            const double gmc = gamma_prime<MODE>(sg.x, sg.y, alpha);
            const double gsc = gmc * g1.y;
            f[0] -= gmc * g0.x;
            f[1] -= gmc * g0.y;
            f[2] -= gmc * g1.x;
            m[0] -= gsc * g0.x;
            m[1] -= gsc * g0.y;
            m[2] -= gsc * g1.x;
        }
    }
#pragma unroll
    for (int o = 1; o < kRodLanes; o <<= 1) {
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

// One constraint: w = e.(V_i + s_i W_i - V_j - s_j W_j) (+ q), from records
// loaded beforehand so that two constraints' gathers are in flight at once.
struct ConLoads {
    double2 g0, g1, g2, sg;
    int qp;
    double2 i0, i1, i2, j0, j1, j2;
};

template <int MODE>
__device__ __forceinline__ void con_load(const SolveArgs &a, int64_t c, ConLoads &L)
{
    const int2 ij = a.pp[c];
    const double2 *gd = reinterpret_cast<const double2 *>(a.geo + 4 * c);
    L.g0 = gd[0];
    L.g1 = gd[1];
    L.g2 = a.geo2[c];
    if (MODE != kModeApply) L.sg = a.st[c];
    if (MODE == kModeInit || MODE == kModeLoop || MODE == kModeRefresh) L.qp = a.qpos[c];
    const double2 *Vi = reinterpret_cast<const double2 *>(a.V + 6 * (int64_t)ij.x);
    const double2 *Vj = reinterpret_cast<const double2 *>(a.V + 6 * (int64_t)ij.y);
    L.i0 = Vi[0];
    L.i1 = Vi[1];
    L.i2 = Vi[2];
    L.j0 = Vj[0];
    L.j1 = Vj[1];
    L.j2 = Vj[2];
}

template <int MODE>
__device__ __forceinline__ void con_update(const SolveArgs &a, int64_t c, const ConLoads &L, double alpha,
                                           double p[4])
{
    const double si = L.g1.y, sj = L.g2.x;
    // velocity of the contact point on i minus that on j, along e
    const double ux = (L.i0.x + si * L.i1.y) - (L.j0.x + sj * L.j1.y);
    const double uy = (L.i0.y + si * L.i2.x) - (L.j0.y + sj * L.j2.x);
    const double uz = (L.i1.x + si * L.i2.y) - (L.j1.x + sj * L.j2.y);
    double w = L.g0.x * ux + L.g0.y * uy + L.g1.x * uz;
    if (MODE == kModeApply) {
        a.out[c] = w + L.g2.y;
    } else if (MODE == kModeInit) {
        w += L.g2.y;
        const double gp = gamma_prime<kModeInit>(L.sg.x, 0.0, 0.0);
        a.st[c] = make_double2(gp, w);
        a.stq[L.qp] = make_double2(gp, w);
        p[2] += w * w;
        p[3] = fmax(p[3], fabs(gp < w ? gp : w));
    } else if (MODE == kModeAlpha0) {
        const double gh = gamma_prime<kModeAlpha0>(L.sg.x, L.sg.y, 0.0);
        p[0] += gh * gh;
        p[1] += gh * w;
    } else if (MODE == kModeRefresh) {
        // FP64 gradient of the accumulated iterate; the FP32 correction restarts at 0
        w += L.g2.y;
        const double gp = gamma_prime<kModeInit>(L.sg.x, 0.0, 0.0);
        a.st[c] = make_double2(gp, w);
        a.stq[L.qp] = make_double2(gp, w);
        const float hw = (float)w, bg = -(float)gp;
        a.st32[c] = make_float4(0.0f, hw, bg, hw);
        a.stq32[L.qp] = make_float4(0.0f, hw, bg, 0.0f);
        p[2] += w * w;
        p[3] = fmax(p[3], fabs(gp < w ? gp : w));
    } else {
        w += L.g2.y;
        const double gp = gamma_prime<kModeLoop>(L.sg.x, L.sg.y, alpha);
        const double sc = gp - L.sg.x, yc = w - L.sg.y;
        a.st[c] = make_double2(gp, w);
        a.stq[L.qp] = make_double2(gp, w);
        p[0] += sc * sc;
        p[1] += sc * yc;
        p[2] += yc * yc;
        p[3] = fmax(p[3], fabs(gp < w ? gp : w));
    }
}

}  // namespace rl
