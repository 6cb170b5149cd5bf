// BBPGD solve of the unilateral constraint problem on gfx950.
//
// The problem is min 1/2 gamma^T Mc gamma + q^T gamma, gamma >= 0, with
// Mc = D^T M D (eq. cqpdef / suppcqpdef; eq. blockdef, block B).  Each
// iteration needs one product Mc gamma, done matrix-free by two kernels:
//
//   rod kernel (four lanes per rod): the contact force D gamma' on the rod,
//     summed over the constraints it takes part in (P side: contiguous range
//     of the pi-sorted list; Q side: incidence list), and the mobility
//     applied in registers: V = M_t F_c and W = Omega_c x dir, so that the
//     velocity of the axis point at arclength s is V + s W.  It then writes,
//     for every contact the rod takes part in, that point's velocity along
//     the contact normal, u = e.(V + s W) (P side in constraint order, Q side
//     in incidence-list order).
//   constraint kernel (contiguous chunk per workgroup, two constraints per
//     lane per round): w = u_P - u_Q + q, the projection, the BB dot products
//     and the natural residual, reduced to one partial per workgroup.  It
//     reads no geometry and gathers no rod data, only u_Q through the
//     constraint's position in the incidence list.
//
// No workgroup ever waits for another inside a launch, so there are no
// device-scope fences in the loop (each one flushes and invalidates the L2
// of the issuing XCD).  Instead every workgroup of the next rod kernel sums
// the previous iteration's partials itself, in a fixed order, and so reaches
// the same step length and stop decision; workgroup 0 publishes them for the
// constraint kernel and latches the stop.  Partials are double-buffered by
// iteration parity.  All sums run in a fixed order (no floating-point
// atomics), so results are bitwise repeatable.
//
// The BB iteration follows Barzilai & Borwein (1988) in its projected form
// (Dai & Fletcher 2005): the paper names the method (Section "Instantiation
// in a massively parallel computing environment"; Appendix
// "Implementation") and leaves its details to earlier work.  Start:
// g0 = Mc gamma0 + q; alpha0 = gh.gh / gh.Mc gh on the projected gradient gh.
// Step k: gamma' = max(0, gamma - alpha g), g' = Mc gamma' + q, stop when
// max |min(gamma', g')| <= tol; s = gamma' - gamma, y = g' - g; alpha =
// s.s/s.y (k even) or s.y/y.y (k odd) when s.y > 0, clamped to
// [1e-12, 1e12] * alpha0.
#include <hip/hip_ext.h>

#include <algorithm>
#include <cmath>
#include <vector>

#include "rl_device.hpp"

namespace rl {

static inline unsigned grid_of(int64_t n, int block) { return (unsigned)((n + block - 1) / block); }
static inline unsigned grid_of(int64_t n) { return grid_of(n, kBlock); }

// ---------------------------------------------------------------------------
// incidence structure and packing
// ---------------------------------------------------------------------------
// Checks 0 <= pi <= pj < n and pi non-decreasing; writes pptr[r] = first c
// with pi[c] >= r (pptr[n] = nc).
__global__ void k_check_pairs(int64_t n, int64_t nc, const int32_t *__restrict__ pi, const int32_t *__restrict__ pj,
                              int32_t *__restrict__ pptr, int *__restrict__ err)
{
    const int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (c > nc) return;
    if (c == nc) {
        // rods after the last constraint's pi (an invalid pi is reported by its own thread)
        int64_t last = nc > 0 ? (int64_t)pi[nc - 1] : -1;
        if (last < -1) last = -1;
        for (int64_t r = last + 1; r <= n; ++r) pptr[r] = (int32_t)nc;
        return;
    }
    const int64_t a = pi[c], b = pj[c];
    if (a < 0 || b >= n || a > b) {
        atomicOr(err, 1);
        return;
    }
    int64_t prev = c > 0 ? (int64_t)pi[c - 1] : -1;
    if (prev > a) {
        atomicOr(err, 2);
        return;
    }
    if (prev < -1) prev = -1;
    for (int64_t r = prev + 1; r <= a; ++r) pptr[r] = (int32_t)c;
}

__global__ void k_qcount(int64_t nc, const int32_t *__restrict__ pj, int *__restrict__ qcnt)
{
    const int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (c >= nc) return;
    atomicAdd(qcnt + pj[c], 1);
}

__global__ void k_qfill(int64_t nc, const int32_t *__restrict__ pj, const int32_t *__restrict__ qptr,
                        int *__restrict__ qcur, int32_t *__restrict__ qidx)
{
    const int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (c >= nc) return;
    const int r = pj[c];
    qidx[qptr[r] + atomicAdd(qcur + r, 1)] = (int32_t)c;
}

// ascending constraint order inside each rod's Q-side list (fixes the
// summation order of the rod kernel)
__global__ void k_qsort(int64_t n, const int32_t *__restrict__ qptr, int32_t *__restrict__ qidx)
{
    const int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (r >= n) return;
    const int b = qptr[r], e = qptr[r + 1];
    for (int k = b + 1; k < e; ++k) {
        const int32_t v = qidx[k];
        int m = k - 1;
        while (m >= b && qidx[m] > v) {
            qidx[m + 1] = qidx[m];
            --m;
        }
        qidx[m + 1] = v;
    }
}

// constraint records: (pi, pj), (ex, ey, ez, s_i) and (s_j, q), q alone,
// (gamma, g = 0)
__global__ void k_pack(int64_t nc, const int32_t *__restrict__ pi, const int32_t *__restrict__ pj,
                       const double *__restrict__ e, const double *__restrict__ arm, const double *__restrict__ q,
                       const double *__restrict__ gamma, int2 *__restrict__ pp, double *__restrict__ geo,
                       double2 *__restrict__ geo2, double *__restrict__ qv, double2 *__restrict__ st)
{
    const int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (c >= nc) return;
    pp[c] = make_int2(pi[c], pj[c]);
    double2 *gd = reinterpret_cast<double2 *>(geo + 4 * c);
    gd[0] = make_double2(e[3 * c], e[3 * c + 1]);
    gd[1] = make_double2(e[3 * c + 2], arm[2 * c]);
    const double qc = q ? q[c] : 0.0;
    geo2[c] = make_double2(arm[2 * c + 1], qc);
    qv[c] = qc;
    st[c] = make_double2(gamma[c], 0.0);
}

// Q-side copies: qpos (inverse of qidx), the geometry a rod needs on its Q
// side in list order, and the start iterate in list order
__global__ void k_pack_q(int64_t nc, const int32_t *__restrict__ qidx, const double *__restrict__ geo,
                         const double2 *__restrict__ geo2, const double2 *__restrict__ st, int32_t *__restrict__ qpos,
                         double *__restrict__ qgeo, double2 *__restrict__ stq)
{
    const int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (k >= nc) return;
    const int c = qidx[k];
    qpos[c] = (int32_t)k;
    const double2 *gd = reinterpret_cast<const double2 *>(geo + 4 * (int64_t)c);
    const double2 g0 = gd[0], g1 = gd[1];
    double2 *qd = reinterpret_cast<double2 *>(qgeo + 4 * k);
    qd[0] = g0;
    qd[1] = make_double2(g1.x, geo2[c].x);
    stq[k] = st[c];
}

__global__ void k_unpack_gamma(int64_t nc, const double2 *__restrict__ st, double *__restrict__ gamma)
{
    const int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (c >= nc) return;
    gamma[c] = st[c].x;
}


// The loop's progress for the host: one relaxed store at system scope to a
// word of coherent pinned host memory (a vector store; the host only polls it).
__device__ __forceinline__ void report_progress(unsigned long long *w, long long k, bool stop)
{
    if (w) __hip_atomic_store(w, 2ull * (unsigned long long)k + (stop ? 1ull : 0ull), __ATOMIC_RELAXED,
                              __HIP_MEMORY_SCOPE_SYSTEM);
}

// The arrays and sizes that the first loads need lead the argument list
// (pptr, qptr, st, stq, geo, qgeo, grid size, n: 14 dwords, what the
// hardware can preload into registers besides the argument block's address),
// so that the first loads do not wait for the argument block.
template <int MODE, bool UNI, bool BIL, int R, int LN>
__global__ void __launch_bounds__(kRodLoopBlock)
    k_rod(const int32_t *__restrict__ pptr, const int32_t *__restrict__ qptr, const double2 *st, const double2 *stq,
          const double *__restrict__ geo, const double *__restrict__ qgeo, unsigned nblk, int n, SolveArgs a,
          long long k)
{
    __shared__ double lds[kRodLoopBlock / 64 + 1][4];
    double alpha = 0.0;
    const int sub = threadIdx.x & (LN - 1);
    const unsigned tile = xcd_tile(blockIdx.x, nblk);
    const int64_t r = (int64_t)tile * (kRodLoopBlock / LN) + (threadIdx.x / LN);
    const bool active = r < n;
    // The previous iteration's partials, the inputs of the step rule and the
    // stop flag go out first (the partials are read for nothing at k = 0),
    // then the incidence records, which depend neither on the step length nor
    // on the flag (after the stop they are read for nothing).  All loads are
    // unconditional, so the step-length reduction waits only for the first
    // group and runs while the records are in flight.
    const double *part = a.partial + (int64_t)((k - 1) & 1) * a.gcon * 4;
    PartFirst pf;
    if (MODE == kModeLoop) partials_first_split<kRodLoopBlock>(part, a.gcon, pf);
    DecideIn din{};
    if (MODE == kModeLoop) din = decide_in(a.state, a.alpha_buf, k);
    const int done = MODE != kModeApply ? a.state->done : 0;
    // a compiler barrier keeps those loads ahead of the records'
    __asm__ volatile("" ::: "memory");
    RodLoads<R> L;
    rod_load<LN>(pptr, qptr, st, stq, geo, qgeo, r, active, sub, L);
    if (BIL) rod_load_split(a, r, active, L);
    // and the rod's direction and mobility, which the reduction does not need
    const int64_t rr = active ? r : 0;
    const double dx = a.dir[3 * rr], dy = a.dir[3 * rr + 1], dz = a.dir[3 * rr + 2];
    double apar, aperp, rperp;
    rod_mob(a, rr, UNI, apar, aperp, rperp);
    // and a second barrier keeps all of them ahead of the stop test (the
    // compiler would otherwise move them past it, behind the flag's latency)
    __asm__ volatile("" ::: "memory");
    const bool lead = blockIdx.x == 0 && threadIdx.x == 0;
    if (MODE != kModeApply && done) {
        if (MODE == kModeLoop && lead) report_progress(a.progress, k, true);
        return;
    }
    if (MODE == kModeLoop) {
        if (k == 0) {
            alpha = a.state->alpha;
            if (lead) {
                a.alpha_buf[0] = alpha;
                report_progress(a.progress, 0, false);
            }
        } else {
            double t[4];
            sum_partials_split_from<kRodLoopBlock / 64>(pf, part, a.gcon, t, lds);
            const Decision d = decide_from(din, k, t);
            if (lead) {
                report_progress(a.progress, k, d.stop);
                if (d.stop) {
                    SolverState *st = a.state;
                    st->iter = k;
                    st->res = t[3];
                    st->ss = t[0];
                    st->sy = t[1];
                    st->yy = t[2];
                    st->status = d.status;
                    st->done = 1;
                } else {
                    a.alpha_buf[k & 1] = d.alpha;
                }
            }
            if (d.stop) return;
            alpha = d.alpha;
        }
    }
    double f[3], m[3];
    rod_accumulate<MODE, BIL, LN>(a, L, alpha, f, m);
    if (!active) return;
    // translation a_perp f + (a_par - a_perp)(d.f) d; rotation Omega =
    // r_perp dir x m (normal to the axis) and Omega x dir = r_perp (m - (d.m) d)
    const double fd = (apar - aperp) * (dx * f[0] + dy * f[1] + dz * f[2]);
    const double md = dx * m[0] + dy * m[1] + dz * m[2];
    const double v[3] = {aperp * f[0] + fd * dx, aperp * f[1] + fd * dy, aperp * f[2] + fd * dz};
    const double w[3] = {rperp * (m[0] - md * dx), rperp * (m[1] - md * dy), rperp * (m[2] - md * dz)};
    rod_emit_u<LN>(a, L, v, w);
}


// ---------------------------------------------------------------------------
// constraint kernel
// ---------------------------------------------------------------------------
// As in k_rod, what the first loads need leads the argument list (qpos, u_P,
// q, st, u_Q, constraint count, grid size, step lengths: 14 dwords).  CB
// threads per workgroup take CPL constraints each per round.
template <int MODE, int CB, int CPL, bool BIL>
__global__ void __launch_bounds__(CB)
    k_con(const int32_t *__restrict__ qpos, const double *__restrict__ uP, const double *__restrict__ qv,
          const double2 *st, const double *__restrict__ uQ, int nc, unsigned nblk, const double *alpha_buf,
          SolveArgs a, long long k)
{
    __shared__ double lds[CB / 64 + 1][4];
    double p[4] = {0.0, 0.0, 0.0, 0.0};
    const ConIn in{qpos, uP, qv, st, uQ};
    // rounds of CPL constraints per lane, swept band by band per XCD
    const ConBand bd = con_band(blockIdx.x, nblk, nc, (int64_t)CPL * CB);
    const int64_t hi = bd.end;
    int64_t base = bd.first;
    // first round peeled: its records are in flight before the stop flag and
    // the step length are read (every thread reaches the test)
    int64_t c0 = base + threadIdx.x;
    ConLoadsU L[CPL];
#pragma unroll
    for (int u = 0; u < CPL; ++u)
        if (c0 + u * CB < hi) {
            if (BIL) con_load_gen(in, a.cmpv, c0 + u * CB, L[u]);
            else con_load_u<MODE>(in, c0 + u * CB, L[u]);
        }
    // the step length too (read for nothing after the stop)
    const double alpha = MODE == kModeLoop ? alpha_buf[k & 1] : 0.0;
    if (MODE != kModeApply && a.state->done) return;
    for (;;) {
#pragma unroll
        for (int u = 0; u < CPL; ++u)
            if (c0 + u * CB < hi) {
                if (BIL) con_update_gen<MODE>(a, c0 + u * CB, L[u], alpha, p);
                else con_update_u<MODE>(a, c0 + u * CB, L[u], alpha, p);
            }
        base += bd.stride;
        if (base >= hi) break;
        c0 = base + threadIdx.x;
#pragma unroll
        for (int u = 0; u < CPL; ++u)
            if (c0 + u * CB < hi) {
                if (BIL) con_load_gen(in, a.cmpv, c0 + u * CB, L[u]);
                else con_load_u<MODE>(in, c0 + u * CB, L[u]);
            }
    }
    if (MODE == kModeApply) return;
    block_total4<CB / 64>(p, lds);
    if (threadIdx.x == 0) partial_put(a.partial + (int64_t)(k & 1) * a.gcon * 4, a.gcon, blockIdx.x, p);
}

// One workgroup: totals of the start phases (g0 and the Cauchy step).
template <int MODE>
__global__ void __launch_bounds__(kRodBlock) k_fin(SolveArgs a)
{
    __shared__ double lds[kRodBlock / 64 + 1][4];
    SolverState *st = a.state;
    if (st->done && MODE != kModeRefresh) return;
    double t[4];
    sum_partials_split<kRodBlock / 64>(a.partial, a.gcon, t, lds);
    if (threadIdx.x != 0) return;
    if (MODE == kModeRefresh) {
        st->res = t[3];
        st->rho64 = t[3];
        st->refreshes += 1;
        st->refresh = 0;
        if (!isfinite(t[2]) || !isfinite(t[3])) {
            st->status = RL_ERR_NONFINITE;
            st->done = 1;
        } else if (t[3] <= st->tol) {
            st->status = RL_OK;
            st->done = 1;
        } else {
            // next inner round: one order of magnitude, or the tolerance.
            // Longer FP32 rounds drift further from the FP64 path and need
            // more iterations in all: on the dense 400k-rod workload over
            // five seeds, factors 0.3, 0.03, 1e-3 and 1e-4 took 1.10x,
            // 1.27x, 1.66x and 2.38x the iterations of 0.1
            st->inner_tol = fmax(0.5 * st->tol, 1e-1 * t[3]);
        }
        return;
    }
    if (MODE == kModeInit) {
        st->res = t[3];
        if (!isfinite(t[2]) || !isfinite(t[3])) {
            st->status = RL_ERR_NONFINITE;
            st->done = 1;
        } else if (t[3] <= st->tol) {
            st->status = RL_OK;
            st->done = 1;
        }
    } else {
        if (!isfinite(t[0]) || !isfinite(t[1])) {
            st->status = RL_ERR_NONFINITE;
            st->done = 1;
            return;
        }
        if (t[0] == 0.0) {
            st->status = RL_OK;
            st->done = 1;
            return;
        }
        const double a0 = t[1] > 0.0 ? t[0] / t[1] : 1.0;
        st->alpha0 = a0;
        st->alpha = a0;
        st->amin = 1e-12 * a0;
        st->amax = 1e12 * a0;
        if (st->max_iter <= 0) {
            st->status = RL_NOT_CONVERGED;
            st->done = 1;
        }
    }
}

// U = M (D gamma + F) per rod, with the full 6x6 block (external torques may
// have an axial part; the axial rotational mobility equals the normal one).
// `perm` (may be null) maps the solver's rod order to the caller's.
template <bool UNI>
__global__ void __launch_bounds__(kRodBlock) k_velocity(SolveArgs a, const double *__restrict__ F,
                                                        const int *__restrict__ perm, double *__restrict__ U)
{
    const int sub = threadIdx.x & (kRodLanes - 1);
    const int64_t r = (int64_t)blockIdx.x * (kRodBlock / kRodLanes) + (threadIdx.x / kRodLanes);
    const bool active = r < a.n;
    RodLoads<> L;
    rod_load(a, r, active, sub, L);
    double f[3], m[3];
    rod_accumulate<kModeApply>(a, L, 0.0, f, m);
    if (!active || sub != 0) return;
    const int64_t ro = perm ? (int64_t)perm[r] : r;
    const double dx = a.dir[3 * r], dy = a.dir[3 * r + 1], dz = a.dir[3 * r + 2];
    // torque of the contact forces: dir x m
    double tx = dy * m[2] - dz * m[1], ty = dz * m[0] - dx * m[2], tz = dx * m[1] - dy * m[0];
    if (F) {
        f[0] += F[6 * ro];
        f[1] += F[6 * ro + 1];
        f[2] += F[6 * ro + 2];
        tx += F[6 * ro + 3];
        ty += F[6 * ro + 4];
        tz += F[6 * ro + 5];
    }
    double apar, aperp, rperp;
    rod_mob(a, r, UNI, apar, aperp, rperp);
    const double fd = (apar - aperp) * (dx * f[0] + dy * f[1] + dz * f[2]);
    double *u = U + 6 * ro;
    u[0] = aperp * f[0] + fd * dx;
    u[1] = aperp * f[1] + fd * dy;
    u[2] = aperp * f[2] + fd * dz;
    u[3] = rperp * tx;
    u[4] = rperp * ty;
    u[5] = rperp * tz;
}

__global__ void k_state_init(SolverState *st, double tol, long long max_iter)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        st->alpha = st->alpha0 = 0.0;
        st->amin = st->amax = 0.0;
        st->res = st->ss = st->sy = st->yy = 0.0;
        st->tol = tol;
        st->iter = 0;
        st->max_iter = max_iter;
        st->done = 0;
        st->status = RL_OK;
        st->inner_tol = tol;
        st->rho64 = 0.0;
        st->refreshes = 0;
        st->refresh = 0;
    }
}

// mixed precision: gamma64 <- max(0, gamma64 + delta) in both orders
__global__ void k_mix_accum(int64_t nc, const float4 *__restrict__ st32, const int32_t *__restrict__ qpos,
                            double2 *__restrict__ st, double2 *__restrict__ stq)
{
    const int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (c >= nc) return;
    const double v = st[c].x + (double)st32[c].x;
    const double g = v > 0.0 ? v : 0.0;
    st[c].x = g;
    stq[qpos[c]].x = g;
}

// x += h U_t wrapped into [0, box); theta += h Psi(theta) Omega, renormalised;
// xu (may be null) += h U_t without wrapping.
__global__ void k_integrate(int64_t n, const double *__restrict__ U, double *__restrict__ x, double *__restrict__ quat,
                            double *__restrict__ xu, double dt, double b0, double b1, double b2)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double box[3] = {b0, b1, b2};
    for (int a = 0; a < 3; ++a) {
        const double dx = dt * U[6 * i + a];
        double v = x[3 * i + a] + dx;
        v -= box[a] * floor(v / box[a]);
        if (v >= box[a]) v -= box[a];
        x[3 * i + a] = v;
        if (xu) xu[3 * i + a] += dx;
    }
    const double wx = U[6 * i + 3], wy = U[6 * i + 4], wz = U[6 * i + 5];
    double s = quat[4 * i], px = quat[4 * i + 1], py = quat[4 * i + 2], pz = quat[4 * i + 3];
    // Psi(theta) Omega = 1/2 [ -p.Omega ; s Omega - p x Omega ]
    const double ds = -0.5 * (px * wx + py * wy + pz * wz);
    const double dpx = 0.5 * (s * wx - (py * wz - pz * wy));
    const double dpy = 0.5 * (s * wy - (pz * wx - px * wz));
    const double dpz = 0.5 * (s * wz - (px * wy - py * wx));
    s += dt * ds;
    px += dt * dpx;
    py += dt * dpy;
    pz += dt * dpz;
    const double nrm = sqrt(s * s + px * px + py * py + pz * pz);
    quat[4 * i] = s / nrm;
    quat[4 * i + 1] = px / nrm;
    quat[4 * i + 2] = py / nrm;
    quat[4 * i + 3] = pz / nrm;
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
int prepare_solve(rl_ctx *h, int64_t n, const double *dir, const double *len, double len0, int64_t nc,
                  const int32_t *pi, const int32_t *pj, const double *e, const double *arm, const double *q,
                  double *gamma, SolveArgs *out, bool trusted)
{
    hipStream_t st = h->stream;
    const rl_params &p = h->prm;
    int werr = 0;
    SolveArgs s{};
    s.n = n;
    s.nc = nc;
    s.dir = dir;
    s.mob = mobility_host(len ? 1.0 : len0, p.diam, p.eta);
    // constraint workgroups: about kConPerGroup constraints each (every rod
    // workgroup of the next iteration sums one partial per constraint
    // workgroup, so fewer and fuller groups make that sum cheaper), at most
    // kConGridMax, a multiple of 8 (XCDs)
    int64_t gc = std::min<int64_t>(std::max<int64_t>(grid_of(nc, kConPerGroup), 1), kConGridMax);
    // The mixed-precision loop's constraint kernel runs best at one
    // workgroup per CU: at 400k rods, phi 0.08, 68 us per launch from 256
    // workgroups against 84 us from 512 (its FP64 refreshes take the same
    // grid, and the rod kernel sums half the partials)
    if (p.precision == RL_FP32_MIXED) gc = std::min<int64_t>(gc, kConGridMixed);
    s.gcon = (int)((gc + 7) / 8 * 8);
    const int64_t nb = nc > 0 ? nc : 1, rb = n > 0 ? n : 1;
    int32_t *pptr = (int32_t *)ws_get(h, kWsPptr, sizeof(int32_t) * (n + 1), &werr);
    int32_t *qptr = (int32_t *)ws_get(h, kWsQptr, sizeof(int32_t) * (n + 1), &werr);
    int32_t *qidx = (int32_t *)ws_get(h, kWsQidx, sizeof(int32_t) * nb, &werr);
    int *qcnt = (int *)ws_get(h, kWsQcnt, sizeof(int) * rb, &werr);
    int2 *pp = (int2 *)ws_get(h, kWsPP, sizeof(int2) * nb, &werr);
    double *geo = (double *)ws_get(h, kWsGeo, sizeof(double) * 4 * nb, &werr);
    double2 *geo2 = (double2 *)ws_get(h, kWsGeo2, sizeof(double2) * nb, &werr);
    double *qv = (double *)ws_get(h, kWsQv, sizeof(double) * nb, &werr);
    s.uP = (double *)ws_get(h, kWsUP, sizeof(double) * nb, &werr);
    s.uQ = (double *)ws_get(h, kWsUQ, sizeof(double) * nb, &werr);
    s.st = (double2 *)ws_get(h, kWsSt, sizeof(double2) * nb, &werr);
    s.stq = (double2 *)ws_get(h, kWsStq, sizeof(double2) * nb, &werr);
    int32_t *qpos = (int32_t *)ws_get(h, kWsQpos, sizeof(int32_t) * nb, &werr);
    double *qgeo = (double *)ws_get(h, kWsQgeo, sizeof(double) * 4 * nb, &werr);
    s.partial = (double *)ws_get(h, kWsPartial, sizeof(double) * 8 * s.gcon, &werr);
    s.alpha_buf = (double *)ws_get(h, kWsAlpha, sizeof(double) * 2, &werr);
    double *coef = len ? (double *)ws_get(h, kWsCoef, sizeof(double) * 3 * rb, &werr) : nullptr;
    size_t scan_bytes = 0;
    {
        const int rc = scan_tmp_bytes(n, &scan_bytes);
        if (rc) return rc;
    }
    void *scan_tmp = n > 0 ? ws_get(h, kWsScanTmp, scan_bytes, &werr) : nullptr;
    if (werr) return werr;
    s.coef = coef;
    s.pptr = pptr;
    s.qptr = qptr;
    s.qidx = qidx;
    s.pp = pp;
    s.geo = geo;
    s.geo2 = geo2;
    s.qv = qv;
    s.qpos = qpos;
    s.qgeo = qgeo;
    s.state = h->state;
    if (len) RL_HIP(launch_mobility_coeffs(st, n, len, p.diam, p.eta, coef));
    RL_HIP(hipMemsetAsync(h->flag_dev, 0, sizeof(int), st));
    hipLaunchKernelGGL(k_check_pairs, dim3(grid_of(nc + 1)), dim3(kBlock), 0, st, n, nc, pi, pj, pptr, h->flag_dev);
    RL_HIP(hipGetLastError());
    if (!trusted) {
        // a caller's list: its indices must be valid before k_qcount scatters through pj
        RL_HIP(hipMemcpyAsync(h->host_scratch, h->flag_dev, sizeof(int), hipMemcpyDeviceToHost, st));
        RL_HIP(hipStreamSynchronize(st));
        const int ferr = ((int *)h->host_scratch)[0];
        if (ferr) {
            set_error(ferr & 1 ? "pair indices must satisfy 0 <= pi <= pj < n" : "pi must be non-decreasing");
            return RL_ERR_ARG;
        }
    }
    if (n > 0) {
        RL_HIP(hipMemsetAsync(qcnt, 0, sizeof(int) * n, st));
        if (nc > 0) {
            hipLaunchKernelGGL(k_qcount, dim3(grid_of(nc)), dim3(kBlock), 0, st, nc, pj, qcnt);
            RL_HIP(hipGetLastError());
        }
        const int rc = device_scan(h, qcnt, n, qptr, nullptr, scan_tmp);
        if (rc) return rc;
        if (nc > 0) {
            RL_HIP(hipMemsetAsync(qcnt, 0, sizeof(int) * n, st));
            hipLaunchKernelGGL(k_qfill, dim3(grid_of(nc)), dim3(kBlock), 0, st, nc, pj, (const int32_t *)qptr, qcnt,
                               qidx);
            RL_HIP(hipGetLastError());
            hipLaunchKernelGGL(k_qsort, dim3(grid_of(n)), dim3(kBlock), 0, st, n, (const int32_t *)qptr, qidx);
            RL_HIP(hipGetLastError());
        }
    }
    if (nc > 0) {
        hipLaunchKernelGGL(k_pack, dim3(grid_of(nc)), dim3(kBlock), 0, st, nc, pi, pj, e, arm, q,
                           (const double *)gamma, pp, geo, geo2, qv, s.st);
        RL_HIP(hipGetLastError());
        hipLaunchKernelGGL(k_pack_q, dim3(grid_of(nc)), dim3(kBlock), 0, st, nc, (const int32_t *)qidx,
                           (const double *)geo, (const double2 *)geo2, (const double2 *)s.st, qpos, qgeo, s.stq);
        RL_HIP(hipGetLastError());
    }
    *out = s;
    return RL_OK;
}

// the leading arguments of k_rod and k_con
#define RL_ROD_HOT(a, grid) \
    (const int32_t *)(a).pptr, (const int32_t *)(a).qptr, (const double2 *)(a).st, (const double2 *)(a).stq, \
        (const double *)(a).geo, (const double *)(a).qgeo, (unsigned)(grid).x, (int)(a).n
#define RL_CON_HOT(a) \
    (const int32_t *)(a).qpos, (const double *)(a).uP, (const double *)(a).qv, (const double2 *)(a).st, \
        (const double *)(a).uQ, (int)(a).nc, (unsigned)(a).gcon, (const double *)(a).alpha_buf

// rod kernel grid for LN lanes per rod: a multiple of 8 so that each XCD gets a
// contiguous range of rods
static inline unsigned rod_grid(int64_t n, int ln = kRodLanes)
{
    return (grid_of(n, kRodLoopBlock / ln) + 7) / 8 * 8;
}

// the rod kernel with LN lanes per rod and R rounds of records, with
// dispatch-stamped events when e0 is set
template <int MODE, bool BIL, int R, int LN>
static void launch_rod_r(hipStream_t st, const SolveArgs &a, bool uni, long long k, hipEvent_t e0, hipEvent_t e1)
{
    const dim3 grid(rod_grid(a.n, LN));
    if (e0) {
        if (uni)
            hipExtLaunchKernelGGL(HIP_KERNEL_NAME(k_rod<MODE, true, BIL, R, LN>), grid, dim3(kRodLoopBlock), 0, st,
                                  e0, e1, 0, RL_ROD_HOT(a, grid), a, k);
        else
            hipExtLaunchKernelGGL(HIP_KERNEL_NAME(k_rod<MODE, false, BIL, R, LN>), grid, dim3(kRodLoopBlock), 0, st,
                                  e0, e1, 0, RL_ROD_HOT(a, grid), a, k);
    } else {
        if (uni)
            hipLaunchKernelGGL(HIP_KERNEL_NAME(k_rod<MODE, true, BIL, R, LN>), grid, dim3(kRodLoopBlock), 0, st,
                               RL_ROD_HOT(a, grid), a, k);
        else
            hipLaunchKernelGGL(HIP_KERNEL_NAME(k_rod<MODE, false, BIL, R, LN>), grid, dim3(kRodLoopBlock), 0, st,
                               RL_ROD_HOT(a, grid), a, k);
    }
}

// the loop kernel takes eight lanes per rod on dense contact systems (the
// phases that run once per solve keep four, and so do general sets)
template <int MODE, bool BIL>
static void launch_rod_t(hipStream_t st, const SolveArgs &a, bool uni, long long k, hipEvent_t e0 = nullptr,
                         hipEvent_t e1 = nullptr)
{
    if constexpr (MODE == kModeLoop && !BIL) {
        if (rod_dense(a.n, a.nc)) {
            launch_rod_r<MODE, BIL, kRodRounds, kRodLanesDense>(st, a, uni, k, e0, e1);
            return;
        }
    }
    launch_rod_r<MODE, BIL, kRodRounds, kRodLanes>(st, a, uni, k, e0, e1);
}

template <int MODE>
static hipError_t launch_rod(hipStream_t st, const SolveArgs &a, bool uni, long long k)
{
    if (a.n <= 0) return hipSuccess;
    if (a.gen) launch_rod_t<MODE, true>(st, a, uni, k);
    else launch_rod_t<MODE, false>(st, a, uni, k);
    return hipGetLastError();
}

// Constraint kernel shape: while a workgroup's share fits one round of four
// per lane in 512 threads, that; beyond it, eight per lane in 512 threads
// (rounds of 4,096).  Measured on the band sweep: nematic 400k rods (3,673
// per group) 31.8 -> 28.5 us and isotropic phi 0.08 (9,439 per group)
// 95.6 -> 92.1 us against eight per lane in 256 threads; rounds of 3,072
// (six per lane) were slower than either.
static inline bool con_wide(const SolveArgs &a)
{
    const int64_t per = (a.nc + a.gcon - 1) / a.gcon;
    return per > 4 * 512;
}

template <int MODE, bool BIL>
static void launch_con_t(hipStream_t st, const SolveArgs &a, long long k)
{
    if (con_wide(a))
        hipLaunchKernelGGL(HIP_KERNEL_NAME(k_con<MODE, 512, 8, BIL>), dim3(a.gcon), dim3(512), 0, st, RL_CON_HOT(a),
                           a, k);
    else
        hipLaunchKernelGGL(HIP_KERNEL_NAME(k_con<MODE, 512, 4, BIL>), dim3(a.gcon), dim3(512), 0, st, RL_CON_HOT(a),
                           a, k);
}

template <int MODE>
static hipError_t launch_con(hipStream_t st, const SolveArgs &a, long long k)
{
    if (a.gen) launch_con_t<MODE, true>(st, a, k);
    else launch_con_t<MODE, false>(st, a, k);
    return hipGetLastError();
}

int apply_impl(rl_ctx *h, SolveArgs &a, double *w)
{
    if (a.nc == 0) return RL_OK;
    a.out = w;
    RL_HIP(launch_rod<kModeApply>(h->stream, a, a.coef == nullptr, 0));
    RL_HIP(launch_con<kModeApply>(h->stream, a, 0));
    return RL_OK;
}

template <bool BIL>
static void record_sample_t(rl_ctx *h, int v, long long it, const SolveArgs &a, bool uni)
{
    hipStream_t st = h->stream;
    if (a.n > 0) launch_rod_t<kModeLoop, BIL>(st, a, uni, it, h->ev[v][0], h->ev[v][1]);
    if (con_wide(a))
        hipExtLaunchKernelGGL(k_con<kModeLoop, 512, 8, BIL>, dim3(a.gcon), dim3(512), 0, st, h->ev[v][2],
                              h->ev[v][3], 0, RL_CON_HOT(a), a, (long long)it);
    else
        hipExtLaunchKernelGGL(k_con<kModeLoop, 512, 4, BIL>, dim3(a.gcon), dim3(512), 0, st, h->ev[v][2],
                              h->ev[v][3], 0, RL_CON_HOT(a), a, (long long)it);
}

// One loop iteration whose two kernels are launched with start/stop events
// taken by the dispatch itself (the same span a kernel trace reports).
static hipError_t record_sample(rl_ctx *h, int v, long long it, const SolveArgs &a, bool uni)
{
    for (int k = 0; k < 4; ++k)
        if (!h->ev[v][k]) {
            hipError_t e = hipEventCreateWithFlags(&h->ev[v][k], hipEventDisableSystemFence);
            if (e != hipSuccess) return e;
        }
    h->ev_iter[v] = it;
    if (a.gen) record_sample_t<true>(h, v, it, a, uni);
    else record_sample_t<false>(h, v, it, a, uni);
    return hipGetLastError();
}

// U = M (D gamma + F) in the caller's order (perm may be null)
static hipError_t launch_velocity(hipStream_t st, const SolveArgs &a, bool uni, const double *F, const int *perm,
                                  double *U)
{
    const dim3 grid(grid_of(a.n, kRodBlock / kRodLanes));
    if (uni)
        hipLaunchKernelGGL(HIP_KERNEL_NAME(k_velocity<true>), grid, dim3(kRodBlock), 0, st, a, F, perm, U);
    else
        hipLaunchKernelGGL(HIP_KERNEL_NAME(k_velocity<false>), grid, dim3(kRodBlock), 0, st, a, F, perm, U);
    return hipGetLastError();
}

int solve_impl(rl_ctx *h, SolveArgs &a, const double *F, double *U, double *gamma_out, rl_solve_info *info,
               const int *perm)
{
    hipStream_t st = h->stream;
    const rl_params &p = h->prm;
    const bool uni = a.coef == nullptr;
    hipLaunchKernelGGL(k_state_init, dim3(1), dim3(64), 0, st, h->state, p.tol, (long long)p.max_iter);
    RL_HIP(hipGetLastError());
    long long iters = 0, refreshes = 0;
    bool vel_queued = false;
    if (a.nc > 0 && p.precision == RL_FP32_MIXED) {
        int rc = prepare_mixed(h, a);
        if (rc) return rc;
        rc = solve_mixed_impl(h, a, &refreshes);
        if (rc) return rc;
        iters = h->state_host->iter;
        if (gamma_out) {
            hipLaunchKernelGGL(k_unpack_gamma, dim3(grid_of(a.nc)), dim3(kBlock), 0, st, a.nc,
                               (const double2 *)a.st, gamma_out);
            RL_HIP(hipGetLastError());
        }
    } else if (a.nc > 0) {
        RL_HIP(launch_rod<kModeInit>(st, a, uni, 0));
        RL_HIP(launch_con<kModeInit>(st, a, 0));
        hipLaunchKernelGGL(HIP_KERNEL_NAME(k_fin<kModeInit>), dim3(1), dim3(kRodBlock), 0, st, a);
        RL_HIP(hipGetLastError());
        RL_HIP(launch_rod<kModeAlpha0>(st, a, uni, 0));
        RL_HIP(launch_con<kModeAlpha0>(st, a, 0));
        hipLaunchKernelGGL(HIP_KERNEL_NAME(k_fin<kModeAlpha0>), dim3(1), dim3(kRodBlock), 0, st, a);
        RL_HIP(hipGetLastError());
        // The host follows the loop through the progress word that workgroup 0
        // of each rod kernel stores (2 k + stop), keeping `ahead` iterations
        // queued past the one running: the GPU never waits for the host, no
        // copy enters the stream, and at most ahead + 1 iterations are
        // launched after the stop (they exit at once).
        const int every = p.check_every > 0 ? p.check_every : 32;
        const long long ahead = std::min(every, 7);
        volatile unsigned long long *prog = h->progress_host;
        constexpr unsigned long long kNone = ~0ull;
        *prog = kNone;
        a.progress = h->progress_dev;
        // the stop is decided at k = max_iter at the latest
        const long long limit = p.max_iter + 1;
        long long launched = 0;
        // event slots of sampled iterations not yet read (no sampling in an
        // allocation-free call: its events would be created on first use)
        int pend[rl_ctx::kMaxEv], npend = 0;
        bool used[rl_ctx::kMaxEv] = {};
        const int prof_every = h->arena_on ? 0 : h->prof_every;
        auto enqueue = [&](long long count) -> int {
            for (long long k = 0; k < count && launched < limit; ++k, ++launched) {
                int slot = -1;
                if (prof_every > 0 && launched % prof_every == 0)
                    for (int v = 0; v < rl_ctx::kMaxEv && slot < 0; ++v)
                        if (!used[v]) slot = v;
                if (slot >= 0) {
                    RL_HIP(record_sample(h, slot, launched, a, uni));
                    used[slot] = true;
                    pend[npend++] = slot;
                } else {
                    RL_HIP(launch_rod<kModeLoop>(st, a, uni, launched));
                    RL_HIP(launch_con<kModeLoop>(st, a, launched));
                }
            }
            return RL_OK;
        };
        // a sampled iteration counts once its kernels have finished and the
        // loop was still running in it (live < the first iteration known to
        // be dead, or any earlier one once the stop is known)
        auto drain = [&](bool all, long long live) -> int {
            int nkeep = 0;
            for (int u = 0; u < npend; ++u) {
                const int v = pend[u];
                if (!all && (h->ev_iter[v] >= live || hipEventQuery(h->ev[v][3]) != hipSuccess)) {
                    pend[nkeep++] = v;
                    continue;
                }
                if (h->ev_iter[v] < live) {
                    float t0 = 0.f, t1 = 0.f;
                    if (a.n > 0) RL_HIP(hipEventElapsedTime(&t0, h->ev[v][0], h->ev[v][1]));
                    RL_HIP(hipEventElapsedTime(&t1, h->ev[v][2], h->ev[v][3]));
                    h->prof_ms[0] += t0;
                    h->prof_ms[1] += t1;
                    h->prof_cnt[0] += 1.0;
                    h->prof_cnt[1] += 1.0;
                }
                used[v] = false;
            }
            npend = nkeep;
            return RL_OK;
        };
        {
            int rc = enqueue(ahead + 1);
            if (rc) return rc;
            unsigned spins = 0;
            for (;;) {
                const unsigned long long w = *prog;
                const long long cur = w == kNone ? -1 : (long long)(w >> 1);
                if (w != kNone && (w & 1ull)) break;
                if (npend && (rc = drain(false, cur))) return rc;
                if (launched < limit && launched - cur <= ahead) {
                    if ((rc = enqueue(1))) return rc;
                    spins = 0;
                    continue;
                }
                if (launched >= limit && ++spins > (1u << 20)) {
                    // everything is queued: wait for the stream, then the stop
                    // must have been stored
                    RL_HIP(hipStreamSynchronize(st));
                    const unsigned long long w2 = *prog;
                    if (w2 == kNone || !(w2 & 1ull)) {
                        set_error("rl_solve_lcp: stop flag never raised");
                        return RL_ERR_HIP;
                    }
                    break;
                }
                __builtin_ia32_pause();
            }
        }
        // the state copy, the forces and the velocities are queued together
        // and waited for once
        RL_HIP(hipMemcpyAsync(h->state_host, h->state, sizeof(SolverState), hipMemcpyDeviceToHost, st));
        if (gamma_out) {
            hipLaunchKernelGGL(k_unpack_gamma, dim3(grid_of(a.nc)), dim3(kBlock), 0, st, a.nc,
                               (const double2 *)a.st, gamma_out);
            RL_HIP(hipGetLastError());
        }
        if (U && a.n > 0) {
            RL_HIP(launch_velocity(st, a, uni, F, perm, U));
            vel_queued = true;
        }
        RL_HIP(hipStreamSynchronize(st));
        {
            const int rc = drain(true, h->state_host->iter);
            if (rc) return rc;
        }
        iters = h->state_host->iter;
    } else {
        RL_HIP(hipMemcpyAsync(h->state_host, h->state, sizeof(SolverState), hipMemcpyDeviceToHost, st));
    }
    if (U && a.n > 0 && !vel_queued) RL_HIP(launch_velocity(st, a, uni, F, perm, U));
    RL_HIP(hipStreamSynchronize(st));
    const SolverState &s = *h->state_host;
    const int status = a.nc > 0 ? s.status : RL_OK;
    if (info) {
        info->iterations = a.nc > 0 ? iters : 0;
        info->residual = a.nc > 0 ? s.res : 0.0;
        info->alpha0 = s.alpha0;
        info->status = status;
        info->fp64_refreshes = (int32_t)refreshes;
    }
    if (status == RL_ERR_NONFINITE) set_error("rl_solve_lcp: non-finite value in q or an iterate");
    return status;
}

hipError_t launch_refresh64(rl_ctx *h, const SolveArgs &a, bool accum)
{
    hipStream_t st = h->stream;
    const bool uni = a.coef == nullptr;
    if (accum) {
        hipLaunchKernelGGL(k_mix_accum, dim3(grid_of(a.nc)), dim3(kBlock), 0, st, a.nc, (const float4 *)a.st32,
                           a.qpos, a.st, a.stq);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    hipError_t e = launch_rod<kModeApply>(st, a, uni, 0);
    if (e != hipSuccess) return e;
    if ((e = launch_con<kModeRefresh>(st, a, 0)) != hipSuccess) return e;
    hipLaunchKernelGGL(HIP_KERNEL_NAME(k_fin<kModeRefresh>), dim3(1), dim3(kRodBlock), 0, st, a);
    return hipGetLastError();
}

hipError_t launch_alpha0_64(rl_ctx *h, const SolveArgs &a)
{
    hipStream_t st = h->stream;
    hipError_t e = launch_rod<kModeAlpha0>(st, a, a.coef == nullptr, 0);
    if (e != hipSuccess) return e;
    if ((e = launch_con<kModeAlpha0>(st, a, 0)) != hipSuccess) return e;
    hipLaunchKernelGGL(HIP_KERNEL_NAME(k_fin<kModeAlpha0>), dim3(1), dim3(kRodBlock), 0, st, a);
    return hipGetLastError();
}

hipError_t launch_velocity_on(hipStream_t st, const SolveArgs &a, const double *F, const int *perm, double *U)
{
    if (a.n <= 0) return hipSuccess;
    const dim3 grid(grid_of(a.n, kRodBlock / kRodLanes));
    if (a.coef == nullptr)
        hipLaunchKernelGGL(HIP_KERNEL_NAME(k_velocity<true>), grid, dim3(kRodBlock), 0, st, a, F, perm, U);
    else
        hipLaunchKernelGGL(HIP_KERNEL_NAME(k_velocity<false>), grid, dim3(kRodBlock), 0, st, a, F, perm, U);
    return hipGetLastError();
}

hipError_t launch_velocity64(rl_ctx *h, const SolveArgs &a, const double *F, const int *perm, double *U)
{
    return launch_velocity_on(h->stream, a, F, perm, U);
}

hipError_t launch_unpack_gamma(hipStream_t st, const SolveArgs &a, double *gamma)
{
    if (a.nc <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_unpack_gamma, dim3(grid_of(a.nc)), dim3(kBlock), 0, st, a.nc, (const double2 *)a.st, gamma);
    return hipGetLastError();
}

// the iterate back to the caller's start (after trial iterations)
__global__ void k_restore_start(int64_t nc, const double *__restrict__ gamma_in, const int32_t *__restrict__ qpos,
                                double2 *__restrict__ st, double2 *__restrict__ stq)
{
    const int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (c >= nc) return;
    const double2 v = make_double2(gamma_in[c], 0.0);
    st[c] = v;
    stq[qpos[c]] = v;
}

int integrate_impl(rl_ctx *h, int64_t n, const double *U, double *x, double *quat, double *xu)
{
    if (n <= 0) return RL_OK;
    const rl_params &p = h->prm;
    hipLaunchKernelGGL(k_integrate, dim3(grid_of(n)), dim3(kBlock), 0, h->stream, n, U, x, quat, xu, p.dt,
                       p.box[0], p.box[1], p.box[2]);
    RL_HIP(hipGetLastError());
    return RL_OK;
}

}  // namespace rl
