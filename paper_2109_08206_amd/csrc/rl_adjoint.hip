// Adjoint of the steric step on gfx950 (the differentiation form).
//
// Where the step is differentiable, the constraint rows of the active set
// A hold as equalities (eq. linearconstraints): Mc_AA gamma_A + q_A = 0,
// with gamma = 0 off A.  Here c is in A when gamma_c > w_c.  With the pair
// list and A held fixed, the velocities U = M (D gamma + F) (eq.
// constrainedeom_euler) are then a smooth function of the geometry, the
// mobility, q and F.  For a cotangent U_bar, let
//     lambda = Mc_AA^{-1} D_A^T M U_bar      (conjugate gradients below).
// Taking derivatives of U_bar . U through gamma_A = -Mc_AA^{-1} q_A and
// Mc = D^T M D (eq. blockdef, block B) gives
//     q_bar = -lambda,
//     column c of D:  d_bar_c = gamma_c P - lambda_c Q on the rods of c,
//     M:              M_bar   = (U_bar - D lambda) G^T  (and the terms below),
// with P = M (U_bar - D lambda) and G = D gamma + F.  The two readings of q:
//   * solve: q is an input in its own right.  Then Q = M D gamma,
//     F_bar = M U_bar, and M_bar = U_bar G^T - (D lambda)(D gamma)^T.
//   * step: q = phi/h + D^T M F (eq. blockdef, block A).  Then Q = U,
//     F_bar = P, phi_bar = -lambda / h, and M_bar = (U_bar - D lambda) G^T.
// The mobility depends on the director only through the translational
// block a_perp I + (a_par - a_perp) d d^T, so
// dir_bar = (a_par - a_perp) (M_bar_t + M_bar_t^T) d.
//
// lambda: Mc_AA is symmetric positive semi-definite and the right-hand side
// lies in its range.  Conjugate gradients from 0 therefore converge to the
// minimum-norm solution.  The recurrence is that of Chronopoulos & Gear
// (1989): one product w = Mc_AA r and one fused reduction (r.r, r.w) per
// iteration.  It runs as two launches, like the BBPGD loop.  The rod kernel
// forms the next residual of each incident constraint on the fly, sums
// D r into V = M_t F and W = Omega x dir in registers, writes each contact
// point's velocity along the normal, u = e.(V + s W), and publishes the step
// scalars.  The constraint kernel applies the update, takes w = u_P - u_Q on
// A and writes the partial sums.  No workgroup waits for another: every
// workgroup of the next rod kernel sums the previous partials itself in a
// fixed order.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>

#include "rl_device.hpp"
#include "rl_vec.hpp"

namespace rl {

static inline unsigned grid_of(int64_t n, int block) { return (unsigned)((n + block - 1) / block); }
static inline unsigned rod_grid8(int64_t n) { return (grid_of(n, kRodLoopBlock / kRodLanes) + 7) / 8 * 8; }

// CG state.  P order: cs = (lambda, p, mask, 0), cr = (r, s, w, 0);
// Q-side list order: cq = (r, s, w, lambda).  s = Mc_AA p, w = Mc_AA r.
struct CgArgs {
    SolveArgs a;
    double *cs;
    double *cr;
    double *cq;
    double *sc;  // (rho_j, alpha_j) of iteration j at 2 * (j & 1)
    double *ab;  // (alpha_j, beta_j) of iteration j at 2 * (j & 1)
};

// r_{j+1} = r_j - alpha_j (w_j + beta_j s_{j-1}); the same expression on
// both kernels so that they agree bit for bit
__device__ __forceinline__ double cg_next_r(double r, double s, double w, double alpha, double beta)
{
    return fma(-alpha, fma(beta, s, w), r);
}

__device__ __forceinline__ void lane_sum(double *v, int m)
{
#pragma unroll
    for (int o = 1; o < kRodLanes; o <<= 1)
        for (int d = 0; d < m; ++d) v[d] += __shfl_xor(v[d], o, 64);
}

// M U_bar in the rod kernel's output layout (V = M_t u, W = (r_perp w) x d)
template <bool UNI>
__global__ void k_adj_prep(SolveArgs a, const double *__restrict__ Ubar)
{
    const int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (r >= a.n) return;
    const V3 d = load3(a.dir + 3 * r);
    double apar, aperp, rperp;
    rod_mob(a, r, UNI, apar, aperp, rperp);
    const V3 ut = load3(Ubar + 6 * r), ur = load3(Ubar + 6 * r + 3);
    const V3 v = aperp * ut + ((apar - aperp) * dot(d, ut)) * d;
    const V3 w = cross(rperp * ur, d);
    double *o = a.V + 6 * r;
    store3(o, v);
    store3(o + 3, w);
}

// w = D^T (V, W) of one constraint from the geometry record
__device__ __forceinline__ double con_rate(const SolveArgs &a, int64_t c, int2 ij, double2 g0, double2 g1, double2 g2)
{
    const double2 *Vi = reinterpret_cast<const double2 *>(a.V + 6 * (int64_t)ij.x);
    const double2 *Vj = reinterpret_cast<const double2 *>(a.V + 6 * (int64_t)ij.y);
    const double2 i0 = Vi[0], i1 = Vi[1], i2 = Vi[2], j0 = Vj[0], j1 = Vj[1], j2 = Vj[2];
    const double si = g1.y, sj = g2.x;
    const double ux = (i0.x + si * i1.y) - (j0.x + sj * j1.y);
    const double uy = (i0.y + si * i2.x) - (j0.y + sj * j2.x);
    const double uz = (i1.x + si * i2.y) - (j1.x + sj * j2.y);
    return g0.x * ux + g0.y * uy + g1.x * uz;
}

// Start: mask of A, b = D_A^T M U_bar, r0 = b, partials (b.b, 0, |A|, 0)
// into parity 1 (read by the first rod kernel).
__global__ void __launch_bounds__(kConBlock) k_cg_start(CgArgs g, const double *__restrict__ wsol)
{
    __shared__ double lds[kConBlock / 64 + 1][4];
    const SolveArgs &a = g.a;
    double p[4] = {0.0, 0.0, 0.0, 0.0};
    const unsigned tile = xcd_tile(blockIdx.x, gridDim.x);
    const int64_t per = (a.nc + gridDim.x - 1) / gridDim.x;
    const int64_t lo = (int64_t)tile * per, hi = lo + per < a.nc ? lo + per : a.nc;
    for (int64_t c = lo + threadIdx.x; c < hi; c += kConBlock) {
        const int2 ij = a.pp[c];
        const double2 *gd = reinterpret_cast<const double2 *>(a.geo + 4 * c);
        const double m = a.st[c].x > wsol[c] ? 1.0 : 0.0;
        const double b = m > 0.0 ? con_rate(a, c, ij, gd[0], gd[1], a.geo2[c]) : 0.0;
        double2 *cs = reinterpret_cast<double2 *>(g.cs + 4 * c);
        double2 *cr = reinterpret_cast<double2 *>(g.cr + 4 * c);
        double2 *cq = reinterpret_cast<double2 *>(g.cq + 4 * (int64_t)a.qpos[c]);
        cs[0] = make_double2(0.0, 0.0);
        cs[1] = make_double2(m, 0.0);
        cr[0] = make_double2(b, 0.0);
        cr[1] = make_double2(0.0, 0.0);
        cq[0] = make_double2(b, 0.0);
        cq[1] = make_double2(0.0, 0.0);
        p[0] += b * b;
        p[2] += m;
    }
    block_total4<kConBlock / 64>(p, lds);
    if (threadIdx.x == 0) partial_put(a.partial + (int64_t)a.gcon * 4, a.gcon, blockIdx.x, p);
}

// One incidence record of the CG rod kernel: (r, s) and w of the constraint
// in the side's order, and its geometry (ex, ey), (ez, s).
struct CgRec {
    double2 rs, g0, g1;
    double w;
};

__device__ __forceinline__ void cg_rec_load(const double *cr, const double *geo, int c, int end, CgRec &R)
{
    const double2 z = make_double2(0.0, 0.0);
    R.rs = R.g0 = R.g1 = z;
    R.w = 0.0;
    if (c < end) {
        const double2 *x = reinterpret_cast<const double2 *>(cr + 4 * (int64_t)c);
        const double2 *gd = reinterpret_cast<const double2 *>(geo + 4 * (int64_t)c);
        R.rs = x[0];
        R.w = x[1].x;
        R.g0 = gd[0];
        R.g1 = gd[1];
    }
}

// f += +-r_{k} e, m += +-r_{k} s e over one side's incidences of the lane
__device__ __forceinline__ void cg_side(double sign, const double *cr, const double *geo, int b, int e,
                                        const CgRec *rr, double alpha, double beta, double f[3], double m[3])
{
#pragma unroll
    for (int i = 0; i < kRodRounds; ++i) {
        if (b + i * kRodLanes >= e) return;
        rod_add(sign, cg_next_r(rr[i].rs.x, rr[i].rs.y, rr[i].w, alpha, beta), rr[i].g0, rr[i].g1, f, m);
    }
    for (int c = b + kRodRounds * kRodLanes; c < e; c += kRodLanes) {
        CgRec R;
        cg_rec_load(cr, geo, c, e, R);
        rod_add(sign, cg_next_r(R.rs.x, R.rs.y, R.w, alpha, beta), R.g0, R.g1, f, m);
    }
}

// u = e.(V + s W) at every incidence of the lane, in the same order
__device__ __forceinline__ void cg_emit(double *u, const double *geo, int b, int e, const CgRec *rr,
                                        const double v[3], const double w[3])
{
#pragma unroll
    for (int i = 0; i < kRodRounds; ++i) {
        if (b + i * kRodLanes >= e) return;
        u[b + i * kRodLanes] = u_along(rr[i].g0, rr[i].g1, v, w);
    }
    for (int c = b + kRodRounds * kRodLanes; c < e; c += kRodLanes) {
        const double2 *gd = reinterpret_cast<const double2 *>(geo + 4 * (int64_t)c);
        u[c] = u_along(gd[0], gd[1], v, w);
    }
}

// Rod kernel of CG iteration k: D r_k summed per rod (four lanes per rod),
// then V = M_t F and W = Omega x dir, projected on e at every incidence of
// the rod (u = e.(V + s W), the rod's share of w = Mc_AA r).  The first
// records of each lane and the previous partials are loaded before anything
// else: they depend on neither the step scalars nor the stop flag.  Every
// workgroup then sums the partials of iteration k-1 and takes the stop
// decision; workgroup 0 publishes the step scalars and latches the stop.
// The arrays of the first loads, the grid size and n lead the argument list
// (14 dwords, preloaded into registers).
template <bool UNI>
__global__ void __launch_bounds__(kRodLoopBlock)
    k_cg_rod(const int32_t *__restrict__ pptr, const int32_t *__restrict__ qptr, const double *cr0,
             const double *cq0, const double *__restrict__ geo, const double *__restrict__ qgeo, unsigned nblk, int n,
             CgArgs g, long long k)
{
    __shared__ double lds[kRodLoopBlock / 64 + 1][4];
    const SolveArgs &a = g.a;
    SolverState *st = a.state;
    const int sub = threadIdx.x & (kRodLanes - 1);
    const unsigned tile = xcd_tile(blockIdx.x, nblk);
    const int64_t r = (int64_t)tile * (kRodLoopBlock / kRodLanes) + (threadIdx.x / kRodLanes);
    const bool active = r < n;
    int pb = 0, pe = 0, qb = 0, qe = 0;
    if (active) {
        pb = pptr[r] + sub;
        pe = pptr[r + 1];
        qb = qptr[r] + sub;
        qe = qptr[r + 1];
    }
    CgRec P[kRodRounds], Q[kRodRounds];
#pragma unroll
    for (int i = 0; i < kRodRounds; ++i) {
        cg_rec_load(cr0, geo, pb + i * kRodLanes, pe, P[i]);
        cg_rec_load(cq0, qgeo, qb + i * kRodLanes, qe, Q[i]);
    }
    const double *part = a.partial + (int64_t)((k - 1) & 1) * a.gcon * 4;
    PartFirst pf;
    partials_first_split<kRodLoopBlock>(part, a.gcon, pf);
    // the recurrence's other inputs and the rod's direction and mobility do
    // not depend on the partials either
    const double bb0 = st->alpha0, tol = st->tol;
    const long long max_iter = st->max_iter;
    const int ps = 2 * (int)((k - 2) & 1);  // (rho, alpha) of iteration k - 2
    const double rho_prev = g.sc[ps], a_prev = g.sc[ps + 1];
    const int64_t rr = active ? r : 0;
    const V3 d = load3(a.dir + 3 * rr);
    double apar, aperp, rperp;
    rod_mob(a, rr, UNI, apar, aperp, rperp);
    if (st->done) return;
    double t[4];
    sum_partials_split_from<kRodLoopBlock / 64>(pf, part, a.gcon, t, lds);
    double alpha = 0.0, beta = 0.0;
    const bool lead = blockIdx.x == 0 && threadIdx.x == 0;
    if (k == 0) {
        const double bb = t[0];
        const bool stop = !(bb > 0.0);
        if (lead) {
            st->alpha0 = bb;
            st->ss = t[2];
            if (stop) {
                st->iter = 0;
                st->res = 0.0;
                st->status = isfinite(bb) ? RL_OK : RL_ERR_NONFINITE;
                st->done = 1;
            }
        }
        if (stop) return;
    } else {
        const long long j = k - 1;
        const double rho = t[0], del = t[1], bb = bb0;
        if (j == 0) {
            alpha = rho / del;
        } else {
            beta = rho / rho_prev;
            alpha = rho / (del - beta * rho / a_prev);
        }
        int status = 1000;
        if (!isfinite(rho) || !isfinite(del)) status = RL_ERR_NONFINITE;
        else if (rho <= tol * tol * bb) status = RL_OK;
        else if (j >= max_iter) status = RL_NOT_CONVERGED;
        else if (!(alpha > 0.0) || !isfinite(alpha)) status = RL_STAGNATED;
        const bool stop = status != 1000;
        if (lead) {
            if (stop) {
                st->iter = j;
                st->res = sqrt(rho / bb);
                st->status = status;
                st->done = 1;
            } else {
                g.sc[2 * (j & 1)] = rho;
                g.sc[2 * (j & 1) + 1] = alpha;
                g.ab[2 * (j & 1)] = alpha;
                g.ab[2 * (j & 1) + 1] = beta;
            }
        }
        if (stop) return;
    }
    double f[3] = {0.0, 0.0, 0.0}, m[3] = {0.0, 0.0, 0.0};
    cg_side(1.0, g.cr, a.geo, pb, pe, P, alpha, beta, f, m);
    cg_side(-1.0, g.cq, a.qgeo, qb, qe, Q, alpha, beta, f, m);
#pragma unroll
    for (int o = 1; o < kRodLanes; o <<= 1) {
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            f[c] += __shfl_xor(f[c], o, 64);
            m[c] += __shfl_xor(m[c], o, 64);
        }
    }
    if (!active) return;
    // translation M_t f; rotation Omega = r_perp d x m and Omega x d = r_perp (m - (d.m) d)
    const double fd = (apar - aperp) * (d.x * f[0] + d.y * f[1] + d.z * f[2]);
    const double md = d.x * m[0] + d.y * m[1] + d.z * m[2];
    const double v[3] = {aperp * f[0] + fd * d.x, aperp * f[1] + fd * d.y, aperp * f[2] + fd * d.z};
    const double w[3] = {rperp * (m[0] - md * d.x), rperp * (m[1] - md * d.y), rperp * (m[2] - md * d.z)};
    cg_emit(a.uP, a.geo, pb, pe, P, v, w);
    cg_emit(a.uQ, a.qgeo, qb, qe, Q, v, w);
}

struct CgConLoads {
    double2 lp, mk, rs, w0;  // (lambda, p), (mask, 0), (r, s), (w, 0)
    double up, uq;
    int qp;
};

// the CG constraint kernel's inputs (preloaded leading arguments)
struct CgConIn {
    const int32_t *qpos;
    const double *uP, *uQ, *cs, *cr;
};

__device__ __forceinline__ void cg_con_load(const CgConIn &in, int64_t c, CgConLoads &L)
{
    const double2 *cs = reinterpret_cast<const double2 *>(in.cs + 4 * c);
    const double2 *cr = reinterpret_cast<const double2 *>(in.cr + 4 * c);
    L.qp = in.qpos[c];
    L.up = in.uP[c];
    L.lp = cs[0];
    L.mk = cs[1];
    L.rs = cr[0];
    L.w0 = cr[1];
    L.uq = in.uQ[L.qp];
}

__device__ __forceinline__ void cg_con_update(const CgArgs &g, int64_t c, const CgConLoads &L, long long k,
                                              double alpha, double beta, double p[4])
{
    double lam = L.lp.x, pv = L.lp.y, rv = L.rs.x, sv = L.rs.y;
    if (k > 0) {
        const double s1 = fma(beta, sv, L.w0.x);
        const double p1 = fma(beta, pv, rv);
        lam = fma(alpha, p1, lam);
        rv = cg_next_r(rv, sv, L.w0.x, alpha, beta);
        sv = s1;
        pv = p1;
    }
    const double w = L.mk.x > 0.0 ? L.up - L.uq : 0.0;
    double2 *cs = reinterpret_cast<double2 *>(g.cs + 4 * c);
    double2 *cr = reinterpret_cast<double2 *>(g.cr + 4 * c);
    cs[0] = make_double2(lam, pv);
    cr[0] = make_double2(rv, sv);
    cr[1] = make_double2(w, 0.0);
    double2 *cq = reinterpret_cast<double2 *>(g.cq + 4 * (int64_t)L.qp);
    cq[0] = make_double2(rv, sv);
    cq[1] = make_double2(w, lam);
    p[0] += rv * rv;
    p[1] += rv * w;
}

// Constraint kernel of CG iteration k: the update of iteration k-1 (lambda,
// p, s, r), then w_k = Mc_AA r_k = u_P - u_Q on A and the partials
// (r_k.r_k, r_k.w_k).  Like the BBPGD constraint kernel, each lane takes
// kConCpl constraints per round, and the first round's loads and the step
// scalars are in flight before the stop flag is read.
__global__ void __launch_bounds__(kConBlock)
    k_cg_con(const int32_t *__restrict__ qpos, const double *__restrict__ uP, const double *__restrict__ uQ,
             const double *cs0, const double *cr0, int nc, unsigned nblk, const double *ab, CgArgs g, long long k)
{
    __shared__ double lds[kConBlock / 64 + 1][4];
    const SolveArgs &a = g.a;
    double p[4] = {0.0, 0.0, 0.0, 0.0};
    const CgConIn in{qpos, uP, uQ, cs0, cr0};
    const unsigned tile = xcd_tile(blockIdx.x, nblk);
    const int64_t per = (nc + nblk - 1) / nblk;
    const int64_t lo = (int64_t)tile * per, hi = lo + per < nc ? lo + per : nc;
    const int64_t step = (int64_t)kConCpl * kConBlock;
    int64_t c0 = lo + threadIdx.x;
    CgConLoads L[kConCpl];
#pragma unroll
    for (int u = 0; u < kConCpl; ++u)
        if (c0 + u * kConBlock < hi) cg_con_load(in, c0 + u * kConBlock, L[u]);
    const double alpha = k > 0 ? ab[2 * ((k - 1) & 1)] : 0.0;
    const double beta = k > 0 ? ab[2 * ((k - 1) & 1) + 1] : 0.0;
    if (a.state->done) return;
    for (;;) {
#pragma unroll
        for (int u = 0; u < kConCpl; ++u)
            if (c0 + u * kConBlock < hi) cg_con_update(g, c0 + u * kConBlock, L[u], k, alpha, beta, p);
        c0 += step;
        if (c0 >= hi) break;
#pragma unroll
        for (int u = 0; u < kConCpl; ++u)
            if (c0 + u * kConBlock < hi) cg_con_load(in, c0 + u * kConBlock, L[u]);
    }
    block_total4<kConBlock / 64>(p, lds);
    if (threadIdx.x == 0) partial_put(a.partial + (int64_t)(k & 1) * a.gcon * 4, a.gcon, blockIdx.x, p);
}

// Per rod: G_c = D gamma and G_l = D lambda (force and torque), then
// P = M (U_bar - G_l), Q (M G_c, or U in the step reading), F_bar and the
// mobility part of dir_bar.
template <bool UNI, bool STEP>
__global__ void __launch_bounds__(kRodBlock) k_adj_rod(CgArgs g, const double *__restrict__ Ubar,
                                                       const double *__restrict__ F, const int *__restrict__ perm,
                                                       double *__restrict__ PQ, double *__restrict__ Fbar,
                                                       double *__restrict__ dmob)
{
    const SolveArgs &a = g.a;
    const int sub = threadIdx.x & (kRodLanes - 1);
    const int64_t r = (int64_t)blockIdx.x * (kRodBlock / kRodLanes) + (threadIdx.x / kRodLanes);
    const bool active = r < a.n;
    double acc[12] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    if (active) {
        const int pe = a.pptr[r + 1];
        for (int c = a.pptr[r] + sub; c < pe; c += kRodLanes) {
            const double2 *gd = reinterpret_cast<const double2 *>(a.geo + 4 * (int64_t)c);
            const double2 g0 = gd[0], g1 = gd[1];
            const double gm = a.st[c].x, lm = g.cs[4 * (int64_t)c];
            const double e3[3] = {g0.x, g0.y, g1.x};
            for (int d = 0; d < 3; ++d) {
                acc[d] += gm * e3[d];
                acc[3 + d] += gm * g1.y * e3[d];
                acc[6 + d] += lm * e3[d];
                acc[9 + d] += lm * g1.y * e3[d];
            }
        }
        const int qe = a.qptr[r + 1];
        for (int kq = a.qptr[r] + sub; kq < qe; kq += kRodLanes) {
            const double2 *gd = reinterpret_cast<const double2 *>(a.qgeo + 4 * (int64_t)kq);
            const double2 g0 = gd[0], g1 = gd[1];
            const double gm = a.stq[kq].x, lm = g.cq[4 * (int64_t)kq + 3];
            const double e3[3] = {g0.x, g0.y, g1.x};
            for (int d = 0; d < 3; ++d) {
                acc[d] -= gm * e3[d];
                acc[3 + d] -= gm * g1.y * e3[d];
                acc[6 + d] -= lm * e3[d];
                acc[9 + d] -= lm * g1.y * e3[d];
            }
        }
    }
    lane_sum(acc, 12);
    if (!active || sub != 0) return;
    const int64_t ro = perm ? (int64_t)perm[r] : r;
    const V3 d = load3(a.dir + 3 * r);
    double apar, aperp, rperp;
    rod_mob(a, r, UNI, apar, aperp, rperp);
    // contact force and torque d x m of gamma and of lambda
    const V3 gcf = v3(acc[0], acc[1], acc[2]), gct = cross(d, v3(acc[3], acc[4], acc[5]));
    const V3 glf = v3(acc[6], acc[7], acc[8]), glt = cross(d, v3(acc[9], acc[10], acc[11]));
    V3 Ff = v3(0.0, 0.0, 0.0), Ft = v3(0.0, 0.0, 0.0);
    if (F) {
        Ff = load3(F + 6 * ro);
        Ft = load3(F + 6 * ro + 3);
    }
    const V3 ubt = load3(Ubar + 6 * r), ubr = load3(Ubar + 6 * r + 3);
    const V3 u1t = ubt - glf, u1r = ubr - glt;
    const double k2 = apar - aperp;
    const V3 Pt = aperp * u1t + (k2 * dot(d, u1t)) * d, Pr = rperp * u1r;
    const V3 Gt = gcf + Ff, Gr = gct + Ft;
    V3 Qt, Qr, FBt, FBr, dm;
    if (STEP) {
        Qt = aperp * Gt + (k2 * dot(d, Gt)) * d;
        Qr = rperp * Gr;
        FBt = Pt;
        FBr = Pr;
        dm = k2 * (dot(Gt, d) * u1t + dot(u1t, d) * Gt);
    } else {
        Qt = aperp * gcf + (k2 * dot(d, gcf)) * d;
        Qr = rperp * gct;
        FBt = aperp * ubt + (k2 * dot(d, ubt)) * d;
        FBr = rperp * ubr;
        dm = k2 * (dot(Gt, d) * ubt + dot(ubt, d) * Gt - dot(gcf, d) * glf - dot(glf, d) * gcf);
    }
    double *o = PQ + 12 * r;
    store3(o, Pt);
    store3(o + 3, Pr);
    store3(o + 6, Qt);
    store3(o + 9, Qr);
    store3(Fbar + 6 * ro, FBt);
    store3(Fbar + 6 * ro + 3, FBr);
    store3(dmob + 3 * r, dm);
}

// Per constraint: X = gamma_c P - lambda_c Q on each rod (gamma_c taken as 0
// off A), then the gradients with respect to e, the arclengths, q and the
// lever-arm directors of the column [e; y_i x e; -e; -(y_j x e)].
__global__ void k_adj_con(CgArgs g, const double *__restrict__ PQ, double *__restrict__ qbar,
                          double *__restrict__ ebar, double *__restrict__ armbar, double *__restrict__ dbar)
{
    const SolveArgs &a = g.a;
    const int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (c >= a.nc) return;
    const int2 ij = a.pp[c];
    const double2 *gd = reinterpret_cast<const double2 *>(a.geo + 4 * c);
    const double2 g0 = gd[0], g1 = gd[1], g2 = a.geo2[c];
    const V3 e = v3(g0.x, g0.y, g1.x);
    const double si = g1.y, sj = g2.x;
    const double lam = g.cs[4 * c], gam = g.cs[4 * c + 2] > 0.0 ? a.st[c].x : 0.0;
    const double *pi = PQ + 12 * (int64_t)ij.x, *pj = PQ + 12 * (int64_t)ij.y;
    const V3 xa = gam * load3(pi) - lam * load3(pi + 6), xb = gam * load3(pi + 3) - lam * load3(pi + 9);
    const V3 xc = gam * load3(pj) - lam * load3(pj + 6), xd = gam * load3(pj + 3) - lam * load3(pj + 9);
    const V3 di = load3(a.dir + 3 * (int64_t)ij.x), dj = load3(a.dir + 3 * (int64_t)ij.y);
    const V3 yi = si * di, yj = sj * dj;
    const V3 eb = (xa - xc) + cross(xb, yi) - cross(xd, yj);
    const V3 ybi = cross(e, xb), ybj = -1.0 * cross(e, xd);
    qbar[c] = -lam;
    store3(ebar + 3 * c, eb);
    armbar[2 * c] = dot(ybi, di);
    armbar[2 * c + 1] = dot(ybj, dj);
    store3(dbar + 6 * c, si * ybi);
    store3(dbar + 6 * c + 3, sj * ybj);
}

// dir_bar = dmob + lever-arm parts, summed over each rod's constraints in a
// fixed order (P side, then Q side)
__global__ void k_dir_bar(SolveArgs a, const double *__restrict__ dmob, const double *__restrict__ dbar,
                          double *__restrict__ dir_bar)
{
    const int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (r >= a.n) return;
    V3 s = load3(dmob + 3 * r);
    for (int c = a.pptr[r]; c < a.pptr[r + 1]; ++c) s = s + load3(dbar + 6 * (int64_t)c);
    for (int k = a.qptr[r]; k < a.qptr[r + 1]; ++k) s = s + load3(dbar + 6 * (int64_t)a.qidx[k] + 3);
    store3(dir_bar + 3 * r, s);
}

// Adjoint of x' = x + h U_t and theta' = u / |u|, u = theta + h Psi(theta)
// Omega, Psi(theta) Omega = 1/2 [-p.Omega ; s Omega - p x Omega]:
// U_bar (solver order) and the direct part of theta_bar.
__global__ void k_integrate_adj(int64_t n, const int *__restrict__ perm, const double *__restrict__ xbar,
                                const double *__restrict__ quatbar, const double *__restrict__ quat,
                                const double *__restrict__ U, double dt, double *__restrict__ Ubar,
                                double *__restrict__ qbd)
{
    const int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (r >= n) return;
    const int64_t ro = perm ? (int64_t)perm[r] : r;
    const double s = quat[4 * ro];
    const V3 p = load3(quat + 4 * ro + 1), om = load3(U + 6 * ro + 3);
    const double us = s - 0.5 * dt * dot(p, om);
    const V3 uv = p + (0.5 * dt) * (s * om - cross(p, om));
    const double nrm = sqrt(us * us + dot(uv, uv));
    const double qs = us / nrm;
    const V3 qv = (1.0 / nrm) * uv;
    const double bs = quatbar[4 * ro];
    const V3 bv = load3(quatbar + 4 * ro + 1);
    const double pr = qs * bs + dot(qv, bv);
    const double ubs = (bs - pr * qs) / nrm;
    const V3 ubv = (1.0 / nrm) * (bv - pr * qv);
    const V3 omb = (0.5 * dt) * (s * ubv + cross(p, ubv) - ubs * p);
    store3(Ubar + 6 * r, dt * load3(xbar + 3 * ro));
    store3(Ubar + 6 * r + 3, omb);
    qbd[4 * r] = ubs + 0.5 * dt * dot(om, ubv);
    store3(qbd + 4 * r + 1, ubv + (0.5 * dt) * (cross(ubv, om) - ubs * om));
}

// Final per-rod sums of the step adjoint, written in the caller's order:
// x_bar += sum over the rod's constraints of +-r0_bar; theta_bar = direct
// part + J^T dir_bar with J the Jacobian of R(theta) e_z, projected on the
// tangent space of the unit sphere at theta.
__global__ void k_step_bar(SolveArgs a, const int *__restrict__ perm, const double *__restrict__ gbar,
                           const double *__restrict__ dmob, const double *__restrict__ qbd,
                           const double *__restrict__ quat, double *__restrict__ xbar, double *__restrict__ quatbar)
{
    const int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (r >= a.n) return;
    const int64_t ro = perm ? (int64_t)perm[r] : r;
    V3 xb = load3(xbar + 3 * ro), db = load3(dmob + 3 * r);
    for (int c = a.pptr[r]; c < a.pptr[r + 1]; ++c) {
        xb = xb + load3(gbar + 9 * (int64_t)c);
        db = db + load3(gbar + 9 * (int64_t)c + 3);
    }
    for (int k = a.qptr[r]; k < a.qptr[r + 1]; ++k) {
        const int64_t c = a.qidx[k];
        xb = xb - load3(gbar + 9 * c);
        db = db + load3(gbar + 9 * c + 6);
    }
    store3(xbar + 3 * ro, xb);
    const double s = quat[4 * ro], px = quat[4 * ro + 1], py = quat[4 * ro + 2], pz = quat[4 * ro + 3];
    double b0 = qbd[4 * r] + 2.0 * (py * db.x - px * db.y + s * db.z);
    double b1 = qbd[4 * r + 1] + 2.0 * (pz * db.x - s * db.y - px * db.z);
    double b2 = qbd[4 * r + 2] + 2.0 * (s * db.x + pz * db.y - py * db.z);
    double b3 = qbd[4 * r + 3] + 2.0 * (px * db.x + py * db.y + pz * db.z);
    const double qq = s * s + px * px + py * py + pz * pz;
    const double pr = (b0 * s + b1 * px + b2 * py + b3 * pz) / qq;
    quatbar[4 * ro] = b0 - pr * s;
    quatbar[4 * ro + 1] = b1 - pr * px;
    quatbar[4 * ro + 2] = b2 - pr * py;
    quatbar[4 * ro + 3] = b3 - pr * pz;
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
int adjoint_core(rl_ctx *h, SolveArgs &a, bool step, const double *Ubar, const double *F, const int *perm,
                 double cg_tol, const AdjOut &o, rl_adjoint_info *info)
{
    hipStream_t st = h->stream;
    const rl_params &p = h->prm;
    const bool uni = a.coef == nullptr;
    const int64_t n = a.n, nc = a.nc, nb = nc > 0 ? nc : 1, rb = n > 0 ? n : 1;
    int err = 0;
    double *wsol = (double *)ws_get(h, kWsAdjG, sizeof(double) * nb, &err);
    CgArgs g;
    g.cs = (double *)ws_get(h, kWsAdjCs, sizeof(double) * 4 * nb, &err);
    g.cr = (double *)ws_get(h, kWsAdjCr, sizeof(double) * 4 * nb, &err);
    g.cq = (double *)ws_get(h, kWsAdjCq, sizeof(double) * 4 * nb, &err);
    g.sc = (double *)ws_get(h, kWsAdjSc, sizeof(double) * 8, &err);
    double *PQ = (double *)ws_get(h, kWsAdjPQ, sizeof(double) * 12 * rb, &err);
    a.V = (double *)ws_get(h, kWsV, sizeof(double) * 6 * rb, &err);
    if (err) return err;
    g.ab = g.sc + 4;
    if (!(cg_tol > 0.0)) cg_tol = 1e-10;
    // w = Mc gamma + q at the solution: A = {gamma_c > w_c}
    int rc = apply_impl(h, a, wsol);
    if (rc) return rc;
    g.a = a;
    if (n > 0) {
        if (uni)
            hipLaunchKernelGGL(HIP_KERNEL_NAME(k_adj_prep<true>), dim3(grid_of(n, kBlock)), dim3(kBlock), 0, st, a,
                               Ubar);
        else
            hipLaunchKernelGGL(HIP_KERNEL_NAME(k_adj_prep<false>), dim3(grid_of(n, kBlock)), dim3(kBlock), 0, st, a,
                               Ubar);
        RL_HIP(hipGetLastError());
    }
    hipLaunchKernelGGL(k_state_init, dim3(1), dim3(64), 0, st, h->state, cg_tol, (long long)p.max_iter);
    RL_HIP(hipGetLastError());
    long long iters = 0, nact = 0;
    double res = 0.0;
    int status = RL_OK;
    if (nc > 0) {
        hipLaunchKernelGGL(k_cg_start, dim3(a.gcon), dim3(kConBlock), 0, st, g, (const double *)wsol);
        RL_HIP(hipGetLastError());
        const int every = p.check_every > 0 ? p.check_every : 32;
        const dim3 rgrid(rod_grid8(n > 0 ? n : 1));
        long long launched = 0;
        auto enqueue = [&](int cnt) -> int {
            for (int k = 0; k < cnt; ++k, ++launched) {
                if (uni)
                    hipLaunchKernelGGL(HIP_KERNEL_NAME(k_cg_rod<true>), rgrid, dim3(kRodLoopBlock), 0, st,
                                       (const int32_t *)a.pptr, (const int32_t *)a.qptr, (const double *)g.cr,
                                       (const double *)g.cq, a.geo, a.qgeo, (unsigned)rgrid.x, (int)a.n, g, launched);
                else
                    hipLaunchKernelGGL(HIP_KERNEL_NAME(k_cg_rod<false>), rgrid, dim3(kRodLoopBlock), 0, st,
                                       (const int32_t *)a.pptr, (const int32_t *)a.qptr, (const double *)g.cr,
                                       (const double *)g.cq, a.geo, a.qgeo, (unsigned)rgrid.x, (int)a.n, g, launched);
                RL_HIP(hipGetLastError());
                hipLaunchKernelGGL(k_cg_con, dim3(a.gcon), dim3(kConBlock), 0, st, (const int32_t *)a.qpos,
                                   (const double *)a.uP, (const double *)a.uQ, (const double *)g.cs,
                                   (const double *)g.cr, (int)a.nc, (unsigned)a.gcon, (const double *)g.ab, g,
                                   launched);
                RL_HIP(hipGetLastError());
            }
            return RL_OK;
        };
        // the state is copied after every `every` iterations; a few more are
        // queued behind each copy before the host waits for it, so the GPU
        // never idles on the host (iterations after the stop return at once)
        const int la = std::min(every, 8);
        if (!h->chk_ev) RL_HIP(hipEventCreateWithFlags(&h->chk_ev, hipEventDisableTiming));
        if ((rc = enqueue(every))) return rc;
        for (;;) {
            RL_HIP(hipMemcpyAsync(h->state_host, h->state, sizeof(SolverState), hipMemcpyDeviceToHost, st));
            RL_HIP(hipEventRecord(h->chk_ev, st));
            const long long checked = launched;
            if ((rc = enqueue(la))) return rc;
            RL_HIP(hipEventSynchronize(h->chk_ev));
            if (h->state_host->done) break;
            if (checked > p.max_iter + every + 1) {
                set_error("adjoint: CG stop flag never raised");
                return RL_ERR_HIP;
            }
            if ((rc = enqueue(every - la))) return rc;
        }
        iters = h->state_host->iter;
        res = h->state_host->res;
        nact = (long long)h->state_host->ss;
        status = h->state_host->status;
    }
    if (n > 0) {
        const dim3 grid(grid_of(n, kRodBlock / kRodLanes));
#define RL_ADJ_ROD(U_, S_)                                                                                      \
    hipLaunchKernelGGL(HIP_KERNEL_NAME(k_adj_rod<U_, S_>), grid, dim3(kRodBlock), 0, st, g, Ubar, F, perm, PQ, \
                       o.F_bar, o.dmob)
        if (uni && step) RL_ADJ_ROD(true, true);
        else if (uni) RL_ADJ_ROD(true, false);
        else if (step) RL_ADJ_ROD(false, true);
        else RL_ADJ_ROD(false, false);
#undef RL_ADJ_ROD
        RL_HIP(hipGetLastError());
    }
    if (nc > 0) {
        hipLaunchKernelGGL(k_adj_con, dim3(grid_of(nc, kBlock)), dim3(kBlock), 0, st, g, (const double *)PQ, o.q_bar,
                           o.e_bar, o.arm_bar, o.d_bar);
        RL_HIP(hipGetLastError());
    }
    if (info) {
        info->cg_iterations = iters;
        info->cg_residual = res;
        info->n_active = nact;
        info->status = status;
    }
    if (status == RL_ERR_NONFINITE) {
        set_error("adjoint: non-finite value in the CG iteration");
        return status;
    }
    return status;
}

hipError_t launch_dir_bar(hipStream_t st, const SolveArgs &a, const double *dmob, const double *d_bar, double *dir_bar)
{
    if (a.n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_dir_bar, dim3(grid_of(a.n, kBlock)), dim3(kBlock), 0, st, a, dmob, d_bar, dir_bar);
    return hipGetLastError();
}

hipError_t launch_integrate_adj(hipStream_t st, int64_t n, const int *perm, const double *x_bar,
                                const double *quat_bar, const double *quat, const double *U, double dt, double *Ubar,
                                double *qbd)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_integrate_adj, dim3(grid_of(n, kBlock)), dim3(kBlock), 0, st, n, perm, x_bar, quat_bar, quat,
                       U, dt, Ubar, qbd);
    return hipGetLastError();
}

hipError_t launch_step_bar(hipStream_t st, const SolveArgs &a, const int *perm, const double *gbar, const double *dmob,
                           const double *qbd, const double *quat, double *x_bar, double *quat_bar)
{
    if (a.n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_step_bar, dim3(grid_of(a.n, kBlock)), dim3(kBlock), 0, st, a, perm, gbar, dmob, qbd, quat,
                       x_bar, quat_bar);
    return hipGetLastError();
}

}  // namespace rl
