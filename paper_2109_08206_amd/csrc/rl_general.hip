// General constraint sets: unilateral and bilateral constraints together,
// some of them against fixed bodies (eq. linearconstraints a and b; eq.
// blockdef, all four blocks; Appendix "Equation of motion with geometric
// constraints" for one-sided columns).
//
// The loop kernels of the plain solve run unchanged in their general mode:
// the constraints are merged into one list ordered by (P rod, kind), so each
// rod's P-side records are its unilateral ones followed by its bilateral
// ones, and each Q-side list holds the unilateral before the bilateral
// records; two per-rod split indices tell the rod kernel where projection
// stops.  The constraint kernel reads one more number per constraint, the
// compliance 1/(kappa h) of a bilateral row (or -1 for a unilateral one), and
// a constraint without a Q side (qpos < 0) reads no contact velocity there.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>

#include "rl_device.hpp"

namespace rl {

static inline unsigned grid_of(int64_t n) { return (unsigned)((n + kBlock - 1) / kBlock); }

// bit 0: an index outside the rods; bit 1: a bad kind; bit 2: a bad
// compliance (negative or not finite)
__global__ void k_gen_check(int64_t n, int64_t nc, const int32_t *__restrict__ pi, const int32_t *__restrict__ pj,
                            const uint8_t *__restrict__ kind, const double *__restrict__ cmp, int *__restrict__ err)
{
    const int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (c >= nc) return;
    const int a = pi[c], b = pj[c];
    if (a < 0 || a >= n || b < -1 || b >= n) atomicOr(err, 1);
    const int k = kind ? kind[c] : 0;
    if (k != 0 && k != 1) atomicOr(err, 2);
    if (k == 1 && (!cmp || !(cmp[c] >= 0.0) || !isfinite(cmp[c]))) atomicOr(err, 4);
}

// sort key: P rod, then kind (unilateral first)
__global__ void k_gen_keys(int64_t nc, const int32_t *__restrict__ pi, const uint8_t *__restrict__ kind,
                           int *__restrict__ key)
{
    const int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (c >= nc) return;
    key[c] = 2 * pi[c] + (kind ? (int)kind[c] : 0);
}

// the merged list: constraint m is the input's ord[m]
__global__ void k_gen_gather(int64_t nc, const int *__restrict__ ord, const int32_t *__restrict__ pi,
                             const int32_t *__restrict__ pj, const double *__restrict__ e,
                             const double *__restrict__ arm, const double *__restrict__ q,
                             const uint8_t *__restrict__ kind, const double *__restrict__ cmp,
                             const double *__restrict__ gamma, int32_t *__restrict__ mpi, int32_t *__restrict__ mpj,
                             double *__restrict__ me, double *__restrict__ marm, double *__restrict__ mq,
                             double *__restrict__ mcmp, double *__restrict__ mgamma)
{
    const int64_t m = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (m >= nc) return;
    const int64_t c = ord[m];
    mpi[m] = pi[c];
    mpj[m] = pj[c];
    for (int a = 0; a < 3; ++a) me[3 * m + a] = e[3 * c + a];
    marm[2 * m] = arm[2 * c];
    marm[2 * m + 1] = arm[2 * c + 1];
    mq[m] = q[c];
    const bool bil = kind && kind[c] == 1;
    mcmp[m] = bil ? cmp[c] : -1.0;
    mgamma[m] = gamma ? gamma[c] : 0.0;
}

// pptr[r] = first merged constraint with pi >= r (pi sorted)
__global__ void k_gen_pptr(int64_t n, int64_t nc, const int32_t *__restrict__ pi, int32_t *__restrict__ pptr)
{
    const int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (c > nc) return;
    const int64_t a = c < nc ? (int64_t)pi[c] : n;
    const int64_t prev = c > 0 ? (int64_t)pi[c - 1] : -1;
    for (int64_t r = prev + 1; r <= a; ++r) pptr[r] = (int32_t)c;
}

__global__ void k_gen_qcount(int64_t nc, const int32_t *__restrict__ pj, int *__restrict__ qcnt)
{
    const int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (c >= nc) return;
    if (pj[c] >= 0) atomicAdd(qcnt + pj[c], 1);
}

__global__ void k_gen_qfill(int64_t nc, const int32_t *__restrict__ pj, const int32_t *__restrict__ qptr,
                            int *__restrict__ qcur, int32_t *__restrict__ qidx)
{
    const int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (c >= nc) return;
    const int r = pj[c];
    if (r < 0) return;
    qidx[qptr[r] + atomicAdd(qcur + r, 1)] = (int32_t)c;
}

// Each rod's Q list in (kind, constraint) order, its first bilateral
// position, and the first bilateral constraint of its P range.
__global__ void k_gen_rodlists(int64_t n, const int32_t *__restrict__ pptr, const int32_t *__restrict__ qptr,
                               const double *__restrict__ cmpv, int32_t *__restrict__ qidx,
                               int32_t *__restrict__ psplit, int32_t *__restrict__ qsplit)
{
    const int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (r >= n) return;
    const int b = qptr[r], e = qptr[r + 1];
    auto key = [&](int32_t c) -> long long { return ((long long)(cmpv[c] >= 0.0) << 32) | (long long)c; };
    for (int k = b + 1; k < e; ++k) {
        const int32_t v = qidx[k];
        const long long kv = key(v);
        int m = k - 1;
        while (m >= b && key(qidx[m]) > kv) {
            qidx[m + 1] = qidx[m];
            --m;
        }
        qidx[m + 1] = v;
    }
    int qs = e;
    for (int k = b; k < e; ++k)
        if (cmpv[qidx[k]] >= 0.0) {
            qs = k;
            break;
        }
    qsplit[r] = qs;
    const int pb = pptr[r], pe = pptr[r + 1];
    int ps = pe;
    for (int c = pb; c < pe; ++c)
        if (cmpv[c] >= 0.0) {
            ps = c;
            break;
        }
    psplit[r] = ps;
}

// records (as the plain solve's k_pack; q alone, state (gamma, 0))
__global__ void k_gen_pack(int64_t nc, const int32_t *__restrict__ pi, const int32_t *__restrict__ pj,
                           const double *__restrict__ e, const double *__restrict__ arm, const double *__restrict__ q,
                           const double *__restrict__ gamma, int2 *__restrict__ pp, double *__restrict__ geo,
                           double2 *__restrict__ geo2, double *__restrict__ qv, double2 *__restrict__ st,
                           int32_t *__restrict__ qpos)
{
    const int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (c >= nc) return;
    pp[c] = make_int2(pi[c], pj[c]);
    double2 *gd = reinterpret_cast<double2 *>(geo + 4 * c);
    gd[0] = make_double2(e[3 * c], e[3 * c + 1]);
    gd[1] = make_double2(e[3 * c + 2], arm[2 * c]);
    geo2[c] = make_double2(arm[2 * c + 1], q[c]);
    qv[c] = q[c];
    st[c] = make_double2(gamma[c], 0.0);
    qpos[c] = -1;  // filled below for constraints with a Q side
}

// Q-side copies for the qptr[n] entries of the Q lists
__global__ void k_gen_pack_q(int64_t n, int64_t nc, const int32_t *__restrict__ qptr,
                             const int32_t *__restrict__ qidx, const double *__restrict__ geo,
                             const double2 *__restrict__ geo2, const double2 *__restrict__ st,
                             int32_t *__restrict__ qpos, double *__restrict__ qgeo, double2 *__restrict__ stq)
{
    const int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (k >= nc || k >= qptr[n]) return;
    const int c = qidx[k];
    qpos[c] = (int32_t)k;
    const double2 *gd = reinterpret_cast<const double2 *>(geo + 4 * (int64_t)c);
    const double2 g0 = gd[0], g1 = gd[1];
    double2 *qd = reinterpret_cast<double2 *>(qgeo + 4 * k);
    qd[0] = g0;
    qd[1] = make_double2(g1.x, geo2[c].x);
    stq[k] = st[c];
}

__global__ void k_gen_scatter_gamma(int64_t nc, const double2 *__restrict__ st, const int *__restrict__ ord,
                                    double *__restrict__ gamma)
{
    const int64_t m = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (m >= nc) return;
    gamma[ord[m]] = st[m].x;
}

hipError_t launch_scatter_gamma(hipStream_t st, const SolveArgs &a, const int *order, double *gamma)
{
    if (a.nc <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_gen_scatter_gamma, dim3(grid_of(a.nc)), dim3(kBlock), 0, st, a.nc, (const double2 *)a.st,
                       order, gamma);
    return hipGetLastError();
}

int prepare_general(rl_ctx *h, int64_t n, const double *dir, const double *len, double len0, int64_t nc,
                    const int32_t *pi, const int32_t *pj, const double *e, const double *arm, const double *q,
                    const uint8_t *kind, const double *cmp, const double *gamma, bool trusted, SolveArgs *out,
                    const int **order)
{
    hipStream_t st = h->stream;
    const rl_params &p = h->prm;
    int werr = 0;
    if (!trusted && nc > 0) {
        RL_HIP(hipMemsetAsync(h->flag_dev, 0, sizeof(int), st));
        hipLaunchKernelGGL(k_gen_check, dim3(grid_of(nc)), dim3(kBlock), 0, st, n, nc, pi, pj, kind, cmp,
                           h->flag_dev);
        RL_HIP(hipGetLastError());
        RL_HIP(hipMemcpyAsync(h->host_scratch, h->flag_dev, sizeof(int), hipMemcpyDeviceToHost, st));
        RL_HIP(hipStreamSynchronize(st));
        const int f = ((int *)h->host_scratch)[0];
        if (f) {
            set_error(f & 1 ? "constraint rods must satisfy 0 <= pi < n and -1 <= pj < n"
                            : (f & 2 ? "kind must be 0 (unilateral) or 1 (bilateral)"
                                     : "a bilateral constraint needs a finite compliance cmp >= 0"));
            return RL_ERR_ARG;
        }
    }
    const int64_t nb = nc > 0 ? nc : 1, rb = n > 0 ? n : 1;
    int *key = (int *)ws_get(h, kWsGenKey, sizeof(int) * nb, &werr);
    int *key_out = (int *)ws_get(h, kWsGenKeyOut, sizeof(int) * nb, &werr);
    int *ord = (int *)ws_get(h, kWsGenOrd, sizeof(int) * nb, &werr);
    int32_t *mpi = (int32_t *)ws_get(h, kWsGenPi, sizeof(int32_t) * nb, &werr);
    int32_t *mpj = (int32_t *)ws_get(h, kWsGenPj, sizeof(int32_t) * nb, &werr);
    double *me = (double *)ws_get(h, kWsGenE, sizeof(double) * 3 * nb, &werr);
    double *marm = (double *)ws_get(h, kWsGenArm, sizeof(double) * 2 * nb, &werr);
    double *mq = (double *)ws_get(h, kWsGenQ, sizeof(double) * nb, &werr);
    double *mcmp = (double *)ws_get(h, kWsGenCmp, sizeof(double) * nb, &werr);
    double *mgam = (double *)ws_get(h, kWsGenGamma, sizeof(double) * nb, &werr);
    int32_t *psplit = (int32_t *)ws_get(h, kWsGenPsplit, sizeof(int32_t) * rb, &werr);
    int32_t *qsplit = (int32_t *)ws_get(h, kWsGenQsplit, sizeof(int32_t) * rb, &werr);
    if (werr) return werr;
    if (nc > 0) {
        hipLaunchKernelGGL(k_gen_keys, dim3(grid_of(nc)), dim3(kBlock), 0, st, nc, pi, kind, key);
        RL_HIP(hipGetLastError());
        int bits = 1;
        while ((1LL << bits) < 2 * n + 2) ++bits;
        const int rc = stable_sort_by_key(h, nc, key, bits, key_out, ord);
        if (rc) return rc;
        hipLaunchKernelGGL(k_gen_gather, dim3(grid_of(nc)), dim3(kBlock), 0, st, nc, (const int *)ord, pi, pj, e, arm,
                           q, kind, cmp, gamma, mpi, mpj, me, marm, mq, mcmp, mgam);
        RL_HIP(hipGetLastError());
    }
    SolveArgs s{};
    s.n = n;
    s.nc = nc;
    s.dir = dir;
    s.mob = mobility_host(len ? 1.0 : len0, p.diam, p.eta);
    int64_t gc = std::min<int64_t>(std::max<int64_t>((nc + kConPerGroup - 1) / kConPerGroup, 1), kConGridMax);
    s.gcon = (int)((gc + 7) / 8 * 8);
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
    s.gen = true;
    s.psplit = psplit;
    s.qsplit = qsplit;
    s.cmpv = mcmp;
    if (len) RL_HIP(launch_mobility_coeffs(st, n, len, p.diam, p.eta, coef));
    hipLaunchKernelGGL(k_gen_pptr, dim3(grid_of(nc + 1)), dim3(kBlock), 0, st, n, nc, (const int32_t *)mpi, pptr);
    RL_HIP(hipGetLastError());
    if (n > 0) {
        RL_HIP(hipMemsetAsync(qcnt, 0, sizeof(int) * n, st));
        if (nc > 0) {
            hipLaunchKernelGGL(k_gen_qcount, dim3(grid_of(nc)), dim3(kBlock), 0, st, nc, (const int32_t *)mpj, qcnt);
            RL_HIP(hipGetLastError());
        }
        const int rc = device_scan(h, qcnt, n, qptr, nullptr, scan_tmp);
        if (rc) return rc;
        if (nc > 0) {
            RL_HIP(hipMemsetAsync(qcnt, 0, sizeof(int) * n, st));
            hipLaunchKernelGGL(k_gen_qfill, dim3(grid_of(nc)), dim3(kBlock), 0, st, nc, (const int32_t *)mpj,
                               (const int32_t *)qptr, qcnt, qidx);
            RL_HIP(hipGetLastError());
        }
        hipLaunchKernelGGL(k_gen_rodlists, dim3(grid_of(n)), dim3(kBlock), 0, st, n, (const int32_t *)pptr,
                           (const int32_t *)qptr, (const double *)mcmp, qidx, psplit, qsplit);
        RL_HIP(hipGetLastError());
    }
    if (nc > 0) {
        hipLaunchKernelGGL(k_gen_pack, dim3(grid_of(nc)), dim3(kBlock), 0, st, nc, (const int32_t *)mpi,
                           (const int32_t *)mpj, (const double *)me, (const double *)marm, (const double *)mq,
                           (const double *)mgam, pp, geo, geo2, qv, s.st, qpos);
        RL_HIP(hipGetLastError());
        if (n > 0) {
            hipLaunchKernelGGL(k_gen_pack_q, dim3(grid_of(nc)), dim3(kBlock), 0, st, n, nc, (const int32_t *)qptr,
                               (const int32_t *)qidx, (const double *)geo, (const double2 *)geo2,
                               (const double2 *)s.st, qpos, qgeo, s.stq);
            RL_HIP(hipGetLastError());
        }
    }
    *out = s;
    *order = ord;
    return RL_OK;
}

// ---------------------------------------------------------------------------
// Multi-step pieces of a step
// ---------------------------------------------------------------------------
// Brownian force per rod, caller order: F_B = sqrt(2 kT/h) M^(-1/2) xi with
// M^(-1/2) = a_perp^(-1/2) I + (a_par^(-1/2) - a_perp^(-1/2)) d d^T on the
// translation and r^(-1/2) I on the rotation (axial = normal mobility).
__global__ void k_brownian(int64_t n, const double *__restrict__ dir, const double *__restrict__ len, double len0,
                           double diam, double eta, double amp, const double *__restrict__ xi,
                           const double *__restrict__ F, double *__restrict__ Ftot)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double L = len ? len[i] : len0;
    const double lg = log(2.0 * L / diam);
    const double aperp = lg / (4.0 * M_PI * eta * L), apar = 2.0 * aperp;
    const double rperp = 3.0 * lg / (M_PI * eta * L * L * L);
    const double sn = 1.0 / sqrt(aperp), sp = 1.0 / sqrt(apar), sr = 1.0 / sqrt(rperp);
    const double dx = dir[3 * i], dy = dir[3 * i + 1], dz = dir[3 * i + 2];
    const double *z = xi + 6 * i;
    const double dz3 = (sp - sn) * (dx * z[0] + dy * z[1] + dz * z[2]);
    const double fb[6] = {sn * z[0] + dz3 * dx, sn * z[1] + dz3 * dy, sn * z[2] + dz3 * dz,
                          sr * z[3], sr * z[4], sr * z[5]};
    for (int a = 0; a < 6; ++a) Ftot[6 * i + a] = (F ? F[6 * i + a] : 0.0) + amp * fb[a];
}

hipError_t launch_brownian(hipStream_t st, int64_t n, const double *dir, const double *len, double len0, double diam,
                           double eta, double dt, double kT, const double *noise, const double *F, double *Ftot)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_brownian, dim3(grid_of(n)), dim3(kBlock), 0, st, n, dir, len, len0, diam, eta,
                       sqrt(2.0 * kT / dt), noise, F, Ftot);
    return hipGetLastError();
}

// Key of input constraint c in the caller's numbering: a contact by its two
// rods (smaller caller index first, the shift negated when they swap) and
// shift, a link by its key (or index); wall contacts have no key (0).
__device__ __forceinline__ unsigned long long step_key(const StepList &L, int64_t c)
{
    if (c < L.np) {
        unsigned long long a = (unsigned)L.perm[L.pi[c]], b = (unsigned)L.perm[L.pj[c]];
        int img = L.img[c];
        if (a > b) {
            const unsigned long long t = a;
            a = b;
            b = t;
            const int sx = ((img >> 8) & 15) - 8, sy = ((img >> 4) & 15) - 8, sz = (img & 15) - 8;
            img = ((-sx + 8) << 8) | ((-sy + 8) << 4) | (-sz + 8);
        }
        return (1ull << 62) | (a << 37) | (b << 12) | (unsigned long long)img;
    }
    if (c < L.np + L.nl) {
        const int64_t k = c - L.np;
        return (2ull << 62) | ((unsigned long long)(L.link_key ? L.link_key[k] : k) & ((1ull << 62) - 1ull));
    }
    return 0ull;
}

__global__ void k_warm_lookup(StepList L, const unsigned long long *__restrict__ keys,
                              const double *__restrict__ gam, int64_t m, double *__restrict__ gamma0)
{
    const int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (c >= L.nc) return;
    const unsigned long long k = step_key(L, c);
    double g = 0.0;
    if (k != 0ull && m > 0) {
        int64_t lo = 0, hi = m;  // first stored key >= k
        while (lo < hi) {
            const int64_t mid = (lo + hi) >> 1;
            if (keys[mid] < k) lo = mid + 1;
            else hi = mid;
        }
        if (lo < m && keys[lo] == k) g = gam[lo];
    }
    gamma0[c] = g;
}

__global__ void k_warm_keys(StepList L, const double *__restrict__ gamma, unsigned long long *__restrict__ keys,
                            double *__restrict__ vals)
{
    const int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (c >= L.nc) return;
    keys[c] = step_key(L, c);
    vals[c] = gamma[c];
}

int warm_lookup(rl_ctx *h, const StepList &L, double *gamma0)
{
    if (L.nc <= 0) return RL_OK;
    const bool have = h->warm_count >= 0 && h->warm_n == L.n;
    hipLaunchKernelGGL(k_warm_lookup, dim3(grid_of(L.nc)), dim3(kBlock), 0, h->stream, L,
                       (const unsigned long long *)h->buf[kWsWarmKeys], (const double *)h->buf[kWsWarmGam],
                       have ? h->warm_count : (int64_t)0, gamma0);
    RL_HIP(hipGetLastError());
    return RL_OK;
}

int warm_store(rl_ctx *h, const StepList &L, const double *gamma)
{
    int werr = 0;
    const int64_t nb = L.nc > 0 ? L.nc : 1;
    auto *kn = (unsigned long long *)ws_get(h, kWsWarmKeysNew, sizeof(unsigned long long) * nb, &werr);
    auto *vn = (double *)ws_get(h, kWsWarmGamNew, sizeof(double) * nb, &werr);
    auto *ks = (unsigned long long *)ws_get(h, kWsWarmKeys, sizeof(unsigned long long) * nb, &werr);
    auto *vs = (double *)ws_get(h, kWsWarmGam, sizeof(double) * nb, &werr);
    if (werr) return werr;
    if (L.nc > 0) {
        hipLaunchKernelGGL(k_warm_keys, dim3(grid_of(L.nc)), dim3(kBlock), 0, h->stream, L, gamma, kn, vn);
        RL_HIP(hipGetLastError());
        const int rc = sort_key_values(h, L.nc, kn, vn, ks, vs);
        if (rc) return rc;
    }
    h->warm_count = L.nc;
    h->warm_n = L.n;
    return RL_OK;
}

// per-workgroup partial sums of gamma (x_P - x_Q') e^T over contacts [0..8]
// and two-sided links [9..17] (walls and links to fixed points are external)
constexpr int kStressBlock = 256;

__global__ void __launch_bounds__(kStressBlock) k_stress(StepList L, double diam, const double *__restrict__ gamma,
                                                        double *__restrict__ part)
{
    __shared__ double lds[kStressBlock / 64][18];
    double acc[18];
    for (int k = 0; k < 18; ++k) acc[k] = 0.0;
    for (int64_t c = blockIdx.x * (int64_t)kStressBlock + threadIdx.x; c < L.np + L.nl;
         c += (int64_t)gridDim.x * kStressBlock) {
        const double g = gamma[c];
        const double e[3] = {L.e[3 * c], L.e[3 * c + 1], L.e[3 * c + 2]};
        const double si = L.arm[2 * c], sj = L.arm[2 * c + 1];
        const int P = L.pi[c], Q = L.pj[c];
        if (Q < 0) continue;
        // x_P - x_Q' = r - s_P d_P + s_Q d_Q with r the vector between the two
        // points: (phi + diam) e for a contact, length e for a link
        const double rl = c < L.np ? L.phi[c] + diam : L.link_len[c - L.np];
        const int off = c < L.np ? 0 : 9;
        for (int a = 0; a < 3; ++a) {
            const double ra = rl * e[a] - si * L.dir[3 * (int64_t)P + a] + sj * L.dir[3 * (int64_t)Q + a];
            for (int b = 0; b < 3; ++b) acc[off + 3 * a + b] += g * ra * e[b];
        }
    }
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    for (int k = 0; k < 18; ++k) {
        double v = acc[k];
        for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
        if (lane == 0) lds[w][k] = v;
    }
    __syncthreads();
    if (threadIdx.x < 18) {
        double v = 0.0;
        for (int k = 0; k < kStressBlock / 64; ++k) v += lds[k][threadIdx.x];
        part[18 * (int64_t)blockIdx.x + threadIdx.x] = v;
    }
}

int step_stress(rl_ctx *h, const StepList &L, const double *gamma, double *out)
{
    const rl_params &p = h->prm;
    const int64_t m = L.np + L.nl;
    const unsigned grid = (unsigned)std::max<int64_t>(1, std::min<int64_t>((m + kStressBlock - 1) / kStressBlock, 512));
    int werr = 0;
    double *part = (double *)ws_get(h, kWsStress, sizeof(double) * 18 * grid, &werr);
    if (werr) return werr;
    int err = 0;
    double *host = (double *)ws_get_host(h, sizeof(double) * 18 * grid, &err);
    if (err) return err;
    hipLaunchKernelGGL(k_stress, dim3(grid), dim3(kStressBlock), 0, h->stream, L, p.diam, gamma, part);
    RL_HIP(hipGetLastError());
    RL_HIP(hipMemcpyAsync(host, part, sizeof(double) * 18 * grid, hipMemcpyDeviceToHost, h->stream));
    RL_HIP(hipStreamSynchronize(h->stream));
    const double V = p.box[0] * p.box[1] * p.box[2];
    for (int k = 0; k < 18; ++k) {
        double v = 0.0;
        for (unsigned b = 0; b < grid; ++b) v += host[18 * b + k];
        out[k] = v / V;
    }
    return RL_OK;
}

int wall_set(int n_walls, const rl_wall *walls, WallSet *W)
{
    *W = WallSet{};
    if (n_walls < 0 || n_walls > RL_MAX_WALLS || (n_walls > 0 && !walls)) {
        set_error("walls: need 0 <= n_walls <= %d and a wall array", RL_MAX_WALLS);
        return RL_ERR_ARG;
    }
    W->n = n_walls;
    for (int w = 0; w < n_walls; ++w) {
        const rl_wall &src = walls[w];
        const double an = sqrt(src.a[0] * src.a[0] + src.a[1] * src.a[1] + src.a[2] * src.a[2]);
        const bool needs_a = src.kind == RL_WALL_PLANE || src.kind == RL_WALL_CYLINDER_IN;
        const bool needs_r = src.kind == RL_WALL_SPHERE_IN || src.kind == RL_WALL_CYLINDER_IN;
        if (src.kind < RL_WALL_PLANE || src.kind > RL_WALL_CYLINDER_IN || (needs_a && !(fabs(an - 1.0) < 1e-12)) ||
            (needs_r && !(src.r > 0.0)) || !std::isfinite(src.p[0] + src.p[1] + src.p[2])) {
            set_error("walls: wall %d has an unknown kind, a normal or axis that is not a unit vector, or a "
                      "radius <= 0", w);
            return RL_ERR_ARG;
        }
        W->kind[w] = src.kind;
        W->r[w] = src.r;
        for (int k = 0; k < 3; ++k) {
            W->p[w][k] = src.p[k];
            W->a[w][k] = src.a[k];
        }
    }
    return RL_OK;
}

}  // namespace rl

using namespace rl;

extern "C" {

int rl_assemble_walls(rl_handle h, int64_t n, const double *x, const double *dir, const double *len, double len0,
                      const double *F, int32_t n_walls, const rl_wall *walls, int64_t capacity, int32_t *rod,
                      double *e, double *arm, double *phi, double *q, uint8_t *flags, int64_t *n_contacts)
{
    if (!h) {
        set_error("handle is NULL");
        return RL_ERR_ARG;
    }
    RL_HIP(hipSetDevice(h->device));
    if (n < 0 || n >= 0x7fffffff || capacity < 0 || (n > 0 && (!x || !dir)) || (!len && !(len0 > 0.0)) ||
        (capacity > 0 && (!rod || !e || !arm || !phi || !q))) {
        set_error("rl_assemble_walls: bad sizes or NULL array");
        return RL_ERR_ARG;
    }
    WallSet W;
    int rc = wall_set(n_walls, walls, &W);
    if (rc) return rc;
    int werr = 0;
    double *Unc = (double *)ws_get(h, kWsUnc, sizeof(double) * 6 * (n > 0 ? n : 1), &werr);
    if (werr) return werr;
    if (F) RL_HIP(launch_unc(h->stream, n, dir, len, len0, h->prm.diam, h->prm.eta, F, Unc));
    else RL_HIP(hipMemsetAsync(Unc, 0, sizeof(double) * 6 * (n > 0 ? n : 1), h->stream));
    int64_t m = 0;
    rc = walls_impl(h, n, x, dir, len, len0, Unc, W, capacity, rod, e, arm, phi, q, flags, &m);
    if (n_contacts) *n_contacts = m;
    if (rc) return rc;
    RL_HIP(hipStreamSynchronize(h->stream));
    return RL_OK;
}

int rl_assemble_links(rl_handle h, int64_t n, const double *x, const double *dir, const double *len, double len0,
                      const rl_links *links, const double *F, double *length, double *e, double *q, double *cmp,
                      uint8_t *flags)
{
    if (!h) {
        set_error("handle is NULL");
        return RL_ERR_ARG;
    }
    RL_HIP(hipSetDevice(h->device));
    if (!links || links->n_links < 0 || links->n_links >= 0x7fffffff || n < 0 || n >= 0x7fffffff) {
        set_error("rl_assemble_links: bad links or sizes");
        return RL_ERR_ARG;
    }
    const int64_t nl = links->n_links;
    if (nl == 0) return RL_OK;
    if (!x || !dir || !links->p || !links->q || !links->arm || !links->kappa || !links->rest || !length || !e ||
        !q || !cmp || (!len && !(len0 > 0.0))) {
        set_error("rl_assemble_links: NULL array");
        return RL_ERR_ARG;
    }
    hipStream_t st = h->stream;
    int werr = 0;
    double *Unc = (double *)ws_get(h, kWsUnc, sizeof(double) * 6 * (n > 0 ? n : 1), &werr);
    int32_t *lpi = (int32_t *)ws_get(h, kWsGenPi, sizeof(int32_t) * nl, &werr);
    int32_t *lpj = (int32_t *)ws_get(h, kWsGenPj, sizeof(int32_t) * nl, &werr);
    double *larm = (double *)ws_get(h, kWsGenArm, sizeof(double) * 2 * nl, &werr);
    if (werr) return werr;
    if (F) RL_HIP(launch_unc(st, n, dir, len, len0, h->prm.diam, h->prm.eta, F, Unc));
    else RL_HIP(hipMemsetAsync(Unc, 0, sizeof(double) * 6 * (n > 0 ? n : 1), st));
    RL_HIP(hipMemsetAsync(h->flag_dev, 0, sizeof(int), st));
    RL_HIP(launch_links(st, nl, n, x, dir, nullptr, links, h->prm.box, h->prm.dt, Unc, lpi, lpj, length, e, larm, q,
                        cmp, flags, h->flag_dev));
    RL_HIP(hipMemcpyAsync(h->host_scratch, h->flag_dev, sizeof(int), hipMemcpyDeviceToHost, st));
    RL_HIP(hipStreamSynchronize(st));
    if (((int *)h->host_scratch)[0]) {
        set_error("rl_assemble_links: a link has a rod index outside [0, n), p == q, kappa <= 0, a bad rest "
                  "length or no anchor");
        return RL_ERR_ARG;
    }
    return RL_OK;
}

int rl_solve_general(rl_handle h, int64_t n, const double *dir, const double *len, double len0, int64_t nc,
                     const int32_t *pi, const int32_t *pj, const double *e, const double *arm, const double *q,
                     const uint8_t *kind, const double *cmp, const double *F, double *gamma, double *U,
                     rl_solve_info *info)
{
    if (!h) {
        set_error("handle is NULL");
        return RL_ERR_ARG;
    }
    RL_HIP(hipSetDevice(h->device));
    if (n < 0 || n >= 0x7fffffff || nc < 0 || nc >= 0x7fffffff) {
        set_error("rl_solve_general: bad sizes");
        return RL_ERR_ARG;
    }
    if ((nc > 0 && (!dir || !pi || !pj || !e || !arm || !q || !gamma)) || (n > 0 && U && !dir) ||
        (!len && !(len0 > 0.0))) {
        set_error("rl_solve_general: NULL array or len0 <= 0 without len");
        return RL_ERR_ARG;
    }
    if (h->prm.precision != RL_FP64) {
        set_error("rl_solve_general: RL_FP64 only");
        return RL_ERR_ARG;
    }
    SolveArgs a;
    const int *ord = nullptr;
    int rc = prepare_general(h, n, dir, len, len0, nc, pi, pj, e, arm, q, kind, cmp, gamma, false, &a, &ord);
    if (rc) return rc;
    rc = solve_impl(h, a, F, U, nullptr, info);
    if (rc < 0) return rc;
    RL_HIP(launch_scatter_gamma(h->stream, a, ord, gamma));
    RL_HIP(hipStreamSynchronize(h->stream));
    return rc;
}

}  // extern "C"
