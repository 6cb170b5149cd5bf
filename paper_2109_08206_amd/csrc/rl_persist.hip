// Persistent BBPGD loop (FP64, single system) on gfx950.
//
// The two-kernel loop (rl_solver.hip) pays, in every launch, a chain of
// dependent loads: the rods' list offsets, then their records, then the
// step-length partials.  Here one cooperative launch runs the whole loop.
// Each workgroup (one per compute unit) owns a block of consecutive rods (cell
// order) and the constraints whose P rod it owns, and keeps in LDS, for the
// whole solve, its rods' list offsets, the geometry (e, s) of their P-side
// and Q-side incidences, and the P-side contact velocities u_P.  An iteration
// is then
//   rod phase:        f, m of each own rod from its incidences (state of the
//                     own P side from global memory, Q side written by the
//                     owners of the other rods), V, W, and u for each of its
//                     contacts: u_P into LDS, u_Q to global memory in the
//                     constraint's own slot;
//   grid barrier;
//   constraint phase: w = u_P - u_Q + q for the own constraints, projection,
//                     BB dot products and residual; the new state, its Q-side
//                     copy for the owner of pj, one partial per workgroup;
//   grid barrier;
//   every workgroup sums all partials in the same order and takes the same
//   step-length and stop decision (the rule of rl_device.hpp).
//
// The L2 caches of the eight XCDs are not coherent with each other, and a
// device-scope fence writes back and invalidates the whole L2 of the issuing
// XCD.  So the arrays one workgroup writes and another reads (u_Q, the Q-side
// state copy, the partials) are written and read with device-scope relaxed
// atomic stores and loads, which go through to the memory side, and the grid
// barrier is a two-level counter (one per XCD group, then one global) of
// relaxed device-scope atomics: no fences.  Data each workgroup keeps to
// itself (its P-side state) stays in ordinary loads and stores.  Every wait is
// bounded: a workgroup that waits longer than the spin limit raises an error
// flag, and every waiting workgroup leaves as soon as it sees the flag.
//
// Chosen by rl_set_loop(RL_LOOP_PERSISTENT) when the rods split into at most
// one block per compute unit whose records fit the LDS.  It is correct and
// bitwise repeatable, but on this part it is no faster than two launches per
// iteration: the device-scope accesses that cross XCDs are slow, and the two
// barriers cost about as much as the two kernel boundaries.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <vector>

#include "rl_device.hpp"

namespace rl {

constexpr int kPBlock = 1024;                  // threads per workgroup
constexpr int kPLdsBytes = 160 * 1024 - 4096;  // dynamic LDS per workgroup (the rest: static)
constexpr int kPSpin = 1 << 22;                // polls before a barrier wait gives up (seconds)

struct PersistArgs {
    const int *wr0;  // [G+1] first rod of each workgroup
    int cap;         // records per side kept in LDS
    int rmax;        // most rods in a workgroup
    int *bar;        // [9][32] barrier counters: global, then one per XCD group
    int *err;        // set when a barrier wait times out
    double *wpart;   // [2][G][4] workgroup partials by iteration parity
};

__device__ __forceinline__ double ld_dev(const double *p)
{
    return __hip_atomic_load(const_cast<double *>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_dev(double *p, double v)
{
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Grid barrier number b (counted by the caller).  Returns false after a
// time-out anywhere in the grid.
__device__ __forceinline__ bool grid_barrier(const PersistArgs &p, int &b, int *ok)
{
    __syncthreads();  // every wave's stores have completed
    if (threadIdx.x == 0) {
        const int G = gridDim.x, x = blockIdx.x & 7, per = (G - x + 7) / 8;
        const int old = __hip_atomic_fetch_add(p.bar + 32 * (1 + x), 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (old == (b + 1) * per - 1) __hip_atomic_fetch_add(p.bar, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        const int groups = G < 8 ? G : 8, target = (b + 1) * groups;
        int good = 1;
        for (int n = 0; __hip_atomic_load(p.bar, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target; ++n) {
            if (n >= kPSpin || __hip_atomic_load(p.err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
                __hip_atomic_store(p.err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                good = 0;
                break;
            }
            __builtin_amdgcn_s_sleep(1);
        }
        *ok = good;
    }
    ++b;
    __syncthreads();
    return *ok != 0;
}

// One record's state for the rod phase: the own P side with a plain load,
// the Q side (written by the owner of the other rod) with device-scope loads.
__device__ __forceinline__ double2 p_state(const SolveArgs &a, int c, int e)
{
    return c < e ? a.st[c] : make_double2(0.0, 0.0);
}
__device__ __forceinline__ double2 q_state(const SolveArgs &a, int c, int e)
{
    return c < e ? make_double2(ld_dev(&a.stq[c].x), ld_dev(&a.stq[c].y)) : make_double2(0.0, 0.0);
}

template <bool UNI>
__global__ void __launch_bounds__(kPBlock) k_persist(SolveArgs a, PersistArgs p)
{
    extern __shared__ double sm[];
    __shared__ double red[kPBlock / 64 + 1][4];
    __shared__ int ok;
    constexpr int kRpp = kPBlock / kRodLanes;  // rods per pass
    const int G = gridDim.x, wg = blockIdx.x, t = threadIdx.x;
    const int R0 = p.wr0[wg], nr = p.wr0[wg + 1] - R0, cap = p.cap;
    double *pg = sm;            // [cap][4] (ex, ey, ez, s_i) of the own P-side records
    double *qg = sm + 4 * cap;  // [cap][4] (ex, ey, ez, s_j) of the own Q-side records
    double *up = sm + 8 * cap;  // [cap] u_P of the own constraints
    int *qi = reinterpret_cast<int *>(sm + 9 * cap);  // [cap] constraint of each own Q-side record
    int *rp = qi + cap;                                 // [rmax+1] P offsets of the own rods
    int *rq = rp + p.rmax + 1;                          // [rmax+1] Q offsets
    for (int i = t; i <= nr; i += kPBlock) {
        rp[i] = a.pptr[R0 + i];
        rq[i] = a.qptr[R0 + i];
    }
    __syncthreads();
    const int P0 = rp[0], np = rp[nr] - P0, Q0 = rq[0], nq = rq[nr] - Q0;
    for (int j = t; j < np; j += kPBlock) {
        const double2 *s = reinterpret_cast<const double2 *>(a.geo + 4 * (int64_t)(P0 + j));
        double2 *d = reinterpret_cast<double2 *>(pg + 4 * j);
        d[0] = s[0];
        d[1] = s[1];
    }
    for (int j = t; j < nq; j += kPBlock) {
        const double2 *s = reinterpret_cast<const double2 *>(a.qgeo + 4 * (int64_t)(Q0 + j));
        double2 *d = reinterpret_cast<double2 *>(qg + 4 * j);
        d[0] = s[0];
        d[1] = s[1];
        qi[j] = a.qidx[Q0 + j];
    }
    SolverState *st = a.state;
    if (st->done) return;  // written by an earlier launch: the same in every workgroup
    const double tol = st->tol, amin = st->amin, amax = st->amax;
    const long long max_iter = st->max_iter;
    double alpha = st->alpha;
    int b = 0;
    __syncthreads();
    const int sub = t & (kRodLanes - 1);
    for (long long k = 0;; ++k) {
        // ---- rod phase: two rods per lane group, their first two records of
        // each side loaded together
        for (int base = 0; base < nr; base += 2 * kRpp) {
            int pb[2], pe[2], qb[2], qe[2];
            double2 ps[2][2], qs[2][2];
#pragma unroll
            for (int i = 0; i < 2; ++i) {
                const int lr = base + i * kRpp + t / kRodLanes;
                pb[i] = pe[i] = qb[i] = qe[i] = 0;
                if (lr < nr) {
                    pb[i] = rp[lr] + sub;
                    pe[i] = rp[lr + 1];
                    qb[i] = rq[lr] + sub;
                    qe[i] = rq[lr + 1];
                }
#pragma unroll
                for (int u = 0; u < 2; ++u) {
                    ps[i][u] = p_state(a, pb[i] + u * kRodLanes, pe[i]);
                    qs[i][u] = q_state(a, qb[i] + u * kRodLanes, qe[i]);
                }
            }
#pragma unroll
            for (int i = 0; i < 2; ++i) {
                const int lr = base + i * kRpp + t / kRodLanes;
                double f[3] = {0.0, 0.0, 0.0}, m[3] = {0.0, 0.0, 0.0};
                for (int c = pb[i], u = 0; c < pe[i]; c += kRodLanes, ++u) {
                    const double2 sg = u < 2 ? ps[i][u] : a.st[c];
                    const double *g = pg + 4 * (c - P0);
                    rod_add(1.0, gamma_prime<kModeLoop>(sg.x, sg.y, alpha), make_double2(g[0], g[1]),
                            make_double2(g[2], g[3]), f, m);
                }
                for (int c = qb[i], u = 0; c < qe[i]; c += kRodLanes, ++u) {
                    const double2 sg = u < 2 ? qs[i][u] : q_state(a, c, qe[i]);
                    const double *g = qg + 4 * (c - Q0);
                    rod_add(-1.0, gamma_prime<kModeLoop>(sg.x, sg.y, alpha), make_double2(g[0], g[1]),
                            make_double2(g[2], g[3]), f, m);
                }
#pragma unroll
                for (int o = 1; o < kRodLanes; o <<= 1) {
#pragma unroll
                    for (int d = 0; d < 3; ++d) {
                        f[d] += __shfl_xor(f[d], o, 64);
                        m[d] += __shfl_xor(m[d], o, 64);
                    }
                }
                if (lr < nr) {
                    const int64_t r = R0 + lr;
                    const double dx = a.dir[3 * r], dy = a.dir[3 * r + 1], dz = a.dir[3 * r + 2];
                    double apar, aperp, rperp;
                    rod_mob(a, r, UNI, apar, aperp, rperp);
                    const double fd = (apar - aperp) * (dx * f[0] + dy * f[1] + dz * f[2]);
                    const double md = dx * m[0] + dy * m[1] + dz * m[2];
                    const double v[3] = {aperp * f[0] + fd * dx, aperp * f[1] + fd * dy, aperp * f[2] + fd * dz};
                    const double w[3] = {rperp * (m[0] - md * dx), rperp * (m[1] - md * dy),
                                         rperp * (m[2] - md * dz)};
                    for (int c = pb[i]; c < pe[i]; c += kRodLanes) {
                        const double *g = pg + 4 * (c - P0);
                        up[c - P0] = u_along(make_double2(g[0], g[1]), make_double2(g[2], g[3]), v, w);
                    }
                    // u_Q goes to the constraint's own slot (P order), where its owner reads it
                    for (int c = qb[i]; c < qe[i]; c += kRodLanes) {
                        const double *g = qg + 4 * (c - Q0);
                        st_dev(a.uQ + qi[c - Q0], u_along(make_double2(g[0], g[1]), make_double2(g[2], g[3]), v, w));
                    }
                }
            }
        }
        if (!grid_barrier(p, b, &ok)) return;
        // ---- constraint phase: two constraints per thread, loads first
        double ps4[4] = {0.0, 0.0, 0.0, 0.0};
        for (int j0 = 0; j0 < np; j0 += 2 * kPBlock) {
            int qp[2];
            double uq[2], qv[2];
            double2 sg[2];
#pragma unroll
            for (int i = 0; i < 2; ++i) {
                const int j = j0 + i * kPBlock + t;
                if (j < np) {
                    const int64_t c = P0 + j;
                    qp[i] = a.qpos[c];
                    uq[i] = ld_dev(a.uQ + c);
                    sg[i] = a.st[c];
                    qv[i] = a.qv[c];
                }
            }
#pragma unroll
            for (int i = 0; i < 2; ++i) {
                const int j = j0 + i * kPBlock + t;
                if (j >= np) continue;
                const int64_t c = P0 + j;
                const double wv = up[j] - uq[i] + qv[i];
                const double gp = gamma_prime<kModeLoop>(sg[i].x, sg[i].y, alpha);
                const double sc = gp - sg[i].x, yc = wv - sg[i].y;
                a.st[c] = make_double2(gp, wv);
                st_dev(&a.stq[qp[i]].x, gp);
                st_dev(&a.stq[qp[i]].y, wv);
                ps4[0] += sc * sc;
                ps4[1] += sc * yc;
                ps4[2] += yc * yc;
                ps4[3] = fmax(ps4[3], fabs(gp < wv ? gp : wv));
            }
        }
        block_reduce4_all<kPBlock / 64>(ps4, red);
        double *part = p.wpart + ((int64_t)(k & 1) * G + wg) * 4;
        if (t < 4) st_dev(part + t, ps4[t]);
        if (!grid_barrier(p, b, &ok)) return;
        // ---- totals (workgroups in index order, the same tree everywhere) and the decision
        double tt[4] = {0.0, 0.0, 0.0, 0.0};
        for (int v = t; v < G; v += kPBlock) {
            const double *src = p.wpart + ((int64_t)(k & 1) * G + v) * 4;
            tt[0] += ld_dev(src);
            tt[1] += ld_dev(src + 1);
            tt[2] += ld_dev(src + 2);
            tt[3] = fmax(tt[3], ld_dev(src + 3));
        }
        block_reduce4_all<kPBlock / 64>(tt, red);
        const Decision d = decide_from(DecideIn{tol, amin, amax, alpha, max_iter}, k + 1, tt);
        if (d.stop) {
            if (wg == 0 && t == 0) {
                st->iter = k + 1;
                st->res = tt[3];
                st->ss = tt[0];
                st->sy = tt[1];
                st->yy = tt[2];
                st->status = d.status;
                st->done = 1;
            }
            return;
        }
        alpha = d.alpha;
    }
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
// Greedy split of the rods (in order) into at most G blocks with at most L
// records per side each; returns the number of blocks, or G + 1 if it fails.
static int split_rods(const std::vector<int> &pp, const std::vector<int> &qp, int64_t n, int G, int L,
                      std::vector<int> *start)
{
    int blocks = 0;
    int64_t r = 0;
    if (start) start->clear();
    while (r < n) {
        if (blocks == G) return G + 1;
        if (start) start->push_back((int)r);
        const int p0 = pp[r], q0 = qp[r];
        int64_t e = r;
        while (e < n && pp[e + 1] - p0 <= L && qp[e + 1] - q0 <= L) ++e;
        if (e == r) return G + 1;  // one rod alone exceeds L
        r = e;
        ++blocks;
    }
    return blocks;
}

int persistent_plan(rl_ctx *h, const SolveArgs &a, PersistPlan *plan)
{
    plan->ok = false;
    if (a.n <= 0 || a.nc <= 0) return RL_OK;
    int dev = 0;
    RL_HIP(hipGetDevice(&dev));
    hipDeviceProp_t prop;
    RL_HIP(hipGetDeviceProperties(&prop, dev));
    if (!prop.cooperativeLaunch) return RL_OK;
    // the kernels may use more than the default 64 KB of dynamic LDS (a
    // setting of the current device; repeating it is harmless)
    RL_HIP(hipFuncSetAttribute((const void *)k_persist<true>, hipFuncAttributeMaxDynamicSharedMemorySize,
                               kPLdsBytes));
    RL_HIP(hipFuncSetAttribute((const void *)k_persist<false>, hipFuncAttributeMaxDynamicSharedMemorySize,
                               kPLdsBytes));
    int per_cu = 0;
    RL_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void *)k_persist<true>, kPBlock,
                                                        kPLdsBytes));
    const int G = std::min(per_cu, 1) * prop.multiProcessorCount;
    if (G < 8) return RL_OK;
    // the rods' offsets on the host
    const int64_t n = a.n;
    int werr = 0;
    int *hp = (int *)ws_get_host(h, sizeof(int) * 2 * (n + 1), &werr);
    if (werr) return werr;
    RL_HIP(hipMemcpyAsync(hp, a.pptr, sizeof(int) * (n + 1), hipMemcpyDeviceToHost, h->stream));
    RL_HIP(hipMemcpyAsync(hp + n + 1, a.qptr, sizeof(int) * (n + 1), hipMemcpyDeviceToHost, h->stream));
    RL_HIP(hipStreamSynchronize(h->stream));
    std::vector<int> pp(hp, hp + n + 1), qp(hp + n + 1, hp + 2 * (n + 1));
    // the smallest per-side limit L that splits the rods into G blocks (which
    // balances them), then whether L record slots (76 bytes each: two
    // geometries, u_P and a Q-side constraint index) and the blocks' offsets
    // fit the LDS
    const int budget = kPLdsBytes / 76;
    if (split_rods(pp, qp, n, G, budget, nullptr) > G) return RL_OK;
    int lo = (int)((a.nc + G - 1) / G), L = budget;
    while (lo < L) {
        const int mid = (lo + L) / 2;
        if (split_rods(pp, qp, n, G, mid, nullptr) <= G) L = mid;
        else lo = mid + 1;
    }
    std::vector<int> s;
    split_rods(pp, qp, n, G, L, &s);
    int rmax = 0;
    std::vector<int> &wr = plan->wr0;
    wr.assign(G + 1, (int)n);
    for (size_t i = 0; i < s.size(); ++i) wr[i] = s[i];
    for (int i = 0; i < G; ++i) rmax = std::max(rmax, wr[i + 1] - wr[i]);
    if (76 * (size_t)L + 8 * (size_t)(rmax + 1) > (size_t)kPLdsBytes) return RL_OK;
    plan->G = G;
    plan->cap = L;
    plan->rmax = rmax;
    plan->ok = true;
    return RL_OK;
}

int solve_loop_persistent(rl_ctx *h, const SolveArgs &a, const PersistPlan &plan, float *ms)
{
    hipStream_t st = h->stream;
    int werr = 0;
    const int G = plan.G;
    int *wr0 = (int *)ws_get(h, kWsPersistMap, sizeof(int) * (G + 1), &werr);
    int *bar = (int *)ws_get(h, kWsPersistBar, sizeof(int) * (9 * 32 + 32), &werr);
    double *wpart = (double *)ws_get(h, kWsPersistPart, sizeof(double) * 8 * G, &werr);
    if (werr) return werr;
    int *hm = (int *)ws_get_host(h, sizeof(int) * (G + 1), &werr);
    if (werr) return werr;
    std::copy(plan.wr0.begin(), plan.wr0.end(), hm);
    RL_HIP(hipMemcpyAsync(wr0, hm, sizeof(int) * (G + 1), hipMemcpyHostToDevice, st));
    RL_HIP(hipMemsetAsync(bar, 0, sizeof(int) * (9 * 32 + 32), st));
    PersistArgs p{wr0, plan.cap, plan.rmax, bar, bar + 9 * 32, wpart};
    SolveArgs args = a;
    void *kargs[] = {&args, &p};
    for (int v = 0; v < 2; ++v)
        if (!h->pev[v]) RL_HIP(hipEventCreate(&h->pev[v]));
    RL_HIP(hipEventRecord(h->pev[0], st));
    const void *fn = a.coef == nullptr ? (const void *)k_persist<true> : (const void *)k_persist<false>;
    RL_HIP(hipLaunchCooperativeKernel(fn, dim3(G), dim3(kPBlock), kargs, kPLdsBytes, st));
    RL_HIP(hipEventRecord(h->pev[1], st));
    RL_HIP(hipMemcpyAsync(h->state_host, h->state, sizeof(SolverState), hipMemcpyDeviceToHost, st));
    RL_HIP(hipMemcpyAsync(h->host_scratch, bar + 9 * 32, sizeof(int), hipMemcpyDeviceToHost, st));
    RL_HIP(hipStreamSynchronize(st));
    if (((int *)h->host_scratch)[0]) {
        set_error("rl_solve_lcp: a grid barrier of the persistent loop timed out");
        return RL_ERR_HIP;
    }
    RL_HIP(hipEventElapsedTime(ms, h->pev[0], h->pev[1]));
    return RL_OK;
}

}  // namespace rl
