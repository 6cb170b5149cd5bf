// Batched BBPGD: many independent systems of uneven size solved together.
//
// The systems are concatenated (rods, then constraints, system after
// system), so the incidence structure, the packed records and the per-rod /
// per-constraint work are exactly those of the single-system solver.  What
// is per system is the BB state: every workgroup of both kernels works on
// rods or constraints of one system only (tile tables built on the host),
// constraint workgroups leave one partial per tile, and the rod workgroups of
// a system sum that system's partials to get its step length and stop test.
// The first rod tile of a system publishes its step and latches its stop; a
// finished system's workgroups return at once, so converged systems retire
// while the others continue.
//
// Iterations are replayed from a captured HIP graph of B iterations; the
// iteration number comes from a device counter that a one-thread kernel at
// the end of the graph advances by B (kernel nodes keep fixed arguments).
// Workgroup sizes are chosen by timing the candidates on the problem itself
// (cached per problem-size bucket; optionally persisted to the file named by
// RODLCP_TUNE_CACHE).
//
// A cooperative persistent kernel with grid barriers would avoid the
// launches but needs a device-scope release/acquire at every barrier, which
// on this part writes back and invalidates the L2 of every XCD for each
// workgroup; the launch-per-phase scheme needs none.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <vector>

#include "rl_device.hpp"

namespace rl {

static inline unsigned grid_of(int64_t n, int block) { return (unsigned)((n + block - 1) / block); }

struct BatchArgs {
    SolveArgs a;             // the concatenated system
    SolverState *sst;        // [S]
    double *alpha_s;         // [S][2]
    // Tile records by workgroup (the host has applied the XCD-aware tile map
    // and padded the grid to a multiple of 8 with records of system -1), one
    // load each: the rod tile of workgroup w is rt[2w] = (first rod, end rod,
    // system, publishes) and rt[2w+1] = (the system's first and end
    // constraint tile, 0, 0); the constraint tile of workgroup w is ct[w] =
    // (first constraint, end, system, tile number).
    const int4 *rt;
    const int4 *ct;
    const int *sys_c0;       // [S+1] first constraint tile of each system
    int nrb, ncb;            // tiles (the grids are padded to multiples of 8)
    int S;
    double *partial;         // [2][ncb][4]
    long long *kbase;        // iteration number of graph node 0
    int *ndone;              // systems finished
    int *done_s;             // [S] 1 once system s has stopped
};

static const int kBatchRodBlocks[2] = {256, 1024};
constexpr int kComputeUnits = 256;  // MI355X
static const int kBatchConBlocks[2] = {256, 512};

// stop of system s: results for the host, the flag, the count
__device__ __forceinline__ void latch(const BatchArgs &b, int s, long long k, const double t[4], int status)
{
    SolverState *st = b.sst + s;
    st->iter = k;
    st->res = t[3];
    st->ss = t[0];
    st->sy = t[1];
    st->yy = t[2];
    st->status = status;
    st->done = 1;
    b.done_s[s] = 1;
    atomicAdd(b.ndone, 1);
}

// The tile table and the arrays of the first loads lead the argument list
// (14 dwords, preloaded into registers).
template <int MODE, bool UNI, int RB, int R>
__global__ void __launch_bounds__(RB)
    k_rod_b(const int4 *__restrict__ rt, const int32_t *__restrict__ pptr, const int32_t *__restrict__ qptr,
            const double2 *sg, const double2 *sgq, const double *__restrict__ geo, const double *__restrict__ qgeo,
            BatchArgs b, int i)
{
    __shared__ double lds[RB / 64 + 1][4];
    const int sub = threadIdx.x & (kRodLanes - 1);
    const int4 t0 = rt[2 * blockIdx.x], t1 = rt[2 * blockIdx.x + 1];
    if (t0.z < 0) return;  // padding
    const int64_t r = (int64_t)t0.x + threadIdx.x / kRodLanes;
    const bool active = r < t0.y;
    // records first: they depend neither on the system's state nor on its step
    RodLoads<R> L;
    rod_load(pptr, qptr, sg, sgq, geo, qgeo, r, active, sub, L);
    // the counter and the system's partials are read before the stop flag,
    // so that the three loads are in flight together.  The counter base is
    // even, so the parity of k is that of i: the partials' address does not
    // wait for the counter.
    const long long kb = MODE == kModeLoop ? *b.kbase : 0;
    const double *part = b.partial + ((int64_t)((i - 1) & 1) * b.ncb + t1.x) * 4;
    PartFirst pf;
    if (MODE == kModeLoop) partials_first(part, t1.y - t1.x, pf);
    const int s = t0.z;
    SolverState *st = b.sst + s;
    // the rod's direction and mobility and the system's step-rule inputs
    // (the parity of i is that of k) are read before the flag too
    const SolveArgs &a = b.a;
    const int64_t rr = active ? r : 0;
    const double dx = a.dir[3 * rr], dy = a.dir[3 * rr + 1], dz = a.dir[3 * rr + 2];
    double apar, aperp, rperp;
    rod_mob(a, rr, UNI, apar, aperp, rperp);
    DecideIn din{};
    if (MODE == kModeLoop) din = decide_in(st, b.alpha_s + 2 * s, (long long)i);
    if (MODE != kModeApply && st->done) return;
    const long long k = kb + i;
    double alpha = 0.0;
    if (MODE == kModeLoop) {
        const bool publisher = t0.w && threadIdx.x == 0;
        double *abuf = b.alpha_s + 2 * s;
        if (k == 0) {
            alpha = st->alpha;
            if (publisher) abuf[0] = alpha;
        } else {
            double t[4];
            sum_partials_from<RB / 64>(pf, part, t1.y - t1.x, t, lds);
            const Decision d = decide_from(din, k, t);
            if (publisher) {
                if (d.stop) latch(b, s, k, t, d.status);
                else abuf[k & 1] = d.alpha;
            }
            if (d.stop) return;
            alpha = d.alpha;
        }
    }
    double f[3], m[3];
    rod_accumulate<MODE>(b.a, L, alpha, f, m);
    if (!active) return;
    const double fd = (apar - aperp) * (dx * f[0] + dy * f[1] + dz * f[2]);
    const double md = dx * m[0] + dy * m[1] + dz * m[2];
    const double v[3] = {aperp * f[0] + fd * dx, aperp * f[1] + fd * dy, aperp * f[2] + fd * dz};
    const double w[3] = {rperp * (m[0] - md * dx), rperp * (m[1] - md * dy), rperp * (m[2] - md * dz)};
    rod_emit_u(a, L, v, w);
}

template <int MODE, int CB>
__global__ void __launch_bounds__(CB)
    k_con_b(const int4 *__restrict__ ct, const int32_t *__restrict__ qpos, const double *__restrict__ uP,
            const double *__restrict__ qv, const double2 *sg, const double *__restrict__ uQ, const double *alpha_s,
            BatchArgs b, int i)
{
    __shared__ double lds[CB / 64 + 1][4];
    double p[4] = {0.0, 0.0, 0.0, 0.0};
    const int4 tc = ct[blockIdx.x];
    if (tc.z < 0) return;  // padding
    const ConIn in{qpos, uP, qv, sg, uQ};
    const int64_t hi = tc.y;
    // first round peeled: its records are in flight before the system's stop
    // flag and step are read (every thread reaches the test)
    int64_t c0 = tc.x + threadIdx.x;
    ConLoadsU A, B;
    if (c0 < hi) con_load_u<MODE>(in, c0, A);
    if (c0 + CB < hi) con_load_u<MODE>(in, c0 + CB, B);
    const int s = tc.z;
    SolverState *st = b.sst + s;
    // parity of the iteration = parity of i (the counter base is even); the
    // step length is read with the stop flag (for nothing after the stop)
    const int par = MODE == kModeLoop ? (i & 1) : 0;
    const double alpha = MODE == kModeLoop ? alpha_s[2 * s + par] : 0.0;
    if (MODE != kModeApply && st->done) return;
    for (;;) {
        if (c0 < hi) con_update_u<MODE>(b.a, c0, A, alpha, p);
        if (c0 + CB < hi) con_update_u<MODE>(b.a, c0 + CB, B, alpha, p);
        c0 += 2 * CB;
        if (c0 >= hi) break;
        con_load_u<MODE>(in, c0, A);
        if (c0 + CB < hi) con_load_u<MODE>(in, c0 + CB, B);
    }
    if (MODE == kModeApply) return;
    block_total4<CB / 64>(p, lds);
    if (threadIdx.x == 0) {
        double2 *dst = reinterpret_cast<double2 *>(b.partial + ((int64_t)par * b.ncb + tc.w) * 4);
        dst[0] = make_double2(p[0], p[1]);
        dst[1] = make_double2(p[2], p[3]);
    }
}

// One workgroup per system: totals of the start phases.
template <int MODE>
__global__ void __launch_bounds__(256) k_fin_b(BatchArgs b)
{
    __shared__ double lds[256 / 64 + 1][4];
    const int s = blockIdx.x;
    SolverState *st = b.sst + s;
    if (st->done) return;
    double t[4];
    const int c0 = b.sys_c0[s], c1 = b.sys_c0[s + 1];
    sum_partials<256 / 64>(b.partial + (int64_t)c0 * 4, c1 - c0, t, lds);
    if (threadIdx.x != 0) return;
    if (MODE == kModeInit) {
        st->res = t[3];
        if (!isfinite(t[2]) || !isfinite(t[3])) latch(b, s, 0, t, RL_ERR_NONFINITE);
        else if (t[3] <= st->tol) latch(b, s, 0, t, RL_OK);
    } else {
        if (!isfinite(t[0]) || !isfinite(t[1])) {
            latch(b, s, 0, t, RL_ERR_NONFINITE);
            return;
        }
        if (t[0] == 0.0) {
            const double r4[4] = {0.0, 0.0, 0.0, st->res};
            latch(b, s, 0, r4, RL_OK);
            return;
        }
        const double a0 = t[1] > 0.0 ? t[0] / t[1] : 1.0;
        st->alpha0 = a0;
        st->alpha = a0;
        st->amin = 1e-12 * a0;
        st->amax = 1e12 * a0;
        if (st->max_iter <= 0) {
            const double r4[4] = {0.0, 0.0, 0.0, st->res};
            latch(b, s, 0, r4, RL_NOT_CONVERGED);
        }
    }
}

__global__ void k_state_init_b(SolverState *sst, int S, double tol, long long max_iter, long long *kbase, int *ndone,
                               int *done_s)
{
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s == 0) {
        *kbase = 0;
        *ndone = 0;
    }
    if (s >= S) return;
    done_s[s] = 0;
    SolverState *st = sst + s;
    st->alpha = st->alpha0 = st->amin = st->amax = 0.0;
    st->res = st->ss = st->sy = st->yy = 0.0;
    st->tol = tol;
    st->max_iter = max_iter;
    st->iter = 0;
    st->done = 0;
    st->status = RL_OK;
    st->inner_tol = tol;
    st->rho64 = 0.0;
    st->refreshes = 0;
    st->refresh = 0;
}

// partials of the surviving systems' tiles to their positions in the
// compacted tile table (one parity)
__global__ void k_remap_partials(int ncb_new, const int *__restrict__ old_of_new, const double *__restrict__ src,
                                 double *__restrict__ dst)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= ncb_new) return;
    const double *a = src + 4 * (int64_t)old_of_new[t];
    double *d = dst + 4 * (int64_t)t;
    d[0] = a[0];
    d[1] = a[1];
    d[2] = a[2];
    d[3] = a[3];
}

__global__ void k_advance(long long *kbase, int B)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) *kbase += B;
}

// each constraint must join two rods of its own system
__global__ void k_check_batch(int64_t nc, int S, const int64_t *__restrict__ rod_off,
                              const int64_t *__restrict__ pair_off, const int32_t *__restrict__ pi,
                              const int32_t *__restrict__ pj, int *__restrict__ err)
{
    const int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (c >= nc) return;
    int lo = 0, hi = S;  // last s with pair_off[s] <= c
    while (hi - lo > 1) {
        const int mid = (lo + hi) / 2;
        if (pair_off[mid] <= c) lo = mid;
        else hi = mid;
    }
    if (pi[c] < rod_off[lo] || pj[c] >= rod_off[lo + 1]) atomicOr(err, 4);
}

// --- host ------------------------------------------------------------------------

struct BatchTables {
    std::vector<int> rsys, rlo, rhi, csys, clo, chi, sc0, sr0;
};

static void build_tables(int S, const int64_t *rod_off, const int64_t *pair_off, int rod_block, int con_block,
                         BatchTables &t, const std::vector<int> *done = nullptr)
{
    const int rods_per = rod_block / kRodLanes, cons_per = 2 * con_block;
    t = BatchTables{};
    t.sc0.assign(S + 1, 0);
    t.sr0.assign(S, 0);
    for (int s = 0; s < S; ++s) {
        const int64_t nc = pair_off[s + 1] - pair_off[s];
        t.sc0[s] = (int)t.csys.size();
        t.sr0[s] = (int)t.rsys.size();
        if (nc == 0) continue;                 // nothing to iterate: U = M F
        if (done && (*done)[s]) continue;      // finished: its tiles are dropped
        for (int64_t c = pair_off[s]; c < pair_off[s + 1]; c += cons_per) {
            t.csys.push_back(s);
            t.clo.push_back((int)c);
            t.chi.push_back((int)std::min<int64_t>(c + cons_per, pair_off[s + 1]));
        }
        for (int64_t r = rod_off[s]; r < rod_off[s + 1]; r += rods_per) {
            t.rsys.push_back(s);
            t.rlo.push_back((int)r);
            t.rhi.push_back((int)std::min<int64_t>(r + rods_per, rod_off[s + 1]));
        }
    }
    t.sc0[S] = (int)t.csys.size();
}

static inline unsigned pad8(int n) { return (unsigned)((std::max(n, 1) + 7) / 8 * 8); }

// the device's xcd_tile on the host
static inline unsigned xcd_tile_host(unsigned b, unsigned nblocks)
{
    if (nblocks % 8 != 0) return b;
    return (b % 8) * (nblocks / 8) + b / 8;
}

template <int MODE, int RB, int R>
static void launch_rod_b_r(hipStream_t st, const BatchArgs &b, bool uni, int i)
{
    const SolveArgs &a = b.a;
    if (uni)
        hipLaunchKernelGGL(HIP_KERNEL_NAME(k_rod_b<MODE, true, RB, R>), dim3(pad8(b.nrb)), dim3(RB), 0, st, b.rt,
                           a.pptr, a.qptr, (const double2 *)a.st, (const double2 *)a.stq, a.geo, a.qgeo, b, i);
    else
        hipLaunchKernelGGL(HIP_KERNEL_NAME(k_rod_b<MODE, false, RB, R>), dim3(pad8(b.nrb)), dim3(RB), 0, st, b.rt,
                           a.pptr, a.qptr, (const double2 *)a.st, (const double2 *)a.stq, a.geo, a.qgeo, b, i);
}

// The loop kernel holds five rounds of records when the batch as a whole is
// dense (four lanes per rod, which the tile tables assume), in 256-thread
// groups (1,024-thread groups leave 128 registers a lane, too few for five
// rounds).
template <int MODE, int RB>
static hipError_t launch_rod_b(hipStream_t st, const BatchArgs &b, bool uni, int i)
{
    if (b.nrb == 0) return hipSuccess;
    if constexpr (MODE == kModeLoop && RB == 256) {
        if (rod_dense(b.a.n, b.a.nc)) {
            launch_rod_b_r<MODE, RB, kRodRoundsDense>(st, b, uni, i);
            return hipGetLastError();
        }
    }
    launch_rod_b_r<MODE, RB, kRodRounds>(st, b, uni, i);
    return hipGetLastError();
}

template <int MODE, int CB>
static hipError_t launch_con_b(hipStream_t st, const BatchArgs &b, int i)
{
    if (b.ncb == 0) return hipSuccess;
    const SolveArgs &a = b.a;
    hipLaunchKernelGGL(HIP_KERNEL_NAME(k_con_b<MODE, CB>), dim3(pad8(b.ncb)), dim3(CB), 0, st, b.ct, a.qpos,
                       (const double *)a.uP, a.qv, (const double2 *)a.st, (const double *)a.uQ,
                       (const double *)b.alpha_s, b, i);
    return hipGetLastError();
}

template <int MODE>
static hipError_t launch_pair_b(hipStream_t st, const BatchArgs &b, bool uni, int rb, int cb, int i)
{
    hipError_t e = rb == 256 ? launch_rod_b<MODE, 256>(st, b, uni, i) : launch_rod_b<MODE, 1024>(st, b, uni, i);
    if (e != hipSuccess) return e;
    return cb == 256 ? launch_con_b<MODE, 256>(st, b, i) : launch_con_b<MODE, 512>(st, b, i);
}

static hipError_t start_phases(hipStream_t st, const BatchArgs &b, bool uni, int rb, int cb, const rl_params &p)
{
    hipLaunchKernelGGL(k_state_init_b, dim3(grid_of(b.S, 256)), dim3(256), 0, st, b.sst, b.S, p.tol,
                       (long long)p.max_iter, b.kbase, b.ndone, b.done_s);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if ((e = launch_pair_b<kModeInit>(st, b, uni, rb, cb, 0)) != hipSuccess) return e;
    hipLaunchKernelGGL(HIP_KERNEL_NAME(k_fin_b<kModeInit>), dim3(b.S), dim3(256), 0, st, b);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if ((e = launch_pair_b<kModeAlpha0>(st, b, uni, rb, cb, 0)) != hipSuccess) return e;
    hipLaunchKernelGGL(HIP_KERNEL_NAME(k_fin_b<kModeAlpha0>), dim3(b.S), dim3(256), 0, st, b);
    return hipGetLastError();
}

// Uploads the tile tables and fills the table pointers of b.
static int upload_tables(rl_ctx *h, hipStream_t st, const BatchTables &t, int S, BatchArgs &b)
{
    int werr = 0;
    const int nrt = (int)t.rsys.size(), nct = (int)t.csys.size();
    const size_t nr = pad8(nrt), ncb = pad8(nct);  // workgroups of the two grids
    // int4 records first (16-byte aligned), then the per-system tile starts
    const size_t words = 4 * (2 * nr + ncb) + (S + 1);
    int *tab = (int *)ws_get(h, kWsBatchTab, sizeof(int) * words, &werr);
    int *host = (int *)ws_get_host(h, sizeof(int) * words, &werr);
    if (werr) return werr;
    std::fill(host, host + words, 0);
    // workgroup w takes tile xcd_tile(w): each XCD a contiguous range of tiles
    for (size_t w = 0; w < nr; ++w) {
        const int j = (int)xcd_tile_host((unsigned)w, (unsigned)nr);
        int *o = host + 8 * w;
        if (j >= nrt) {
            o[2] = -1;
            continue;
        }
        const int s = t.rsys[j];
        o[0] = t.rlo[j];
        o[1] = t.rhi[j];
        o[2] = s;
        o[3] = j == t.sr0[s];
        o[4] = t.sc0[s];
        o[5] = t.sc0[s + 1];
    }
    for (size_t w = 0; w < ncb; ++w) {
        const int j = (int)xcd_tile_host((unsigned)w, (unsigned)ncb);
        int *o = host + 8 * nr + 4 * w;
        if (j >= nct) {
            o[2] = -1;
            continue;
        }
        o[0] = t.clo[j];
        o[1] = t.chi[j];
        o[2] = t.csys[j];
        o[3] = j;
    }
    std::copy(t.sc0.begin(), t.sc0.end(), host + 4 * (2 * nr + ncb));
    b.rt = reinterpret_cast<const int4 *>(tab);
    b.ct = reinterpret_cast<const int4 *>(tab + 8 * nr);
    b.sys_c0 = tab + 4 * (2 * nr + ncb);
    b.nrb = nrt;
    b.ncb = nct;
    RL_HIP(hipMemcpyAsync(tab, host, sizeof(int) * words, hipMemcpyHostToDevice, st));
    RL_HIP(hipStreamSynchronize(st));
    return RL_OK;
}

static int bucket_of(int64_t nc)
{
    int bkt = 0;
    while ((1LL << bkt) < nc && bkt < 62) ++bkt;
    return bkt;
}

static void tune_cache_load(rl_ctx *h)
{
    if (h->tune_loaded) return;
    h->tune_loaded = 1;
    const char *path = getenv("RODLCP_TUNE_CACHE");
    if (!path) return;
    FILE *f = fopen(path, "r");
    if (!f) return;
    int bkt, rb, cb;
    while (fscanf(f, "%d %d %d", &bkt, &rb, &cb) == 3)
        if (bkt >= 0 && bkt < 64 && (rb == 256 || rb == 1024) && (cb == 256 || cb == 512)) {
            h->tune_rb[bkt] = rb;
            h->tune_cb[bkt] = cb;
        }
    fclose(f);
}

static void tune_cache_store(int bkt, int rb, int cb)
{
    const char *path = getenv("RODLCP_TUNE_CACHE");
    if (!path) return;
    FILE *f = fopen(path, "a");
    if (!f) return;
    fprintf(f, "%d %d %d\n", bkt, rb, cb);
    fclose(f);
}

int solve_batched_impl(rl_ctx *h, int S, const int64_t *rod_off, const int64_t *pair_off, SolveArgs &a,
                       const int32_t *pi, const int32_t *pj, const double *e, const double *arm, const double *q,
                       const double *gamma_in, const double *F, double *gamma_out, double *U, rl_solve_info *infos)
{
    const rl_params &p = h->prm;
    int werr = 0;
    // capture needs a stream of our own (the null stream cannot be captured)
    RL_HIP(hipStreamSynchronize(h->stream));
    if (!h->own_stream) RL_HIP(hipStreamCreateWithFlags(&h->own_stream, hipStreamNonBlocking));
    hipStream_t st = h->own_stream;
    const bool uni = a.coef == nullptr;
    // device copies of the offsets for the ownership check
    int64_t *offs = (int64_t *)ws_get(h, kWsBatchOff, sizeof(int64_t) * 2 * (S + 1), &werr);
    BatchArgs b{};
    b.a = a;
    b.S = S;
    b.sst = (SolverState *)ws_get(h, kWsBatchState, sizeof(SolverState) * S, &werr);
    b.alpha_s = (double *)ws_get(h, kWsBatchAlpha, sizeof(double) * 2 * S, &werr);
    long long *ctr = (long long *)ws_get(h, kWsBatchCtr, sizeof(long long) * 2, &werr);
    b.done_s = (int *)ws_get(h, kWsBatchDone, sizeof(int) * S, &werr);
    if (werr) return werr;
    b.kbase = ctr;
    b.ndone = (int *)(ctr + 1);
    RL_HIP(hipMemcpyAsync(offs, rod_off, sizeof(int64_t) * (S + 1), hipMemcpyHostToDevice, st));
    RL_HIP(hipMemcpyAsync(offs + S + 1, pair_off, sizeof(int64_t) * (S + 1), hipMemcpyHostToDevice, st));
    RL_HIP(hipMemsetAsync(h->flag_dev, 0, sizeof(int), st));
    if (a.nc > 0) {
        hipLaunchKernelGGL(k_check_batch, dim3(grid_of(a.nc, 256)), dim3(256), 0, st, a.nc, S, offs, offs + S + 1,
                           pi, pj, h->flag_dev);
        RL_HIP(hipGetLastError());
    }
    RL_HIP(hipMemcpyAsync(h->host_scratch, h->flag_dev, sizeof(int), hipMemcpyDeviceToHost, st));
    RL_HIP(hipStreamSynchronize(st));
    if (((int *)h->host_scratch)[0]) {
        set_error("rl_solve_lcp_batched: a constraint joins rods of another system");
        return RL_ERR_ARG;
    }
    // workgroup sizes: fixed by the caller, cached, or timed now
    tune_cache_load(h);
    const int bkt = bucket_of(a.nc);
    int rb = h->batch_rb, cb = h->batch_cb;
    BatchTables tab;
    if (rb == 0 || cb == 0) {
        rb = h->tune_rb[bkt];
        cb = h->tune_cb[bkt];
    }
    const int max_tiles_con = (int)(a.nc / 512 + S + 8);
    const size_t part_words = 8 * (size_t)(a.nc / 256 + S + 8);
    double *parts[2] = {(double *)ws_get(h, kWsBatchPartial, sizeof(double) * part_words, &werr),
                        (double *)ws_get(h, kWsBatchPartial2, sizeof(double) * part_words, &werr)};
    if (werr) return werr;
    int cur_part = 0;
    b.partial = parts[0];
    (void)max_tiles_con;
    if (rb == 0 || cb == 0) {
        hipEvent_t e0, e1;
        RL_HIP(hipEventCreate(&e0));
        RL_HIP(hipEventCreate(&e1));
        float best = 1e30f;
        for (int ir = 0; ir < 2; ++ir)
            for (int ic = 0; ic < 2; ++ic) {
                const int trb = kBatchRodBlocks[ir], tcb = kBatchConBlocks[ic];
                build_tables(S, rod_off, pair_off, trb, tcb, tab);
                int rc = upload_tables(h, st, tab, S, b);
                if (rc) return rc;
                RL_HIP(start_phases(st, b, uni, trb, tcb, p));
                for (int it = 0; it < 4; ++it) RL_HIP(launch_pair_b<kModeLoop>(st, b, uni, trb, tcb, it));
                RL_HIP(hipEventRecord(e0, st));
                for (int it = 4; it < 24; ++it) RL_HIP(launch_pair_b<kModeLoop>(st, b, uni, trb, tcb, it));
                RL_HIP(hipEventRecord(e1, st));
                RL_HIP(hipEventSynchronize(e1));
                float ms = 0.f;
                RL_HIP(hipEventElapsedTime(&ms, e0, e1));
                // The trial times the first iterations of the full batch, but
                // the wall time is spent once most systems have stopped; the
                // first candidate (the smallest groups, the better choice there)
                // gives way only to a clear win.
                if (ms < 0.97f * best) {
                    best = ms;
                    rb = trb;
                    cb = tcb;
                }
                // the trial moved the iterate: restore it from the caller's start
                hipLaunchKernelGGL(k_restore_start, dim3(grid_of(a.nc, 256)), dim3(256), 0, st, a.nc, gamma_in,
                                   a.qpos, a.st, a.stq);
                RL_HIP(hipGetLastError());
            }
        RL_HIP(hipEventDestroy(e0));
        RL_HIP(hipEventDestroy(e1));
        h->tune_rb[bkt] = rb;
        h->tune_cb[bkt] = cb;
        tune_cache_store(bkt, rb, cb);
    }
    h->batch_rb_used = rb;
    h->batch_cb_used = cb;
    build_tables(S, rod_off, pair_off, rb, cb, tab);
    int rc = upload_tables(h, st, tab, S, b);
    if (rc) return rc;
    RL_HIP(start_phases(st, b, uni, rb, cb, p));
    // graph of B iterations plus the counter advance; re-captured whenever
    // the tile table is compacted to the systems still iterating
    // iterations per graph: even, so that every graph starts at an even count
    const int B = p.check_every > 0 ? (p.check_every + 1) / 2 * 2 : 32;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    auto capture = [&]() -> int {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
        exec = nullptr;
        graph = nullptr;
        RL_HIP(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
        for (int it = 0; it < B; ++it) {
            hipError_t ee = launch_pair_b<kModeLoop>(st, b, uni, rb, cb, it);
            if (ee != hipSuccess) {
                (void)hipStreamEndCapture(st, &graph);
                if (graph) (void)hipGraphDestroy(graph);
                graph = nullptr;
                RL_HIP(ee);
            }
        }
        hipLaunchKernelGGL(k_advance, dim3(1), dim3(64), 0, st, b.kbase, B);
        RL_HIP(hipStreamEndCapture(st, &graph));
        RL_HIP(hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0));
        return RL_OK;
    };
    if ((rc = capture())) return rc;
    if (!h->chk_ev) RL_HIP(hipEventCreateWithFlags(&h->chk_ev, hipEventDisableTiming));
    int ndone = 0, last_ndone = 0;
    long long replays = 0;
    std::vector<int> done_host(S, 0);
    // The count of finished systems is copied after every replay, and the
    // next replay is queued behind the copy before the host waits for it, so
    // the GPU never idles on the host.  A replay after the last stop returns
    // at once in every workgroup.
    RL_HIP(hipGraphLaunch(exec, st));
    ++replays;
    for (;;) {
        RL_HIP(hipMemcpyAsync(h->host_scratch, b.ndone, sizeof(int), hipMemcpyDeviceToHost, st));
        RL_HIP(hipEventRecord(h->chk_ev, st));
        const long long checked = replays;
        RL_HIP(hipGraphLaunch(exec, st));
        ++replays;
        RL_HIP(hipEventSynchronize(h->chk_ev));
        ndone = ((int *)h->host_scratch)[0];
        if (ndone >= S) break;
        if (checked * B > p.max_iter + 2 * B) {
            (void)hipStreamSynchronize(st);
            (void)hipGraphExecDestroy(exec);
            (void)hipGraphDestroy(graph);
            set_error("rl_solve_lcp_batched: systems did not all stop");
            return RL_ERR_HIP;
        }
        if (ndone > last_ndone) {
            last_ndone = ndone;
            // every queued replay has ended once the copy of the flags is in
            RL_HIP(hipMemcpyAsync(done_host.data(), b.done_s, sizeof(int) * S, hipMemcpyDeviceToHost, st));
            RL_HIP(hipStreamSynchronize(st));
            int live = 0;
            for (int s = 0; s < S; ++s)
                if (!done_host[s]) live += tab.sc0[s + 1] - tab.sc0[s];
            // Finished systems' workgroups still read their records before
            // they see the flag: the table drops them once they are an
            // eighth of it.
            if (8 * (b.ncb - live) >= b.ncb) {
                // Once fewer constraint tiles than compute units are left (the
                // tail of a few slow systems), tuned rod groups give way to the
                // smallest, for more workgroups on the little work that remains
                // (the rod tiling carries no state between iterations).
                if (h->batch_rb == 0 && live < kComputeUnits) rb = kBatchRodBlocks[0];
                // carry the last iteration's partials of the live systems to the new tiles
                BatchTables nt;
                build_tables(S, rod_off, pair_off, rb, cb, nt, &done_host);
                std::vector<int> old_of_new(nt.csys.size());
                for (size_t t = 0; t < nt.csys.size(); ++t) {
                    const int s = nt.csys[t];
                    old_of_new[t] = tab.sc0[s] + (int)t - nt.sc0[s];
                }
                const long long knext = replays * B;
                const int par = (int)((knext - 1) & 1);
                int *map = (int *)ws_get(h, kWsBatchMap, sizeof(int) * std::max<size_t>(old_of_new.size(), 1),
                                         &werr);
                if (werr) return werr;
                const int old_ncb = b.ncb;
                const int new_ncb = (int)nt.csys.size();
                if (new_ncb > 0) {
                    int *hm = (int *)ws_get_host(h, sizeof(int) * new_ncb, &werr);
                    if (werr) return werr;
                    std::copy(old_of_new.begin(), old_of_new.end(), hm);
                    RL_HIP(hipMemcpyAsync(map, hm, sizeof(int) * new_ncb, hipMemcpyHostToDevice, st));
                    double *dst = parts[cur_part ^ 1];
                    hipLaunchKernelGGL(k_remap_partials, dim3(grid_of(new_ncb, 256)), dim3(256), 0, st, new_ncb,
                                       (const int *)map, b.partial + (int64_t)par * old_ncb * 4,
                                       dst + (int64_t)par * new_ncb * 4);
                    RL_HIP(hipGetLastError());
                    RL_HIP(hipStreamSynchronize(st));
                }
                cur_part ^= 1;
                b.partial = parts[cur_part];
                tab = nt;
                if ((rc = upload_tables(h, st, tab, S, b))) return rc;
                if ((rc = capture())) return rc;
            }
            // after a full wait nothing is queued: start the next replay
            RL_HIP(hipGraphLaunch(exec, st));
            ++replays;
        }
    }
    RL_HIP(hipStreamSynchronize(st));
    RL_HIP(hipGraphExecDestroy(exec));
    RL_HIP(hipGraphDestroy(graph));
    if (gamma_out && a.nc > 0) RL_HIP(launch_unpack_gamma(st, a, gamma_out));
    if (U) RL_HIP(launch_velocity_on(st, a, F, nullptr, U));
    std::vector<SolverState> host(S);
    RL_HIP(hipMemcpyAsync(host.data(), b.sst, sizeof(SolverState) * S, hipMemcpyDeviceToHost, st));
    RL_HIP(hipStreamSynchronize(st));
    int worst = RL_OK;
    for (int s = 0; s < S; ++s) {
        const bool empty = pair_off[s + 1] == pair_off[s];
        if (infos) {
            infos[s].iterations = empty ? 0 : host[s].iter;
            infos[s].residual = empty ? 0.0 : host[s].res;
            infos[s].alpha0 = host[s].alpha0;
            infos[s].status = empty ? RL_OK : host[s].status;
            infos[s].fp64_refreshes = 0;
        }
        const int stt = empty ? RL_OK : host[s].status;
        if (stt < 0) worst = stt;
        else if (worst >= 0 && stt > worst) worst = stt;
    }
    if (worst == RL_ERR_NONFINITE) set_error("rl_solve_lcp_batched: non-finite value in a system");
    return worst;
}

}  // namespace rl
