// Mixed-precision BBPGD (RL_FP32_MIXED) on gfx950.
//
// The iterate is split as gamma = gamma64 + delta.  gamma64 and g64 =
// Mc gamma64 + q are double precision and are recomputed only by FP64
// "refresh" products; between refreshes the BB iteration runs in single
// precision on the correction delta >= b = -gamma64, with h = h0 +
// Mc32 delta standing in for the gradient (h0 = g64 at the refresh).  Only
// the BB dot products s.s, s.y, y.y and the residual are accumulated in
// double precision (from single-precision differences), as is every
// refresh.  Because delta and its product shrink as the solve converges,
// single-precision rounding stays below the residual it has to resolve;
// each inner round ends when its residual has dropped by 1e-4 (or to the
// tolerance, or it stalls), and the solve ends only when an FP64 refresh
// certifies residual <= tol.
//
// The kernels mirror the FP64 ones (rl_solver.hip) with single-precision
// records: 16-byte (delta, h, b, h0) state and 16-byte (e, s) geometry per
// incidence instead of 16 + 32 bytes, and 4-byte contact velocities.
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>

#include "rl_device.hpp"

namespace rl {

static inline unsigned grid_of(int64_t n, int block) { return (unsigned)((n + block - 1) / block); }
static inline unsigned rod_grid32(int64_t n, int ln) { return (grid_of(n, kRodLoopBlock / ln) + 7) / 8 * 8; }

constexpr long long kInnerRoundCap = 4000;  // inner iterations before a forced refresh

// single-precision geometry records from the FP64 ones
__global__ void k_pack32(int64_t nc, const double *__restrict__ geo, const double *__restrict__ qgeo,
                         float4 *__restrict__ geo32, float4 *__restrict__ qgeo32)
{
    const int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (c >= nc) return;
    const double *g = geo + 4 * c;
    geo32[c] = make_float4((float)g[0], (float)g[1], (float)g[2], (float)g[3]);
    const double *qg = qgeo + 4 * c;  // list order, same length
    qgeo32[c] = make_float4((float)qg[0], (float)qg[1], (float)qg[2], (float)qg[3]);
}

__device__ __forceinline__ float delta_prime(float4 s, float alpha)
{
    const float v = fmaf(-alpha, s.y, s.x);
    return v > s.z ? v : s.z;
}

// one incidence record: state (delta, h, b, h0) and geometry (e, s)
struct Rec32 {
    float4 s, g;
};

// unconditional, like the FP64 records: a lane past its list reads zeros
__device__ __forceinline__ void rec32_load(const float4 *__restrict__ st, const float4 *__restrict__ geo, int c,
                                           int end, Rec32 &R)
{
    const bool ok = c < end;
    const float4 *z = reinterpret_cast<const float4 *>(kZeroRecord);
    R.s = *(ok ? st + c : z);
    R.g = *(ok ? geo + c : z);
}

// Records of each side held in registers across the step-length wait: as
// in the FP64 rod kernel, three rounds over four lanes per rod where rods
// have a few constraints and over eight lanes on dense systems (rod_dense).

__device__ __forceinline__ void add32(float sign, float dp, float4 g, float f[3], float m[3])
{
    const float dv = sign * dp, ds = dv * g.w;
    f[0] += dv * g.x;
    f[1] += dv * g.y;
    f[2] += dv * g.z;
    m[0] += ds * g.x;
    m[1] += ds * g.y;
    m[2] += ds * g.z;
}

template <int R, int LN>
__device__ __forceinline__ void side32(float sign, const float4 *__restrict__ st, const float4 *__restrict__ geo,
                                       int b, int e, const Rec32 *rr, float a32, float f[3], float m[3])
{
#pragma unroll
    for (int i = 0; i < R; ++i) {
        if (b + i * LN >= e) return;
        add32(sign, delta_prime(rr[i].s, a32), rr[i].g, f, m);
    }
    for (int c = b + R * LN; c < e; c += LN) add32(sign, delta_prime(st[c], a32), geo[c], f, m);
}

__device__ __forceinline__ float u32_along(float4 g, const float v[3], const float w[3])
{
    return g.x * (v[0] + g.w * w[0]) + g.y * (v[1] + g.w * w[1]) + g.z * (v[2] + g.w * w[2]);
}

template <int R, int LN>
__device__ __forceinline__ void emit32(float *__restrict__ u, const float4 *__restrict__ geo, int b, int e,
                                       const Rec32 *rr, const float v[3], const float w[3])
{
#pragma unroll
    for (int i = 0; i < R; ++i) {
        if (b + i * LN >= e) return;
        u[b + i * LN] = u32_along(rr[i].g, v, w);
    }
    for (int c = b + R * LN; c < e; c += LN) u[c] = u32_along(geo[c], v, w);
}

// Rod kernel of the inner FP32 iteration: the force of delta' on the rod,
// then the velocity of each of its contact points along e (contact-velocity
// form, as in the FP64 rod kernel).
// The arrays of the first loads, the grid size and n lead the argument list
// (14 dwords), so that they arrive in preloaded registers.
template <bool UNI, int R, int LN>
__global__ void __launch_bounds__(kRodLoopBlock)
    k_rod32(const int32_t *__restrict__ pptr, const int32_t *__restrict__ qptr, const float4 *s32, const float4 *sq32,
            const float4 *__restrict__ g32, const float4 *__restrict__ gq32, unsigned nblk, int n, SolveArgs a,
            long long k, int first, long long round_start)
{
    __shared__ double lds[kRodLoopBlock / 64 + 1][4];
    SolverState *st = a.state;
    const int sub = threadIdx.x & (LN - 1);
    const unsigned tile = xcd_tile(blockIdx.x, nblk);
    const int64_t r = (int64_t)tile * (kRodLoopBlock / LN) + (threadIdx.x / LN);
    const bool active = r < n;
    // the previous iteration's partials (read for nothing on a first
    // iteration) and the flags first, then the offsets and the records, all
    // unconditional, so that the step-length reduction waits only for the
    // first group
    const double *part = a.partial + (int64_t)((k - 1) & 1) * a.gcon * 4;
    PartFirst pf;
    partials_first_split<kRodLoopBlock>(part, a.gcon, pf);
    const bool halt = st->done || st->refresh;
    const double aprev = a.alpha_buf[(k - 1) & 1], inner_tol = st->inner_tol, amin = st->amin, amax = st->amax;
    const long long max_iter = st->max_iter;
    const double alpha_first = st->alpha;
    __asm__ volatile("" ::: "memory");
    const int64_t rr = active ? r : 0;
    const int pb0 = pptr[rr], pe0 = pptr[rr + 1], qb0 = qptr[rr], qe0 = qptr[rr + 1];
    const int pb = active ? pb0 + sub : 0, pe = active ? pe0 : 0;
    const int qb = active ? qb0 + sub : 0, qe = active ? qe0 : 0;
    // R rounds of both sides in flight before the flags are read
    Rec32 P[R], Q[R];
#pragma unroll
    for (int i = 0; i < R; ++i) {
        rec32_load(s32, g32, pb + i * LN, pe, P[i]);
        rec32_load(sq32, gq32, qb + i * LN, qe, Q[i]);
    }
    // keeps the loads ahead of the flag test (see k_rod)
    __asm__ volatile("" ::: "memory");
    if (halt) return;
    double alpha;
    if (first) {
        alpha = alpha_first;
        if (blockIdx.x == 0 && threadIdx.x == 0) a.alpha_buf[k & 1] = alpha;
    } else {
        double t[4];
        sum_partials_split_from<kRodLoopBlock / 64>(pf, part, a.gcon, t, lds);
        const double ss = t[0], sy = t[1], yy = t[2], res = t[3];
        int done = 0, refresh = 0, status = RL_OK;
        if (!isfinite(ss) || !isfinite(sy) || !isfinite(yy) || !isfinite(res)) {
            done = 1;
            status = RL_ERR_NONFINITE;
        } else if (k >= max_iter) {
            done = 1;
            status = RL_NOT_CONVERGED;
        } else if (res <= inner_tol || ss == 0.0 || k - round_start >= kInnerRoundCap) {
            refresh = 1;
        }
        double al = aprev;
        if (sy > 0.0) {
            al = ((k - 1) % 2 == 0) ? ss / sy : sy / yy;
            al = al < amin ? amin : (al > amax ? amax : al);
        }
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            if (done || refresh) {
                st->iter = k;
                st->res = res;
                st->alpha = al;
                if (done) {
                    st->status = status;
                    st->done = 1;
                } else {
                    st->refresh = 1;
                }
            } else {
                a.alpha_buf[k & 1] = al;
            }
        }
        if (done || refresh) return;
        alpha = al;
    }
    const float a32 = (float)alpha;
    float f[3] = {0.f, 0.f, 0.f}, m[3] = {0.f, 0.f, 0.f};
    side32<R, LN>(1.f, a.st32, a.geo32, pb, pe, P, a32, f, m);
    side32<R, LN>(-1.f, a.stq32, a.qgeo32, qb, qe, Q, a32, f, m);
#pragma unroll
    for (int o = 1; o < LN; o <<= 1) {
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            f[d] += __shfl_xor(f[d], o, 64);
            m[d] += __shfl_xor(m[d], o, 64);
        }
    }
    if (!active) return;
    const float dx = (float)a.dir[3 * r], dy = (float)a.dir[3 * r + 1], dz = (float)a.dir[3 * r + 2];
    float apar, aperp, rperp;
    if (UNI) {
        apar = (float)a.mob.apar;
        aperp = (float)a.mob.aperp;
        rperp = (float)a.mob.rperp;
    } else {
        apar = (float)a.coef[3 * r];
        aperp = (float)a.coef[3 * r + 1];
        rperp = (float)a.coef[3 * r + 2];
    }
    const float fd = (apar - aperp) * (dx * f[0] + dy * f[1] + dz * f[2]);
    const float md = dx * m[0] + dy * m[1] + dz * m[2];
    const float v[3] = {aperp * f[0] + fd * dx, aperp * f[1] + fd * dy, aperp * f[2] + fd * dz};
    const float w[3] = {rperp * (m[0] - md * dx), rperp * (m[1] - md * dy), rperp * (m[2] - md * dz)};
    emit32<R, LN>(a.uP32, a.geo32, pb, pe, P, v, w);
    emit32<R, LN>(a.uQ32, a.qgeo32, qb, qe, Q, v, w);
}

struct Con32Loads {
    float4 s;
    float up, uq;
    int qp;
};

// One round of CPL constraints per lane: the list positions first, then the
// records, then the gathers of u_Q.  Lanes past the end read constraint
// `last` instead (their values go unused), so that no load sits behind a
// branch: with a branch around each constraint's loads the compiler keeps
// them in program order, and each gather of u_Q, which needs its list
// position, waits for every load issued before it (the memory counter
// completes in order), one memory round trip per constraint of the lane.
// At 400k rods, phi 0.08: 88 -> 84 us per launch.
template <int CB, int CPL>
__device__ __forceinline__ void con32_load_round(const int32_t *qpos, const float *uP32, const float4 *st32,
                                                 const float *uQ32, int64_t c0, int64_t last, Con32Loads (&L)[CPL])
{
    int64_t cc[CPL];
#pragma unroll
    for (int u = 0; u < CPL; ++u) {
        const int64_t c = c0 + (int64_t)u * CB;
        cc[u] = c < last ? c : last;
        L[u].qp = qpos[cc[u]];
    }
    // compiler barriers keep the three groups in this order (the scheduler
    // would otherwise wait for the first position right after its load)
    __asm__ volatile("" ::: "memory");
#pragma unroll
    for (int u = 0; u < CPL; ++u) {
        L[u].up = uP32[cc[u]];
        L[u].s = st32[cc[u]];
    }
    __asm__ volatile("" ::: "memory");
#pragma unroll
    for (int u = 0; u < CPL; ++u) L[u].uq = uQ32[L[u].qp];
}

__device__ __forceinline__ void con32_update(const SolveArgs &a, int64_t c, const Con32Loads &L, float a32,
                                             double p[4])
{
    // h = h0 + Mc32 delta, the rate being the difference of the two contact velocities
    const float h = L.s.w + (L.up - L.uq);
    const float dp = delta_prime(L.s, a32);
    a.st32[c] = make_float4(dp, h, L.s.z, L.s.w);
    a.stq32[L.qp] = make_float4(dp, h, L.s.z, 0.f);
    const double sc = (double)dp - (double)L.s.x, yc = (double)h - (double)L.s.y;
    const double gam = (double)dp - (double)L.s.z;
    p[0] += sc * sc;
    p[1] += sc * yc;
    p[2] += yc * yc;
    p[3] = fmax(p[3], fabs(gam < (double)h ? gam : (double)h));
}

// CB threads per workgroup take CPL constraints each per round; the shape is
// chosen per launch like that of the FP64 constraint kernel.
// As in k_rod32, what the first loads need leads the argument list.
template <int CB, int CPL>
__global__ void __launch_bounds__(CB)
    k_con32(const int32_t *__restrict__ qpos, const float *__restrict__ uP32, const float4 *s32,
            const float *__restrict__ uQ32, int nc, unsigned nblk, const double *alpha_buf, SolveArgs a, long long k)
{
    __shared__ double lds[CB / 64 + 1][4];
    double p[4] = {0.0, 0.0, 0.0, 0.0};
    // rounds of CPL constraints per lane, swept band by band per XCD
    const ConBand bd = con_band(blockIdx.x, nblk, nc, (int64_t)CPL * CB);
    const int64_t hi = bd.end;
    int64_t base = bd.first;
    // the step length and the flags are read first (scalar loads), then the
    // first round goes out before the flags are tested; nothing in this
    // launch writes the flags, so the early return is uniform (a workgroup
    // without constraints loads nothing; nc >= 1 whenever it has some)
    const double a64 = alpha_buf[k & 1];
    const int halt = a.state->done | a.state->refresh;  // both read, no branch
    const int64_t last = (int64_t)nc - 1;
    int64_t c0 = base + threadIdx.x;
    Con32Loads L[CPL];
    if (base < hi) con32_load_round<CB, CPL>(qpos, uP32, s32, uQ32, c0, last, L);
    __asm__ volatile("" ::: "memory");
    if (halt) return;
    const float a32 = (float)a64;
    for (;;) {
#pragma unroll
        for (int u = 0; u < CPL; ++u)
            if (c0 + u * CB < hi) con32_update(a, c0 + u * CB, L[u], a32, p);
        base += bd.stride;
        if (base >= hi) break;
        c0 = base + threadIdx.x;
        con32_load_round<CB, CPL>(qpos, uP32, s32, uQ32, c0, last, L);
    }
    block_total4<CB / 64>(p, lds);
    if (threadIdx.x == 0) partial_put(a.partial + (int64_t)(k & 1) * a.gcon * 4, a.gcon, blockIdx.x, p);
}

// the leading arguments of k_rod32 and k_con32
#define RL_ROD32_HOT(a, grid)                                                                              \
    (const int32_t *)(a).pptr, (const int32_t *)(a).qptr, (const float4 *)(a).st32, (const float4 *)(a).stq32, \
        (const float4 *)(a).geo32, (const float4 *)(a).qgeo32, (unsigned)(grid).x, (int)(a).n
#define RL_CON32_HOT(a)                                                                                   \
    (const int32_t *)(a).qpos, (const float *)(a).uP32, (const float4 *)(a).st32, (const float *)(a).uQ32, \
        (int)(a).nc, (unsigned)(a).gcon, (const double *)(a).alpha_buf

// more than 2,048 constraints per workgroup: 256 threads with 8 each, else
// 512 threads with 2 each
static inline bool con32_wide(const SolveArgs &a) { return (a.nc + a.gcon - 1) / a.gcon > 2048; }

// the FP32 rod kernel with LN lanes per rod and R rounds of records, with
// dispatch-stamped events when e0 is set
template <int R, int LN>
static void launch_rod32(hipStream_t st, const SolveArgs &a, bool uni, long long k, int fl, long long round_start,
                         hipEvent_t e0, hipEvent_t e1)
{
    const dim3 g(rod_grid32(a.n, LN));
    if (e0) {
        if (uni)
            hipExtLaunchKernelGGL(HIP_KERNEL_NAME(k_rod32<true, R, LN>), g, dim3(kRodLoopBlock), 0, st, e0, e1, 0,
                                  RL_ROD32_HOT(a, g), a, k, fl, round_start);
        else
            hipExtLaunchKernelGGL(HIP_KERNEL_NAME(k_rod32<false, R, LN>), g, dim3(kRodLoopBlock), 0, st, e0, e1, 0,
                                  RL_ROD32_HOT(a, g), a, k, fl, round_start);
    } else {
        if (uni)
            hipLaunchKernelGGL(HIP_KERNEL_NAME(k_rod32<true, R, LN>), g, dim3(kRodLoopBlock), 0, st,
                               RL_ROD32_HOT(a, g), a, k, fl, round_start);
        else
            hipLaunchKernelGGL(HIP_KERNEL_NAME(k_rod32<false, R, LN>), g, dim3(kRodLoopBlock), 0, st,
                               RL_ROD32_HOT(a, g), a, k, fl, round_start);
    }
}

static void launch_rod32_r(hipStream_t st, const SolveArgs &a, bool uni, bool dense, long long k, int fl,
                           long long round_start, hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr)
{
    if (dense) launch_rod32<kRodRounds, kRodLanesDense>(st, a, uni, k, fl, round_start, e0, e1);
    else launch_rod32<kRodRounds, kRodLanes>(st, a, uni, k, fl, round_start, e0, e1);
}

int prepare_mixed(rl_ctx *h, SolveArgs &a)
{
    int werr = 0;
    const int64_t nb = a.nc > 0 ? a.nc : 1;
    a.st32 = (float4 *)ws_get(h, kWsSt32, sizeof(float4) * nb, &werr);
    a.stq32 = (float4 *)ws_get(h, kWsStq32, sizeof(float4) * nb, &werr);
    float4 *geo32 = (float4 *)ws_get(h, kWsGeo32, sizeof(float4) * nb, &werr);
    float4 *qgeo32 = (float4 *)ws_get(h, kWsQgeo32, sizeof(float4) * nb, &werr);
    a.uP32 = (float *)ws_get(h, kWsUP32, sizeof(float) * nb, &werr);
    a.uQ32 = (float *)ws_get(h, kWsUQ32, sizeof(float) * nb, &werr);
    if (werr) return werr;
    a.geo32 = geo32;
    a.qgeo32 = qgeo32;
    if (a.nc > 0) {
        hipLaunchKernelGGL(k_pack32, dim3(grid_of(a.nc, kBlock)), dim3(kBlock), 0, h->stream, a.nc, a.geo, a.qgeo,
                           geo32, qgeo32);
        RL_HIP(hipGetLastError());
    }
    return RL_OK;
}

static int read_state(rl_ctx *h)
{
    RL_HIP(hipMemcpyAsync(h->state_host, h->state, sizeof(SolverState), hipMemcpyDeviceToHost, h->stream));
    RL_HIP(hipStreamSynchronize(h->stream));
    return RL_OK;
}

int solve_mixed_impl(rl_ctx *h, SolveArgs &a, long long *refreshes)
{
    hipStream_t st = h->stream;
    const rl_params &p = h->prm;
    const bool uni = a.coef == nullptr;
    // start: FP64 g0 and residual (also fills the FP32 state), then alpha0
    RL_HIP(launch_refresh64(h, a, false));
    RL_HIP(launch_alpha0_64(h, a));
    int rc = read_state(h);
    if (rc) return rc;
    const int every = p.check_every > 0 ? p.check_every : 32;
    long long k = 0, round_start = 0, launched = 0;
    bool first = true;
    const bool wide = con32_wide(a);
    const bool dense = rod_dense(a.n, a.nc);
    while (!h->state_host->done) {
        if (launched > p.max_iter + 4 * every + 64) {
            set_error("rl_solve_lcp: mixed-precision loop did not stop");
            return RL_ERR_HIP;
        }
        int nev = 0;
        const long long k_block = k;
        for (int i = 0; i < every; ++i, ++k, ++launched) {
            const int fl = first ? 1 : 0;
            first = false;
            const bool samp = h->prof_every > 0 && k % h->prof_every == 0 && nev < rl_ctx::kMaxEv;
            if (samp) {
                // dispatch-stamped events around both kernels of this iteration
                for (int e = 0; e < 4; ++e)
                    if (!h->ev[nev][e]) RL_HIP(hipEventCreateWithFlags(&h->ev[nev][e], hipEventDisableSystemFence));
                h->ev_iter[nev] = k;
                launch_rod32_r(st, a, uni, dense, k, fl, round_start, h->ev[nev][0], h->ev[nev][1]);
                if (wide)
                    hipExtLaunchKernelGGL(HIP_KERNEL_NAME(k_con32<256, 8>), dim3(a.gcon), dim3(256), 0, st,
                                          h->ev[nev][2], h->ev[nev][3], 0, RL_CON32_HOT(a), a, (long long)k);
                else
                    hipExtLaunchKernelGGL(HIP_KERNEL_NAME(k_con32<512, 2>), dim3(a.gcon), dim3(512), 0, st,
                                          h->ev[nev][2], h->ev[nev][3], 0, RL_CON32_HOT(a), a, (long long)k);
                ++nev;
            } else {
                launch_rod32_r(st, a, uni, dense, k, fl, round_start);
                if (wide)
                    hipLaunchKernelGGL(HIP_KERNEL_NAME(k_con32<256, 8>), dim3(a.gcon), dim3(256), 0, st,
                                       RL_CON32_HOT(a), a, k);
                else
                    hipLaunchKernelGGL(HIP_KERNEL_NAME(k_con32<512, 2>), dim3(a.gcon), dim3(512), 0, st,
                                       RL_CON32_HOT(a), a, k);
            }
            RL_HIP(hipGetLastError());
        }
        if ((rc = read_state(h))) return rc;
        const SolverState &s = *h->state_host;
        {
            // samples at or after a stop/refresh decision ran kernels that exited at once
            const long long valid = (s.refresh || s.done) ? s.iter : k;
            for (int v = 0; v < nev; ++v) {
                if (h->ev_iter[v] >= valid || h->ev_iter[v] < k_block) continue;
                float t0 = 0.f, t1 = 0.f;
                RL_HIP(hipEventElapsedTime(&t0, h->ev[v][0], h->ev[v][1]));
                RL_HIP(hipEventElapsedTime(&t1, h->ev[v][2], h->ev[v][3]));
                h->prof_ms[0] += t0;
                h->prof_ms[1] += t1;
                h->prof_cnt[0] += 1.0;
                h->prof_cnt[1] += 1.0;
            }
        }
        if (s.done && s.status == RL_ERR_NONFINITE) break;
        if (s.refresh || s.done) {
            // the stop iteration: continue from there after the FP64 refresh
            k = s.iter;
            const bool was_done = s.done;
            const int status = s.status;
            RL_HIP(launch_refresh64(h, a, true));
            if ((rc = read_state(h))) return rc;
            if (was_done && !h->state_host->done) {
                // iteration cap: keep the refreshed FP64 iterate, report the cap
                SolverState fix = *h->state_host;
                fix.done = 1;
                fix.status = status;
                fix.iter = k;
                *h->state_host = fix;
                break;
            }
            round_start = k;
            first = true;
        }
    }
    h->state_host->iter = std::max<long long>(h->state_host->iter, 0);
    *refreshes = h->state_host->refreshes;
    return RL_OK;
}

}  // namespace rl
