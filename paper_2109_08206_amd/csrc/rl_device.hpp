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

__device__ __forceinline__ Decision decide(const SolveArgs &a, long long k, const double t[4])
{
    const SolverState *st = a.state;
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
    double al = a.alpha_buf[(k - 1) & 1];
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

}  // namespace rl
