// Stable key-value radix sort (rocPRIM through hipCUB), used to put rods in
// cell order deterministically: equal cells keep ascending rod index.
#include <hipcub/hipcub.hpp>

#include "rl_internal.hpp"

namespace rl {

__global__ void k_iota(int64_t n, int *__restrict__ v)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < n) v[i] = (int)i;
}

// perm[t] = rod with the t-th smallest (key, index); keys_out receives the keys.
int stable_sort_by_key(rl_ctx *h, int64_t n, const int *keys, int bits, int *keys_out, int *perm)
{
    hipStream_t st = h->stream;
    int werr = 0;
    int *idx = (int *)ws_get(h, kWsSortIdx, sizeof(int) * (n > 0 ? n : 1), &werr);
    if (werr) return werr;
    hipLaunchKernelGGL(k_iota, dim3((unsigned)((n + kBlock - 1) / kBlock)), dim3(kBlock), 0, st, n, idx);
    RL_HIP(hipGetLastError());
    size_t tmp_bytes = 0;
    RL_HIP(hipcub::DeviceRadixSort::SortPairs(nullptr, tmp_bytes, keys, keys_out, idx, perm, (int)n, 0, bits, st));
    void *tmp = ws_get(h, kWsSortTmp, tmp_bytes, &werr);
    if (werr) return werr;
    RL_HIP(hipcub::DeviceRadixSort::SortPairs(tmp, tmp_bytes, keys, keys_out, idx, perm, (int)n, 0, bits, st));
    return RL_OK;
}

}  // namespace rl
