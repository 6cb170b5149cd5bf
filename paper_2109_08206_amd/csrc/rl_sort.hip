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

__global__ void k_scan_ends(int64_t m, int *__restrict__ out, int64_t *__restrict__ total)
{
    if (blockIdx.x != 0 || threadIdx.x != 0) return;
    out[0] = 0;
    if (total) *total = out[m];
}

int scan_tmp_bytes(int64_t m, size_t *bytes)
{
    *bytes = 0;
    if (m <= 0) return RL_OK;
    RL_HIP(hipcub::DeviceScan::InclusiveSum(nullptr, *bytes, (const int *)nullptr, (int *)nullptr, (int)m,
                                            (hipStream_t)0));
    return RL_OK;
}

int device_scan(rl_ctx *h, const int *in, int64_t m, int *out, int64_t *total, void *tmp)
{
    hipStream_t st = h->stream;
    if (m > 0) {
        int werr = 0;
        size_t tmp_bytes = 0;
        RL_HIP(hipcub::DeviceScan::InclusiveSum(nullptr, tmp_bytes, in, out + 1, (int)m, st));
        if (!tmp) tmp = ws_get(h, kWsScanTmp, tmp_bytes, &werr);
        if (werr) return werr;
        RL_HIP(hipcub::DeviceScan::InclusiveSum(tmp, tmp_bytes, in, out + 1, (int)m, st));
    }
    hipLaunchKernelGGL(k_scan_ends, dim3(1), dim3(64), 0, st, m, out, total);
    RL_HIP(hipGetLastError());
    return RL_OK;
}

// sorts m (key, value) pairs by key into keys_out / vals_out
int sort_key_values(rl_ctx *h, int64_t m, const unsigned long long *keys, const double *vals,
                    unsigned long long *keys_out, double *vals_out)
{
    hipStream_t st = h->stream;
    if (m <= 0) return RL_OK;
    int werr = 0;
    size_t tmp_bytes = 0;
    RL_HIP(hipcub::DeviceRadixSort::SortPairs(nullptr, tmp_bytes, keys, keys_out, vals, vals_out, (int)m, 0, 64, st));
    void *tmp = ws_get(h, kWsSortTmp, tmp_bytes, &werr);
    if (werr) return werr;
    RL_HIP(hipcub::DeviceRadixSort::SortPairs(tmp, tmp_bytes, keys, keys_out, vals, vals_out, (int)m, 0, 64, st));
    return RL_OK;
}

}  // namespace rl
