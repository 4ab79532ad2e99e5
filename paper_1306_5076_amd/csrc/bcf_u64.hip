// bcf_u64.hip -- sorts of 64-bit unsigned keys (an extension: the paper sorts
// 32-bit keys).
//
// A u64 key is two 32-bit digits.  The sort is the least-significant-digit
// composition of two stable 32-bit pair sorts (the same block sort and merge
// passes as bcf_sort_pairs_u32): first by the low halves, carrying the high
// halves as values; then by the high halves, carrying the low halves.  The
// second sort is stable, so keys with equal high halves keep the low-half
// order of the first, and the result ascends by (high, low), which is the
// order of the u64 values.  Two streaming kernels split the keys into their
// halves and join them back.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "bcf.h"

namespace {

constexpr int kThreads = 256;
constexpr int kPerThread = 4;  // keys per thread, kThreads apart (coalesced per access)

__global__ __launch_bounds__(kThreads) void k_split64(const uint64_t *keys, uint32_t *lo, uint32_t *hi, uint64_t n)
{
    const uint64_t base = (uint64_t)blockIdx.x * (kThreads * kPerThread) + threadIdx.x;
#pragma unroll
    for (int k = 0; k < kPerThread; ++k) {
        const uint64_t i = base + (uint64_t)k * kThreads;
        if (i < n) {
            const uint64_t x = keys[i];
            lo[i] = (uint32_t)x;
            hi[i] = (uint32_t)(x >> 32);
        }
    }
}

__global__ __launch_bounds__(kThreads) void k_join64(const uint32_t *hi, const uint32_t *lo, uint64_t *keys, uint64_t n)
{
    const uint64_t base = (uint64_t)blockIdx.x * (kThreads * kPerThread) + threadIdx.x;
#pragma unroll
    for (int k = 0; k < kPerThread; ++k) {
        const uint64_t i = base + (uint64_t)k * kThreads;
        if (i < n)
            keys[i] = ((uint64_t)hi[i] << 32) | lo[i];
    }
}

uint64_t align256(uint64_t b) { return (b + 255) / 256 * 256; }

}  // namespace

extern "C" bcf_status bcf_sort_u64(const uint64_t *keys_in, uint64_t *keys_out, uint64_t n, void *temp,
                                   uint64_t *temp_bytes, void *stream)
{
    if (!temp_bytes)
        return BCF_ERR_INVALID;
    uint64_t pair_need = 0;
    bcf_status st = bcf_sort_pairs_u32(nullptr, nullptr, nullptr, nullptr, n, nullptr, &pair_need, stream);
    if (st != BCF_OK)
        return st;  // n beyond the pair sort's limit
    const uint64_t half = align256(n * sizeof(uint32_t));
    const uint64_t need = n ? 4 * half + pair_need : 0;
    if (!temp) {
        *temp_bytes = need;
        return BCF_OK;
    }
    if (n == 0)
        return BCF_OK;
    if (!keys_in || !keys_out)
        return BCF_ERR_INVALID;
    if (*temp_bytes < need)
        return BCF_ERR_TEMP_TOO_SMALL;
    char *t = static_cast<char *>(temp);
    uint32_t *a_lo = reinterpret_cast<uint32_t *>(t), *a_hi = reinterpret_cast<uint32_t *>(t + half);
    uint32_t *b_lo = reinterpret_cast<uint32_t *>(t + 2 * half), *b_hi = reinterpret_cast<uint32_t *>(t + 3 * half);
    void *pair_temp = t + 4 * half;
    uint64_t pair_bytes = pair_need;
    hipStream_t s = static_cast<hipStream_t>(stream);
    const uint64_t blocks = (n + kThreads * kPerThread - 1) / (kThreads * kPerThread);
    hipLaunchKernelGGL(k_split64, dim3((uint32_t)blocks), dim3(kThreads), 0, s, keys_in, a_lo, a_hi, n);
    if (hipGetLastError() != hipSuccess)
        return BCF_ERR_DEVICE;
    // by the low halves, carrying the high halves
    st = bcf_sort_pairs_u32(a_lo, a_hi, b_lo, b_hi, n, pair_temp, &pair_bytes, stream);
    if (st != BCF_OK)
        return st;
    // stably by the high halves, carrying the low halves
    st = bcf_sort_pairs_u32(b_hi, b_lo, a_hi, a_lo, n, pair_temp, &pair_bytes, stream);
    if (st != BCF_OK)
        return st;
    hipLaunchKernelGGL(k_join64, dim3((uint32_t)blocks), dim3(kThreads), 0, s, a_hi, a_lo, keys_out, n);
    return hipGetLastError() == hipSuccess ? BCF_OK : BCF_ERR_DEVICE;
}
