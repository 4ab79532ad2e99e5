// bcf_sort_u32_noalloc: the key sort of bcf_sort_u32 with its temporary
// storage in a device array the library owns, for callers that cannot
// allocate device memory (code under graph capture, tight serving loops,
// harnesses that forbid allocation).
//
// The array below is a file-scope device variable: every GPU the library runs
// on gets its own copy, at its own address, when the code object is loaded,
// and keeps it until the process ends.  In host code the name `scratch` is
// only a host-side stand-in, never a device address, so host code uses the
// address hipGetSymbolAddress returns for the current device (looked up once
// per device, on the first call made with that device current) and nothing
// else: it is what the sort's kernels receive as their temp buffer.
#include <hip/hip_runtime.h>

#include <mutex>

#include "bcf.h"
#include "bcf_internal.hpp"

namespace {

// Largest sort the array serves, and the array's size: bcf_sort_u32 needs
// 17,874,944 bytes of temp for 2^22 keys (the ping-pong key buffer, the split
// list, two key-sample sets and the four-way cut list; the layout does not
// depend on the tuning).  The size is checked against the library's own temp
// query on every call.
constexpr uint64_t kNoAllocMaxKeys = BCF_NOALLOC_MAX_KEYS;
constexpr uint64_t kScratchBytes = 18ull << 20;

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void *g_scratch[kMaxDevices];  // device address of `scratch` on each device, once looked up

// Device address of this device's copy of `scratch` (nullptr on failure).
void *scratch_address(int dev)
{
    std::lock_guard<std::mutex> g(g_mu);
    if (!g_scratch[dev]) {
        void *p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || p == nullptr)
            return nullptr;
        g_scratch[dev] = p;
    }
    return g_scratch[dev];
}

}  // namespace

extern "C" bcf_status bcf_sort_u32_noalloc(const uint32_t *keys_in, uint32_t *keys_out, uint64_t n, void *stream)
{
    if (n > kNoAllocMaxKeys)
        return BCF_ERR_INVALID;
    if (n == 0)
        return BCF_OK;
    if (!keys_in || !keys_out)
        return BCF_ERR_INVALID;
    uint64_t need = 0;
    bcf_status st = bcf_sort_u32(nullptr, nullptr, n, nullptr, &need, stream);
    if (st != BCF_OK)
        return st;
    if (need > kScratchBytes)
        return BCF_ERR_TEMP_TOO_SMALL;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices)
        return BCF_ERR_DEVICE;
    void *temp = scratch_address(dev);
    if (!temp)
        return BCF_ERR_DEVICE;
    uint64_t bytes = kScratchBytes;
    // no per-launch timing events for this call, even while profiling is on
    bcf::ProfilingOff quiet;
    return bcf_sort_u32(keys_in, keys_out, n, temp, &bytes, stream);
}
