// LDS bank-geometry and HBM copy microbenchmark for gfx950 (CDNA4).
//
// The paper's framework (Sec. 2.1) views shared memory as a matrix whose rows
// are the memory banks, filled column-major, and designs accesses so that the
// threads of one warp touch distinct rows.  On the paper's GPU warp width and
// bank count were both 32; on gfx950 the wave is 64 lanes wide and the bank
// count, bank width and the group of lanes serviced together must be measured
// before any conflict-free layout can be derived.  This program measures them.
//
// For every access pattern (word address as a function of the lane) and
// access width (4, 8, 16 bytes per lane) it times a long chain of independent
// LDS reads (a) inside one wave with the shader clock and (b) across the whole
// chip with events, and prints cycles per wave-instruction.  Each pattern is a
// separate kernel instantiation so that a counter run (rocprofv3 --pmc
// SQ_LDS_BANK_CONFLICT SQ_INSTS_LDS) attributes conflict cycles to it.
// It also times a plain streaming copy to give the achievable HBM rate.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <vector>

#define CHECK(x)                                                                          \
    do {                                                                                  \
        hipError_t e_ = (x);                                                              \
        if (e_ != hipSuccess) {                                                           \
            std::fprintf(stderr, "HIP error %s at %s:%d\n", hipGetErrorString(e_), __FILE__, \
                         __LINE__);                                                       \
            std::exit(1);                                                                 \
        }                                                                                 \
    } while (0)

constexpr int kLdsWords = 9216;   // 36 KiB of LDS per work-group (4 groups fit a CU)
constexpr int kUnroll = 8;        // independent reads per loop trip
constexpr int kSpread = 64;       // word distance between the 8 reads (bank-neutral)

// word address for lane `l` under pattern `p`
__host__ __device__ constexpr uint32_t pattern_addr(int p, uint32_t l)
{
    switch (p) {
    case 0: return l;                              // stride 1
    case 1: return 2 * l;                          // stride 2
    case 2: return 4 * l;                          // stride 4
    case 3: return 8 * l;                          // stride 8
    case 4: return 16 * l;                         // stride 16
    case 5: return 32 * l;                         // stride 32
    case 6: return 64 * l;                         // stride 64
    case 7: return 65 * l;                         // stride 65 (one pad word per 64)
    case 8: return 33 * l;                         // stride 33 (one pad word per 32)
    case 9: return (l & 31) + 2048 * (l >> 5);     // lanes l and l+32 share a bank, distinct words
    case 10: return 2 * (l & 31) + (l >> 5);       // upper half on odd words, lower on even
    case 11: return 0;                             // broadcast
    case 12: return 128 * l;                       // stride 128
    case 13: return (l & 15) + 2048 * (l >> 4);    // 16-lane groups on the same banks
    case 14: return 17 * l;                        // stride 17 (b128: 68 words, four pad words per 64)
    default: return l;
    }
}
constexpr int kPatterns = 15;
const char *pattern_name(int p)
{
    static const char *n[] = {"stride1", "stride2", "stride4", "stride8", "stride16",
                              "stride32", "stride64", "stride65", "stride33",
                              "half_alias(l&31)+2048*(l>>5)", "interleave 2*(l&31)+(l>>5)",
                              "broadcast", "stride128", "quarter_alias(l&15)+2048*(l>>4)", "stride17"};
    return n[p];
}

typedef unsigned v2u __attribute__((ext_vector_type(2)));
typedef unsigned v4u __attribute__((ext_vector_type(4)));

// eight independent reads of W words at byte offsets k*4*kSpread, then a wait
#define LDS_READ8(OP, T, FOLD)                                                                   \
    {                                                                                            \
        T r0, r1, r2, r3, r4, r5, r6, r7;                                                        \
        asm volatile(OP " %0, %8 offset:0\n" OP " %1, %8 offset:256\n" OP " %2, %8 offset:512\n"      \
                     OP " %3, %8 offset:768\n" OP " %4, %8 offset:1024\n" OP                       \
                     " %5, %8 offset:1280\n" OP " %6, %8 offset:1536\n" OP " %7, %8 offset:1792\n"   \
                     "s_waitcnt lgkmcnt(0)"                                                       \
                     : "=&v"(r0), "=&v"(r1), "=&v"(r2), "=&v"(r3), "=&v"(r4), "=&v"(r5), "=&v"(r6), \
                       "=&v"(r7)                                                                 \
                     : "v"(addr));                                                               \
        acc += FOLD(r0) + FOLD(r1) + FOLD(r2) + FOLD(r3) + FOLD(r4) + FOLD(r5) + FOLD(r6) + FOLD(r7); \
    }

__device__ inline uint32_t f1(uint32_t v) { return v; }
__device__ inline uint32_t f2(v2u v) { return v.x ^ v.y; }
__device__ inline uint32_t f4(v4u v) { return v.x ^ v.y ^ v.z ^ v.w; }

// W words per lane; the pattern address is scaled by W so each lane reads W
// consecutive, W-aligned words.  The eight reads of one trip are kSpread words
// apart (a multiple of 64, so they fall on the same banks).
template <int P, int W>
__global__ __launch_bounds__(64) void lds_probe(uint32_t *sink, unsigned long long *cycles, int iters)
{
    __shared__ uint32_t lds[kLdsWords];
    const uint32_t lane = threadIdx.x;
    for (int i = lane; i < kLdsWords; i += 64)
        lds[i] = (uint32_t)i * 2654435761u;
    __syncthreads();
    // LDS byte offset of this lane's first word
    typedef __attribute__((address_space(3))) uint32_t lds_word;
    const uint32_t lds_base = (uint32_t)(uintptr_t)(lds_word *)lds;
    const uint32_t addr = lds_base + 4u * W * pattern_addr(P, lane);
    uint32_t acc = 0;
    unsigned long long t0 = clock64();
    for (int it = 0; it < iters; ++it) {
        if constexpr (W == 1)
            LDS_READ8("ds_read_b32", uint32_t, f1)
        else if constexpr (W == 2)
            LDS_READ8("ds_read_b64", v2u, f2)
        else
            LDS_READ8("ds_read_b128", v4u, f4)
    }
    unsigned long long t1 = clock64();
    if (lane == 0 && blockIdx.x == 0)
        cycles[P * 8 + W] = t1 - t0;
    if (acc == 0x12345678u)
        sink[blockIdx.x * 64 + lane] = acc;
}

__global__ void copy_u32x4(const uint4 *__restrict__ in, uint4 *__restrict__ out, size_t n4)
{
    size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
    size_t stride = (size_t)gridDim.x * blockDim.x;
    for (; i < n4; i += stride)
        out[i] = in[i];
}

// One wave copies one 4096-element tile, lane l moving elements 64r + l
// (r = 0..63): the access pattern of the sort kernels' STRIDED tile I/O.
template <bool NT>
__global__ __launch_bounds__(128) void copy_tiles_strided(const uint32_t *__restrict__ in, uint32_t *__restrict__ out,
                                                          size_t ntiles)
{
    const uint32_t lane = threadIdx.x & 63;
    const size_t tile = (size_t)blockIdx.x * 2 + (threadIdx.x >> 6);
    if (tile >= ntiles)
        return;
    const uint32_t *src = in + tile * 4096 + lane;
    uint32_t *dst = out + tile * 4096 + lane;
    uint32_t v[64];
#pragma unroll
    for (int r = 0; r < 64; ++r)
        v[r] = NT ? __builtin_nontemporal_load(src + 64 * r) : src[64 * r];
#pragma unroll
    for (int r = 0; r < 64; ++r) {
        if (NT)
            __builtin_nontemporal_store(v[r], dst + 64 * r);
        else
            dst[64 * r] = v[r];
    }
}

// Same tiles, lane l moving 16-byte groups 256q + 4l .. +3 (q = 0..15).
template <bool NT>
__global__ __launch_bounds__(128) void copy_tiles_x4(const v4u *__restrict__ in, v4u *__restrict__ out, size_t ntiles)
{
    const uint32_t lane = threadIdx.x & 63;
    const size_t tile = (size_t)blockIdx.x * 2 + (threadIdx.x >> 6);
    if (tile >= ntiles)
        return;
    const v4u *src = in + tile * 1024 + lane;
    v4u *dst = out + tile * 1024 + lane;
    v4u v[16];
#pragma unroll
    for (int q = 0; q < 16; ++q)
        v[q] = NT ? __builtin_nontemporal_load(src + 64 * q) : src[64 * q];
#pragma unroll
    for (int q = 0; q < 16; ++q) {
        if (NT)
            __builtin_nontemporal_store(v[q], dst + 64 * q);
        else
            dst[64 * q] = v[q];
    }
}

template <class F>
double time_ms(F launch, int reps)
{
    hipEvent_t a, b;
    CHECK(hipEventCreate(&a));
    CHECK(hipEventCreate(&b));
    for (int w = 0; w < 3; ++w)
        launch();
    CHECK(hipEventRecord(a));
    for (int r = 0; r < reps; ++r)
        launch();
    CHECK(hipEventRecord(b));
    CHECK(hipEventSynchronize(b));
    CHECK(hipGetLastError());
    float ms;
    CHECK(hipEventElapsedTime(&ms, a, b));
    CHECK(hipEventDestroy(a));
    CHECK(hipEventDestroy(b));
    return ms / reps;
}

// Copy bandwidth as a function of the working set (in + out bytes), to see
// where the 256 MB last-level cache (MALL) stops holding both buffers.
void copy_working_set(int cus)
{
    for (int lg = 20; lg <= 27; ++lg) {
        const size_t n = (size_t)1 << lg, ntiles = n / 4096;
        uint32_t *in, *out;
        CHECK(hipMalloc(&in, n * 4));
        CHECK(hipMalloc(&out, n * 4));
        CHECK(hipMemset(in, 1, n * 4));
        const dim3 grid((unsigned)((ntiles + 1) / 2)), block(128);
        const int reps = lg <= 24 ? 200 : 20;
        const double plain = time_ms([&] { hipLaunchKernelGGL(copy_tiles_strided<false>, grid, block, 0, 0, in, out, ntiles); }, reps);
        const double nt = time_ms([&] { hipLaunchKernelGGL(copy_tiles_strided<true>, grid, block, 0, 0, in, out, ntiles); }, reps);
        std::printf("working set %7.1f MiB (2^%d u32 in + out): plain %8.1f GB/s  nontemporal %8.1f GB/s\n",
                    2.0 * n * 4 / 1048576.0, lg, 2.0 * n * 4 / (plain * 1e-3) / 1e9, 2.0 * n * 4 / (nt * 1e-3) / 1e9);
        CHECK(hipFree(in));
        CHECK(hipFree(out));
    }
    (void)cus;
}

void copy_variants(int cus)
{
    copy_working_set(cus);
    for (int lg : {26, 28}) {
        const size_t n = (size_t)1 << lg, ntiles = n / 4096;
        uint32_t *in, *out;
        CHECK(hipMalloc(&in, n * 4));
        CHECK(hipMalloc(&out, n * 4));
        CHECK(hipMemset(in, 1, n * 4));
        const dim3 grid((unsigned)((ntiles + 1) / 2)), block(128);
        struct V {
            const char *name;
            double ms;
        } vs[6];
        vs[0] = {"tile copy, dword per lane (64 loads)", time_ms([&] { hipLaunchKernelGGL(copy_tiles_strided<false>, grid, block, 0, 0, in, out, ntiles); }, 20)};
        vs[1] = {"tile copy, dword per lane, nontemporal", time_ms([&] { hipLaunchKernelGGL(copy_tiles_strided<true>, grid, block, 0, 0, in, out, ntiles); }, 20)};
        vs[2] = {"tile copy, dwordx4 per lane (16 loads)", time_ms([&] { hipLaunchKernelGGL(copy_tiles_x4<false>, grid, block, 0, 0, (const v4u *)in, (v4u *)out, ntiles); }, 20)};
        vs[3] = {"tile copy, dwordx4 per lane, nontemporal", time_ms([&] { hipLaunchKernelGGL(copy_tiles_x4<true>, grid, block, 0, 0, (const v4u *)in, (v4u *)out, ntiles); }, 20)};
        vs[4] = {"grid-stride dwordx4, 64 groups/CU", time_ms([&] { hipLaunchKernelGGL(copy_u32x4, dim3(cus * 64), dim3(256), 0, 0, (const uint4 *)in, (uint4 *)out, n / 4); }, 20)};
        vs[5] = {"hipMemcpyAsync device to device", time_ms([&] { CHECK(hipMemcpyAsync(out, in, n * 4, hipMemcpyDeviceToDevice, 0)); }, 20)};
        for (auto &v : vs)
            std::printf("copy 2^%d u32 %-44s %8.1f us %8.1f GB/s\n", lg, v.name, v.ms * 1e3, 2.0 * n * 4 / (v.ms * 1e-3) / 1e9);
        CHECK(hipFree(in));
        CHECK(hipFree(out));
    }
}

template <int P, int W>
void run_one(uint32_t *sink, unsigned long long *cyc_d, std::vector<unsigned long long> &cyc_h, int cus,
             double clk_hz)
{
    // host-side bounds check of every address the kernel will touch
    for (uint32_t l = 0; l < 64; ++l) {
        uint32_t last = W * pattern_addr(P, l) + (kUnroll - 1) * kSpread + W - 1;
        if (last >= (uint32_t)kLdsWords)
            return;  // pattern does not fit at this width: skipped
        if ((W * pattern_addr(P, l)) % W != 0) {
            std::fprintf(stderr, "pattern %d width %d misaligned\n", P, W);
            std::exit(2);
        }
    }
    const int iters = 2048;
    hipLaunchKernelGGL((lds_probe<P, W>), dim3(1), dim3(64), 0, 0, sink, cyc_d, iters);
    CHECK(hipGetLastError());
    CHECK(hipDeviceSynchronize());
    CHECK(hipMemcpy(cyc_h.data(), cyc_d, cyc_h.size() * sizeof(unsigned long long), hipMemcpyDeviceToHost));
    double per_instr_wave = (double)cyc_h[P * 8 + W] / (double)(iters * kUnroll);
    // chip-wide throughput: 8 one-wave groups per CU
    const int blocks = cus * 8;
    hipEvent_t a, b;
    CHECK(hipEventCreate(&a));
    CHECK(hipEventCreate(&b));
    CHECK(hipEventRecord(a));
    hipLaunchKernelGGL((lds_probe<P, W>), dim3(blocks), dim3(64), 0, 0, sink, cyc_d, iters);
    CHECK(hipEventRecord(b));
    CHECK(hipEventSynchronize(b));
    CHECK(hipGetLastError());
    float ms = 0;
    CHECK(hipEventElapsedTime(&ms, a, b));
    double instr_per_cu = (double)blocks / cus * iters * kUnroll;
    double cyc_per_instr_cu = ms * 1e-3 * clk_hz / instr_per_cu;
    std::printf("%-34s b%-4d wave_cycles/instr %7.2f   CU_cycles/instr %7.2f   bytes/clk/CU %7.1f\n",
                pattern_name(P), 32 * W, per_instr_wave, cyc_per_instr_cu,
                64.0 * 4 * W / cyc_per_instr_cu);
    CHECK(hipEventDestroy(a));
    CHECK(hipEventDestroy(b));
}

template <int P>
void run_pattern(uint32_t *sink, unsigned long long *cyc_d, std::vector<unsigned long long> &cyc_h, int cus,
                 double clk)
{
    run_one<P, 1>(sink, cyc_d, cyc_h, cus, clk);
    if constexpr (P != 7 && P != 10 && P != 9 && P != 13) {
        run_one<P, 2>(sink, cyc_d, cyc_h, cus, clk);
        run_one<P, 4>(sink, cyc_d, cyc_h, cus, clk);
    }
}

template <int... Ps>
void run_all(std::integer_sequence<int, Ps...>, uint32_t *sink, unsigned long long *cyc_d,
             std::vector<unsigned long long> &cyc_h, int cus, double clk)
{
    (run_pattern<Ps>(sink, cyc_d, cyc_h, cus, clk), ...);
}

int main()
{
    hipDeviceProp_t prop;
    CHECK(hipGetDeviceProperties(&prop, 0));
    int clk_khz = 0;
    CHECK(hipDeviceGetAttribute(&clk_khz, hipDeviceAttributeClockRate, 0));
    std::printf("device %s arch %s CUs %d warpSize %d sharedMemPerBlock %zu maxSharedPerMP %zu clock %d kHz "
                "memclk %d kHz busWidth %d L2 %d\n",
                prop.name, prop.gcnArchName, prop.multiProcessorCount, prop.warpSize, prop.sharedMemPerBlock,
                prop.maxSharedMemoryPerMultiProcessor, clk_khz, prop.memoryClockRate, prop.memoryBusWidth,
                prop.l2CacheSize);
    const int cus = prop.multiProcessorCount;
    const double clk = clk_khz * 1e3;
    uint32_t *sink;
    unsigned long long *cyc_d;
    CHECK(hipMalloc(&sink, (size_t)cus * 8 * 64 * sizeof(uint32_t)));
    CHECK(hipMalloc(&cyc_d, 16 * 8 * sizeof(unsigned long long)));
    CHECK(hipMemset(cyc_d, 0, 16 * 8 * sizeof(unsigned long long)));
    std::vector<unsigned long long> cyc_h(16 * 8);
    const bool copy_only = std::getenv("PROBE_COPY_ONLY") != nullptr;
    if (!copy_only)
        run_all(std::make_integer_sequence<int, kPatterns>{}, sink, cyc_d, cyc_h, cus, clk);

    // streaming copy: achievable HBM rate
    for (int lg : {26, 28}) {
        size_t n = (size_t)1 << lg;
        uint32_t *in, *out;
        CHECK(hipMalloc(&in, n * 4));
        CHECK(hipMalloc(&out, n * 4));
        CHECK(hipMemset(in, 1, n * 4));
        size_t n4 = n / 4;
        int threads = 256;
        int blocks = cus * 16;
        hipEvent_t a, b;
        CHECK(hipEventCreate(&a));
        CHECK(hipEventCreate(&b));
        for (int w = 0; w < 3; ++w)
            hipLaunchKernelGGL(copy_u32x4, dim3(blocks), dim3(threads), 0, 0, (const uint4 *)in, (uint4 *)out, n4);
        const int reps = 20;
        CHECK(hipEventRecord(a));
        for (int r = 0; r < reps; ++r)
            hipLaunchKernelGGL(copy_u32x4, dim3(blocks), dim3(threads), 0, 0, (const uint4 *)in, (uint4 *)out, n4);
        CHECK(hipEventRecord(b));
        CHECK(hipEventSynchronize(b));
        CHECK(hipGetLastError());
        float ms;
        CHECK(hipEventElapsedTime(&ms, a, b));
        double s = ms * 1e-3 / reps;
        std::printf("copy 2^%d u32: %.1f us  %.1f GB/s (read+write)\n", lg, s * 1e6, 2.0 * n * 4 / s / 1e9);
        CHECK(hipFree(in));
        CHECK(hipFree(out));
        CHECK(hipEventDestroy(a));
        CHECK(hipEventDestroy(b));
    }
    copy_variants(cus);
    CHECK(hipFree(sink));
    CHECK(hipFree(cyc_d));
    std::printf("done\n");
    return 0;
}
