// Drives the host-side paths of the C ABI (include/bcf.h) that run without a
// GPU: temp-size queries, argument validation, the host planners of the
// table-driven calls (segmented sorts, merges of runs and of run groups, the
// distribution step), pass counts and tuning.  Built with AddressSanitizer and
// UndefinedBehaviorSanitizer on the host side only (no device code), so that
// the planners' index arithmetic and table building are checked for
// out-of-bounds accesses and undefined behaviour.  No call here launches a
// kernel or touches device memory.  Exit status 0 on success.
#include <algorithm>
#include <cstdint>
#include <cstdio>
#include <random>
#include <vector>

#include "bcf.h"

static int failures = 0;
#define CHECK(c)                                                         \
    do {                                                                 \
        if (!(c)) {                                                      \
            std::fprintf(stderr, "check failed line %d: %s\n", __LINE__, #c); \
            failures++;                                                  \
        }                                                                \
    } while (0)

static std::vector<uint64_t> offsets(std::mt19937_64 &g, uint32_t parts, uint64_t n, bool empties)
{
    std::vector<uint64_t> off(parts + 1, 0);
    for (uint32_t r = 1; r < parts; r++)
        off[r] = n ? g() % (n + 1) : 0;
    off[parts] = n;
    std::sort(off.begin(), off.end());
    if (!empties)  // spread duplicates: strictly rising where possible
        for (uint32_t r = 1; r <= parts && n >= parts; r++)
            if (off[r] <= off[r - 1])
                off[r] = off[r - 1] + 1 <= n ? off[r - 1] + 1 : n;
    off[parts] = n;
    return off;
}

int main()
{
    std::mt19937_64 g(12345);
    uint64_t need = 0;
    // sorts: queries over sizes, and errors
    const uint64_t sizes[] = {0, 1, 4095, 4096, 4097, 1u << 16, (1u << 19) + 3, 1u << 25, (1ull << 32) - 1};
    for (uint64_t n : sizes) {
        CHECK(bcf_sort_u32(nullptr, nullptr, n, nullptr, &need, nullptr) == BCF_OK);
        CHECK(bcf_sort_pairs_u32(nullptr, nullptr, nullptr, nullptr, n, nullptr, &need, nullptr) == BCF_OK);
        CHECK(bcf_sort_i32(nullptr, nullptr, n, nullptr, &need, nullptr) == BCF_OK);
        CHECK(bcf_sort_f32(nullptr, nullptr, n, nullptr, &need, nullptr) == BCF_OK);
        CHECK(bcf_sort_u64(nullptr, nullptr, n, nullptr, &need, nullptr) == BCF_OK);
        for (int pairs = 0; pairs <= 1; pairs++)
            CHECK(bcf_sort_passes(n, pairs) <= 64);
    }
    CHECK(bcf_sort_u32(nullptr, nullptr, 1ull << 32, nullptr, &need, nullptr) == BCF_ERR_INVALID);
    CHECK(bcf_sort_u32(nullptr, nullptr, 10, nullptr, nullptr, nullptr) == BCF_ERR_INVALID);
    for (int s = 0; s <= 5; s++)
        CHECK(bcf_status_string((bcf_status)s) != nullptr);

    // host planners: segmented sorts and merges of runs with random offsets,
    // with binary and fan-in 4 merge steps
    const uint64_t totals[] = {0, 1, 100, 4096, 4097, 70000, 1u << 20, (1u << 22) + 77};
    bcf_tuning saved{};
    bcf_get_tuning(&saved);
    for (int fan_in : {2, 4})
    for (uint64_t n : totals)
        for (uint32_t parts : {1u, 2u, 3u, 17u, 300u, 5000u})
            for (int empties = 0; empties <= 1; empties++) {
                auto off = offsets(g, parts, n, empties);
                CHECK(bcf_segmented_sort_host(nullptr, nullptr, off.data(), parts, nullptr, &need, nullptr) ==
                      BCF_OK);
                CHECK(bcf_segmented_sort_pairs_host(nullptr, nullptr, nullptr, nullptr, off.data(), parts, nullptr,
                                                    &need, nullptr) == BCF_OK);
                CHECK(bcf_segmented_upload(off.data(), parts, 0, nullptr, &need, nullptr) == BCF_OK);
                CHECK(bcf_merge_runs_host(nullptr, nullptr, off.data(), parts, nullptr, nullptr, nullptr, &need,
                                          nullptr) == BCF_OK);
                const void *vdummy = reinterpret_cast<const void *>(1);
                CHECK(bcf_merge_runs_host(nullptr, static_cast<const uint32_t *>(vdummy), off.data(), parts, nullptr,
                                          nullptr, nullptr, &need, nullptr) == BCF_OK);
                // groups of consecutive runs
                std::vector<uint32_t> gs{0};
                while (gs.back() < parts)
                    gs.push_back(std::min<uint32_t>(parts, gs.back() + 1 + uint32_t(g() % 7)));
                CHECK(bcf_merge_run_groups(nullptr, nullptr, off.data(), parts, gs.data(), uint32_t(gs.size() - 1),
                                           nullptr, nullptr, nullptr, &need, nullptr) == BCF_OK);
                for (uint32_t P : {1u, 4u, 256u})
                    for (int pb = 0; pb <= 1; pb++)
                        (void)bcf_distribute_runs(nullptr, off.data(), parts, P, P, pb, nullptr, nullptr, nullptr,
                                                  nullptr, &need, nullptr);
                bcf_tuning t4 = saved;
                t4.merge_fan_in = fan_in;
                CHECK(bcf_set_tuning(&t4) == BCF_OK);
            }
    CHECK(bcf_set_tuning(&saved) == BCF_OK);
    // invalid offsets are refused before any device access
    std::vector<uint64_t> bad{0, 5, 3, 9};
    CHECK(bcf_segmented_sort_host(nullptr, nullptr, bad.data(), 3, nullptr, &need, nullptr) == BCF_ERR_INVALID);
    CHECK(bcf_merge_runs_host(nullptr, nullptr, bad.data(), 3, nullptr, nullptr, nullptr, &need, nullptr) ==
          BCF_ERR_INVALID);
    std::vector<uint64_t> nz{1, 5};
    CHECK(bcf_merge_runs_host(nullptr, nullptr, nz.data(), 1, nullptr, nullptr, nullptr, &need, nullptr) ==
          BCF_ERR_INVALID);
    // sort by distribution: queries over its limits
    for (uint64_t n : {0ull, 1ull, 1ull << 20, 1ull << 26})
        for (uint32_t P : {1u, 16u, 256u})
            (void)bcf_sort_u32_pb(nullptr, nullptr, n, P, 1u << 18, 1, nullptr, &need, nullptr);
    // tuning round trip
    bcf_tuning t{}, back{};
    bcf_get_tuning(&t);
    CHECK(bcf_set_tuning(&t) == BCF_OK);
    bcf_get_tuning(&back);
    CHECK(back.merge_fan_in == t.merge_fan_in && back.block_sort == t.block_sort);
    if (failures)
        return 1;
    std::printf("host ABI sanitizer run: ok\n");
    return 0;
}
