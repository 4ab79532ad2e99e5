/*
 * Drives every function of the CPU oracle (oracle/bcf_oracle.c) on seeded
 * inputs of many sizes, edge cases included, so that a build with
 * AddressSanitizer and UndefinedBehaviorSanitizer sees every code path:
 * out-of-bounds accesses, use after free, signed overflow, bad shifts.  The
 * results are checked only loosely here (sortedness, multiset hash); the
 * oracle's pins live in the Python tests.  Exit status 0 on success.
 */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

int oracle_sort_u32(const uint32_t *in, uint32_t *out, uint64_t n);
int oracle_sort_pairs_u32(const uint32_t *kin, const uint32_t *vin, uint32_t *kout, uint32_t *vout, uint64_t n);
int oracle_sort_typed(int kind, const uint32_t *kin, const uint32_t *vin, uint32_t *kout, uint32_t *vout,
                      uint64_t n);
int oracle_colored_prefix_sums(const uint32_t *values, const uint8_t *colors, uint32_t *out, uint64_t n, uint32_t d);
int oracle_sort_u64(const uint64_t *in, uint64_t *out, uint64_t n);
int oracle_merge_runs(const uint32_t *kin, const uint32_t *vin, const uint64_t *off, uint32_t k, uint32_t *kout,
                      uint32_t *vout);
int oracle_segmented_sort(const uint32_t *kin, uint32_t *kout, const uint64_t *off, uint32_t nseg);
void oracle_multiset_hash(const uint32_t *keys, const uint32_t *vals, uint64_t n, uint64_t *sum_out,
                          uint64_t *xor_out);
int oracle_is_sorted_u32(const uint32_t *keys, uint64_t n);
int oracle_distribute_runs(const uint32_t *keys, const uint64_t *off, uint32_t s, uint32_t P, uint32_t t, int pb,
                           uint32_t *out, uint64_t *piece_off, uint32_t *splitters);

static uint64_t state = 0x9E3779B97F4A7C15ull;
static uint64_t next(void)
{
    uint64_t z = (state += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

static int failures = 0;
#define CHECK(c)                                                     \
    do {                                                             \
        if (!(c)) {                                                  \
            fprintf(stderr, "check failed line %d: %s\n", __LINE__, #c); \
            failures++;                                              \
        }                                                            \
    } while (0)

static void fill(uint32_t *a, uint64_t n, int mode)
{
    for (uint64_t i = 0; i < n; i++) {
        uint32_t x = (uint32_t)(next() >> 32);
        a[i] = mode == 0 ? x : mode == 1 ? x % 3u : mode == 2 ? 0xFFFFFFFFu : (uint32_t)(n - i);
    }
}

static void same_multiset(const uint32_t *a, const uint32_t *va, const uint32_t *b, const uint32_t *vb, uint64_t n)
{
    uint64_t s1, x1, s2, x2;
    oracle_multiset_hash(a, va, n, &s1, &x1);
    oracle_multiset_hash(b, vb, n, &s2, &x2);
    CHECK(s1 == s2 && x1 == x2);
}

int main(void)
{
    static const uint64_t sizes[] = {0, 1, 2, 3, 7, 64, 65, 4095, 4096, 4097, 12345, 100003};
    for (size_t si = 0; si < sizeof(sizes) / sizeof(sizes[0]); si++) {
        const uint64_t n = sizes[si];
        const size_t b = (size_t)(n ? n : 1) * sizeof(uint32_t);
        uint32_t *k = malloc(b), *v = malloc(b), *ko = malloc(b), *vo = malloc(b);
        uint64_t *k64 = malloc((size_t)(n ? n : 1) * 8), *o64 = malloc((size_t)(n ? n : 1) * 8);
        uint8_t *col = malloc(n ? n : 1);
        for (int mode = 0; mode < 4; mode++) {
            fill(k, n, mode);
            for (uint64_t i = 0; i < n; i++)
                v[i] = (uint32_t)i;
            CHECK(oracle_sort_u32(k, ko, n) == 0);
            CHECK(oracle_is_sorted_u32(ko, n));
            same_multiset(k, 0, ko, 0, n);
            memcpy(ko, k, b);
            CHECK(oracle_sort_u32(ko, ko, n) == 0);  // in place
            CHECK(oracle_is_sorted_u32(ko, n));
            CHECK(oracle_sort_pairs_u32(k, v, ko, vo, n) == 0);
            same_multiset(k, v, ko, vo, n);
            for (int kind = 1; kind <= 2; kind++) {
                CHECK(oracle_sort_typed(kind, k, v, ko, vo, n) == 0);
                CHECK(oracle_sort_typed(kind, k, 0, ko, 0, n) == 0);
            }
            CHECK(oracle_sort_typed(7, k, 0, ko, 0, n) == -2);
            for (uint64_t i = 0; i < n; i++) {
                k64[i] = next();
                col[i] = (uint8_t)(next() & 255u);
            }
            CHECK(oracle_sort_u64(k64, o64, n) == 0);
            for (uint64_t i = 1; i < n; i++)
                CHECK(o64[i - 1] <= o64[i]);
            for (uint32_t d = 1; d <= 256; d *= 4)
                CHECK(oracle_colored_prefix_sums(v, col, ko, n, d) == 0);
            CHECK(oracle_colored_prefix_sums(v, col, ko, n, 0) == -2);
            // runs / segments: up to 9 pieces, some empty
            for (uint32_t parts = 1; parts <= 9; parts += 4) {
                uint64_t off[10];
                off[0] = 0;
                for (uint32_t r = 1; r < parts; r++) {
                    uint64_t c = n ? next() % (n + 1) : 0;
                    off[r] = c < off[r - 1] ? off[r - 1] : c;
                }
                off[parts] = n;
                CHECK(oracle_segmented_sort(k, ko, off, parts) == 0);
                memcpy(vo, ko, b);  // every segment sorted: a valid merge input
                uint32_t *mk = malloc(b), *mv = malloc(b);
                CHECK(oracle_merge_runs(vo, v, off, parts, mk, mv) == 0);
                CHECK(oracle_is_sorted_u32(mk, n));
                CHECK(oracle_merge_runs(vo, 0, off, parts, mk, 0) == 0);
                for (uint32_t P = 1; P <= 8; P *= 2)
                    for (int pb = 0; pb <= 1; pb++) {
                        const uint64_t nb = pb ? 2 * P - 1 : P;
                        uint64_t *po = malloc((size_t)(nb * parts + 1) * 8);
                        uint32_t spl[8];
                        CHECK(oracle_distribute_runs(vo, off, parts, P, 3, pb, mk, po, spl) == 0);
                        free(po);
                    }
                free(mk);
                free(mv);
            }
        }
        free(k), free(v), free(ko), free(vo), free(k64), free(o64), free(col);
    }
    // bad offsets are refused
    uint32_t a[4] = {1, 2, 3, 4}, o[4];
    uint64_t bad[3] = {0, 3, 2};
    CHECK(oracle_merge_runs(a, 0, bad, 2, o, 0) != 0);
    if (failures)
        return 1;
    printf("oracle sanitizer run: ok\n");
    return 0;
}
