/* Drives every entry point of the oracle (oracle/sr4.c) on small seeded inputs
 * and its edge cases, for a build under AddressSanitizer and
 * UndefinedBehaviorSanitizer.  The checks here are only that each call
 * succeeds and that its output is ordered and a permutation of its input;
 * the oracle's values are pinned by the other oracle tests.  Prints OK. */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

int lsd_u32(const uint32_t*, const uint32_t*, size_t, int, int, int, uint32_t*, uint32_t*);
int lsd_u64(const uint64_t*, const uint32_t*, size_t, int, int, int, uint64_t*, uint32_t*);
int digit_counts_u32(const uint32_t*, size_t, int, int, uint64_t*);
int digit_counts_u64(const uint64_t*, size_t, int, int, uint64_t*);
int segmented_u32(const uint32_t*, const uint32_t*, const uint64_t*, size_t, uint32_t*, uint32_t*);
int segmented_u64(const uint64_t*, const uint32_t*, const uint64_t*, size_t, uint64_t*, uint32_t*);
int gsd_u32(const uint32_t*, const uint32_t*, size_t, int, int, uint32_t*, uint32_t*,
            uint64_t*, uint32_t*, uint64_t*, int*);
int ger_u32(const uint32_t*, const uint32_t*, size_t, int, int, const uint32_t*, size_t,
            uint32_t*, uint32_t*, uint64_t*, uint32_t*, uint64_t*, int*);
int gvr_u32(const uint32_t*, const uint32_t*, size_t, int, int, const uint32_t*, size_t,
            uint32_t*, uint32_t*, uint64_t*, uint32_t*, uint64_t*, int*);
int sort_kind(uint64_t*, uint32_t*, size_t, int, int);

static uint64_t state = 0x9E3779B97F4A7C15ull;

static uint64_t next(void)   /* xorshift64* */
{
    state ^= state >> 12;
    state ^= state << 25;
    state ^= state >> 27;
    return state * 0x2545F4914F6CDD1Dull;
}

static int fails;

#define CHECK(c)                                                              \
    do {                                                                      \
        if (!(c)) {                                                           \
            fprintf(stderr, "check failed line %d: %s\n", __LINE__, #c);      \
            ++fails;                                                          \
        }                                                                     \
    } while (0)

/* keys sorted and the payloads a permutation of 0..n-1 that maps back */
static void check_u32(const uint32_t* in, const uint32_t* k, const uint32_t* v, size_t n)
{
    for (size_t i = 1; i < n; ++i) CHECK(k[i - 1] <= k[i]);
    if (!v) return;
    char* seen = calloc(n ? n : 1, 1);
    for (size_t i = 0; i < n; ++i) {
        CHECK(v[i] < n);
        if (v[i] < n) {
            CHECK(!seen[v[i]]);
            seen[v[i]] = 1;
            CHECK(in[v[i]] == k[i]);
        }
    }
    free(seen);
}

static void fill_u32(uint32_t* a, size_t n, int kind)
{
    for (size_t i = 0; i < n; ++i) {
        uint64_t r = next();
        a[i] = kind == 0 ? (uint32_t)r : kind == 1 ? (uint32_t)(r % 7) : 42u;
    }
}

static void plain_sorts(void)
{
    const size_t sizes[] = {0, 1, 2, 3, 255, 256, 257, 1000, 4097};
    for (size_t si = 0; si < sizeof sizes / sizeof *sizes; ++si)
        for (int kind = 0; kind < 3; ++kind) {
            size_t n = sizes[si];
            uint32_t* k = malloc((n ? n : 1) * 4);
            uint32_t* v = malloc((n ? n : 1) * 4);
            uint32_t* ko = malloc((n ? n : 1) * 4);
            uint32_t* vo = malloc((n ? n : 1) * 4);
            uint64_t* k64 = malloc((n ? n : 1) * 8);
            uint64_t* k64o = malloc((n ? n : 1) * 8);
            fill_u32(k, n, kind);
            for (size_t i = 0; i < n; ++i) {
                v[i] = (uint32_t)i;
                k64[i] = ((uint64_t)k[i] << 32) | (next() & 3);
            }
            for (int bits = 8; bits <= 16; bits += 8) {
                CHECK(lsd_u32(k, v, n, bits, 0, 32, ko, vo) == 0);
                check_u32(k, ko, vo, n);
                CHECK(lsd_u32(k, NULL, n, bits, 4, 28, ko, NULL) == 0);
                CHECK(lsd_u64(k64, v, n, bits, 0, 64, k64o, vo) == 0);
                for (size_t i = 1; i < n; ++i) CHECK(k64o[i - 1] <= k64o[i]);
            }
            memcpy(ko, k, n * 4);
            memcpy(vo, v, n * 4);
            CHECK(lsd_u32(ko, vo, n, 8, 0, 32, ko, vo) == 0);   /* in place */
            check_u32(k, ko, vo, n);
            uint64_t cnt[1 << 16];
            CHECK(digit_counts_u32(k, n, 8, 8, cnt) == 0);
            uint64_t tot = 0;
            for (int d = 0; d < 256; ++d) tot += cnt[d];
            CHECK(tot == n);
            CHECK(digit_counts_u64(k64, n, 48, 16, cnt) == 0);
            for (size_t i = 0; i < n; ++i) k64[i] = (uint64_t)k[i] | ((uint64_t)(i & 1) << 63);
            CHECK(sort_kind(k64, vo, n, 64, 1) == 0);
            CHECK(sort_kind(k64, NULL, n, 32, 2) == 0);
            free(k); free(v); free(ko); free(vo); free(k64); free(k64o);
        }
    CHECK(lsd_u32(NULL, NULL, 0, 8, 0, 32, NULL, NULL) == 0);
    CHECK(lsd_u32(NULL, NULL, 5, 8, 0, 32, NULL, NULL) != 0);
    CHECK(lsd_u32(NULL, NULL, 0, 8, 0, 33, NULL, NULL) != 0);
}

static void segmented(void)
{
    const uint64_t off[] = {0, 0, 1, 5, 300, 300, 1300, 1301};
    const size_t nseg = sizeof off / sizeof *off - 1, n = off[nseg];
    uint32_t k[1301], v[1301], ko[1301], vo[1301];
    uint64_t k64[1301], k64o[1301];
    fill_u32(k, n, 0);
    for (size_t i = 0; i < n; ++i) {
        v[i] = (uint32_t)i;
        k64[i] = next();
    }
    CHECK(segmented_u32(k, v, off, nseg, ko, vo) == 0);
    for (size_t s = 0; s < nseg; ++s)
        for (uint64_t i = off[s] + 1; i < off[s + 1]; ++i) CHECK(ko[i - 1] <= ko[i]);
    CHECK(segmented_u64(k64, v, off, nseg, k64o, vo) == 0);
    const uint64_t bad[] = {0, 10, 5};
    CHECK(segmented_u32(k, NULL, bad, 2, ko, NULL) != 0);
}

static void sample_sorts(void)
{
    const size_t sizes[] = {1, 2, 7, 100, 1000, 5003};
    const int ps[] = {1, 2, 3, 16, 64};
    for (size_t si = 0; si < sizeof sizes / sizeof *sizes; ++si)
        for (size_t pi = 0; pi < sizeof ps / sizeof *ps; ++pi)
            for (int kind = 0; kind < 3; ++kind) {
                const size_t n = sizes[si];
                const int p = ps[pi], s = 4;
                uint32_t* k = malloc(n * 4);
                uint32_t* v = malloc(n * 4);
                uint32_t* ko = malloc(n * 4);
                uint32_t* vo = malloc(n * 4);
                uint64_t* cnt = calloc((size_t)p * p, 8);
                uint32_t* sk = calloc((size_t)p, 4);
                uint64_t* sg = calloc((size_t)p, 8);
                const size_t npos = (size_t)s * p;
                uint32_t* pos = malloc(npos * 4);
                fill_u32(k, n, kind);
                for (size_t i = 0; i < n; ++i) v[i] = (uint32_t)i;
                for (size_t i = 0; i < npos; ++i) pos[i] = (uint32_t)(next() % n);
                int pu = 0;
                CHECK(gsd_u32(k, v, n, p, 2, ko, vo, cnt, sk, sg, &pu) == 0);
                check_u32(k, ko, vo, n);
                CHECK(ger_u32(k, v, n, p, s, pos, npos, ko, vo, cnt, sk, sg, &pu) == 0);
                check_u32(k, ko, vo, n);
                CHECK(gvr_u32(k, v, n, p, s, pos, npos, ko, vo, cnt, sk, sg, &pu) == 0);
                check_u32(k, ko, vo, n);
                CHECK(gvr_u32(k, NULL, n, p, s, pos, npos, ko, NULL, cnt, sk, sg, &pu) == 0);
                CHECK(ger_u32(k, v, n, p, s, pos, 0, ko, vo, cnt, sk, sg, &pu) != 0 || s * p < 2);
                free(k); free(v); free(ko); free(vo); free(cnt); free(sk); free(sg); free(pos);
            }
}

int main(void)
{
    plain_sorts();
    segmented();
    sample_sorts();
    if (fails) {
        fprintf(stderr, "%d checks failed\n", fails);
        return 1;
    }
    puts("OK");
    return 0;
}
