/*
 * Driver that runs every oracle entry point on small inputs, built together
 * with oracle/oracle.c under AddressSanitizer and UndefinedBehaviorSanitizer
 * by tests/test_sanitize.py. It checks memory safety and defined behaviour of
 * the checker itself, plus a few self-consistency facts (round trips, levels
 * equal between the queue search and Algorithm 3). Inputs come from a small
 * linear congruential generator; nothing here computes the method.
 */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

typedef struct oracle_adj oracle_adj;
oracle_adj *oracle_adj_build(int64_t n, int64_t m, const int64_t *src, const int64_t *dst);
void oracle_adj_free(oracle_adj *a);
int64_t oracle_adj_n(const oracle_adj *a);
int64_t oracle_adj_degree(const oracle_adj *a, int64_t v);
int64_t oracle_bfs(const oracle_adj *a, int64_t root, int32_t *level);
int oracle_parents_max(const oracle_adj *a, const int32_t *level, int64_t root, int32_t *parent);
int oracle_validate(int64_t n, int64_t m, const int64_t *src, const int64_t *dst, int64_t root,
                    const int32_t *level, const int32_t *parent, const int32_t *ref_level);
int oracle_directory(int64_t n, int32_t p, int64_t m, const int64_t *src, const int64_t *dst, uint8_t *V);
int64_t oracle_wah_encode(const uint8_t *bits, int64_t nbits, int32_t w, int32_t fill_bit_field,
                          uint64_t *out, int64_t cap);
int oracle_wah_decode(const uint64_t *words, int64_t nw, int64_t nbits, int32_t w, int32_t fill_bit_field,
                      uint8_t *bits);
int64_t oracle_alg3_cap(int64_t n, int32_t p);
int64_t oracle_alg3(const oracle_adj *a, int32_t p, const uint8_t *V, int64_t root, int32_t max_levels,
                    int32_t *level, int32_t *parent, int64_t *words, int64_t *sieved_bits,
                    int64_t *unsieved_words, uint64_t *dump);
int64_t oracle_teps_m(int64_t m, const int64_t *src, const int64_t *dst, const int32_t *level);

static uint64_t lcg_state = 0x9E3779B97F4A7C15ull;
static uint64_t next_u64(void)
{
    lcg_state = lcg_state * 6364136223846793005ull + 1442695040888963407ull;
    return lcg_state ^ (lcg_state >> 29);
}

#define CHECK(c)                                                           \
    do {                                                                   \
        if (!(c)) {                                                        \
            fprintf(stderr, "check failed at line %d: %s\n", __LINE__, #c); \
            return 1;                                                      \
        }                                                                  \
    } while (0)

static int wah_cases(void)
{
    static const int widths[] = {4, 5, 8, 32, 64};
    for (int wi = 0; wi < 5; ++wi) {
        const int w = widths[wi];
        for (int fb = 0; fb < 2; ++fb) {
            for (int t = 0; t < 60; ++t) {
                const int64_t nbits = (int64_t)(next_u64() % 700);
                uint8_t *bits = malloc((size_t)(nbits > 0 ? nbits : 1));
                uint8_t *back = malloc((size_t)(nbits > 0 ? nbits : 1));
                const int kind = (int)(next_u64() % 4);
                for (int64_t k = 0; k < nbits; ++k) {
                    const uint64_t r = next_u64();
                    bits[k] = kind == 0 ? 0 : kind == 1 ? 1 : kind == 2 ? (uint8_t)(r & 1)
                                                                        : (uint8_t)((k / 97) & 1);
                }
                const int64_t cap = nbits / (w - 1) + 2;
                uint64_t *out = malloc(sizeof(uint64_t) * (size_t)cap);
                const int64_t nw = oracle_wah_encode(bits, nbits, w, fb, out, cap);
                CHECK(nw >= 0 && nw <= cap);
                CHECK(oracle_wah_decode(out, nw, nbits, w, fb, back) == 0);
                CHECK(nbits == 0 || memcmp(bits, back, (size_t)nbits) == 0);
                /* corrupted streams: decode must reject or accept without faults */
                for (int c = 0; c < 4 && nw > 0; ++c) {
                    out[next_u64() % (uint64_t)nw] ^= (uint64_t)1 << (next_u64() % (uint64_t)w);
                    (void)oracle_wah_decode(out, nw, nbits, w, fb, back);
                }
                CHECK(oracle_wah_encode(bits, nbits, w, fb, out, 0) < 0 || nbits == 0);
                free(out);
                free(bits);
                free(back);
            }
        }
    }
    CHECK(oracle_wah_encode(NULL, 5, 64, 1, NULL, 0) < 0);
    CHECK(oracle_wah_decode(NULL, 3, 5, 64, 1, NULL) < 0);
    return 0;
}

static int graph_cases(void)
{
    static const int32_t ps[] = {1, 2, 4, 8};
    for (int t = 0; t < 12; ++t) {
        const int64_t n = 512 << (t % 3);
        const int64_t m = (int64_t)(next_u64() % (uint64_t)(3 * n)) + 1;
        int64_t *src = malloc(sizeof(int64_t) * (size_t)m), *dst = malloc(sizeof(int64_t) * (size_t)m);
        for (int64_t e = 0; e < m; ++e) {
            src[e] = (int64_t)(next_u64() % (uint64_t)(n / 2));
            dst[e] = (e % 11 == 0) ? src[e] : (int64_t)(next_u64() % (uint64_t)(n / 2));
        }
        oracle_adj *a = oracle_adj_build(n, m, src, dst);
        CHECK(a && oracle_adj_n(a) == n);
        CHECK(oracle_adj_degree(a, -1) < 0 && oracle_adj_degree(a, n) < 0);
        int32_t *level = malloc(sizeof(int32_t) * (size_t)n), *parent = malloc(sizeof(int32_t) * (size_t)n);
        int32_t *l3 = malloc(sizeof(int32_t) * (size_t)n), *p3 = malloc(sizeof(int32_t) * (size_t)n);
        const int64_t root = src[0];
        const int64_t nl = oracle_bfs(a, root, level);
        CHECK(nl >= 1);
        CHECK(oracle_parents_max(a, level, root, parent) == 0);
        CHECK(oracle_validate(n, m, src, dst, root, level, parent, level) == 0);
        CHECK(oracle_teps_m(m, src, dst, level) >= 0);
        const int32_t p = ps[t % 4];
        uint8_t *V = malloc((size_t)(p * n));
        CHECK(oracle_directory(n, p, m, src, dst, V) == 0);
        const int32_t L = 64;
        const int64_t cap = oracle_alg3_cap(n, p);
        int64_t *words = calloc((size_t)L * p * p, sizeof(int64_t));
        int64_t *sb = calloc((size_t)L * p * p, sizeof(int64_t));
        int64_t *uw = calloc((size_t)L * p, sizeof(int64_t));
        uint64_t *dump = calloc((size_t)L * p * p * (size_t)cap, sizeof(uint64_t));
        const int64_t nl3 = oracle_alg3(a, p, V, root, L, l3, p3, words, sb, uw, dump);
        CHECK(nl3 == nl);
        CHECK(memcmp(level, l3, sizeof(int32_t) * (size_t)n) == 0);
        CHECK(memcmp(parent, p3, sizeof(int32_t) * (size_t)n) == 0);
        CHECK(oracle_alg3(a, p, V, root, 1, l3, p3, words, NULL, NULL, NULL) == (nl > 1 ? -2 : 1));
        CHECK(oracle_alg3(a, p, V, n, L, l3, p3, words, NULL, NULL, NULL) == -1);
        /* planted mistake: the validator must flag it */
        for (int64_t v = 0; v < n; ++v)
            if (v != root && level[v] > 0) {
                parent[v] = -1;
                break;
            }
        CHECK(nl == 1 || oracle_validate(n, m, src, dst, root, level, parent, NULL) != 0);
        free(V);
        free(words);
        free(sb);
        free(uw);
        free(dump);
        free(level);
        free(parent);
        free(l3);
        free(p3);
        oracle_adj_free(a);
        free(src);
        free(dst);
    }
    CHECK(oracle_adj_build(0, 0, NULL, NULL) == NULL);
    int64_t bad = 5;
    CHECK(oracle_adj_build(4, 1, &bad, &bad) == NULL);
    oracle_adj_free(NULL);
    return 0;
}

int main(void)
{
    if (wah_cases() || graph_cases())
        return 1;
    printf("oracle sanitizer check ok\n");
    return 0;
}
