/*
 * Driver that runs the seeded input generator (rmat.c) on small sizes under
 * AddressSanitizer and UndefinedBehaviorSanitizer, built by
 * tests/test_sanitize.py: permutation, R-MAT and Erdos-Renyi tuples, root
 * picking, and the argument checks. Checks only ranges and distinctness.
 */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

uint64_t rmat_rng(uint64_t seed, uint64_t ctr);
int rmat_permutation(int64_t n, uint64_t seed, int64_t *perm);
int rmat_edges(int32_t scale, int64_t m, double a, double b, double c, uint64_t seed, const int64_t *perm,
               int64_t *src, int64_t *dst);
int er_edges(int64_t n, int64_t m, uint64_t seed, int64_t *src, int64_t *dst);
int64_t rmat_pick_roots(int64_t n, int64_t m, const int64_t *src, const int64_t *dst, int64_t count,
                        uint64_t seed, int64_t *roots);

#define CHECK(c)                                                           \
    do {                                                                   \
        if (!(c)) {                                                        \
            fprintf(stderr, "check failed at line %d: %s\n", __LINE__, #c); \
            return 1;                                                      \
        }                                                                  \
    } while (0)

int main(void)
{
    for (int scale = 1; scale <= 12; ++scale) {
        const int64_t n = (int64_t)1 << scale, m = 16 * n;
        int64_t *perm = malloc(sizeof(int64_t) * (size_t)n);
        uint8_t *seen = calloc((size_t)n, 1);
        int64_t *src = malloc(sizeof(int64_t) * (size_t)m), *dst = malloc(sizeof(int64_t) * (size_t)m);
        int64_t roots[16];
        CHECK(rmat_permutation(n, 7 + (uint64_t)scale, perm) == 0);
        for (int64_t i = 0; i < n; ++i) {
            CHECK(perm[i] >= 0 && perm[i] < n && !seen[perm[i]]);
            seen[perm[i]] = 1;
        }
        CHECK(rmat_edges(scale, m, 0.57, 0.19, 0.19, 11, perm, src, dst) == 0);
        for (int64_t t = 0; t < m; ++t)
            CHECK(src[t] >= 0 && src[t] < n && dst[t] >= 0 && dst[t] < n);
        const int64_t got = rmat_pick_roots(n, m, src, dst, 16, 3, roots);
        CHECK(got >= 0 && got <= 16);
        for (int64_t k = 0; k < got; ++k) {
            CHECK(roots[k] >= 0 && roots[k] < n);
            for (int64_t q = 0; q < k; ++q)
                CHECK(roots[q] != roots[k]);
        }
        CHECK(er_edges(n, m, 5, src, dst) == 0);
        for (int64_t t = 0; t < m; ++t)
            CHECK(src[t] >= 0 && src[t] < n && dst[t] >= 0 && dst[t] < n);
        free(perm);
        free(seen);
        free(src);
        free(dst);
    }
    int64_t x = 0;
    CHECK(rmat_permutation(0, 1, &x) < 0);
    CHECK(rmat_edges(0, 1, 0.5, 0.2, 0.2, 1, NULL, &x, &x) < 0);
    CHECK(rmat_edges(4, 1, 0.9, 0.2, 0.2, 1, NULL, &x, &x) < 0);
    CHECK(er_edges(0, 1, 1, &x, &x) < 0);
    CHECK(rmat_pick_roots(4, 1, NULL, NULL, 1, 1, &x) < 0);
    (void)rmat_rng(1, 2);
    printf("generator sanitizer check ok\n");
    return 0;
}
