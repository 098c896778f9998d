/*
 * Seeded synthetic graph inputs: R-MAT (Kronecker-style) and Erdos-Renyi
 * tuple lists, a seeded vertex permutation and a seeded root picker.
 *
 * This module only produces inputs. It holds none of the BFS, sieve or
 * compression arithmetic and is shared by the CPU oracle tests and the GPU
 * path alike, so that both see the same tuples.
 *
 * Workload shape follows the paper's experimental setup (Sec. VII.A): the
 * vertex count is 2^scale, the tuple count is edgefactor * 2^scale with
 * edgefactor 16, degrees follow a power law. Self-loops and duplicate tuples
 * are kept, as the TEPS definition counts them.
 *
 * Random numbers come from a counter-based generator: the SplitMix64 output
 * function (Steele, Lea and Flood, "Fast splittable pseudorandom number
 * generators", OOPSLA 2014) applied to seed + (counter + 1) * golden gamma.
 * Every draw is a pure function of (seed, counter), so results do not depend
 * on the number of threads.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define RMAT_GAMMA 0x9E3779B97F4A7C15ULL

uint64_t rmat_rng(uint64_t seed, uint64_t ctr)
{
    uint64_t z = seed + (ctr + 1ULL) * RMAT_GAMMA;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

/* Uniform integer in [0, range) by the multiply-shift method. */
static inline uint64_t bounded(uint64_t x, uint64_t range)
{
    return (uint64_t)(((unsigned __int128)x * range) >> 64);
}

/* Seeded uniform permutation of [0, n) by Fisher-Yates; draw i uses counter i. */
int rmat_permutation(int64_t n, uint64_t seed, int64_t *perm)
{
    if (n <= 0 || !perm)
        return -1;
    for (int64_t i = 0; i < n; ++i)
        perm[i] = i;
    for (int64_t i = n - 1; i > 0; --i) {
        int64_t j = (int64_t)bounded(rmat_rng(seed, (uint64_t)i), (uint64_t)i + 1);
        int64_t t = perm[i];
        perm[i] = perm[j];
        perm[j] = t;
    }
    return 0;
}

/*
 * R-MAT tuples. Tuple t picks one quadrant of the adjacency matrix at each of
 * `scale` recursion levels with probabilities (a, b, c, 1-a-b-c); level l sets
 * bit (scale-1-l) of the source (row half) and of the destination (column
 * half). Level l of tuple t uses the 32-bit half (d & 1) of draw d >> 1, with
 * d = t * scale + l. If perm is given, ids are mapped through it.
 */
int rmat_edges(int32_t scale, int64_t m, double a, double b, double c,
               uint64_t seed, const int64_t *perm, int64_t *src, int64_t *dst)
{
    if (scale < 1 || scale > 40 || m < 0 || !src || !dst)
        return -1;
    if (a < 0 || b < 0 || c < 0 || a + b + c > 1.0)
        return -1;
    const double two32 = 4294967296.0;
    const uint64_t ta = (uint64_t)(a * two32);
    const uint64_t tab = (uint64_t)((a + b) * two32);
    const uint64_t tabc = (uint64_t)((a + b + c) * two32);
#pragma omp parallel for schedule(static)
    for (int64_t t = 0; t < m; ++t) {
        uint64_t u = 0, v = 0;
        for (int l = 0; l < scale; ++l) {
            uint64_t d = (uint64_t)t * (uint64_t)scale + (uint64_t)l;
            uint64_t x = rmat_rng(seed, d >> 1);
            uint64_t r = (d & 1) ? (x >> 32) : (x & 0xffffffffULL);
            int q = r < ta ? 0 : r < tab ? 1 : r < tabc ? 2 : 3;
            u |= (uint64_t)(q >> 1) << (scale - 1 - l);
            v |= (uint64_t)(q & 1) << (scale - 1 - l);
        }
        if (perm) {
            u = (uint64_t)perm[u];
            v = (uint64_t)perm[v];
        }
        src[t] = (int64_t)u;
        dst[t] = (int64_t)v;
    }
    return 0;
}

/*
 * Erdos-Renyi style tuples: both endpoints of tuple t are independent uniform
 * draws in [0, n) (counters 2t and 2t+1). Self-loops and duplicates are kept.
 */
int er_edges(int64_t n, int64_t m, uint64_t seed, int64_t *src, int64_t *dst)
{
    if (n <= 0 || m < 0 || !src || !dst)
        return -1;
#pragma omp parallel for schedule(static)
    for (int64_t t = 0; t < m; ++t) {
        src[t] = (int64_t)bounded(rmat_rng(seed, 2 * (uint64_t)t), (uint64_t)n);
        dst[t] = (int64_t)bounded(rmat_rng(seed, 2 * (uint64_t)t + 1), (uint64_t)n);
    }
    return 0;
}

/*
 * Pick up to `count` distinct roots, uniform over vertices that have at least
 * one incident tuple which is not a self-loop. Candidate c is
 * bounded(rng(seed, c), n); candidates are tried in counter order. Returns the
 * number of roots written (fewer than count if the graph has too few
 * eligible vertices), or -1 on bad arguments.
 */
int64_t rmat_pick_roots(int64_t n, int64_t m, const int64_t *src, const int64_t *dst,
                        int64_t count, uint64_t seed, int64_t *roots)
{
    if (n <= 0 || m < 0 || count < 0 || !src || !dst || !roots)
        return -1;
    uint8_t *ok = (uint8_t *)calloc((size_t)n, 1);
    uint8_t *taken = (uint8_t *)calloc((size_t)n, 1);
    if (!ok || !taken) {
        free(ok);
        free(taken);
        return -1;
    }
    int64_t eligible = 0;
    for (int64_t t = 0; t < m; ++t) {
        int64_t u = src[t], v = dst[t];
        if (u == v || u < 0 || v < 0 || u >= n || v >= n)
            continue;
        ok[u] = 1;
        ok[v] = 1;
    }
    for (int64_t v = 0; v < n; ++v)
        eligible += ok[v];
    int64_t want = count < eligible ? count : eligible;
    int64_t got = 0;
    for (uint64_t ctr = 0; got < want; ++ctr) {
        int64_t v = (int64_t)bounded(rmat_rng(seed, ctr), (uint64_t)n);
        if (ok[v] && !taken[v]) {
            taken[v] = 1;
            roots[got++] = v;
        }
    }
    free(ok);
    free(taken);
    return got;
}
