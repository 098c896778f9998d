/*
 * Oracle for the compression + sieve breadth-first search of Lv, Tan, Chen and
 * Sun, "Compression and Sieve: Reducing Communication in Parallel Breadth
 * First Search on Distributed Memory Systems" (2012).
 *
 * TEST INFRASTRUCTURE, NOT PART OF THE PRODUCT. Only the test suite, the
 * smoke check and the benchmark's CPU-baseline leg may load this library.
 * It is plain, serial and slow on purpose, keeps one byte per bit in every
 * bit vector, and shares no code, header, table or helper with the GPU path.
 *
 * What each function follows:
 *   oracle_adj_build    the undirected adjacency of a tuple list; the paper
 *                       turns the generator's tuple list into CSR (Sec. VII.A)
 *   oracle_bfs          hop levels from the source by a FIFO queue; BFS finds
 *                       every vertex reachable from s (Sec. II)
 *   oracle_parents_max  the parent chosen by the (select, max) semiring: the
 *                       highest-labelled neighbour on the previous level
 *                       (Sec. III.A)
 *   oracle_validate     validity rules of a BFS parent tree
 *   oracle_directory    directory vectors V_{i,j} (Sec. V.A, Eq. dir-vec)
 *   oracle_wah_encode   word-aligned hybrid compression (Sec. IV, Table 3)
 *   oracle_wah_decode   its inverse
 *   oracle_alg3         the level loop of Algorithm 3 (Sec. V.B) over p
 *                       virtual processors: SpMV, mask, update, reduction,
 *                       sieve, compress, exchange, uncompress
 *   oracle_teps_m       TEPS numerator: input tuples inside the traversed
 *                       component, duplicates and self-loops included
 *                       (Sec. VII.A)
 *
 * Readings where the paper is silent (stated once here):
 *   - Processor P_i owns the contiguous vertex range R_i = [i*n/p, (i+1)*n/p).
 *   - A 64-bit WAH word keeps bit 63 as the literal/fill flag and, in a fill,
 *     bit 62 as the fill bit and bits 61..0 as the run length counted in
 *     groups; the toy format of Table 3 (fill_bit_field = 0) has no fill bit.
 *   - Literal payloads are most-significant-bit first: bit t of a group goes
 *     to bit (w-2-t) of the word, as Table 3 shows. The active word holds the
 *     last r bits right-aligned, in the same order (bit t to bit r-1-t), as
 *     the 128-bit, 32-bit-word example kept commented out in the source of
 *     Table 3 shows (its four trailing ones become 0000000F).
 *   - The frontier count is reduced right after the update; the sieve and the
 *     exchange run only when the new frontier is non-empty. The source is set
 *     in every processor's incoming frontier without a message.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------------ */
/* Undirected adjacency: tuple (u, v) puts v in the list of u and u in the   */
/* list of v; a self-loop (u, u) therefore appears twice in the list of u.   */
/* ------------------------------------------------------------------------ */

typedef struct oracle_adj {
    int64_t n;
    int64_t *off; /* n + 1 offsets */
    int32_t *nbr; /* off[n] neighbour ids */
} oracle_adj;

oracle_adj *oracle_adj_build(int64_t n, int64_t m, const int64_t *src, const int64_t *dst)
{
    if (n <= 0 || n >= ((int64_t)1 << 31) || m < 0 || (m > 0 && (!src || !dst)))
        return NULL;
    for (int64_t t = 0; t < m; ++t)
        if (src[t] < 0 || src[t] >= n || dst[t] < 0 || dst[t] >= n)
            return NULL;
    oracle_adj *a = (oracle_adj *)calloc(1, sizeof(oracle_adj));
    int64_t *cursor = (int64_t *)calloc((size_t)n + 1, sizeof(int64_t));
    if (!a || !cursor) {
        free(a);
        free(cursor);
        return NULL;
    }
    a->n = n;
    a->off = (int64_t *)calloc((size_t)n + 1, sizeof(int64_t));
    a->nbr = (int32_t *)malloc(sizeof(int32_t) * (size_t)(2 * m > 0 ? 2 * m : 1));
    if (!a->off || !a->nbr) {
        free(a->off);
        free(a->nbr);
        free(a);
        free(cursor);
        return NULL;
    }
    for (int64_t t = 0; t < m; ++t) {
        a->off[src[t] + 1] += 1;
        a->off[dst[t] + 1] += 1;
    }
    for (int64_t v = 0; v < n; ++v)
        a->off[v + 1] += a->off[v];
    for (int64_t v = 0; v < n; ++v)
        cursor[v] = a->off[v];
    for (int64_t t = 0; t < m; ++t) {
        a->nbr[cursor[src[t]]++] = (int32_t)dst[t];
        a->nbr[cursor[dst[t]]++] = (int32_t)src[t];
    }
    free(cursor);
    return a;
}

void oracle_adj_free(oracle_adj *a)
{
    if (!a)
        return;
    free(a->off);
    free(a->nbr);
    free(a);
}

int64_t oracle_adj_n(const oracle_adj *a) { return a ? a->n : -1; }

/* Number of adjacency entries of v (a self-loop counts twice). */
int64_t oracle_adj_degree(const oracle_adj *a, int64_t v)
{
    if (!a || v < 0 || v >= a->n)
        return -1;
    return a->off[v + 1] - a->off[v];
}

/* ------------------------------------------------------------------------ */
/* Serial FIFO-queue BFS: level[v] = hop distance from root, -1 if           */
/* unreachable. Returns the number of levels (max level + 1), or -1.         */
/* ------------------------------------------------------------------------ */

int64_t oracle_bfs(const oracle_adj *a, int64_t root, int32_t *level)
{
    if (!a || !level || root < 0 || root >= a->n)
        return -1;
    int32_t *queue = (int32_t *)malloc(sizeof(int32_t) * (size_t)a->n);
    if (!queue)
        return -1;
    for (int64_t v = 0; v < a->n; ++v)
        level[v] = -1;
    int64_t head = 0, tail = 0;
    level[root] = 0;
    queue[tail++] = (int32_t)root;
    int32_t maxlev = 0;
    while (head < tail) {
        int32_t u = queue[head++];
        for (int64_t e = a->off[u]; e < a->off[u + 1]; ++e) {
            int32_t v = a->nbr[e];
            if (level[v] < 0) {
                level[v] = level[u] + 1;
                if (level[v] > maxlev)
                    maxlev = level[v];
                queue[tail++] = v;
            }
        }
    }
    free(queue);
    return (int64_t)maxlev + 1;
}

/* ------------------------------------------------------------------------ */
/* (select, max) parent: parent[root] = root; for every other reached v the   */
/* largest neighbour u with level[u] = level[v] - 1; -1 if unreached.        */
/* ------------------------------------------------------------------------ */

int oracle_parents_max(const oracle_adj *a, const int32_t *level, int64_t root, int32_t *parent)
{
    if (!a || !level || !parent || root < 0 || root >= a->n)
        return -1;
    for (int64_t v = 0; v < a->n; ++v) {
        parent[v] = -1;
        if (v == root) {
            parent[v] = (int32_t)root;
            continue;
        }
        if (level[v] <= 0)
            continue;
        for (int64_t e = a->off[v]; e < a->off[v + 1]; ++e) {
            int32_t u = a->nbr[e];
            if (level[u] == level[v] - 1 && u > parent[v])
                parent[v] = u;
        }
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Validity of a BFS parent tree, checked against the tuple list itself.     */
/* Returns 0 if valid, else an OR of:                                        */
/*   1  the root is not its own parent or is not on level 0                  */
/*   2  a reached vertex lacks a parent, or an unreached one has one         */
/*   4  a tree edge {parent[v], v} is not among the tuples                   */
/*   8  a tree edge does not join consecutive levels                         */
/*  16  some tuple joins levels that differ by more than one                 */
/*  32  some tuple joins a reached and an unreached vertex                   */
/*  64  the reached set differs from ref_level's (when ref_level is given)   */
/* ------------------------------------------------------------------------ */

int oracle_validate(int64_t n, int64_t m, const int64_t *src, const int64_t *dst, int64_t root,
                    const int32_t *level, const int32_t *parent, const int32_t *ref_level)
{
    if (n <= 0 || m < 0 || !level || !parent || root < 0 || root >= n)
        return -1;
    int bad = 0;
    if (parent[root] != root || level[root] != 0)
        bad |= 1;
    for (int64_t v = 0; v < n; ++v) {
        if (v == root)
            continue;
        if (level[v] >= 0) {
            if (parent[v] < 0 || parent[v] >= n)
                bad |= 2;
            else if (level[parent[v]] != level[v] - 1)
                bad |= 8;
        } else if (parent[v] != -1) {
            bad |= 2;
        }
        if (ref_level && ((ref_level[v] >= 0) != (level[v] >= 0)))
            bad |= 64;
    }
    uint8_t *seen = (uint8_t *)calloc((size_t)n, 1);
    if (!seen)
        return -1;
    for (int64_t t = 0; t < m; ++t) {
        int64_t u = src[t], v = dst[t];
        if (u < 0 || u >= n || v < 0 || v >= n)
            continue;
        if (parent[v] == u)
            seen[v] = 1;
        if (parent[u] == v)
            seen[u] = 1;
        int32_t lu = level[u], lv = level[v];
        if ((lu >= 0) != (lv >= 0))
            bad |= 32;
        else if (lu >= 0 && (lu - lv > 1 || lv - lu > 1))
            bad |= 16;
    }
    for (int64_t v = 0; v < n; ++v)
        if (v != root && level[v] >= 0 && parent[v] >= 0 && parent[v] < n && !seen[v])
            bad |= 4;
    free(seen);
    return bad;
}

/* ------------------------------------------------------------------------ */
/* Directory vectors (Sec. V.A, Eq. dir-vec). The matrix is split into p     */
/* block-rows and each block-row into p sub-blocks; A_{i,j} has rows R_i and */
/* columns R_j, and A[v][u] = 1 for every tuple {u, v}. Entry k of V_{i,j} is */
/* one iff column k of A_{i,j} has a non-zero. Output: one byte per entry,   */
/* V[(i * p + j) * (n / p) + k].                                             */
/* ------------------------------------------------------------------------ */

int oracle_directory(int64_t n, int32_t p, int64_t m, const int64_t *src, const int64_t *dst,
                     uint8_t *V)
{
    if (n <= 0 || p <= 0 || n % p != 0 || m < 0 || !V)
        return -1;
    int64_t R = n / p;
    memset(V, 0, (size_t)(p * n));
    for (int64_t t = 0; t < m; ++t) {
        int64_t u = src[t], v = dst[t];
        if (u < 0 || u >= n || v < 0 || v >= n)
            return -1;
        /* A[v][u] = 1: row v in R_{v/R}, column u in R_{u/R}. */
        V[((v / R) * p + (u / R)) * R + (u % R)] = 1;
        /* A[u][v] = 1 (the matrix of an undirected graph is symmetric). */
        V[((u / R) * p + (v / R)) * R + (v % R)] = 1;
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* WAH codec (Sec. IV, Table 3). Words are w bits wide (4 <= w <= 64), held  */
/* in uint64. A group is w-1 consecutive bits. The most significant bit of a */
/* word tells a literal (0) from a fill (1). A literal holds one group, most */
/* significant bit first. A fill stands for a run of c identical all-0 or    */
/* all-1 groups and stores c (the number of groups, not bits); with          */
/* fill_bit_field the bit below the flag is the fill bit, without it only    */
/* 0-fills exist and all-1 groups are written as literals. The bits after    */
/* the last full group go to one right-aligned active word.                 */
/* ------------------------------------------------------------------------ */

static int group_class(const uint8_t *bits, int64_t start, int g)
{
    int ones = 0;
    for (int t = 0; t < g; ++t)
        ones += bits[start + t] ? 1 : 0;
    if (ones == 0)
        return 0; /* all zero */
    if (ones == g)
        return 1; /* all one */
    return 2;     /* mixed */
}

int64_t oracle_wah_encode(const uint8_t *bits, int64_t nbits, int32_t w, int32_t fill_bit_field,
                          uint64_t *out, int64_t cap)
{
    if (w < 4 || w > 64 || nbits < 0 || (nbits > 0 && !bits) || cap < 0 || (cap > 0 && !out))
        return -1;
    const int g = w - 1;
    const uint64_t flag = (uint64_t)1 << (w - 1);
    const int count_bits = fill_bit_field ? w - 2 : w - 1;
    const uint64_t max_count = (count_bits >= 64) ? ~(uint64_t)0 : (((uint64_t)1 << count_bits) - 1);
    const int64_t G = nbits / g;
    const int64_t r = nbits - G * g;
    int64_t nw = 0;
    int64_t x = 0;
    while (x < G) {
        int cls = group_class(bits, x * g, g);
        if (cls == 1 && !fill_bit_field)
            cls = 2; /* no 1-fills in the toy format */
        if (cls == 2) {
            uint64_t word = 0;
            for (int t = 0; t < g; ++t)
                if (bits[x * g + t])
                    word |= (uint64_t)1 << (g - 1 - t);
            if (nw >= cap)
                return -2;
            out[nw++] = word;
            x += 1;
        } else {
            int64_t c = 1;
            while (x + c < G && group_class(bits, (x + c) * g, g) == cls && (uint64_t)c < max_count)
                c += 1;
            uint64_t word = flag | (uint64_t)c;
            if (fill_bit_field && cls == 1)
                word |= (uint64_t)1 << (w - 2);
            if (nw >= cap)
                return -2;
            out[nw++] = word;
            x += c;
        }
    }
    if (r > 0) {
        uint64_t word = 0;
        for (int t = 0; t < r; ++t)
            if (bits[G * g + t])
                word |= (uint64_t)1 << (r - 1 - t);
        if (nw >= cap)
            return -2;
        out[nw++] = word;
    }
    return nw;
}

/* Decode nw words into nbits bytes (0/1). Returns 0, or -1 if the stream is  */
/* not a valid encoding of exactly nbits bits.                               */
int oracle_wah_decode(const uint64_t *words, int64_t nw, int64_t nbits, int32_t w,
                      int32_t fill_bit_field, uint8_t *bits)
{
    if (w < 4 || w > 64 || nbits < 0 || nw < 0 || (nw > 0 && !words) || (nbits > 0 && !bits))
        return -1;
    const int g = w - 1;
    const uint64_t flag = (uint64_t)1 << (w - 1);
    const int count_bits = fill_bit_field ? w - 2 : w - 1;
    const uint64_t count_mask = (count_bits >= 64) ? ~(uint64_t)0 : (((uint64_t)1 << count_bits) - 1);
    const uint64_t word_mask = (w == 64) ? ~(uint64_t)0 : (((uint64_t)1 << w) - 1);
    const int64_t G = nbits / g;
    const int64_t r = nbits - G * g;
    const int64_t regular = r > 0 ? nw - 1 : nw; /* words before the active word */
    if (regular < 0)
        return -1;
    int64_t pos = 0;
    for (int64_t k = 0; k < regular; ++k) {
        uint64_t word = words[k];
        if (word & ~word_mask)
            return -1;
        if (word & flag) {
            uint64_t c = word & count_mask;
            int fb = fill_bit_field ? (int)((word >> (w - 2)) & 1) : 0;
            if (c == 0 || (uint64_t)(G * g - pos) / (uint64_t)g < c)
                return -1;
            for (int64_t b = 0; b < (int64_t)c * g; ++b)
                bits[pos + b] = (uint8_t)fb;
            pos += (int64_t)c * g;
        } else {
            if (pos + g > G * g)
                return -1;
            for (int t = 0; t < g; ++t)
                bits[pos + t] = (uint8_t)((word >> (g - 1 - t)) & 1);
            pos += g;
        }
    }
    if (pos != G * g)
        return -1;
    if (r > 0) {
        uint64_t word = words[nw - 1];
        if (word & flag || word & ~word_mask)
            return -1;
        if (word >> r)
            return -1; /* bits above the r active bits must be zero */
        for (int t = 0; t < r; ++t)
            bits[pos + t] = (uint8_t)((word >> (r - 1 - t)) & 1);
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Algorithm 3 (Sec. V.B) over p virtual processors, one level at a time.    */
/*                                                                          */
/* Processor P_i owns R_i; it keeps its visited vector pi_i, its frontier    */
/* piece f_i and, for every j, the incoming piece f_{i,j} over R_j (its view */
/* of P_j's frontier). At level k:                                           */
/*   t_i = sum_j A_{i,j} (x) f_{i,j} over the (select, max) semiring, i.e.   */
/*         t_i[v] = max{u in R_j : A[v][u] = 1, f_{i,j}[u] = 1}              */
/*   t_i = t_i . not(pi_i);  pi_i = pi_i + t_i;  f_i = t_i                   */
/*   reduction of |f| = sum_i |f_i|; stop if zero                            */
/*   for every j: f_{i,j}' = Compress(f_i . V_{j,i})   (sieve, then WAH-64)  */
/*   Alltoallv: P_j receives g_{j,i}' = f_{i,j}'                             */
/*   for every i: P_j's incoming f_{j,i} = Uncompress(g_{j,i}')              */
/* The new vertices v of level k + 1 get level k + 1 and parent t_i[v].      */
/*                                                                          */
/* V is the byte directory of oracle_directory. Outputs: level and parent    */
/* (n entries); words[(k * p + i) * p + j] = 64-bit words of the stream from */
/* P_i to P_j carrying level k (zero for k = 0, which is never sent);        */
/* optional sieved_bits (same index) = ones in f_i . V_{j,i}; optional       */
/* unsieved_words[k * p + i] = words of WAH-64(f_i) without the sieve;       */
/* optional dump[((k * p + i) * p + j) * cap + w] = the streams themselves,  */
/* cap = floor((n/p)/63) + 1 words per stream. Returns the number of levels  */
/* (max level + 1), -1 on bad arguments, -2 if max_levels is too small, -3   */
/* if a stream fails to decode.                                              */
/* ------------------------------------------------------------------------ */

int64_t oracle_alg3_cap(int64_t n, int32_t p) { return (n / p) / 63 + 1; }

int64_t oracle_alg3(const oracle_adj *a, int32_t p, const uint8_t *V, int64_t root, int32_t max_levels,
                    int32_t *level, int32_t *parent, int64_t *words, int64_t *sieved_bits,
                    int64_t *unsieved_words, uint64_t *dump)
{
    if (!a || p <= 0 || a->n % p != 0 || !V || root < 0 || root >= a->n || max_levels < 1 || !level ||
        !parent || !words)
        return -1;
    const int64_t n = a->n;
    const int64_t R = n / p;
    const int64_t cap = oracle_alg3_cap(n, p);
    uint8_t *pi = (uint8_t *)calloc((size_t)n, 1);       /* pi_i over R_i, all i */
    uint8_t *f = (uint8_t *)calloc((size_t)n, 1);        /* f_i over R_i, all i */
    uint8_t *in = (uint8_t *)calloc((size_t)(p * n), 1); /* in[i * n + u] = f_{i,owner(u)}[u] */
    int32_t *t = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    uint8_t *piece = (uint8_t *)malloc((size_t)R);
    uint8_t *back = (uint8_t *)malloc((size_t)R);
    uint64_t *stream = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)cap);
    int64_t ret = 0;
    if (!pi || !f || !in || !t || !piece || !back || !stream) {
        ret = -1;
        goto done;
    }
    memset(words, 0, sizeof(int64_t) * (size_t)max_levels * p * p);
    if (sieved_bits)
        memset(sieved_bits, 0, sizeof(int64_t) * (size_t)max_levels * p * p);
    if (unsieved_words)
        memset(unsieved_words, 0, sizeof(int64_t) * (size_t)max_levels * p);
    if (dump)
        memset(dump, 0, sizeof(uint64_t) * (size_t)max_levels * p * p * cap);

    for (int64_t v = 0; v < n; ++v) {
        level[v] = -1;
        parent[v] = -1;
    }
    /* f(s) <- s: the source is known to every processor. */
    level[root] = 0;
    parent[root] = (int32_t)root;
    pi[root] = 1;
    for (int32_t i = 0; i < p; ++i)
        in[i * n + root] = 1;

    int32_t k = 0;
    for (;;) {
        /* t_i = sum_j A_{i,j} (x) f_{i,j}, evaluated column by column. */
        for (int64_t v = 0; v < n; ++v)
            t[v] = -1;
        for (int32_t i = 0; i < p; ++i) {
            for (int64_t u = 0; u < n; ++u) {
                if (!in[i * n + u])
                    continue;
                for (int64_t e = a->off[u]; e < a->off[u + 1]; ++e) {
                    int32_t v = a->nbr[e];
                    if (v / R != i)
                        continue; /* row v is not in block-row i */
                    if ((int32_t)u > t[v])
                        t[v] = (int32_t)u;
                }
            }
        }
        /* Mask with the visited vector, update it, and take the new frontier. */
        int64_t count = 0;
        for (int64_t v = 0; v < n; ++v) {
            if (pi[v])
                t[v] = -1;
            f[v] = 0;
            if (t[v] >= 0) {
                pi[v] = 1;
                f[v] = 1;
                level[v] = k + 1;
                parent[v] = t[v];
                count += 1;
            }
        }
        /* Reduction of the frontier size: stop on an empty frontier. */
        if (count == 0)
            break;
        k += 1;
        if (k >= max_levels) {
            ret = -2;
            goto done;
        }
        memset(in, 0, (size_t)(p * n));
        for (int32_t i = 0; i < p; ++i) {
            const uint8_t *fi = f + i * R;
            if (unsieved_words) {
                int64_t nw = oracle_wah_encode(fi, R, 64, 1, stream, cap);
                if (nw < 0) {
                    ret = -3;
                    goto done;
                }
                unsieved_words[(int64_t)k * p + i] = nw;
            }
            for (int32_t j = 0; j < p; ++j) {
                /* Sieve: f_{i,j} = f_i . V_{j,i}. */
                const uint8_t *vji = V + ((int64_t)j * p + i) * R;
                int64_t ones = 0;
                for (int64_t x = 0; x < R; ++x) {
                    piece[x] = (uint8_t)(fi[x] & vji[x]);
                    ones += piece[x];
                }
                int64_t nw = oracle_wah_encode(piece, R, 64, 1, stream, cap);
                if (nw < 0) {
                    ret = -3;
                    goto done;
                }
                int64_t idx = ((int64_t)k * p + i) * p + j;
                words[idx] = nw;
                if (sieved_bits)
                    sieved_bits[idx] = ones;
                if (dump)
                    memcpy(dump + idx * cap, stream, sizeof(uint64_t) * (size_t)nw);
                /* Exchange and uncompress on the receiving side P_j. */
                if (oracle_wah_decode(stream, nw, R, 64, 1, back) != 0) {
                    ret = -3;
                    goto done;
                }
                memcpy(in + (int64_t)j * n + (int64_t)i * R, back, (size_t)R);
            }
        }
    }
    ret = (int64_t)k + 1;
done:
    free(pi);
    free(f);
    free(in);
    free(t);
    free(piece);
    free(back);
    free(stream);
    return ret;
}

/* ------------------------------------------------------------------------ */
/* TEPS numerator (Sec. VII.A): tuples inside the traversed component,       */
/* multiple edges and self-loops included.                                   */
/* ------------------------------------------------------------------------ */

int64_t oracle_teps_m(int64_t m, const int64_t *src, const int64_t *dst, const int32_t *level)
{
    if (m < 0 || !level || (m > 0 && (!src || !dst)))
        return -1;
    int64_t c = 0;
    for (int64_t t = 0; t < m; ++t)
        if (level[src[t]] >= 0)
            c += 1;
    (void)dst;
    return c;
}
