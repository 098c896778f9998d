/*
 * csbfs -- compression + sieve breadth-first search on one MI355X (gfx950).
 *
 * C ABI of the library built from paper_1208_5542_amd/csrc/csbfs. It follows
 * Lv, Tan, Chen and Sun, "Compression and Sieve: Reducing Communication in
 * Parallel Breadth First Search on Distributed Memory Systems" (2012):
 * Algorithm 3 (Sec. V.B) over p virtual processors held as buffers on one
 * GPU. Processor P_i owns the contiguous vertex range
 * R_i = [i*n/p, (i+1)*n/p). Every level runs the expansion over the
 * sub-blocks A_{i,j} (Eq. sub-block; a top-down push, or a bottom-up pull
 * over the same entries, chosen per level), the mask and update of the visited
 * vector, the frontier-size reduction, the sieve of every outgoing message
 * with the cross directory (Eq. dir-vec, Eq. cross-dir), WAH compression
 * (Sec. IV, Table 3), and decompression into the receivers' frontier views.
 * Messages are never sent anywhere: their bytes are counted.
 *
 * Conventions shared by every entry point:
 *   - Every function returns an int status: CSBFS_OK (0) or a negative
 *     CSBFS_E* code. csbfs_last_error() gives a thread-local message for the
 *     most recent failure on the calling thread. No C++ exception crosses the
 *     ABI. On failure the contents of output buffers are unspecified, and
 *     nothing the caller owns is freed.
 *   - Pointers documented as "device" are HIP device (or managed) memory of
 *     the current device; "host" pointers are ordinary CPU memory.
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *     Device work is enqueued on it only; calls documented as blocking
 *     synchronize that stream (and nothing else) before returning.
 *   - Bit vectors are arrays of uint64 words: bit k of a vector is bit k % 64
 *     of word k / 64.
 *   - Vertex ids are int64 at the interface and must be < 2^31.
 *   - Memory. Every device buffer can be the caller's: csbfs_layout_query
 *     gives the exact sizes, csbfs_graph_build_into builds a graph in a
 *     caller buffer and csbfs_bfs_ws searches in a caller workspace; neither
 *     allocates device memory nor synchronizes anything but its own stream.
 *     The convenience calls csbfs_graph_build and csbfs_engine_create
 *     allocate those same buffers themselves (hipMalloc) and free them in
 *     csbfs_graph_free and csbfs_engine_free. The codec calls allocate nothing.
 *
 * The WAH-64 stream format (Sec. IV, Table 3 and the 32-bit example in the
 * source of that table). A stream encodes N bits b[0..N) as 63-bit groups;
 * G = floor(N/63) full groups, r = N - 63*G bits left over.
 *   literal word: bit 63 = 0; bit (62 - t) = b[63x + t], t = 0..62, for one
 *                 group x that is neither all 0 nor all 1;
 *   fill word:    bit 63 = 1; bit 62 = the fill bit; bits 61..0 = c >= 1, a
 *                 maximal run of c groups that are all equal to the fill bit
 *                 (a run of one group is a fill too);
 *   active word:  present iff r > 0, always the last word; bit (r - 1 - t) =
 *                 b[63G + t] for t < r, all other bits 0.
 * A stream of N bits never has more than floor(N/63) + 1 words.
 */
#ifndef CSBFS_H
#define CSBFS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define CSBFS_VERSION 10200 /* 1.2.0 */

#define CSBFS_OK 0
#define CSBFS_EINVAL (-1)    /* null pointer, bad size or bad flag */
#define CSBFS_ERANGE (-2)    /* root or tuple id outside [0, n); n, p not admissible */
#define CSBFS_ENOSPACE (-3)  /* caller buffer or workspace too small */
#define CSBFS_EHIP (-4)      /* HIP runtime error; see csbfs_last_error() */
#define CSBFS_EOVERFLOW (-5) /* a sub-block has 2^31 or more adjacency entries */
#define CSBFS_ECORRUPT (-6)  /* a WAH stream failed validation while decoding */

/* Library version as CSBFS_VERSION. */
int csbfs_version(void);

/* Static text for a status code (never NULL). */
const char *csbfs_strerror(int status);

/* Thread-local message describing the last failure on this thread ("" if none). */
const char *csbfs_last_error(void);

/* ======================================================================== */
/* Graph: the p x p sub-block grid of an undirected graph.                  */
/* ======================================================================== */

typedef struct csbfs_graph csbfs_graph;

/*
 * Partition and store an undirected graph (Sec. V.A, Eq. abc and Eq.
 * sub-block; the tuple list to CSR step of Sec. VII.A).
 *
 *   src, dst  device int64[n_tuples]: tuple t is the undirected edge
 *             {src[t], dst[t]}; duplicates and self-loops are kept (a
 *             self-loop is stored twice in its row).
 *   n         vertex count; 64 <= n < 2^31.
 *   p         virtual processor count; n % p == 0 and (n / p) % 64 == 0.
 *   out       host: receives the graph handle.
 *
 * Block (i, j) holds, for every source u in R_j, its neighbours in R_i as a
 * CSR row (int32 row offsets, uint32 local column ids). The directory vector
 * V_{i,j} (Eq. dir-vec) is the non-empty-row bitmap of block (i, j). The
 * input buffers are only read and may be freed after the call. Blocking.
 * Errors: EINVAL (null pointers, n_tuples < 0), ERANGE (n or p not
 * admissible, a tuple id outside [0, n)), EOVERFLOW, ECORRUPT (the built
 * CSR failed its consistency check: a column id outside its block or an
 * adjacency total other than 2 * n_tuples), EHIP.
 */
int csbfs_graph_build(const int64_t *src, const int64_t *dst, int64_t n_tuples, int64_t n,
                      int32_t p, void *stream, csbfs_graph **out);

/*
 * The same partition built in caller-owned device memory (Sec. V.A; the
 * problem statement of Sec. II: the caller holds the graph and the search's
 * state, the library computes). graph_mem (graph_bytes) receives the graph
 * and must stay valid and unmodified while the handle is used; scratch
 * (scratch_bytes) holds the build's temporaries and is free again when the
 * call returns. Sizes come from csbfs_layout_query (same n, n_tuples, p);
 * both buffers must start at a multiple of 256 bytes. The handle itself is
 * small host memory; csbfs_graph_free releases it and never frees the
 * caller's buffer. No device allocation; synchronizes `stream` only
 * (blocking). Errors: as csbfs_graph_build, plus EINVAL (null or misaligned
 * buffer) and ENOSPACE (a buffer smaller than the query gives).
 */
int csbfs_graph_build_into(const int64_t *src, const int64_t *dst, int64_t n_tuples, int64_t n, int32_t p,
                           void *graph_mem, size_t graph_bytes, void *scratch, size_t scratch_bytes,
                           void *stream, csbfs_graph **out);

/* Release a graph handle. A graph built by csbfs_graph_build also frees its
 * device memory (hipFree, which waits for work still using it); one built by
 * csbfs_graph_build_into leaves the caller's buffer alone and makes no HIP
 * call. NULL is accepted. */
int csbfs_graph_free(csbfs_graph *g);

typedef struct csbfs_graph_info {
    int64_t n;              /* vertices */
    int32_t p;              /* virtual processors; p * p sub-blocks */
    int32_t reserved;
    int64_t range;          /* |R_i| = n / p */
    int64_t n_tuples;       /* input tuples */
    int64_t nnz;            /* adjacency entries over all blocks = 2 * n_tuples */
    int64_t max_block_nnz;  /* largest sub-block */
    int64_t device_bytes;   /* device memory held by the graph */
} csbfs_graph_info;

/* Sizes of a built graph (host call, no device work). */
int csbfs_graph_get_info(const csbfs_graph *g, csbfs_graph_info *info);

/*
 * Copy the directory out: dst device uint64[p * p * (n / p) / 64]; the words
 * of V_{i,j} start at (i * p + j) * (n / p) / 64 (Eq. dir-vec). cap_words is
 * the capacity of dst. Errors: EINVAL, ENOSPACE, EHIP. Asynchronous.
 */
int csbfs_graph_copy_directory(const csbfs_graph *g, uint64_t *dst, int64_t cap_words,
                               void *stream);

/*
 * Copy sub-block (i, j) out: row_ptr device int32[n/p + 1] (row_ptr[0] = 0),
 * col device uint32[cap] (local ids in R_i; order within a row unspecified),
 * nnz_out host int64. Blocking. Errors: EINVAL, ERANGE (i or j outside
 * [0, p)), ENOSPACE (cap < block size; nnz_out still set), EHIP.
 */
int csbfs_graph_copy_block(const csbfs_graph *g, int32_t i, int32_t j, int32_t *row_ptr,
                           uint32_t *col, int64_t cap, int64_t *nnz_out, void *stream);

/*
 * TEPS numerator (Sec. VII.A): the number of input tuples inside the
 * component reached by a search whose level vector is `level` (device
 * int32[n], -1 = unreached), duplicates and self-loops included. Blocking.
 * Errors: EINVAL, EHIP.
 */
int csbfs_count_traversed_tuples(const csbfs_graph *g, const int32_t *level, int64_t *m_out,
                                 void *stream);

/* ======================================================================== */
/* Engine: per-graph workspace for repeated single-source searches.          */
/* ======================================================================== */

typedef struct csbfs_engine csbfs_engine;

/* Engine flags. */
#define CSBFS_FLAG_TIMING 1u       /* record per-kernel times into the level stats */
#define CSBFS_FLAG_KEEP_STREAMS 2u /* keep every level's WAH streams for copy-out */
#define CSBFS_FLAG_NO_SIEVE 4u     /* all-ones directory: Alg. 2 messages (no sieve) */
/* The (select, max) product t_i = sum_j A_{i,j} (x) f_{i,j} of a level has
 * three exact evaluations, all giving identical level[] and parent[]:
 *   top-down ("sparse"): every frontier source in the views pushes itself
 *       into parent[] of its unvisited neighbours with atomicMax;
 *   bottom-up: every unvisited vertex scans its rows, sorted by decreasing
 *       id, and stops at the first neighbour set in its views (the highest
 *       one); the direction-optimizing search of Beamer et al., which the
 *       paper names as future work (Sec. VIII);
 *   dense: the push only marks targets seen, then each new vertex pulls its
 *       parent as in bottom-up.
 * By default each level is top-down or bottom-up, chosen on the device from
 * the frontier (see csbfs_engine_set_direction). These flags force one
 * evaluation for every level. */
#define CSBFS_FLAG_SPARSE_ONLY 8u
#define CSBFS_FLAG_DENSE_ONLY 16u
#define CSBFS_FLAG_BOTTOM_UP_ONLY 32u
/* How a top-down level applies its (target, source) pairs. The atomic push
 * relaxes each pair in place: an atomicMax into parent[] and an atomicOr
 * into the new-vertex bitmap, random accesses that go to the memory side.
 * The binned push (propagation blocking, Beamer, Asanovic and Patterson,
 * IPDPS 2017) relaxes the short rows so but writes the pairs of the long
 * rows (over 128 entries in a block), sorted in on-chip memory, into one
 * bin per 2^15 target vertices, then resolves each bin in on-chip memory:
 * from the parents the atomic part left, the highest source per target,
 * and the new vertices' parents and bitmap words, each written once. Both
 * give identical results. By default a top-down level is binned when its
 * frontier has at least 2^23 adjacency entries, at least 64 per frontier
 * vertex, and at most half the bins' capacity; the workspace has bins only
 * for graphs of at most 2^26 vertices whose half capacity is at least 2^24
 * pairs (by default an nnz of about 2^28 or more). Pairs past a segment's
 * capacity go to the atomic push. BINNED_PUSH bins every top-down level that
 * fits the bins (and always gives a workspace bins); ATOMIC_PUSH never bins
 * and the workspace holds no bins. */
#define CSBFS_FLAG_BINNED_PUSH 64u
#define CSBFS_FLAG_ATOMIC_PUSH 128u

/*
 * Parameters of one search on a caller workspace (csbfs_bfs_ws); a zeroed
 * struct (or NULL) gives the defaults.
 *   flags           CSBFS_FLAG_KEEP_STREAMS, NO_SIEVE, at most one of
 *                   SPARSE_ONLY, DENSE_ONLY, BOTTOM_UP_ONLY and at most one
 *                   of BINNED_PUSH, ATOMIC_PUSH (TIMING is an engine
 *                   feature and is rejected here).
 *   max_levels      levels whose counters (and, with KEEP_STREAMS, streams)
 *                   are kept, 1..65536; 0 means 64. Deeper searches still run
 *                   to the end; their extra levels are not reported.
 *   alpha, beta     the direction rule of csbfs_engine_set_direction; both 0
 *                   mean alpha = 16, beta = 48; alpha < 0 keeps every level
 *                   top-down; beta >= 0.
 *   segment_groups  groups of 63 bits per encoder segment: 1024 or 2048, or
 *                   0 to choose from the sizes (same streams either way).
 *   push_bin_pairs  capacity of the binned push in (target, source) pairs
 *                   (8 bytes each, split evenly over the bins and over 256
 *                   segments per bin), >= 0; 0 means nnz / 8 + 65536 (nnz:
 *                   adjacency entries). A level is binned only if its
 *                   frontier's entries fit. Ignored with ATOMIC_PUSH.
 */
typedef struct csbfs_search_config {
    uint32_t flags;
    int32_t max_levels;
    float alpha;
    float beta;
    int32_t segment_groups;
    int32_t push_bin_pairs;
} csbfs_search_config;

/* Byte sizes of the caller-owned device buffers. */
typedef struct csbfs_sizes {
    int64_t graph_bytes;          /* a built graph (csbfs_graph_build_into graph_mem) */
    int64_t build_scratch_bytes;  /* temporaries of csbfs_graph_build_into */
    int64_t workspace_bytes;      /* one search (csbfs_bfs_ws workspace) */
    int64_t alignment;            /* every buffer starts at a multiple of this (256) */
} csbfs_sizes;

/*
 * Exact sizes of the buffers for a graph of n vertices and n_tuples tuples
 * on p processors, and of a search workspace for config cfg (NULL =
 * defaults). Host arithmetic only: no device is touched. The sizes depend on
 * (n, n_tuples, p, cfg) alone, never on the tuples themselves. Errors: EINVAL
 * (out NULL, bad config, n_tuples < 0), ERANGE (n or p not admissible, as in
 * csbfs_graph_build).
 */
int csbfs_layout_query(int64_t n, int64_t n_tuples, int32_t p, const csbfs_search_config *cfg,
                       csbfs_sizes *out);

/* Level directions reported in csbfs_level_stats.direction. */
#define CSBFS_DIR_TOP_DOWN 0
#define CSBFS_DIR_BOTTOM_UP 1
#define CSBFS_DIR_DENSE 2

/*
 * Allocate (hipMalloc) a search workspace of Algorithm 3 for graph g, the
 * one csbfs_bfs_ws takes for a config of these flags and max_levels:
 * visited vector pi, the bitmaps of the vertices discovered by the last two
 * expansions (t_i, which becomes f_i; one per level parity), a mark per
 * 4096 vertices per level parity telling which parts of them may be
 * non-zero, the p frontier views (p * n bits), the WAH stream arena (p * p
 * streams of floor((n/p)/63) + 1 words, times max_levels with
 * CSBFS_FLAG_KEEP_STREAMS), the expansion work queue, the binned push's
 * bins (only where a level can be binned, see CSBFS_FLAG_BINNED_PUSH) and
 * the per-level counters for up to max_levels levels (1 <= max_levels <=
 * 65536); plus a pinned two-word mailbox and, with CSBFS_FLAG_TIMING, five
 * events per level. The graph must outlive the engine. The encoder's segment size is
 * chosen from n/p and p. Errors: EINVAL, EHIP.
 */
int csbfs_engine_create(const csbfs_graph *g, int32_t max_levels, uint32_t flags,
                        csbfs_engine **out);

/*
 * Parameters of the per-level direction choice (Beamer, Asanovic and
 * Patterson's rule). After the update that produced f^{k+1}, with m_f the
 * adjacency entries of f^{k+1} and m_u those of the still unvisited
 * vertices: a top-down search turns bottom-up when m_f * alpha > m_u and
 * the frontier did not shrink; a
 * bottom-up search turns top-down again when |f^{k+1}| * beta < n and the
 * frontier shrank. Level 0 is top-down. alpha <= 0 keeps every level
 * top-down. Defaults: alpha = 16, beta = 48. Takes effect at the next
 * csbfs_bfs. Errors: EINVAL (NULL engine, beta <= 0 or a NaN).
 */
int csbfs_engine_set_direction(csbfs_engine *e, float alpha, float beta);

/* Release an engine (hipFree waits for work still using it). NULL is accepted. */
int csbfs_engine_free(csbfs_engine *e);

/* Counters of one BFS level k: the frontier f^k, its expansion, and the
 * messages carrying it (which exist for k >= 1; level 0 is seeded). */
typedef struct csbfs_level_stats {
    int64_t frontier;           /* |f^k|; 1 at level 0 */
    int64_t edges;              /* adjacency entries read when expanding f^k (top-down:
                                   the rows of its sources; bottom-up: the entries the
                                   unvisited vertices read before their first hit) */
    int64_t view_bits;          /* ones over all p x p views the expansion of f^k reads:
                                   sum over all i, j of ones(f_i^k . V_{j,i}); p at level 0 */
    int64_t sieved_bits;        /* sum over i != j of ones(f_i^k . V_{j,i}) */
    int64_t unsieved_bits;      /* (p - 1) * |f^k|: ones the Allgatherv of Alg. 1 carries */
    int64_t raw_bytes;          /* p (p - 1) 8 ceil(|R|/64): Alg. 1 bitmap bytes */
    int64_t wah_unsieved_bytes; /* sum over i != j of 8 |WAH(f_i^k)|: Alg. 2 bytes */
    int64_t wah_sieved_bytes;   /* sum over i != j of 8 |WAH(f_i^k . V_{j,i})|: Alg. 3 bytes */
    int64_t self_bytes;         /* sum over i of 8 |WAH(f_i^k . V_{i,i})| (never sent) */
    int64_t max_rank_bytes;     /* max over i of Alg. 3 bytes sent plus received by P_i */
    int64_t pulled;             /* bottom-up: unvisited vertices that scanned their rows */
    float ms_expand;            /* expansion of f^k: csbfs_bfs, its main kernel (the push or the
                                   pull); batched, every expansion kernel (TIMING) */
    float ms_update;            /* batched: mask, visit update and reduction; csbfs_bfs: 0,
                                   its update runs inside the encode (TIMING) */
    float ms_compress;          /* sieve + WAH encode of the f^k messages; csbfs_bfs: with
                                   the update that forms f^k (TIMING) */
    float ms_decode;            /* decode/merge of the f^k messages (TIMING) */
    int32_t direction;          /* CSBFS_DIR_* used to expand f^k */
    float ms_long_rows;         /* csbfs_bfs: the top-down long-row (chunk queue) kernel of the
                                   expansion of f^k (with the binned push: the pairs written
                                   into the bins and the bins resolved), and the parent pull
                                   of the dense evaluation; 0 for batched searches (TIMING) */
    int32_t push;               /* csbfs_bfs, top-down levels: CSBFS_PUSH_BINNED if the
                                   expansion of f^k used the binned push, else
                                   CSBFS_PUSH_ATOMIC (and for every other level) */
    int32_t reserved;           /* 0 */
} csbfs_level_stats;

#define CSBFS_PUSH_ATOMIC 0
#define CSBFS_PUSH_BINNED 1

/*
 * One breadth-first search from `root` (Algorithm 3; the problem statement of
 * Sec. II and Algorithm 1: discover every vertex reachable from s).
 *
 *   level   device int32[n]: hop distance from root, -1 if unreachable.
 *   parent  device int32[n]: parent[root] = root; for every other reached v,
 *           the highest-labelled neighbour on level[v] - 1 (the (select, max)
 *           semiring of Sec. III.A); -1 if unreachable.
 *   stats   host csbfs_level_stats[stats_cap] or NULL: stats[k] for levels
 *           k < min(n_levels, stats_cap, max_levels of the engine).
 *   n_levels host: number of levels (max level + 1), whatever stats_cap is.
 *
 * Blocking: the level loop reads each level's frontier size back (the
 * "reducing" step of Sec. VII.B), one level behind the GPU. Concurrent calls on one engine race;
 * distinct engines may run concurrently on distinct streams. Errors: EINVAL,
 * ERANGE (root outside [0, n)), ECORRUPT, EHIP.
 */
int csbfs_bfs(csbfs_engine *e, int64_t root, int32_t *level, int32_t *parent,
              csbfs_level_stats *stats, int32_t stats_cap, int32_t *n_levels, void *stream);

/*
 * One breadth-first search in a caller-owned workspace: the same search,
 * results and statistics as csbfs_bfs (Algorithm 3; the problem statement
 * of Sec. II), with every device buffer supplied by the caller.
 *   g            a built graph (either build call).
 *   cfg          search parameters (NULL = defaults); the same cfg must be
 *                given to csbfs_layout_query and to the stream copy-outs.
 *   level, parent, stats, stats_cap, n_levels: as csbfs_bfs.
 *   workspace    device buffer of ws_bytes >= workspace_bytes of
 *                csbfs_layout_query (256-byte aligned, any contents: the
 *                search clears what it needs). It holds the search's state
 *                and, afterwards, its streams and counters until the next
 *                search on it. One search at a time per workspace; searches
 *                on distinct workspaces may run concurrently on distinct
 *                streams.
 *   host_mailbox pinned host memory of two uint64 words (hipHostMalloc, or a
 *                torch tensor with pin_memory=True) through which the GPU
 *                posts each level's frontier size, or NULL: the host then
 *                copies each level's count back after the stream drains,
 *                which costs a round trip per level. One search at a time
 *                per mailbox.
 * No device allocation; synchronizes `stream` only. Blocking (the level
 * loop reads each level's frontier size one level behind the GPU). Errors:
 * EINVAL (null or misaligned argument, bad cfg, a mailbox that is not pinned
 * host memory), ENOSPACE (workspace too small), ERANGE (root outside
 * [0, n)), ECORRUPT, EHIP.
 */
int csbfs_bfs_ws(const csbfs_graph *g, int64_t root, const csbfs_search_config *cfg, int32_t *level,
                 int32_t *parent, csbfs_level_stats *stats, int32_t stats_cap, int32_t *n_levels,
                 void *workspace, size_t ws_bytes, uint64_t *host_mailbox, void *stream);

/* Word counts of the streams of the last csbfs_bfs_ws search on workspace,
 * which had n_levels levels; layout as csbfs_engine_stream_words. Blocking
 * on `stream`. Errors: EINVAL, ENOSPACE (workspace too small for cfg). */
int csbfs_ws_stream_words(const csbfs_graph *g, const csbfs_search_config *cfg, const void *workspace,
                          size_t ws_bytes, int32_t n_levels, int32_t *words, int32_t cap_levels, void *stream);

/* Copy the stream from P_i to P_j carrying level k of the last csbfs_bfs_ws
 * search on workspace (cfg with CSBFS_FLAG_KEEP_STREAMS); as
 * csbfs_engine_copy_stream. */
int csbfs_ws_copy_stream(const csbfs_graph *g, const csbfs_search_config *cfg, const void *workspace,
                         size_t ws_bytes, int32_t n_levels, int32_t k, int32_t i, int32_t j, uint64_t *dst,
                         int64_t cap_words, int64_t *n_words_out, void *stream);

/*
 * Word counts of the last search's streams: words host int32[cap_levels * p
 * * p]; words[(k * p + i) * p + j] = words of the stream from P_i to P_j
 * carrying level k (0 for k = 0, which is seeded and never sent). Levels
 * beyond the engine's max_levels read 0. Blocking. Errors: EINVAL.
 */
int csbfs_engine_stream_words(const csbfs_engine *e, int32_t *words, int32_t cap_levels);

/*
 * Copy the stream from P_i to P_j that carried level k in the last search
 * (needs CSBFS_FLAG_KEEP_STREAMS): dst device uint64[cap_words]; n_words_out
 * host. Blocking. Errors: EINVAL (flag missing, k/i/j out of range),
 * ENOSPACE, EHIP.
 */
int csbfs_engine_copy_stream(const csbfs_engine *e, int32_t k, int32_t i, int32_t j,
                             uint64_t *dst, int64_t cap_words, int64_t *n_words_out,
                             void *stream);

/* ======================================================================== */
/* Batched searches: up to 64 roots at once (multi-source BFS).             */
/* ======================================================================== */

/*
 * A batched search runs Algorithm 3 for up to 64 roots together. Every
 * vertex carries a 64-bit visit mask (bit r: reached by root r's search).
 * A top-down level pushes a source's mask of frontier roots along each edge
 * once; a bottom-up level lets every vertex still missing some roots OR its
 * neighbours' frontier masks until all of them are found (the direction-
 * optimizing search the paper names as future work, Sec. VIII, over the
 * union of the roots' frontiers), chosen per level on the device. Each root
 * keeps its own frontier bitmap (one bit-plane per root), so every root's
 * messages are exactly those of its single-root search: p x p streams per
 * root and level, sieved by the same directory and WAH-64 compressed, all
 * in one launch per step. Levels only (no parents).
 */
typedef struct csbfs_batch_engine csbfs_batch_engine;

/* Workspace for batches of up to max_roots (1..64) roots and max_levels
 * levels of counters (1..65536). Flags: CSBFS_FLAG_TIMING,
 * CSBFS_FLAG_KEEP_STREAMS, CSBFS_FLAG_NO_SIEVE, and CSBFS_FLAG_SPARSE_ONLY
 * or CSBFS_FLAG_BOTTOM_UP_ONLY to force one evaluation at every level (the
 * results are identical). The graph must outlive the engine. Blocking.
 * Errors: EINVAL, EHIP. */
int csbfs_batch_engine_create(const csbfs_graph *g, int32_t max_roots, int32_t max_levels,
                              uint32_t flags, csbfs_batch_engine **out);

/* Release a batch engine (hipFree waits for work still using it). NULL is accepted. */
int csbfs_batch_engine_free(csbfs_batch_engine *e);

/*
 * One batched search.
 *   roots   host int64[n_roots], 1 <= n_roots <= max_roots, each in [0, n)
 *           (repeats allowed).
 *   level   device int32[n_roots * n]: level[r * n + v] = hop distance of v
 *           from roots[r], -1 if unreachable.
 *   stats   host csbfs_level_stats[stats_cap] or NULL: per level, summed
 *           over the roots whose frontier at that level is not empty
 *           (frontier, bits and bytes as for csbfs_bfs; edges counts the
 *           adjacency entries the batch read once for all its roots: the
 *           rows of the union frontier top-down, the entries read before
 *           every missing root was found bottom-up; direction as used).
 *   n_levels host: max over roots of (max level + 1).
 * Blocking. Errors: EINVAL, ERANGE (a root outside [0, n)), ECORRUPT, EHIP.
 */
int csbfs_batch_bfs(csbfs_batch_engine *e, const int64_t *roots, int32_t n_roots, int32_t *level,
                    csbfs_level_stats *stats, int32_t stats_cap, int32_t *n_levels, void *stream);

/* Word counts of the last batch's streams: words host int32[cap_levels *
 * n_roots * p * p], words[((k * n_roots + r) * p + i) * p + j] = words of
 * root r's stream from P_i to P_j carrying level k (0 when root r's level-k
 * frontier is empty, and for k = 0). Blocking. Errors: EINVAL. */
int csbfs_batch_stream_words(const csbfs_batch_engine *e, int32_t *words, int32_t cap_levels);

/* Copy root r's stream from P_i to P_j carrying level k of the last batch
 * (needs CSBFS_FLAG_KEEP_STREAMS). As csbfs_engine_copy_stream. */
int csbfs_batch_copy_stream(const csbfs_batch_engine *e, int32_t k, int32_t r, int32_t i,
                            int32_t j, uint64_t *dst, int64_t cap_words, int64_t *n_words_out,
                            void *stream);

/* Device bytes csbfs_batch_engine_create would allocate for these
 * arguments (host only, allocates nothing). Returns -1 on bad arguments. */
int64_t csbfs_batch_engine_bytes(const csbfs_graph *g, int32_t max_roots, int32_t max_levels,
                                 uint32_t flags);

/* ======================================================================== */
/* Serving: a request loop over resident graphs.                             */
/* ======================================================================== */

/*
 * A server answers breadth-first queries (graph, root) -> level[] over graphs
 * registered with it (built once and resident in HBM). Requests wait in one
 * queue per graph; each of `slots` worker threads owns a HIP stream and,
 * whenever it is free, serves the graph whose oldest request has the
 * highest response ratio ((waiting time + expected service time) / expected
 * service time, from the graph's measured search times: short searches go
 * first and long waits are not starved). It takes up to max_batch of that
 * graph's waiting requests and answers them either one by one with the
 * direction-optimizing single-root search or together with one batched
 * search (csbfs_batch_bfs), whichever the graph's measured costs say is
 * cheaper for that many roots. Requests that arrive while others run are
 * admitted as soon as a slot frees up, and the slots' searches overlap on
 * the device. Per (slot, graph) one device block (batched engine, result
 * buffer, single-root workspace) is admitted under an HBM budget; blocks
 * come from the stream-ordered allocator and idle ones are released, least
 * recently used first, to make room, without synchronizing the device.
 * Every result equals that of a search from the same root alone (levels
 * are exact; no parents are returned).
 */
typedef struct csbfs_server csbfs_server;

typedef struct csbfs_server_config {
    int32_t slots;       /* worker threads / HIP streams, 1..16 */
    int32_t max_batch;   /* roots per batched search, 1..64 */
    int32_t max_levels;  /* level counters of each engine, 1..65536 */
    int32_t reserved;    /* 0 */
    int64_t hbm_budget;  /* bytes of engines + result buffers the server may hold */
} csbfs_server_config;

/* Outcome of one request; times in seconds on one steady host clock. */
typedef struct csbfs_request_info {
    int64_t id;
    int64_t root;
    int32_t graph_id;
    int32_t status;      /* CSBFS_OK or a negative status of the batch it ran in */
    int32_t n_levels;    /* max level + 1 of this root's search */
    int32_t batch_size;  /* requests taken together by one worker (one batched search, or
                            single-root searches one after the other) */
    int32_t slot;
    int32_t batched;     /* 1: answered by a batched search; 0: by a single-root search */
    double t_submit;
    double t_start;      /* its batch started */
    double t_done;       /* its levels were in place */
} csbfs_request_info;

/* Start the workers. Errors: EINVAL (bad config), EHIP. */
int csbfs_server_create(const csbfs_server_config *cfg, csbfs_server **out);

/* Register a graph (must outlive the server); *graph_id = 0, 1, ... in the
 * order of registration. Errors: EINVAL, ENOSPACE (one engine plus one
 * result buffer of this graph exceed the budget). */
int csbfs_server_add_graph(csbfs_server *s, const csbfs_graph *g, int32_t *graph_id);

/*
 * Queue a query. level_out: device int32[n of the graph] that receives the
 * levels (-1 unreachable), or NULL for no copy-out; the caller keeps it valid
 * until the request is done. Ordering: the server writes level_out only
 * after all work the caller enqueued on `stream` (NULL: the null stream)
 * before this call (an event recorded on `stream` here, awaited by the
 * worker's stream), and the write is complete when csbfs_server_wait
 * returns for this request. Non-blocking; thread-safe. Errors: EINVAL
 * (stopped server, unknown graph), ERANGE (root outside [0, n)), EHIP.
 */
int csbfs_server_submit(csbfs_server *s, int32_t graph_id, int64_t root, int32_t *level_out, void *stream,
                        int64_t *request_id);

/* Block until the request is done and return its outcome (once per id).
 * Errors: EINVAL (unknown or already collected id). */
int csbfs_server_wait(csbfs_server *s, int64_t request_id, csbfs_request_info *info);

/* Block until no request is waiting or running. */
int csbfs_server_drain(csbfs_server *s);

/* Device bytes of one (slot, graph) block of a registered graph (batched
 * engine, result buffer, single-root workspace, parent scratch), or -1. */
int64_t csbfs_server_graph_bytes(const csbfs_server *s, int32_t graph_id);

/* Device bytes currently held by the server's blocks. */
int64_t csbfs_server_bytes_held(const csbfs_server *s);

/* Drain, stop the workers and release everything. NULL is accepted. */
int csbfs_server_free(csbfs_server *s);

/* ======================================================================== */
/* WAH-64 codec on device buffers (Sec. IV).                                */
/* ======================================================================== */

/* Largest stream for nbits bits: floor(nbits/63) + 1 words. */
int64_t csbfs_wah_capacity(int64_t nbits);

/* Device scratch bytes the two codec calls need for nbits bits. */
size_t csbfs_wah_workspace_bytes(int64_t nbits);

/*
 * Sieve and compress: encode (bits AND mask) over nbits bits (mask NULL means
 * no sieve) as one WAH-64 stream (Alg. 3, sieve then Compress).
 *   bits, mask  device uint64[ceil(nbits/64)]; bits at or past nbits are ignored.
 *   out         device uint64[cap_words], cap_words >= csbfs_wah_capacity(nbits).
 *   n_words     device int64[1]: receives the stream length in words.
 *   workspace   device scratch of ws_bytes >= csbfs_wah_workspace_bytes(nbits);
 *               any contents (the call clears what it needs); one call at a
 *               time per workspace.
 * nbits is at most 63 * (2^29 - 1) (EINVAL above).
 * Asynchronous. Errors: EINVAL, ENOSPACE, EHIP.
 */
int csbfs_wah_encode(const uint64_t *bits, const uint64_t *mask, int64_t nbits, uint64_t *out,
                     int64_t cap_words, int64_t *n_words, void *workspace, size_t ws_bytes,
                     void *stream);

/*
 * Sieve and compress with no workspace argument and no allocation of any
 * kind, for callers that cannot allocate: code under HIP graph capture,
 * tight serving loops, harnesses that forbid hipMalloc. Same arguments,
 * stream and errors as csbfs_wah_encode without the workspace. The
 * encoder's look-back words and tickets live in a fixed 256 KiB device array
 * inside the library (one per GPU, held until the process ends), which
 * bounds nbits by csbfs_wah_noalloc_max_bits() (above 4 * 10^9 bits): a
 * larger nbits fails with EINVAL. The array is cleared by a kernel at every
 * call (no memset node). Every call on one GPU shares that array: calls
 * that overlap in time on one GPU (concurrent streams or threads) race and
 * must be serialized by the caller. Asynchronous.
 */
int csbfs_wah_encode_noalloc(const uint64_t *bits, const uint64_t *mask, int64_t nbits, uint64_t *out,
                             int64_t cap_words, int64_t *n_words, void *stream);

/* Largest nbits csbfs_wah_encode_noalloc accepts (host arithmetic only). */
int64_t csbfs_wah_noalloc_max_bits(void);

/*
 * Uncompress: OR the nbits bits of a WAH-64 stream of n_words words into dst
 * (device uint64[ceil(nbits/64)]; zero it first for a plain decode).
 *   status  device int32[1]: set to 0 if the stream is a valid encoding of
 *           exactly nbits bits, non-zero otherwise (dst then unspecified).
 * Asynchronous. Errors: EINVAL, ENOSPACE, EHIP.
 */
int csbfs_wah_decode_or(const uint64_t *words, int64_t n_words, int64_t nbits, uint64_t *dst,
                        int32_t *status, void *workspace, size_t ws_bytes, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* CSBFS_H */
