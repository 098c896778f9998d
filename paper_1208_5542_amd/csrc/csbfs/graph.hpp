// Internal layout of a partitioned graph (not installed).
#pragma once

#include <memory>
#include <vector>

#include "common.hpp"

namespace csbfs {

// Rows longer than kBigRow adjacency entries are expanded through the chunk
// queue, kBigChunk entries per queue item, instead of inside their frontier
// word's wavefront.
constexpr int kBigRow = 128;
constexpr int kBigChunk = 512;

// Alignment of every array carved out of a caller's buffer.
constexpr int64_t kAlign = 256;
inline int64_t align_up(int64_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

// Upper bound on the chunk-queue items of all rows expanded at once, from
// the adjacency total alone: a row of d > kBigRow entries needs
// ceil(d / kBigChunk) < d / kBigChunk + 1 items, and there are fewer than
// nnz / kBigRow such rows.
inline int64_t big_items_bound(int64_t nnz) { return nnz / kBigChunk + nnz / kBigRow + 2; }

// Byte offsets of the arrays of a graph inside its device buffer, and of the
// build's temporaries inside the build scratch; both depend on (n, p,
// n_tuples) only.
struct GraphLayout {
    int64_t n, P, R, W, B, nnz, ntile;
    // graph buffer
    int64_t row_ptr, col_base, col, dir, deg, pull_off, pull_col, head, live, qoff, small, graph_bytes;
    // build scratch
    int64_t cnt, sums, nnzb, misc, queues, scan, scratch_bytes;
};
int graph_layout(int64_t n, int64_t n_tuples, int32_t p, GraphLayout *out);

}  // namespace csbfs

struct csbfs_graph {
    int device = -1;
    int64_t n = 0;          // vertices
    int32_t P = 1;          // virtual processors
    int64_t R = 0;          // n / P
    int64_t W = 0;          // R / 64 words per piece
    int64_t n_tuples = 0;
    int64_t nnz = 0;
    int64_t max_block_nnz = 0;
    std::vector<int64_t> big_items;  // per block-row: queue items if every row were expanded at once
    int64_t device_bytes = 0;
    void *owned = nullptr;            // the graph buffer when the library allocated it
    // block b = i * P + j: rows are sources u in R_j, columns targets in R_i
    int32_t *row_ptr = nullptr;       // [P*P][R + 1], offsets within the block
    int64_t *col_base = nullptr;      // [P*P + 1], block start in col
    std::vector<int64_t> col_base_host;
    uint32_t *col = nullptr;          // [nnz], local target ids
    uint64_t *dir = nullptr;          // [P*P][W], V_{i,j} = non-empty rows of block (i, j)
    int32_t *deg = nullptr;           // [n], adjacency entries of u over all blocks
    // Pull layout: the rows of v in blocks (j, i), j = P-1 down to 0, merged
    // into one row of global ids in decreasing order (processor i's view of
    // column v of its block-row; by symmetry the same entries as the blocks)
    int64_t *pull_off = nullptr;      // [n + 1]
    uint32_t *pull_col = nullptr;     // [nnz]
    uint32_t *head = nullptr;         // [2n]: the first two ids of v's merged row (0xFFFFFFFF: none)
    uint64_t *live = nullptr;         // [n / 64]: vertices with at least one adjacency entry
    int64_t *qoff = nullptr;          // [P + 1]: processor r's chunk-queue region
    unsigned long long *scratch = nullptr;  // small reduction scratch
};

namespace csbfs {
int graph_device_check(const csbfs_graph *g);
// Sort every block row (descending target id) in place; tmp has nnz entries
// of scratch, queues and q_count come from the build scratch.
int64_t sort_queue_cap(int64_t nnz, int which);
int sort_rows_desc(uint32_t *col, uint32_t *tmp, const int32_t *row_ptr, const int64_t *col_base, int64_t R,
                   int32_t P, int64_t nnz, int64_t *queues, unsigned long long *q_count, int32_t *err,
                   hipStream_t st);
// off[v] = sum of deg[u] for u < v (off has n + 1 entries; off[n] = total);
// tile_sum holds scan_tiles(n) entries of scratch.
int64_t scan_tiles(int64_t n);
int degree_offsets(const int32_t *deg, int64_t n, int64_t *off, int64_t *tile_sum, hipStream_t st);
// A batch engine on caller memory: a device block of csbfs_batch_engine_bytes
// and a pinned two-word host buffer (each may be null: then allocated and
// owned by the engine); `st` runs its initial zeroing.
int batch_engine_make(const csbfs_graph *g, int32_t max_roots, int32_t max_levels, uint32_t flags, void *mem,
                      unsigned long long *host_ctl, hipStream_t st, csbfs_batch_engine **out);
void batch_engine_release(csbfs_batch_engine *e);
}
