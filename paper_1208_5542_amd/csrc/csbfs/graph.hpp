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
    unsigned long long *scratch = nullptr;  // small reduction scratch
};

namespace csbfs {
int graph_device_check(const csbfs_graph *g);
// Sort every block row (descending target id); replaces *col by a new buffer.
int sort_rows_desc(uint32_t **col, const int64_t *col_base_host, const int32_t *row_ptr, int64_t R,
                   int32_t P, int64_t nnz, hipStream_t st);
// off[v] = sum of deg[u] for u < v (off has n + 1 entries; off[n] = total).
int degree_offsets(const int32_t *deg, int64_t n, int64_t *off, hipStream_t st);
}
