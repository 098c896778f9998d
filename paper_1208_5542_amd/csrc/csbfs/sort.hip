// Graph-build helpers: sort every block row in descending order of target id
// with rocPRIM's segmented radix sort, and the offsets of the merged pull
// rows (a scan of the degrees). Setup only; the search never calls them.
// Descending rows let the parent search of a new vertex stop at its first
// frontier neighbour, which is then the highest-labelled one.
#include <algorithm>
#include <cstring>

#include <rocprim/rocprim.hpp>

#include "graph.hpp"

namespace csbfs {
namespace {

// Offset of row s of one block within that block's col (s = R gives its size).
struct RowOffset {
    const int32_t *row_ptr;  // the block's R + 1 row offsets
    __host__ __device__ uint32_t operator()(uint32_t s) const { return (uint32_t)row_ptr[s]; }
};

}  // namespace

int sort_rows_desc(uint32_t **col, const int64_t *col_base_host, const int32_t *row_ptr, int64_t R,
                   int32_t P, int64_t nnz, hipStream_t st) {
    if (nnz == 0) return CSBFS_OK;
    if (R >= ((int64_t)1 << 31) - 1) return fail(CSBFS_EOVERFLOW, "block too large for the row sort");
    rocprim::counting_iterator<uint32_t> cnt(0);
    int bits = 1;
    while (((int64_t)1 << bits) < R) ++bits;
    // one sort per block: every block has fewer than 2^31 entries
    int64_t max_block = 0;
    for (int64_t b = 0; b < (int64_t)P * P; ++b)
        max_block = std::max(max_block, col_base_host[b + 1] - col_base_host[b]);
    size_t ws_bytes = 0;
    {
        RowOffset fo{row_ptr};
        auto begin = rocprim::make_transform_iterator(cnt, fo);
        auto end = rocprim::make_transform_iterator(cnt + 1, fo);
        CSBFS_HIP(rocprim::segmented_radix_sort_keys_desc(nullptr, ws_bytes, *col, *col,
                                                          (unsigned)max_block, (unsigned)R, begin,
                                                          end, 0, bits, st));
    }
    uint32_t *tmp = nullptr;
    void *ws = nullptr;
    CSBFS_HIP(hipMalloc(&tmp, sizeof(uint32_t) * nnz));
    hipError_t e = hipMalloc(&ws, ws_bytes > 0 ? ws_bytes : 1);
    for (int64_t b = 0; e == hipSuccess && b < (int64_t)P * P; ++b) {
        const int64_t base = col_base_host[b], size = col_base_host[b + 1] - base;
        if (size == 0) continue;
        RowOffset fo{row_ptr + b * (R + 1)};
        auto begin = rocprim::make_transform_iterator(cnt, fo);
        auto end = rocprim::make_transform_iterator(cnt + 1, fo);
        size_t need = 0;
        e = rocprim::segmented_radix_sort_keys_desc(nullptr, need, *col + base, tmp + base,
                                                    (unsigned)size, (unsigned)R, begin, end, 0,
                                                    bits, st);
        if (e == hipSuccess && need > ws_bytes) e = hipErrorInvalidValue;
        if (e == hipSuccess)
            e = rocprim::segmented_radix_sort_keys_desc(ws, need, *col + base, tmp + base,
                                                        (unsigned)size, (unsigned)R, begin, end, 0,
                                                        bits, st);
    }
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (ws) (void)hipFree(ws);
    if (e != hipSuccess) {
        (void)hipFree(tmp);
        return hip_fail(e, "segmented_radix_sort_keys_desc", __FILE__, __LINE__);
    }
    (void)hipFree(*col);
    *col = tmp;
    return CSBFS_OK;
}

int degree_offsets(const int32_t *deg, int64_t n, int64_t *off, hipStream_t st) {
    size_t ws_bytes = 0;
    auto in = rocprim::make_transform_iterator(deg, [] __host__ __device__(int32_t d) { return (int64_t)d; });
    CSBFS_HIP(rocprim::inclusive_scan(nullptr, ws_bytes, in, off + 1, (size_t)n, rocprim::plus<int64_t>(), st));
    void *ws = nullptr;
    CSBFS_HIP(hipMalloc(&ws, ws_bytes > 0 ? ws_bytes : 1));
    hipError_t e = hipMemsetAsync(off, 0, sizeof(int64_t), st);
    if (e == hipSuccess)
        e = rocprim::inclusive_scan(ws, ws_bytes, in, off + 1, (size_t)n, rocprim::plus<int64_t>(), st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    (void)hipFree(ws);
    if (e != hipSuccess) return hip_fail(e, "degree_offsets", __FILE__, __LINE__);
    return CSBFS_OK;
}

}  // namespace csbfs
