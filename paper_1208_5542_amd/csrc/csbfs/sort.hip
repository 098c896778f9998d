// Graph-build helper: sort every block row in descending order of target id
// with rocPRIM's segmented radix sort. Setup only; the search never calls it.
// Descending rows let the parent search of a new vertex stop at its first
// frontier neighbour, which is then the highest-labelled one.
#include <cstring>

#include <rocprim/rocprim.hpp>

#include "graph.hpp"

namespace csbfs {
namespace {

// Global col offset of row s = b * R + u (s = P*P*R gives the total).
struct RowOffset {
    const int64_t *col_base;
    const int32_t *row_ptr;
    int64_t R;
    int64_t nrows;
    __host__ __device__ uint32_t operator()(uint32_t s) const {
        if ((int64_t)s >= nrows) return (uint32_t)col_base[nrows / R];
        const int64_t b = s / R, u = s - b * R;
        return (uint32_t)(col_base[b] + row_ptr[b * (R + 1) + u]);
    }
};

}  // namespace

int sort_rows_desc(uint32_t **col, const int64_t *col_base, const int32_t *row_ptr, int64_t R,
                   int32_t P, int64_t nnz, hipStream_t st) {
    const int64_t nrows = (int64_t)P * P * R;
    if (nnz == 0) return CSBFS_OK;
    if (nnz >= ((int64_t)1 << 32) - 1 || nrows >= ((int64_t)1 << 32) - 1)
        return fail(CSBFS_EOVERFLOW, "graph too large for the row sort");
    RowOffset fo{col_base, row_ptr, R, nrows};
    rocprim::counting_iterator<uint32_t> cnt(0);
    auto begin = rocprim::make_transform_iterator(cnt, fo);
    auto end = rocprim::make_transform_iterator(cnt + 1, fo);
    uint32_t *tmp = nullptr;
    void *ws = nullptr;
    size_t ws_bytes = 0;
    int bits = 1;
    while (((int64_t)1 << bits) < R) ++bits;
    CSBFS_HIP(rocprim::segmented_radix_sort_keys_desc(nullptr, ws_bytes, *col, tmp, (unsigned)nnz,
                                                      (unsigned)nrows, begin, end, 0, bits, st));
    CSBFS_HIP(hipMalloc(&tmp, sizeof(uint32_t) * nnz));
    hipError_t e = hipMalloc(&ws, ws_bytes > 0 ? ws_bytes : 1);
    if (e != hipSuccess) {
        (void)hipFree(tmp);
        return hip_fail(e, "hipMalloc(sort workspace)", __FILE__, __LINE__);
    }
    e = rocprim::segmented_radix_sort_keys_desc(ws, ws_bytes, *col, tmp, (unsigned)nnz,
                                                (unsigned)nrows, begin, end, 0, bits, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    (void)hipFree(ws);
    if (e != hipSuccess) {
        (void)hipFree(tmp);
        return hip_fail(e, "segmented_radix_sort_keys_desc", __FILE__, __LINE__);
    }
    (void)hipFree(*col);
    *col = tmp;
    return CSBFS_OK;
}

}  // namespace csbfs
