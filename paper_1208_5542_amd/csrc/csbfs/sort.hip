// Graph-build helpers: sort every block row in descending order of target
// id, and the offsets of the merged pull rows (a scan of the degrees).
// Setup only; the search never calls them. Descending rows let the parent
// search of a new vertex stop at its first frontier neighbour, which is
// then the highest-labelled one.
//
// The row sort is segmented by row length, so that every row runs on the
// unit that fits it and the scratch each class needs is known from the
// sizes alone (no library sort with a device-queried workspace):
//   L <= 32         one thread: bitonic network in registers (8 or 32 slots)
//   33 .. 1024      one wavefront: bitonic network over the row in LDS
//   1025 .. 16384   one workgroup: bitonic network over the row in LDS
//   > 16384         one workgroup: least-significant-bit-first radix sort,
//                   one stable split per bit (ones first), ping-ponging
//                   between the row and the same range of a temp buffer
// Keys in the networks are id + 1 with 0 as padding, so padding sorts last.
#include "graph.hpp"
#include "device.hpp"

namespace csbfs {
namespace {

constexpr int kSortThreads = 256;
constexpr int kWaveRow = 1024;     // longest row of the wavefront class
constexpr int kBlockRow = 16384;   // longest row of the workgroup class
constexpr int kRadixItems = 16;    // elements per thread per radix chunk
constexpr int kRadixChunk = kSortThreads * kRadixItems;

__device__ __forceinline__ void cas_desc(uint32_t &a, uint32_t &b) {
    // after the call a >= b
    const uint32_t hi = a > b ? a : b, lo = a > b ? b : a;
    a = hi;
    b = lo;
}

// Bitonic network over N register slots, descending.
template <int N>
__device__ __forceinline__ void reg_bitonic_desc(uint32_t (&x)[N]) {
#pragma unroll
    for (int k = 2; k <= N; k <<= 1) {
#pragma unroll
        for (int j = k >> 1; j > 0; j >>= 1) {
#pragma unroll
            for (int i = 0; i < N; ++i) {
                const int l = i ^ j;
                if (l > i) {
                    // descending where (i & k) == 0, ascending elsewhere; the
                    // last merge (k == N) is all descending
                    if ((i & k) == 0)
                        cas_desc(x[i], x[l]);
                    else
                        cas_desc(x[l], x[i]);
                }
            }
        }
    }
}

struct SortArgs {
    uint32_t *col;
    uint32_t *tmp;               // nnz entries of scratch (same offsets as col)
    const int32_t *row_ptr;      // [B][R + 1]
    const int64_t *col_base;     // [B + 1]
    int64_t R;
    int64_t rows;                // B * R
    int64_t *q_wave;             // rows of 33 .. 1024 entries
    int64_t *q_block;            // rows of 1025 .. 16384
    int64_t *q_radix;            // rows above 16384
    unsigned long long *q_count; // [3]
    int64_t cap_wave, cap_block, cap_radix;
    int32_t key_bits;            // bits of a local id (ids < R)
    int32_t *err;
};

__device__ __forceinline__ void row_range(const SortArgs &a, int64_t row, int64_t &start, int64_t &len) {
    const int64_t b = row / a.R, u = row - b * a.R;
    const int32_t *rp = a.row_ptr + b * (a.R + 1) + u;
    start = a.col_base[b] + rp[0];
    len = rp[1] - rp[0];
}

// Wave-aggregated append of row to one of the class queues.
__device__ __forceinline__ void enqueue(const SortArgs &a, bool want, int which, int64_t row) {
    int64_t *q = which == 0 ? a.q_wave : which == 1 ? a.q_block : a.q_radix;
    const int64_t cap = which == 0 ? a.cap_wave : which == 1 ? a.cap_block : a.cap_radix;
    const uint64_t m = __ballot(want);
    if (!m) return;
    const int lane = threadIdx.x & 63;
    const int leader = __ffsll((unsigned long long)m) - 1;
    unsigned long long base = 0;
    if (lane == leader) base = atomicAdd(&a.q_count[which], (unsigned long long)__popcll(m));
    base = (unsigned long long)shfl64((int64_t)base, leader);
    if (want) {
        const unsigned long long pos = base + __popcll(m & ((1ull << lane) - 1));
        if ((int64_t)pos < cap)
            q[pos] = row;
        else
            *a.err = 1;  // cannot happen: capacities bound the row counts
    }
}

// Rows of at most 32 entries sorted by their own thread; longer rows queued.
__global__ __launch_bounds__(kSortThreads) void k_sort_short(SortArgs a) {
    for (int64_t base = blockIdx.x * (int64_t)blockDim.x; base < a.rows;
         base += (int64_t)gridDim.x * blockDim.x) {
        const int64_t row = base + threadIdx.x;
        int64_t start = 0, len = 0;
        if (row < a.rows) row_range(a, row, start, len);
        if (len >= 2 && len <= 8) {
            uint32_t x[8];
#pragma unroll
            for (int k = 0; k < 8; ++k) x[k] = k < len ? a.col[start + k] + 1u : 0u;
            reg_bitonic_desc<8>(x);
#pragma unroll
            for (int k = 0; k < 8; ++k)
                if (k < len) a.col[start + k] = x[k] - 1u;
        } else if (len > 8 && len <= 32) {
            uint32_t x[32];
#pragma unroll
            for (int k = 0; k < 32; ++k) x[k] = k < len ? a.col[start + k] + 1u : 0u;
            reg_bitonic_desc<32>(x);
#pragma unroll
            for (int k = 0; k < 32; ++k)
                if (k < len) a.col[start + k] = x[k] - 1u;
        }
        enqueue(a, len > 32 && len <= kWaveRow, 0, row);
        enqueue(a, len > kWaveRow && len <= kBlockRow, 1, row);
        enqueue(a, len > kBlockRow, 2, row);
    }
}

// Bitonic network over m (a power of two) slots of LDS, descending; `sync`
// orders the stages (wave or workgroup).
template <class Sync>
__device__ __forceinline__ void lds_bitonic_desc(uint32_t *s, int m, int t, int nt, Sync sync) {
    for (int k = 2; k <= m; k <<= 1) {
        for (int j = k >> 1; j > 0; j >>= 1) {
            for (int p = t; p < m / 2; p += nt) {
                // the p-th pair of this stage: i has bit j clear
                const int i = ((p / j) * 2 * j) + (p % j);
                const int l = i + j;
                uint32_t x = s[i], y = s[l];
                const bool desc = (i & k) == 0;
                if (desc ? x < y : x > y) {
                    s[i] = y;
                    s[l] = x;
                }
            }
            sync();
        }
    }
}

struct WaveSync {
    __device__ __forceinline__ void operator()() const { wave_lds_sync(); }
};
struct BlockSync {
    __device__ __forceinline__ void operator()() const { __syncthreads(); }
};

__device__ __forceinline__ int pow2_at_least(int64_t v) {
    int m = 1;
    while (m < v) m <<= 1;
    return m;
}

__global__ __launch_bounds__(kSortThreads) void k_sort_wave(SortArgs a) {
    __shared__ uint32_t buf[kSortThreads / 64][kWaveRow];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    uint32_t *s = buf[wid];
    const int64_t count = (int64_t)a.q_count[0] < a.cap_wave ? (int64_t)a.q_count[0] : a.cap_wave;
    const int64_t wave = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) >> 6;
    const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
    for (int64_t q = wave; q < count; q += nwaves) {
        int64_t start, len;
        row_range(a, a.q_wave[q], start, len);
        const int m = pow2_at_least(len);
        for (int k = lane; k < m; k += 64) s[k] = k < len ? a.col[start + k] + 1u : 0u;
        wave_lds_sync();
        lds_bitonic_desc(s, m, lane, 64, WaveSync());
        for (int k = lane; k < len; k += 64) a.col[start + k] = s[k] - 1u;
        wave_lds_sync();
    }
}

__global__ __launch_bounds__(kSortThreads) void k_sort_block(SortArgs a) {
    __shared__ uint32_t s[kBlockRow];
    const int64_t count = (int64_t)a.q_count[1] < a.cap_block ? (int64_t)a.q_count[1] : a.cap_block;
    for (int64_t q = blockIdx.x; q < count; q += gridDim.x) {
        int64_t start, len;
        row_range(a, a.q_block[q], start, len);
        const int m = pow2_at_least(len);
        for (int k = threadIdx.x; k < m; k += blockDim.x) s[k] = k < len ? a.col[start + k] + 1u : 0u;
        __syncthreads();
        lds_bitonic_desc(s, m, threadIdx.x, blockDim.x, BlockSync());
        for (int k = threadIdx.x; k < len; k += blockDim.x) a.col[start + k] = s[k] - 1u;
        __syncthreads();
    }
}

__device__ int block_sum_i32(int v) {
    __shared__ int red[kSortThreads / 64];
    for (int d = 32; d > 0; d >>= 1) v += __shfl_xor(v, d, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    int t = 0;
    for (int k = 0; k < kSortThreads / 64; ++k) t += red[k];
    __syncthreads();
    return t;
}

__device__ int block_excl_i32(int v, int *total) {
    __shared__ int ws[kSortThreads / 64];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    const int incl = wave_incl_scan_i32(v);
    if (lane == 63) ws[wid] = incl;
    __syncthreads();
    int before = 0, tot = 0;
    for (int k = 0; k < kSortThreads / 64; ++k) {
        if (k < wid) before += ws[k];
        tot += ws[k];
    }
    __syncthreads();
    *total = tot;
    return before + incl - v;
}

// Rows above kBlockRow entries: one stable split per key bit, least
// significant first, ones before zeros (so the result is descending).
__global__ __launch_bounds__(kSortThreads) void k_sort_radix(SortArgs a) {
    const int64_t count = (int64_t)a.q_count[2] < a.cap_radix ? (int64_t)a.q_count[2] : a.cap_radix;
    for (int64_t q = blockIdx.x; q < count; q += gridDim.x) {
        int64_t start, len;
        row_range(a, a.q_radix[q], start, len);
        uint32_t *from = a.col + start, *to = a.tmp + start;
        for (int bit = 0; bit < a.key_bits; ++bit) {
            // ones in the whole row
            int ones = 0;
            for (int64_t c = 0; c < len; c += kRadixChunk)
                for (int k = 0; k < kRadixItems; ++k) {
                    const int64_t e = c + (int64_t)threadIdx.x * kRadixItems + k;
                    if (e < len) ones += (from[e] >> bit) & 1u;
                }
            const int64_t total_ones = block_sum_i32(ones);
            int64_t ones_done = 0, zeros_done = 0;
            for (int64_t c = 0; c < len; c += kRadixChunk) {
                const int64_t e0 = c + (int64_t)threadIdx.x * kRadixItems;
                uint32_t v[kRadixItems];
                int mine = 0, have = 0;
#pragma unroll
                for (int k = 0; k < kRadixItems; ++k) {
                    v[k] = 0;
                    if (e0 + k < len) {
                        v[k] = from[e0 + k];
                        mine += (v[k] >> bit) & 1u;
                        ++have;
                    }
                }
                int chunk_ones;
                const int ones_before = block_excl_i32(mine, &chunk_ones);
                const int64_t chunk_len = len - c < kRadixChunk ? len - c : kRadixChunk;
                // zeros before this thread's items in the chunk
                int64_t o = ones_done + ones_before;
                int64_t z = total_ones + zeros_done + ((int64_t)threadIdx.x * kRadixItems - ones_before);
#pragma unroll
                for (int k = 0; k < kRadixItems; ++k) {
                    if (k < have) {
                        if ((v[k] >> bit) & 1u)
                            to[o++] = v[k];
                        else
                            to[z++] = v[k];
                    }
                }
                ones_done += chunk_ones;
                zeros_done += chunk_len - chunk_ones;
            }
            __syncthreads();
            uint32_t *t = from;
            from = to;
            to = t;
        }
        if (from != a.col + start) {
            for (int64_t e = threadIdx.x; e < len; e += blockDim.x) a.col[start + e] = from[e];
        }
        __syncthreads();
    }
}

// Exclusive scan of deg (int32, n entries) into off (int64, n + 1 entries):
// tile sums, a one-workgroup scan of the tile sums, then each tile again.
constexpr int kScanItems = 16;
constexpr int kScanTile = kSortThreads * kScanItems;

__global__ __launch_bounds__(kSortThreads) void k_scan_tiles(const int32_t *deg, int64_t n, int64_t *tile_sum) {
    const int64_t t0 = (int64_t)blockIdx.x * kScanTile;
    long long s = 0;
    for (int k = threadIdx.x; k < kScanTile; k += kSortThreads) {
        const int64_t v = t0 + k;
        if (v < n) s += deg[v];
    }
    for (int d = 32; d > 0; d >>= 1) s += __shfl_xor(s, d, 64);
    __shared__ long long red[kSortThreads / 64];
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        long long t = 0;
        for (int k = 0; k < kSortThreads / 64; ++k) t += red[k];
        tile_sum[blockIdx.x] = t;
    }
}

__device__ long long block_excl_i64(long long v, long long *total) {
    __shared__ long long ws[kSortThreads / 64];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    long long incl = v;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const long long t = __shfl_up(incl, d, 64);
        if (lane >= d) incl += t;
    }
    if (lane == 63) ws[wid] = incl;
    __syncthreads();
    long long before = 0, tot = 0;
    for (int k = 0; k < kSortThreads / 64; ++k) {
        if (k < wid) before += ws[k];
        tot += ws[k];
    }
    __syncthreads();
    *total = tot;
    return before + incl - v;
}

__global__ __launch_bounds__(kSortThreads) void k_scan_top(int64_t *tile_sum, int64_t ntiles) {
    long long carry = 0;
    for (int64_t b = 0; b < ntiles; b += kSortThreads) {
        const int64_t t = b + threadIdx.x;
        const long long v = t < ntiles ? tile_sum[t] : 0;
        long long tot;
        const long long ex = block_excl_i64(v, &tot);
        if (t < ntiles) tile_sum[t] = carry + ex;
        carry += tot;
    }
}

__global__ __launch_bounds__(kSortThreads) void k_scan_apply(const int32_t *deg, int64_t n,
                                                             const int64_t *tile_sum, int64_t *off) {
    const int64_t v0 = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
    long long d[kScanItems], mine = 0;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        d[k] = v0 + k < n ? deg[v0 + k] : 0;
        mine += d[k];
    }
    long long tot;
    long long x = tile_sum[blockIdx.x] + block_excl_i64(mine, &tot);
    if (blockIdx.x == 0 && threadIdx.x == 0) off[0] = 0;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        x += d[k];
        if (v0 + k < n) off[v0 + k + 1] = x;
    }
}

}  // namespace

int64_t sort_queue_cap(int64_t nnz, int which) {
    // a row of a class has more entries than the class below allows
    const int64_t above = which == 0 ? 32 : which == 1 ? kWaveRow : kBlockRow;
    return nnz / (above + 1) + 1;
}

int64_t scan_tiles(int64_t n) { return (n + kScanTile - 1) / kScanTile; }

int sort_rows_desc(uint32_t *col, uint32_t *tmp, const int32_t *row_ptr, const int64_t *col_base, int64_t R,
                   int32_t P, int64_t nnz, int64_t *queues, unsigned long long *q_count, int32_t *err,
                   hipStream_t st) {
    if (nnz == 0) return CSBFS_OK;
    SortArgs a{};
    a.col = col;
    a.tmp = tmp;
    a.row_ptr = row_ptr;
    a.col_base = col_base;
    a.R = R;
    a.rows = (int64_t)P * P * R;
    a.cap_wave = sort_queue_cap(nnz, 0);
    a.cap_block = sort_queue_cap(nnz, 1);
    a.cap_radix = sort_queue_cap(nnz, 2);
    a.q_wave = queues;
    a.q_block = queues + a.cap_wave;
    a.q_radix = a.q_block + a.cap_block;
    a.q_count = q_count;
    int bits = 1;
    while (((int64_t)1 << bits) < R) ++bits;
    a.key_bits = bits;
    a.err = err;
    CSBFS_HIP(hipMemsetAsync(q_count, 0, 3 * sizeof(unsigned long long), st));
    hipLaunchKernelGGL(k_sort_short, dim3(grid_for(a.rows, kSortThreads, 65536)), dim3(kSortThreads), 0, st, a);
    CSBFS_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_sort_wave, dim3(4096), dim3(kSortThreads), 0, st, a);
    CSBFS_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_sort_block, dim3(2048), dim3(kSortThreads), 0, st, a);
    CSBFS_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_sort_radix, dim3(1024), dim3(kSortThreads), 0, st, a);
    CSBFS_HIP(hipGetLastError());
    return CSBFS_OK;
}

int degree_offsets(const int32_t *deg, int64_t n, int64_t *off, int64_t *tile_sum, hipStream_t st) {
    const int64_t nt = scan_tiles(n);
    hipLaunchKernelGGL(k_scan_tiles, dim3((unsigned)nt), dim3(kSortThreads), 0, st, deg, n, tile_sum);
    CSBFS_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(kSortThreads), 0, st, tile_sum, nt);
    CSBFS_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_scan_apply, dim3((unsigned)nt), dim3(kSortThreads), 0, st, deg, n,
                       (const int64_t *)tile_sum, off);
    CSBFS_HIP(hipGetLastError());
    return CSBFS_OK;
}

}  // namespace csbfs
