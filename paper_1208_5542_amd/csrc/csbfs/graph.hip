// Graph partitioning: the p x p sub-block grid of Sec. V.A (Eq. abc, Eq.
// sub-block), one CSR per block, and the directory vectors of Eq. dir-vec.
//
// Block b = i * P + j holds, for every source u in R_j (row u - j*R), its
// neighbours v in R_i as local ids v - i*R. Tuple {u, v} contributes u -> v
// to block (owner(v), owner(u)) and v -> u to block (owner(u), owner(v)); a
// self-loop contributes twice to one row. Rows are built by a counting pass,
// a per-block scan (tile sums, scan of tile sums, local scans) and a scatter.
#include <vector>

#include "graph.hpp"

namespace csbfs {
namespace {

constexpr int kThreads = 256;
constexpr int kTileItems = 4;
constexpr int kTile = kThreads * kTileItems;

__device__ __forceinline__ int wave_incl_scan_ll(long long &v) {
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        long long t = __shfl_up(v, d, 64);
        if (lane >= d) v += t;
    }
    return 0;
}

__device__ long long block_excl_scan_ll(long long v, long long *total) {
    __shared__ long long ws[kThreads / 64];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    long long incl = v;
    wave_incl_scan_ll(incl);
    if (lane == 63) ws[wid] = incl;
    __syncthreads();
    long long before = 0, tot = 0;
    for (int k = 0; k < kThreads / 64; ++k) {
        if (k < wid) before += ws[k];
        tot += ws[k];
    }
    __syncthreads();
    *total = tot;
    return before + incl - v;
}

__global__ void k_count(const int64_t *src, const int64_t *dst, int64_t m, int64_t n, int64_t R,
                        int32_t P, int32_t *cnt, int32_t *err) {
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < m;
         t += (int64_t)gridDim.x * blockDim.x) {
        const int64_t u = src[t], v = dst[t];
        if (u < 0 || u >= n || v < 0 || v >= n) {
            *err = 1;
            continue;
        }
        const int64_t ou = u / R, ov = v / R;
        atomicAdd(&cnt[(ov * P + ou) * R + (u - ou * R)], 1);  // u -> v
        atomicAdd(&cnt[(ou * P + ov) * R + (v - ov * R)], 1);  // v -> u
    }
}

// tile sums of every block's row counts: sums[b * ntile + t]
__global__ __launch_bounds__(kThreads) void k_tile_sum(const int32_t *cnt, int64_t R, int64_t ntile,
                                                       long long *sums) {
    const int64_t t = blockIdx.x, b = blockIdx.y;
    long long s = 0;
    for (int64_t k = threadIdx.x; k < kTile; k += kThreads) {
        const int64_t u = t * kTile + k;
        if (u < R) s += cnt[b * R + u];
    }
    __shared__ long long red[kThreads / 64];
    for (int d = 32; d > 0; d >>= 1) s += __shfl_xor(s, d, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        long long tot = 0;
        for (int k = 0; k < kThreads / 64; ++k) tot += red[k];
        sums[b * ntile + t] = tot;
    }
}

// in-place exclusive scan of each block's tile sums; block totals to nnz[b]
__global__ __launch_bounds__(kThreads) void k_tile_scan(long long *sums, int64_t ntile,
                                                        long long *nnz) {
    const int64_t b = blockIdx.x;
    long long carry = 0;
    for (int64_t base = 0; base < ntile; base += kThreads) {
        const int64_t t = base + threadIdx.x;
        const long long v = t < ntile ? sums[b * ntile + t] : 0;
        long long tot;
        const long long ex = block_excl_scan_ll(v, &tot);
        if (t < ntile) sums[b * ntile + t] = carry + ex;
        carry += tot;
    }
    if (threadIdx.x == 0) nnz[b] = carry;
}

// row_ptr[b * (R + 1) + u] = exclusive prefix of row counts within block b;
// the counts become the scatter cursors (cursor[u] = row_ptr[u]).
__global__ __launch_bounds__(kThreads) void k_tile_apply(int32_t *cnt, int64_t R, int64_t ntile,
                                                         const long long *sums, int32_t *row_ptr) {
    const int64_t t = blockIdx.x, b = blockIdx.y;
    const int64_t u0 = t * kTile + threadIdx.x * kTileItems;
    long long v[kTileItems];
    long long mine = 0;
    for (int k = 0; k < kTileItems; ++k) {
        const int64_t u = u0 + k;
        v[k] = u < R ? cnt[b * R + u] : 0;
        mine += v[k];
    }
    long long tot;
    long long x = sums[b * ntile + t] + block_excl_scan_ll(mine, &tot);
    for (int k = 0; k < kTileItems; ++k) {
        const int64_t u = u0 + k;
        if (u < R) {
            row_ptr[b * (R + 1) + u] = (int32_t)x;
            cnt[b * R + u] = (int32_t)x;
            x += v[k];
            if (u == R - 1) row_ptr[b * (R + 1) + R] = (int32_t)x;
        }
    }
}

__global__ void k_scatter(const int64_t *src, const int64_t *dst, int64_t m, int64_t R, int32_t P,
                          int32_t *cursor, const int64_t *col_base, uint32_t *col) {
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < m;
         t += (int64_t)gridDim.x * blockDim.x) {
        const int64_t u = src[t], v = dst[t];
        const int64_t ou = u / R, ov = v / R;
        const int64_t b1 = ov * P + ou, b2 = ou * P + ov;
        const int32_t p1 = atomicAdd(&cursor[b1 * R + (u - ou * R)], 1);
        col[col_base[b1] + p1] = (uint32_t)(v - ov * R);
        const int32_t p2 = atomicAdd(&cursor[b2 * R + (v - ov * R)], 1);
        col[col_base[b2] + p2] = (uint32_t)(u - ou * R);
    }
}

// V_{i,j}: bit u of block b's vector = row u of block b is non-empty.
__global__ void k_directory(const int32_t *row_ptr, int64_t R, int64_t W, int64_t nblocks,
                            uint64_t *dir) {
    const int lane = threadIdx.x & 63;
    const int64_t wave = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) >> 6;
    const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
    for (int64_t w = wave; w < nblocks * W; w += nwaves) {
        const int64_t b = w / W, q = w - b * W;
        const int32_t *rp = row_ptr + b * (R + 1) + q * 64 + lane;
        const bool nz = rp[1] > rp[0];
        const uint64_t m = __ballot(nz);
        if (lane == 0) dir[w] = m;
    }
}

// deg[u] = adjacency entries of u over all blocks of its column; big[i] +=
// the expansion-queue items that the rows of block-row i would need if every
// row were expanded at once (the capacity of processor i's chunk queue).
__global__ void k_degree(const int32_t *row_ptr, int64_t R, int32_t P, int64_t n, int32_t *deg,
                         unsigned long long *big_items) {
    for (int64_t base = blockIdx.x * (int64_t)blockDim.x; base < n;
         base += (int64_t)gridDim.x * blockDim.x) {
        const int64_t u = base + threadIdx.x;
        const bool ok = u < n;
        const int64_t j = ok ? u / R : 0, ul = ok ? u - j * R : 0;
        int32_t d = 0;
        for (int32_t i = 0; i < P; ++i) {
            unsigned long long items = 0;
            if (ok) {
                const int32_t *rp = row_ptr + ((int64_t)i * P + j) * (R + 1) + ul;
                const int32_t len = rp[1] - rp[0];
                d += len;
                if (len > kBigRow) items = (len + kBigChunk - 1) / kBigChunk;
            }
            for (int s = 32; s > 0; s >>= 1) items += __shfl_xor(items, s, 64);
            if ((threadIdx.x & 63) == 0 && items) atomicAdd(&big_items[i], items);
        }
        if (ok) deg[u] = d;
    }
}

// Consistency of a built graph: the largest column id (must be below R) and
// the degree total (must equal nnz).
__global__ void k_check(const uint32_t *col, int64_t nnz, const int32_t *deg, int64_t n,
                        unsigned long long *out) {
    uint32_t mx = 0;
    unsigned long long ds = 0;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < nnz; k += stride)
        mx = col[k] > mx ? col[k] : mx;
    for (int64_t u = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; u < n; u += stride)
        ds += (unsigned long long)deg[u];
    for (int d = 32; d > 0; d >>= 1) {
        const uint32_t o = __shfl_xor(mx, d, 64);
        mx = o > mx ? o : mx;
        ds += __shfl_xor(ds, d, 64);
    }
    if ((threadIdx.x & 63) == 0) {
        atomicMax(&out[0], (unsigned long long)mx);
        if (ds) atomicAdd(&out[1], ds);
    }
}

__global__ void k_count_m(const int32_t *level, const int32_t *deg, int64_t n,
                          unsigned long long *out) {
    unsigned long long s = 0;
    for (int64_t u = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; u < n;
         u += (int64_t)gridDim.x * blockDim.x)
        if (level[u] >= 0) s += (unsigned long long)deg[u];
    for (int d = 32; d > 0; d >>= 1) s += __shfl_xor(s, d, 64);
    if ((threadIdx.x & 63) == 0 && s) atomicAdd(out, s);
}

// Merge the rows of v in blocks (j, i), j = P-1 down to 0, into one row of
// global ids: each block row is already in decreasing order and block j
// holds the ids of R_j, so the merged row is in decreasing order. The row's
// first two ids are also kept beside each other per vertex (head; 0xFFFFFFFF
// where the row is shorter), so a pull can test them without the row. One
// thread per vertex (setup only).
__global__ void k_pull_fill(const int32_t *row_ptr, const int64_t *col_base, const uint32_t *col,
                            int64_t R, int32_t P, int64_t n, const int64_t *pull_off, uint32_t *pull_col,
                            uint32_t *head) {
    for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < n;
         v += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = v / R, vl = v - i * R;
        const int64_t d0 = pull_off[v];
        int64_t d = d0;
        uint32_t h[2] = {0xFFFFFFFFu, 0xFFFFFFFFu};
        for (int32_t j = P - 1; j >= 0; --j) {
            const int64_t b = (int64_t)j * P + i;
            const int32_t *rp = row_ptr + b * (R + 1) + vl;
            const uint32_t *src = col + col_base[b];
            const uint32_t base = (uint32_t)(j * R);
            for (int32_t e = rp[0]; e < rp[1]; ++e) {
                const uint32_t id = base + src[e];
                if (d - d0 < 2) h[d - d0] = id;
                pull_col[d++] = id;
            }
        }
        head[2 * v] = h[0];
        head[2 * v + 1] = h[1];
    }
}

// Vertices with at least one adjacency entry, one bit each.
__global__ void k_live(const int32_t *deg, int64_t n, uint64_t *live) {
    const int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    const uint64_t b = __ballot(v < n && deg[v] > 0);
    if ((threadIdx.x & 63) == 0 && v < n) live[v >> 6] = b;
}

unsigned grid_for(int64_t items, int64_t per_block, unsigned cap = 65536) {
    int64_t g = (items + per_block - 1) / per_block;
    if (g < 1) g = 1;
    if (g > cap) g = cap;
    return (unsigned)g;
}

constexpr int kMiscWords = 64;  // build flags and counters: err, sort queue counts, check, big items

int check_sizes(int64_t n, int64_t n_tuples, int32_t p, const char *who) {
    if (n_tuples < 0) return fail(CSBFS_EINVAL, std::string(who) + ": negative tuple count");
    if (n < 64 || n >= ((int64_t)1 << 31)) return fail(CSBFS_ERANGE, std::string(who) + ": need 64 <= n < 2^31");
    if (p < 1 || p > 64 || n % p != 0 || (n / p) % 64 != 0)
        return fail(CSBFS_ERANGE, std::string(who) + ": need 1 <= p <= 64, p | n and 64 | n/p");
    if (n_tuples > ((int64_t)1 << 40)) return fail(CSBFS_ERANGE, std::string(who) + ": too many tuples");
    return CSBFS_OK;
}

}  // namespace

int graph_layout(int64_t n, int64_t n_tuples, int32_t p, GraphLayout *L) {
    const int rc = check_sizes(n, n_tuples, p, "graph layout");
    if (rc) return rc;
    GraphLayout g{};
    g.n = n;
    g.P = p;
    g.R = n / p;
    g.W = g.R / 64;
    g.B = (int64_t)p * p;
    g.nnz = 2 * n_tuples;
    g.ntile = (g.R + kTile - 1) / kTile;
    int64_t o = 0;
    auto take = [&o](int64_t bytes) {
        const int64_t at = o;
        o += align_up(bytes > 0 ? bytes : 1);
        return at;
    };
    g.row_ptr = take(4 * g.B * (g.R + 1));
    g.col_base = take(8 * (g.B + 1));
    g.col = take(4 * g.nnz);
    g.dir = take(8 * g.B * g.W);
    g.deg = take(4 * n);
    g.pull_off = take(8 * (n + 1));
    g.pull_col = take(4 * g.nnz);
    g.head = take(8 * n);
    g.live = take(8 * (n / 64));
    g.qoff = take(8 * (g.P + 1));
    g.small = take(8 * 64);
    g.graph_bytes = o;
    o = 0;
    g.cnt = take(4 * g.B * g.R);
    g.sums = take(8 * g.B * g.ntile);
    g.nnzb = take(8 * g.B);
    g.misc = take(8 * (kMiscWords + g.P));
    g.queues = take(8 * (sort_queue_cap(g.nnz, 0) + sort_queue_cap(g.nnz, 1) + sort_queue_cap(g.nnz, 2)));
    g.scan = take(8 * scan_tiles(n));
    g.scratch_bytes = o;
    *L = g;
    return CSBFS_OK;
}

int graph_device_check(const csbfs_graph *g) {
    int dev = -1;
    CSBFS_HIP(hipGetDevice(&dev));
    if (dev != g->device) return fail(CSBFS_EINVAL, "graph was built on another device");
    return CSBFS_OK;
}

}  // namespace csbfs

using namespace csbfs;

extern "C" int csbfs_graph_build_into(const int64_t *src, const int64_t *dst, int64_t n_tuples, int64_t n,
                                      int32_t p, void *graph_mem, size_t graph_bytes, void *scratch,
                                      size_t scratch_bytes, void *stream, csbfs_graph **out) {
    if (!out) return fail(CSBFS_EINVAL, "csbfs_graph_build_into: out is NULL");
    *out = nullptr;
    if (n_tuples < 0 || (n_tuples > 0 && (!src || !dst)))
        return fail(CSBFS_EINVAL, "csbfs_graph_build_into: null tuple arrays or negative count");
    GraphLayout L;
    int rc = graph_layout(n, n_tuples, p, &L);
    if (rc) return rc;
    if (!graph_mem || !scratch) return fail(CSBFS_EINVAL, "csbfs_graph_build_into: null graph or scratch buffer");
    if ((uintptr_t)graph_mem % kAlign || (uintptr_t)scratch % kAlign)
        return fail(CSBFS_EINVAL, "csbfs_graph_build_into: buffers must be 256-byte aligned");
    if ((int64_t)graph_bytes < L.graph_bytes || (int64_t)scratch_bytes < L.scratch_bytes)
        return fail(CSBFS_ENOSPACE, "csbfs_graph_build_into: graph or scratch buffer smaller than "
                                    "csbfs_layout_query gives");
    hipStream_t st = as_stream(stream);
    const int64_t R = L.R, W = L.W, B = L.B, ntile = L.ntile;
    char *gm = (char *)graph_mem, *sm = (char *)scratch;

    std::unique_ptr<csbfs_graph> g(new csbfs_graph());
    CSBFS_HIP(hipGetDevice(&g->device));
    g->n = n;
    g->P = p;
    g->R = R;
    g->W = W;
    g->n_tuples = n_tuples;
    g->row_ptr = (int32_t *)(gm + L.row_ptr);
    g->col_base = (int64_t *)(gm + L.col_base);
    g->col = (uint32_t *)(gm + L.col);
    g->dir = (uint64_t *)(gm + L.dir);
    g->deg = (int32_t *)(gm + L.deg);
    g->pull_off = (int64_t *)(gm + L.pull_off);
    g->pull_col = (uint32_t *)(gm + L.pull_col);
    g->head = (uint32_t *)(gm + L.head);
    g->live = (uint64_t *)(gm + L.live);
    g->qoff = (int64_t *)(gm + L.qoff);
    g->scratch = (unsigned long long *)(gm + L.small);
    int32_t *cnt = (int32_t *)(sm + L.cnt);
    long long *sums = (long long *)(sm + L.sums);
    long long *nnzb = (long long *)(sm + L.nnzb);
    unsigned long long *misc = (unsigned long long *)(sm + L.misc);
    int32_t *err = (int32_t *)misc;
    unsigned long long *qcount = misc + 8, *chk = misc + 16, *big = misc + kMiscWords;

    CSBFS_HIP(hipMemsetAsync(cnt, 0, sizeof(int32_t) * B * R, st));
    CSBFS_HIP(hipMemsetAsync(misc, 0, sizeof(unsigned long long) * (kMiscWords + p), st));
    if (n_tuples > 0) {
        hipLaunchKernelGGL(k_count, dim3(grid_for(n_tuples, kThreads)), dim3(kThreads), 0, st, src,
                           dst, n_tuples, n, R, p, cnt, err);
        CSBFS_HIP(hipGetLastError());
    }
    int32_t herr = 0;
    CSBFS_HIP(hipMemcpyAsync(&herr, err, sizeof(herr), hipMemcpyDeviceToHost, st));
    CSBFS_HIP(hipStreamSynchronize(st));
    if (herr) return fail(CSBFS_ERANGE, "csbfs_graph_build_into: a tuple id is outside [0, n)");

    hipLaunchKernelGGL(k_tile_sum, dim3((unsigned)ntile, (unsigned)B), dim3(kThreads), 0, st,
                       (const int32_t *)cnt, R, ntile, sums);
    CSBFS_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_tile_scan, dim3((unsigned)B), dim3(kThreads), 0, st, sums, ntile, nnzb);
    CSBFS_HIP(hipGetLastError());
    std::vector<long long> nnz(B);
    CSBFS_HIP(hipMemcpyAsync(nnz.data(), nnzb, sizeof(long long) * B, hipMemcpyDeviceToHost, st));
    CSBFS_HIP(hipStreamSynchronize(st));
    std::vector<int64_t> base(B + 1, 0);
    int64_t maxb = 0;
    for (int64_t b = 0; b < B; ++b) {
        if (nnz[b] >= ((long long)1 << 31) - 1)
            return fail(CSBFS_EOVERFLOW, "csbfs_graph_build_into: a sub-block has >= 2^31 entries");
        base[b + 1] = base[b] + nnz[b];
        if (nnz[b] > maxb) maxb = nnz[b];
    }
    const int64_t total = base[B];
    if (total != L.nnz) return fail(CSBFS_ECORRUPT, "csbfs_graph_build_into: adjacency count mismatch");
    CSBFS_HIP(hipMemcpyAsync(g->col_base, base.data(), sizeof(int64_t) * (B + 1), hipMemcpyHostToDevice, st));
    hipLaunchKernelGGL(k_tile_apply, dim3((unsigned)ntile, (unsigned)B), dim3(kThreads), 0, st, cnt, R,
                       ntile, (const long long *)sums, g->row_ptr);
    CSBFS_HIP(hipGetLastError());
    if (n_tuples > 0) {
        hipLaunchKernelGGL(k_scatter, dim3(grid_for(n_tuples, kThreads)), dim3(kThreads), 0, st,
                           src, dst, n_tuples, R, p, cnt, (const int64_t *)g->col_base, g->col);
        CSBFS_HIP(hipGetLastError());
    }
    // rows in decreasing id order; pull_col serves as the sort's temp buffer
    // (it is filled from the sorted blocks afterwards)
    rc = sort_rows_desc(g->col, g->pull_col, g->row_ptr, g->col_base, R, p, total,
                        (int64_t *)(sm + L.queues), qcount, err, st);
    if (rc) return rc;
    hipLaunchKernelGGL(k_directory, dim3(grid_for(B * W * 64, kThreads)), dim3(kThreads), 0, st,
                       (const int32_t *)g->row_ptr, R, W, B, g->dir);
    CSBFS_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_degree, dim3(grid_for(n, kThreads)), dim3(kThreads), 0, st,
                       (const int32_t *)g->row_ptr, R, p, n, g->deg, big);
    CSBFS_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_live, dim3(grid_for(n, 256, 1u << 30)), dim3(256), 0, st, (const int32_t *)g->deg, n,
                       g->live);
    CSBFS_HIP(hipGetLastError());
    // never hand the search a column id outside its block or a lost entry
    hipLaunchKernelGGL(k_check, dim3(4096), dim3(kThreads), 0, st, (const uint32_t *)g->col, total,
                       (const int32_t *)g->deg, n, chk);
    CSBFS_HIP(hipGetLastError());
    rc = degree_offsets(g->deg, n, g->pull_off, (int64_t *)(sm + L.scan), st);
    if (rc) return rc;
    hipLaunchKernelGGL(k_pull_fill, dim3(grid_for(n, kThreads)), dim3(kThreads), 0, st,
                       (const int32_t *)g->row_ptr, (const int64_t *)g->col_base, (const uint32_t *)g->col, R, p,
                       n, (const int64_t *)g->pull_off, g->pull_col, g->head);
    CSBFS_HIP(hipGetLastError());
    std::vector<unsigned long long> tail(kMiscWords + p);
    int64_t pull_total = -1;
    CSBFS_HIP(hipMemcpyAsync(tail.data(), misc, sizeof(unsigned long long) * (kMiscWords + p),
                             hipMemcpyDeviceToHost, st));
    CSBFS_HIP(hipMemcpyAsync(&pull_total, g->pull_off + n, sizeof(int64_t), hipMemcpyDeviceToHost, st));
    CSBFS_HIP(hipStreamSynchronize(st));
    if ((int32_t)tail[0] != 0)
        return fail(CSBFS_ECORRUPT, "csbfs_graph_build_into: internal row-sort queue overflow");
    if (total > 0 && (tail[16] >= (unsigned long long)R || tail[17] != (unsigned long long)total))
        return fail(CSBFS_ECORRUPT, "csbfs_graph_build_into: internal consistency check of the block "
                                    "CSR failed (column id or degree total)");
    if (pull_total != total)
        return fail(CSBFS_ECORRUPT, "csbfs_graph_build_into: pull-row offsets disagree with the blocks");
    // chunk-queue regions per processor, from the long rows each block-row has
    std::vector<int64_t> qoff(p + 1, 0);
    g->big_items.assign(p, 0);
    for (int32_t r = 0; r < p; ++r) {
        g->big_items[r] = (int64_t)tail[kMiscWords + r];
        qoff[r + 1] = qoff[r] + g->big_items[r];
    }
    if (qoff[p] > big_items_bound(total))
        return fail(CSBFS_ECORRUPT, "csbfs_graph_build_into: chunk-queue items above their bound");
    CSBFS_HIP(hipMemcpyAsync(g->qoff, qoff.data(), sizeof(int64_t) * (p + 1), hipMemcpyHostToDevice, st));
    CSBFS_HIP(hipStreamSynchronize(st));
    g->col_base_host = base;
    g->nnz = total;
    g->max_block_nnz = maxb;
    g->device_bytes = L.graph_bytes;
    *out = g.release();
    return CSBFS_OK;
}

extern "C" int csbfs_graph_build(const int64_t *src, const int64_t *dst, int64_t n_tuples,
                                 int64_t n, int32_t p, void *stream, csbfs_graph **out) {
    if (!out) return fail(CSBFS_EINVAL, "csbfs_graph_build: out is NULL");
    *out = nullptr;
    if (n_tuples < 0 || (n_tuples > 0 && (!src || !dst)))
        return fail(CSBFS_EINVAL, "csbfs_graph_build: null tuple arrays or negative count");
    GraphLayout L;
    int rc = graph_layout(n, n_tuples, p, &L);
    if (rc) return rc;
    void *gm = nullptr, *sm = nullptr;
    CSBFS_HIP(hipMalloc(&gm, (size_t)L.graph_bytes));
    hipError_t e = hipMalloc(&sm, (size_t)L.scratch_bytes);
    if (e != hipSuccess) {
        (void)hipFree(gm);
        return hip_fail(e, "hipMalloc(build scratch)", __FILE__, __LINE__);
    }
    rc = csbfs_graph_build_into(src, dst, n_tuples, n, p, gm, (size_t)L.graph_bytes, sm,
                                (size_t)L.scratch_bytes, stream, out);
    (void)hipFree(sm);
    if (rc) {
        (void)hipFree(gm);
        return rc;
    }
    (*out)->owned = gm;
    return CSBFS_OK;
}

extern "C" int csbfs_graph_free(csbfs_graph *g) {
    if (!g) return CSBFS_OK;
    // a caller-owned buffer stays the caller's; hipFree orders itself after
    // the device work that may still use the library's own buffer
    if (g->owned) (void)hipFree(g->owned);
    delete g;
    return CSBFS_OK;
}

extern "C" int csbfs_graph_get_info(const csbfs_graph *g, csbfs_graph_info *info) {
    if (!g || !info) return fail(CSBFS_EINVAL, "csbfs_graph_get_info: null argument");
    info->n = g->n;
    info->p = g->P;
    info->reserved = 0;
    info->range = g->R;
    info->n_tuples = g->n_tuples;
    info->nnz = g->nnz;
    info->max_block_nnz = g->max_block_nnz;
    info->device_bytes = g->device_bytes;
    return CSBFS_OK;
}

extern "C" int csbfs_graph_copy_directory(const csbfs_graph *g, uint64_t *dst, int64_t cap_words,
                                          void *stream) {
    if (!g || !dst) return fail(CSBFS_EINVAL, "csbfs_graph_copy_directory: null argument");
    const int64_t words = (int64_t)g->P * g->P * g->W;
    if (cap_words < words) return fail(CSBFS_ENOSPACE, "csbfs_graph_copy_directory: dst too small");
    CSBFS_HIP(hipMemcpyAsync(dst, g->dir, sizeof(uint64_t) * words, hipMemcpyDeviceToDevice,
                             as_stream(stream)));
    return CSBFS_OK;
}

extern "C" int csbfs_graph_copy_block(const csbfs_graph *g, int32_t i, int32_t j, int32_t *row_ptr,
                                      uint32_t *col, int64_t cap, int64_t *nnz_out, void *stream) {
    if (!g || !row_ptr || !nnz_out || cap < 0)
        return fail(CSBFS_EINVAL, "csbfs_graph_copy_block: null argument");
    if (i < 0 || i >= g->P || j < 0 || j >= g->P)
        return fail(CSBFS_ERANGE, "csbfs_graph_copy_block: block index outside [0, p)");
    const int64_t b = (int64_t)i * g->P + j;
    const int64_t nnz = g->col_base_host[b + 1] - g->col_base_host[b];
    *nnz_out = nnz;
    if (cap < nnz) return fail(CSBFS_ENOSPACE, "csbfs_graph_copy_block: col capacity too small");
    if (nnz > 0 && !col) return fail(CSBFS_EINVAL, "csbfs_graph_copy_block: col is NULL");
    hipStream_t st = as_stream(stream);
    CSBFS_HIP(hipMemcpyAsync(row_ptr, g->row_ptr + b * (g->R + 1), sizeof(int32_t) * (g->R + 1),
                             hipMemcpyDeviceToDevice, st));
    if (nnz > 0)
        CSBFS_HIP(hipMemcpyAsync(col, g->col + g->col_base_host[b], sizeof(uint32_t) * nnz,
                                 hipMemcpyDeviceToDevice, st));
    CSBFS_HIP(hipStreamSynchronize(st));
    return CSBFS_OK;
}

extern "C" int csbfs_count_traversed_tuples(const csbfs_graph *g, const int32_t *level,
                                            int64_t *m_out, void *stream) {
    if (!g || !level || !m_out) return fail(CSBFS_EINVAL, "csbfs_count_traversed_tuples: null argument");
    hipStream_t st = as_stream(stream);
    CSBFS_HIP(hipMemsetAsync(g->scratch, 0, sizeof(unsigned long long), st));
    hipLaunchKernelGGL(k_count_m, dim3(grid_for(g->n, kThreads, 4096)), dim3(kThreads), 0, st,
                       level, (const int32_t *)g->deg, g->n, g->scratch);
    CSBFS_HIP(hipGetLastError());
    unsigned long long s = 0;
    CSBFS_HIP(hipMemcpyAsync(&s, g->scratch, sizeof(s), hipMemcpyDeviceToHost, st));
    CSBFS_HIP(hipStreamSynchronize(st));
    // every tuple contributes two adjacency entries (a self-loop two in one row)
    *m_out = (int64_t)(s / 2);
    return CSBFS_OK;
}
