// The level loop of Algorithm 3 (Sec. V.B) over P virtual processors on one
// GPU. Processor i's state lives in slices of device arrays: visited bits
// pi_i and frontier piece f_i (R bits each), the temporary t_i, and its P
// incoming frontier pieces f_{i,j}, the "views" (bits of R_j as received from
// P_j). One level k:
//
//   expand   t_i = sum_j A_{i,j} (x) f_{i,j} over the (select, max) semiring,
//            top-down: every set bit u of a view is a source whose row in
//            block (i, j) is pushed to its targets v; an unvisited v records
//            u by atomicMax into parent[v] (the highest label wins, Sec.
//            III.A) and the first writer sets bit v of t_i.
//   update   t_i &= ~pi_i; pi_i |= t_i; f_i = t_i; level[v] = k + 1; the
//            frontier size is reduced into a counter that the host reads.
//   sieve + compress   stream i -> j = WAH-64(f_i AND V_{j,i})  (wah.hip)
//   exchange           stream slot (i, j) is P_j's receive buffer from P_i
//   decode/merge       view (j, i) |= WAH^-1(stream i -> j)    (wah.hip)
//
// The expansion reads each view word once and clears it, so the views are
// zero again when the decoder ORs the next level's messages into them.
#include <vector>

#include "graph.hpp"

namespace csbfs {
namespace {

constexpr int kExpThreads = 256;
constexpr int kUpdThreads = 256;
constexpr int kEvPerLevel = 5;

struct BigItem {
    int32_t block;
    int32_t u_local;
    int32_t start;  // offsets within the block's col
    int32_t end;
};

struct ExpandArgs {
    uint64_t *view;
    int64_t view_words;
    const int32_t *row_ptr;
    const int64_t *col_base;
    const uint32_t *col;
    const uint64_t *pi;
    int32_t *parent;
    uint64_t *T;
    BigItem *queue;
    uint32_t *queue_count;
    int64_t queue_cap;
    int64_t R;
    int64_t W;
    int32_t P;
    unsigned long long *edges;
    int32_t *status;
};

__device__ __forceinline__ int wave_incl_scan_i32(int v) {
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        int t = __shfl_up(v, d, 64);
        if (lane >= d) v += t;
    }
    return v;
}

// Record source u for target v (global ids) if v is not yet visited.
__device__ __forceinline__ void relax(const ExpandArgs &a, int64_t v, int32_t u) {
    const uint64_t bit = 1ull << (v & 63);
    if (a.pi[v >> 6] & bit) return;
    const int32_t old = __hip_atomic_load(&a.parent[v], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (old >= u) return;
    atomicMax(&a.parent[v], u);
    if (old < 0) atomicOr((unsigned long long *)&a.T[v >> 6], (unsigned long long)bit);
}

__global__ __launch_bounds__(kExpThreads) void expand_kernel(ExpandArgs a) {
    const int lane = threadIdx.x & 63;
    const int64_t wave = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) >> 6;
    const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
    const int64_t ntiles = (a.view_words + 63) >> 6;
    unsigned long long edges = 0;
    for (int64_t tile = wave; tile < ntiles; tile += nwaves) {
        const int64_t w = (tile << 6) + lane;
        uint64_t bits = w < a.view_words ? a.view[w] : 0;
        if (bits) a.view[w] = 0;
        uint64_t nz = __ballot(bits != 0);
        while (nz) {
            const int src = __ffsll((unsigned long long)nz) - 1;
            nz &= nz - 1;
            const uint64_t wb = __shfl(bits, src, 64);
            const int64_t wi = (tile << 6) + src;
            const int64_t b = wi / a.W;
            const int64_t q = wi - b * a.W;
            const int32_t i = (int32_t)(b / a.P);
            const int32_t j = (int32_t)(b - (int64_t)i * a.P);
            const int64_t ul = (q << 6) + lane;
            int32_t rs = 0, deg = 0;
            if ((wb >> lane) & 1) {
                const int32_t *rp = a.row_ptr + b * (a.R + 1) + ul;
                rs = rp[0];
                deg = rp[1] - rs;
            }
            // long rows go to the chunk queue, one wave-aggregated reservation
            int32_t items = deg > kBigRow ? (deg + kBigChunk - 1) / kBigChunk : 0;
            const int32_t items_incl = wave_incl_scan_i32(items);
            const int32_t items_total = __shfl(items_incl, 63, 64);
            if (items_total) {
                uint32_t base = 0;
                if (lane == 63) base = atomicAdd(a.queue_count, (uint32_t)items_total);
                base = __shfl(base, 63, 64);
                if (items) {
                    int64_t pos = (int64_t)base + items_incl - items;
                    if (pos + items > a.queue_cap) {
                        *a.status = 2;  // cannot happen: the capacity bounds every row at once
                    } else {
                        for (int32_t c = 0; c < items; ++c) {
                            BigItem it;
                            it.block = (int32_t)b;
                            it.u_local = (int32_t)ul;
                            it.start = rs + c * kBigChunk;
                            it.end = min(rs + deg, rs + (c + 1) * kBigChunk);
                            a.queue[pos + c] = it;
                        }
                    }
                    deg = 0;
                }
            }
            const int32_t incl = wave_incl_scan_i32(deg);
            const int32_t total = __shfl(incl, 63, 64);
            const int32_t excl = incl - deg;
            edges += (unsigned long long)total;
            const int32_t u_base = (int32_t)(j * a.R + (q << 6));
            const uint32_t *colb = a.col + a.col_base[b];
            const int64_t vbase = (int64_t)i * a.R;
            for (int32_t e0 = 0; e0 < total; e0 += 64) {
                const int32_t e = e0 + lane;
                // owner: the largest lane L with excl[L] <= e
                int lo = 0;
#pragma unroll
                for (int step = 32; step > 0; step >>= 1) {
                    const int probe = lo + step;
                    const int32_t ex = __shfl(excl, probe < 64 ? probe : 63, 64);
                    if (probe < 64 && ex <= e) lo = probe;
                }
                const int32_t ex_lo = __shfl(excl, lo, 64);
                const int32_t rs_lo = __shfl(rs, lo, 64);
                if (e < total) {
                    const uint32_t vl = colb[rs_lo + (e - ex_lo)];
                    relax(a, vbase + vl, u_base + lo);
                }
            }
        }
    }
    // `total` is wave-uniform, so every lane holds the wave's edge count
    if (lane == 0 && edges) atomicAdd(a.edges, edges);
}

__global__ __launch_bounds__(kExpThreads) void expand_big_kernel(ExpandArgs a) {
    const int lane = threadIdx.x & 63;
    const int64_t wave = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) >> 6;
    const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
    const int64_t queued = *a.queue_count;
    const int64_t count = queued < a.queue_cap ? queued : a.queue_cap;
    unsigned long long edges = 0;
    for (int64_t k = wave; k < count; k += nwaves) {
        const BigItem it = a.queue[k];
        const int64_t b = it.block;
        const int32_t i = (int32_t)(b / a.P);
        const int32_t j = (int32_t)(b - (int64_t)i * a.P);
        const int32_t u = (int32_t)(j * a.R + it.u_local);
        const uint32_t *colb = a.col + a.col_base[b];
        const int64_t vbase = (int64_t)i * a.R;
        for (int32_t e = it.start + lane; e < it.end; e += 64) relax(a, vbase + colb[e], u);
        edges += (unsigned long long)(it.end - it.start);
    }
    if (lane == 0 && edges) atomicAdd(a.edges, edges);
}

struct UpdateArgs {
    uint64_t *T;
    uint64_t *pi;
    uint64_t *f;
    int32_t *level;
    int32_t next_level;
    int64_t words;        // n / 64
    int64_t W;            // words per processor
    int32_t P;
    unsigned long long *rank_count;  // [P]
    unsigned long long *total;       // [1]
    uint32_t *queue_count;
};

__global__ __launch_bounds__(kUpdThreads) void update_kernel(UpdateArgs a) {
    const int lane = threadIdx.x & 63;
    const int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    uint64_t t = 0;
    if (q < a.words) {
        t = a.T[q];
        if (t) {
            a.T[q] = 0;
            const uint64_t p = a.pi[q];
            t &= ~p;
            a.pi[q] = p | t;
        }
        a.f[q] = t;
    }
    if (q == 0) *a.queue_count = 0;
    // frontier size per processor
    const int c = __popcll(t);
    const int64_t q0 = __shfl(q, 0, 64);
    const int64_t q63 = q0 + 63 < a.words ? q0 + 63 : a.words - 1;
    if (q0 / a.W == q63 / a.W) {
        int s = c;
        for (int d = 32; d > 0; d >>= 1) s += __shfl_xor(s, d, 64);
        if (lane == 0 && s && q0 < a.words) {
            atomicAdd(&a.rank_count[q0 / a.W], (unsigned long long)s);
            atomicAdd(a.total, (unsigned long long)s);
        }
    } else if (c) {
        atomicAdd(&a.rank_count[q / a.W], (unsigned long long)c);
        atomicAdd(a.total, (unsigned long long)c);
    }
    // level of every new vertex, one coalesced row of 64 per non-zero word
    uint64_t nz = __ballot(t != 0);
    while (nz) {
        const int src = __ffsll((unsigned long long)nz) - 1;
        nz &= nz - 1;
        const uint64_t tw = __shfl(t, src, 64);
        const int64_t qq = q0 + src;
        if ((tw >> lane) & 1) a.level[(qq << 6) + lane] = a.next_level;
    }
}

struct SeedArgs {
    int32_t *level;
    int32_t *parent;
    uint64_t *pi;
    uint64_t *T;
    uint64_t *view;
    int64_t n;
    int64_t words;
    int64_t view_words;
};

__global__ void seed_fill_kernel(SeedArgs a) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < a.n; k += stride) {
        a.level[k] = -1;
        a.parent[k] = -1;
        if (k < a.words) {
            a.pi[k] = 0;
            a.T[k] = 0;
        }
        if (k < a.view_words) a.view[k] = 0;
    }
    for (int64_t k = a.n + blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < a.view_words;
         k += stride)
        a.view[k] = 0;
}

// f(s) <- s: the source is known to every processor without a message.
__global__ void seed_root_kernel(SeedArgs a, int64_t root, int64_t R, int64_t W, int32_t P,
                                 unsigned long long *frontier0, unsigned long long *rank0) {
    const int64_t own = root / R, rl = root - own * R;
    a.level[root] = 0;
    a.parent[root] = (int32_t)root;
    a.pi[root >> 6] |= 1ull << (root & 63);
    for (int32_t i = 0; i < P; ++i) a.view[((int64_t)i * P + own) * W + (rl >> 6)] |= 1ull << (rl & 63);
    *frontier0 = 1;
    rank0[own] = 1;
}

unsigned grid_for(int64_t items, int64_t per_block, int64_t cap) {
    int64_t g = (items + per_block - 1) / per_block;
    if (g < 1) g = 1;
    if (g > cap) g = cap;
    return (unsigned)g;
}

}  // namespace
}  // namespace csbfs

using namespace csbfs;

// Per-level device counters, slot k for k < L and slot L for levels past the
// engine's capacity (reset before each use).
struct LevelCounters {
    unsigned long long *frontier;   // [L+1]
    unsigned long long *rank;       // [L+1][P]
    unsigned long long *edges;      // [L+1]
    unsigned long long *sbits;      // [L+1][S]
    unsigned long long *uwords;     // [L+1][P]
    int64_t *words;                 // [L+1][S]
};

struct csbfs_engine {
    const csbfs_graph *g = nullptr;
    int device = -1;
    int32_t L = 0;
    uint32_t flags = 0;
    int64_t S = 0, cap = 0, nseg = 0, nchunk = 0;
    uint64_t *pi = nullptr, *f = nullptr, *T = nullptr, *view = nullptr, *arena = nullptr;
    int32_t *seg_count = nullptr, *seg_first = nullptr;
    int64_t *chunk_groups = nullptr;
    BigItem *queue = nullptr;
    uint32_t *queue_count = nullptr;
    int64_t queue_cap = 0;
    void *counters_mem = nullptr;
    size_t counters_bytes = 0;
    LevelCounters lc{};
    int32_t *status = nullptr;
    unsigned long long *host_count = nullptr;  // pinned
    std::vector<hipEvent_t> events;
    int32_t last_levels = 0;
    std::vector<void *> allocs;
};

namespace {

int engine_alloc(csbfs_engine *e, void **p, size_t bytes) {
    CSBFS_HIP(hipMalloc(p, bytes > 0 ? bytes : 1));
    e->allocs.push_back(*p);
    return CSBFS_OK;
}

void engine_release(csbfs_engine *e) {
    (void)hipDeviceSynchronize();
    for (void *p : e->allocs) (void)hipFree(p);
    e->allocs.clear();
    if (e->host_count) (void)hipHostFree(e->host_count);
    for (hipEvent_t ev : e->events) (void)hipEventDestroy(ev);
    e->events.clear();
    delete e;
}

}  // namespace

extern "C" int csbfs_engine_create(const csbfs_graph *g, int32_t max_levels, uint32_t flags,
                                   csbfs_engine **out) {
    if (!out) return fail(CSBFS_EINVAL, "csbfs_engine_create: out is NULL");
    *out = nullptr;
    if (!g) return fail(CSBFS_EINVAL, "csbfs_engine_create: graph is NULL");
    if (max_levels < 1 || max_levels > 65536)
        return fail(CSBFS_EINVAL, "csbfs_engine_create: max_levels outside [1, 65536]");
    if (flags & ~(CSBFS_FLAG_TIMING | CSBFS_FLAG_KEEP_STREAMS | CSBFS_FLAG_NO_SIEVE))
        return fail(CSBFS_EINVAL, "csbfs_engine_create: unknown flag");
    int rc = graph_device_check(g);
    if (rc) return rc;
    csbfs_engine *e = new csbfs_engine();
    e->g = g;
    e->device = g->device;
    e->L = max_levels;
    e->flags = flags;
    const int64_t P = g->P, n = g->n;
    e->S = P * P;
    e->cap = wah_cap(g->R);
    e->nseg = enc_segments(g->R);
    e->nchunk = dec_chunks(g->R);
    const int64_t words = n / 64;
    const int64_t arena_slots = (flags & CSBFS_FLAG_KEEP_STREAMS) ? (int64_t)max_levels + 1 : 1;
    e->queue_cap = g->big_items > 0 ? g->big_items : 1;
#define ALLOC(ptr, bytes)                                                  \
    do {                                                                   \
        void *_p = nullptr;                                                \
        int _rc = engine_alloc(e, &_p, (bytes));                           \
        if (_rc) {                                                         \
            engine_release(e);                                             \
            return _rc;                                                    \
        }                                                                  \
        ptr = reinterpret_cast<decltype(ptr)>(_p);                         \
    } while (0)
    ALLOC(e->pi, sizeof(uint64_t) * words);
    ALLOC(e->f, sizeof(uint64_t) * words);
    ALLOC(e->T, sizeof(uint64_t) * words);
    ALLOC(e->view, sizeof(uint64_t) * P * words);
    ALLOC(e->arena, sizeof(uint64_t) * e->S * e->cap * arena_slots);
    ALLOC(e->seg_count, sizeof(int32_t) * e->S * e->nseg);
    ALLOC(e->seg_first, sizeof(int32_t) * e->S * e->nseg);
    ALLOC(e->chunk_groups, sizeof(int64_t) * e->S * e->nchunk);
    ALLOC(e->queue, sizeof(BigItem) * e->queue_cap);
    ALLOC(e->queue_count, sizeof(uint32_t));
    ALLOC(e->status, sizeof(int32_t));
    const int64_t slots = (int64_t)max_levels + 1;
    const size_t cnt_bytes = sizeof(unsigned long long) * slots * (1 + P + 1 + e->S + P) +
                             sizeof(int64_t) * slots * e->S;
    ALLOC(e->counters_mem, cnt_bytes);
#undef ALLOC
    e->counters_bytes = cnt_bytes;
    unsigned long long *c = (unsigned long long *)e->counters_mem;
    e->lc.frontier = c;
    c += slots;
    e->lc.rank = c;
    c += slots * P;
    e->lc.edges = c;
    c += slots;
    e->lc.sbits = c;
    c += slots * e->S;
    e->lc.uwords = c;
    c += slots * P;
    e->lc.words = (int64_t *)c;
    hipError_t herr = hipHostMalloc((void **)&e->host_count, sizeof(unsigned long long));
    if (herr != hipSuccess) {
        e->host_count = nullptr;
        engine_release(e);
        return hip_fail(herr, "hipHostMalloc", __FILE__, __LINE__);
    }
    if (flags & CSBFS_FLAG_TIMING) {
        e->events.resize((size_t)max_levels * kEvPerLevel);
        for (auto &ev : e->events) {
            herr = hipEventCreate(&ev);
            if (herr != hipSuccess) {
                ev = nullptr;
                engine_release(e);
                return hip_fail(herr, "hipEventCreate", __FILE__, __LINE__);
            }
        }
    }
    *out = e;
    return CSBFS_OK;
}

extern "C" int csbfs_engine_free(csbfs_engine *e) {
    if (!e) return CSBFS_OK;
    engine_release(e);
    return CSBFS_OK;
}

namespace {

struct LevelPtrs {
    int64_t slot;
};

inline int64_t slot_of(const csbfs_engine *e, int64_t k) { return k < e->L ? k : e->L; }

int reset_overflow_slot(csbfs_engine *e, hipStream_t st) {
    const int64_t L = e->L, P = e->g->P, S = e->S;
    CSBFS_HIP(hipMemsetAsync(e->lc.frontier + L, 0, sizeof(unsigned long long), st));
    CSBFS_HIP(hipMemsetAsync(e->lc.rank + L * P, 0, sizeof(unsigned long long) * P, st));
    CSBFS_HIP(hipMemsetAsync(e->lc.edges + L, 0, sizeof(unsigned long long), st));
    CSBFS_HIP(hipMemsetAsync(e->lc.sbits + L * S, 0, sizeof(unsigned long long) * S, st));
    CSBFS_HIP(hipMemsetAsync(e->lc.uwords + L * P, 0, sizeof(unsigned long long) * P, st));
    return CSBFS_OK;
}

}  // namespace

extern "C" int csbfs_bfs(csbfs_engine *e, int64_t root, int32_t *level, int32_t *parent,
                         csbfs_level_stats *stats, int32_t stats_cap, int32_t *n_levels,
                         void *stream) {
    if (!e || !level || !parent || !n_levels || stats_cap < 0 || (stats_cap > 0 && !stats))
        return fail(CSBFS_EINVAL, "csbfs_bfs: null argument or negative stats_cap");
    const csbfs_graph *g = e->g;
    if (root < 0 || root >= g->n) return fail(CSBFS_ERANGE, "csbfs_bfs: root outside [0, n)");
    int rc = graph_device_check(g);
    if (rc) return rc;
    hipStream_t st = as_stream(stream);
    const int64_t P = g->P, n = g->n, R = g->R, W = g->W, S = e->S;
    const int64_t words = n / 64, view_words = P * words;
    const bool timing = (e->flags & CSBFS_FLAG_TIMING) != 0;
    const bool keep = (e->flags & CSBFS_FLAG_KEEP_STREAMS) != 0;

    // a0: seed
    CSBFS_HIP(hipMemsetAsync(e->counters_mem, 0, e->counters_bytes, st));
    CSBFS_HIP(hipMemsetAsync(e->status, 0, sizeof(int32_t), st));
    CSBFS_HIP(hipMemsetAsync(e->queue_count, 0, sizeof(uint32_t), st));
    SeedArgs sa{level, parent, e->pi, e->T, e->view, n, words, view_words};
    const int64_t fill_items = n > view_words ? n : view_words;
    hipLaunchKernelGGL(seed_fill_kernel, dim3(grid_for(fill_items, 256, 8192)), dim3(256), 0, st, sa);
    CSBFS_HIP(hipGetLastError());
    hipLaunchKernelGGL(seed_root_kernel, dim3(1), dim3(1), 0, st, sa, root, R, W, (int32_t)P,
                       e->lc.frontier, e->lc.rank);
    CSBFS_HIP(hipGetLastError());

    ExpandArgs ea{};
    ea.view = e->view;
    ea.view_words = view_words;
    ea.row_ptr = g->row_ptr;
    ea.col_base = g->col_base;
    ea.col = g->col;
    ea.pi = e->pi;
    ea.parent = parent;
    ea.T = e->T;
    ea.queue = e->queue;
    ea.queue_count = e->queue_count;
    ea.queue_cap = e->queue_cap;
    ea.R = R;
    ea.W = W;
    ea.P = (int32_t)P;
    ea.status = e->status;
    const unsigned exp_grid = grid_for((view_words + 63) / 64, kExpThreads / 64, 16384);
    const unsigned big_grid = 2048;
    const unsigned upd_grid = grid_for(words, kUpdThreads, 1u << 30);

    WahBatch wb{};
    wb.bits_base = e->f;
    wb.mask_base = (e->flags & CSBFS_FLAG_NO_SIEVE) ? nullptr : g->dir;
    wb.nbits = R;
    wb.words_per_piece = W;
    wb.cap = e->cap;
    wb.P = (int32_t)P;
    wb.seg_count = e->seg_count;
    wb.seg_first = e->seg_first;
    wb.nseg = e->nseg;
    wb.chunk_groups = e->chunk_groups;
    wb.nchunk = e->nchunk;
    wb.dst_base = e->view;
    wb.status = e->status;

    int64_t k = 0;
    for (;; ++k) {
        const int64_t sk = slot_of(e, k), sn = slot_of(e, k + 1);
        if (k + 1 >= e->L) {
            rc = reset_overflow_slot(e, st);
            if (rc) return rc;
        }
        hipEvent_t *ev = (timing && k < e->L) ? &e->events[(size_t)k * kEvPerLevel] : nullptr;
        if (ev) CSBFS_HIP(hipEventRecord(ev[0], st));
        // a1: expand f^k
        ea.edges = e->lc.edges + sk;
        hipLaunchKernelGGL(expand_kernel, dim3(exp_grid), dim3(kExpThreads), 0, st, ea);
        CSBFS_HIP(hipGetLastError());
        hipLaunchKernelGGL(expand_big_kernel, dim3(big_grid), dim3(kExpThreads), 0, st, ea);
        CSBFS_HIP(hipGetLastError());
        if (ev) CSBFS_HIP(hipEventRecord(ev[1], st));
        // a2: mask, visit, f^{k+1}; a3: reduction of |f^{k+1}|
        UpdateArgs ua{e->T, e->pi, e->f, level, (int32_t)(k + 1), words, W, (int32_t)P,
                      e->lc.rank + sn * P, e->lc.frontier + sn, e->queue_count};
        hipLaunchKernelGGL(update_kernel, dim3(upd_grid), dim3(kUpdThreads), 0, st, ua);
        CSBFS_HIP(hipGetLastError());
        if (ev) CSBFS_HIP(hipEventRecord(ev[2], st));
        CSBFS_HIP(hipMemcpyAsync(e->host_count, e->lc.frontier + sn, sizeof(unsigned long long),
                                 hipMemcpyDeviceToHost, st));
        CSBFS_HIP(hipStreamSynchronize(st));
        if (*e->host_count == 0) break;
        // a4 + a5: sieve and compress every stream i -> j
        const int64_t arena_slot = keep ? sn : 0;
        wb.out_base = e->arena + arena_slot * S * e->cap;
        wb.n_words = e->lc.words + sn * S;
        wb.stat_sieved_bits = e->lc.sbits + sn * S;
        wb.stat_unsieved_words = e->lc.uwords + sn * P;
        rc = launch_wah_encode(wb, st);
        if (rc) return rc;
        if (ev) CSBFS_HIP(hipEventRecord(ev[3], st));
        // a6: the stream slots are the receive buffers; a7: decode into the views
        rc = launch_wah_decode(wb, st);
        if (rc) return rc;
        if (ev) CSBFS_HIP(hipEventRecord(ev[4], st));
    }
    const int64_t nl = k + 1;  // levels 0..k
    *n_levels = (int32_t)(nl < INT32_MAX ? nl : INT32_MAX);
    e->last_levels = *n_levels;

    // statistics
    int32_t hstatus = 0;
    CSBFS_HIP(hipMemcpyAsync(&hstatus, e->status, sizeof(hstatus), hipMemcpyDeviceToHost, st));
    const int64_t have = nl < e->L ? nl : e->L;
    const int64_t want = stats_cap < have ? stats_cap : have;
    std::vector<unsigned long long> fr, rk, ed, sb, uw;
    std::vector<int64_t> wd;
    if (want > 0) {
        fr.resize(want);
        ed.resize(want);
        sb.resize(want * S);
        uw.resize(want * P);
        wd.resize(want * S);
        CSBFS_HIP(hipMemcpyAsync(fr.data(), e->lc.frontier, sizeof(unsigned long long) * want,
                                 hipMemcpyDeviceToHost, st));
        CSBFS_HIP(hipMemcpyAsync(ed.data(), e->lc.edges, sizeof(unsigned long long) * want,
                                 hipMemcpyDeviceToHost, st));
        CSBFS_HIP(hipMemcpyAsync(sb.data(), e->lc.sbits, sizeof(unsigned long long) * want * S,
                                 hipMemcpyDeviceToHost, st));
        CSBFS_HIP(hipMemcpyAsync(uw.data(), e->lc.uwords, sizeof(unsigned long long) * want * P,
                                 hipMemcpyDeviceToHost, st));
        CSBFS_HIP(hipMemcpyAsync(wd.data(), e->lc.words, sizeof(int64_t) * want * S,
                                 hipMemcpyDeviceToHost, st));
    }
    CSBFS_HIP(hipStreamSynchronize(st));
    if (hstatus != 0) return fail(CSBFS_ECORRUPT, "csbfs_bfs: a stream failed validation while decoding");
    for (int64_t lv = 0; lv < want; ++lv) {
        csbfs_level_stats &s = stats[lv];
        s = csbfs_level_stats{};
        s.frontier = (int64_t)fr[lv];
        s.edges = (int64_t)ed[lv];
        if (lv > 0) {
            int64_t sieved = 0, sent = 0, self = 0, uws = 0, maxr = 0;
            for (int64_t i = 0; i < P; ++i) {
                int64_t send = 0, recv = 0;
                for (int64_t j = 0; j < P; ++j) {
                    const int64_t w_ij = wd[lv * S + i * P + j];
                    const int64_t w_ji = wd[lv * S + j * P + i];
                    if (i == j) {
                        self += 8 * w_ij;
                        continue;
                    }
                    sieved += (int64_t)sb[lv * S + i * P + j];
                    sent += 8 * w_ij;
                    send += 8 * w_ij;
                    recv += 8 * w_ji;
                }
                uws += (int64_t)uw[lv * P + i];
                if (send + recv > maxr) maxr = send + recv;
            }
            s.sieved_bits = sieved;
            s.unsieved_bits = (P - 1) * s.frontier;
            s.raw_bytes = P * (P - 1) * 8 * W;
            s.wah_unsieved_bytes = 8 * (P - 1) * uws;
            s.wah_sieved_bytes = sent;
            s.self_bytes = self;
            s.max_rank_bytes = maxr;
        }
    }
    if (timing) {
        for (int64_t lv = 0; lv < nl && lv < e->L; ++lv) {
            hipEvent_t *ev = &e->events[(size_t)lv * kEvPerLevel];
            float a = 0, b = 0;
            CSBFS_HIP(hipEventElapsedTime(&a, ev[0], ev[1]));
            CSBFS_HIP(hipEventElapsedTime(&b, ev[1], ev[2]));
            if (lv < want) {
                stats[lv].ms_expand = a;
                stats[lv].ms_update = b;
            }
            if (lv + 1 < nl && lv + 1 < want) {
                float c = 0, d = 0;
                CSBFS_HIP(hipEventElapsedTime(&c, ev[2], ev[3]));
                CSBFS_HIP(hipEventElapsedTime(&d, ev[3], ev[4]));
                stats[lv + 1].ms_compress = c;
                stats[lv + 1].ms_decode = d;
            }
        }
    }
    return CSBFS_OK;
}

extern "C" int csbfs_engine_stream_words(const csbfs_engine *e, int32_t *words, int32_t cap_levels) {
    if (!e || !words || cap_levels < 0) return fail(CSBFS_EINVAL, "csbfs_engine_stream_words: bad argument");
    const int64_t S = e->S;
    std::vector<int64_t> wd((size_t)e->L * S);
    CSBFS_HIP(hipMemcpy(wd.data(), e->lc.words, sizeof(int64_t) * e->L * S, hipMemcpyDeviceToHost));
    for (int64_t lv = 0; lv < cap_levels; ++lv)
        for (int64_t s = 0; s < S; ++s)
            words[lv * S + s] = (lv < e->L && lv < e->last_levels) ? (int32_t)wd[lv * S + s] : 0;
    return CSBFS_OK;
}

extern "C" int csbfs_engine_copy_stream(const csbfs_engine *e, int32_t k, int32_t i, int32_t j,
                                        uint64_t *dst, int64_t cap_words, int64_t *n_words_out,
                                        void *stream) {
    if (!e || !dst || !n_words_out) return fail(CSBFS_EINVAL, "csbfs_engine_copy_stream: null argument");
    if (!(e->flags & CSBFS_FLAG_KEEP_STREAMS))
        return fail(CSBFS_EINVAL, "csbfs_engine_copy_stream: engine lacks CSBFS_FLAG_KEEP_STREAMS");
    const int64_t P = e->g->P;
    if (k < 0 || k >= e->L || k >= e->last_levels || i < 0 || i >= P || j < 0 || j >= P)
        return fail(CSBFS_EINVAL, "csbfs_engine_copy_stream: level or processor out of range");
    const int64_t s = (int64_t)i * P + j;
    int64_t nw = 0;
    hipStream_t st = as_stream(stream);
    CSBFS_HIP(hipMemcpyAsync(&nw, e->lc.words + (int64_t)k * e->S + s, sizeof(int64_t),
                             hipMemcpyDeviceToHost, st));
    CSBFS_HIP(hipStreamSynchronize(st));
    *n_words_out = nw;
    if (nw > cap_words) return fail(CSBFS_ENOSPACE, "csbfs_engine_copy_stream: dst too small");
    if (nw > 0)
        CSBFS_HIP(hipMemcpyAsync(dst, e->arena + ((int64_t)k * e->S + s) * e->cap,
                                 sizeof(uint64_t) * nw, hipMemcpyDeviceToDevice, st));
    CSBFS_HIP(hipStreamSynchronize(st));
    return CSBFS_OK;
}
