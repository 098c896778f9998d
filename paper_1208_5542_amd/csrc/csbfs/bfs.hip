// The level loop of Algorithm 3 (Sec. V.B) over P virtual processors on one
// GPU. Processor i's state lives in slices of device arrays: visited bits
// pi_i and frontier piece f_i (R bits each), the "seen" bits S_i (pi_i plus
// the vertices discovered during the current level), and its P incoming
// frontier pieces f_{i,j}, the "views" (bits of R_j as received from P_j).
// Level k (launch order: update + sieve + compress, decode + reduction,
// expansion):
//
//   expand   t_i = sum_j A_{i,j} (x) f_{i,j} over the (select, max) semiring
//            (Sec. III.A: the highest-labelled frontier neighbour wins).
//            Three exact evaluations of the same product:
//              top-down (sparse): every set bit u of view (i, j) is a source
//                      whose row in block (i, j) is pushed to its targets v
//                      in R_i; an unvisited v takes u by atomicMax into
//                      parent[v], and its first discoverer sets its S bit;
//              bottom-up: every unvisited v of R_i reads its merged row
//                      (global ids in decreasing order) and stops at the
//                      first neighbour set in P_i's views: the maximum;
//              dense:  a top-down push that only sets S bits (a bitmap small
//                      enough to stay in L2), then every new v pulls its
//                      parent as in bottom-up.
//            By default each level is top-down or bottom-up: the
//            reduction applies Beamer's rule to the frontier's size and
//            adjacency entries and stores the direction (and the top-down
//            tile width) on the device, where the expansion reads it.
//   update   f_i = S_i & ~pi_i, formed while the encoder stages it (never
//            stored); pi_i = S_i (the other parity's copy); level[v] = k;
//            the views are cleared for this level's messages.
//   sieve + compress   stream i -> j = WAH-64(f_i AND V_{j,i})
//   exchange           stream slot (i, j) is P_j's receive buffer from P_i
//   decode/merge       view (j, i) |= WAH^-1(stream i -> j); the decode's
//                      first workgroup reduces |f| (read by the host) and
//                      chooses the direction.
//
// Processor i's pull reads the column of v in its block-row A_{i,*}; by the
// symmetry of A that is the row of v in blocks (j, i), which the graph keeps
// merged per vertex (the pull layout) next to the blocks.
#include <cstdlib>
#include <vector>

#include "wah_device.hpp"
#include "graph.hpp"

namespace csbfs {
namespace {

constexpr int kExpThreads = 512;
constexpr int kPullThreads = 512;
constexpr int kPullRounds = 16;  // per-lane steps (kUnroll entries each) before the wave helps
constexpr int kEvPerLevel = 4;  // before/after the update + encode, after the decode, after the expansion
constexpr int kPullTileDense = 64;  // bitmap words per wave tile of the dense pull
constexpr int kPullTileBU = 8;      // ... and of the bottom-up pull (many more candidates; 8 beat 2 and 4)
constexpr int32_t kDirTD = CSBFS_DIR_TOP_DOWN, kDirBU = CSBFS_DIR_BOTTOM_UP, kDirDense = CSBFS_DIR_DENSE;
// No frontier left: every kernel of the iteration returns at once (the
// host learns of it one iteration late, and that iteration costs nothing).
constexpr int32_t kDirIdle = 3;

struct BigItem {
    int32_t block;
    int32_t u_local;
    int32_t start;  // offsets within the block's col
    int32_t end;
};

struct ExpandArgs {
    const uint64_t *view;
    int64_t rank_words;        // view words per processor: P * W
    const int32_t *row_ptr;
    const int64_t *col_base;
    const uint32_t *col;
    const uint64_t *pi;
    uint64_t *S;
    int32_t *parent;
    BigItem *queue;
    const int64_t *qoff;       // [P + 1]: processor r's chunk queue is queue[qoff[r], qoff[r+1])
    uint32_t *queue_count;     // [P] items pushed
    int32_t tile_words;        // view words per tile (<= 64), read from *tile at kernel entry
    const int32_t *tile;       // device: tile width chosen with the level's direction
    int64_t R;
    int64_t W;
    int32_t P;
    unsigned long long *edges;
    int32_t *status;
    const int32_t *dir;        // device direction of this level; the kernels run if top-down
};


constexpr int kUnroll = 2;  // independent edges in flight per lane (2 beat 4 and 8: scale 26 237 -> 253 GTEPS)

// Relax kUnroll (target v, source u) pairs; every load is issued before any
// result is used, so their latencies overlap.
//   sparse: an unvisited v takes u by atomicMax into parent[v]; the lane
//           that finds it still without a parent also sets its seen bit.
//   dense:  v is only marked seen.
template <bool kDense>
__device__ __forceinline__ void relax_batch(const ExpandArgs &a, const int64_t (&v)[kUnroll],
                                            const int32_t (&u)[kUnroll], const bool (&ok)[kUnroll]) {
    if (kDense) {
        uint64_t w[kUnroll];
#pragma unroll
        for (int k = 0; k < kUnroll; ++k)
            w[k] = ok[k] ? __hip_atomic_load(&a.S[v[k] >> 6], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)
                         : ~0ull;
#pragma unroll
        for (int k = 0; k < kUnroll; ++k) {
            const uint64_t bit = 1ull << (v[k] & 63);
            if (!(w[k] & bit)) atomicOr((unsigned long long *)&a.S[v[k] >> 6], (unsigned long long)bit);
        }
    } else {
        uint64_t pw[kUnroll];
#pragma unroll
        for (int k = 0; k < kUnroll; ++k) pw[k] = ok[k] ? a.pi[v[k] >> 6] : ~0ull;
        int32_t old[kUnroll];
#pragma unroll
        for (int k = 0; k < kUnroll; ++k) {
            const bool need = !((pw[k] >> (v[k] & 63)) & 1);
            old[k] = need ? __hip_atomic_load(&a.parent[v[k]], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)
                          : INT32_MAX;
        }
        // The first atomicMax on a vertex comes from a lane whose load still
        // saw no parent: that lane also marks the vertex seen, so S & ~pi
        // is exactly this level's new vertices.
#pragma unroll
        for (int k = 0; k < kUnroll; ++k) {
            if (old[k] < u[k]) atomicMax(&a.parent[v[k]], u[k]);
            if (old[k] < 0)
                atomicOr((unsigned long long *)&a.S[v[k] >> 6], (unsigned long long)(1ull << (v[k] & 63)));
        }
    }
}

// A wavefront takes 64 view words at a time (lane = word). Their set bits
// are ranked across the tile and taken 64 at a time (lane = source u). Rows
// longer than kBigRow go to the chunk queue (one wave-aggregated
// reservation); the remaining edges of the 64 sources are spread evenly over
// the lanes, kUnroll edges per lane per step.
template <bool kDense>
__device__ __forceinline__ void expand_tile(const ExpandArgs &a, int32_t r, int64_t tile,
                                            unsigned long long &edges) {
    const int lane = threadIdx.x & 63;
    const int64_t wl = tile * a.tile_words + lane;
    const bool in = lane < a.tile_words && wl < a.rank_words;
    const int64_t w0 = (int64_t)r * a.rank_words + tile * a.tile_words;  // word of lane 0
    const uint64_t bits = in ? a.view[w0 + lane] : 0;
    const int cnt = __popcll(bits);
    const int incl_b = wave_incl_scan_i32(cnt);
    const int tot_b = __shfl(incl_b, 63, 64);
    const int excl_b = incl_b - cnt;
    uint32_t *qcount = a.queue_count + r;
    BigItem *queue = a.queue + a.qoff[r];
    const int64_t qcap = a.qoff[r + 1] - a.qoff[r];
    for (int base = 0; base < tot_b; base += 64) {
        const int rk = base + lane;
        const int L = owner_lane(excl_b, rk < tot_b ? rk : tot_b - 1);
        const uint64_t wb = __shfl(bits, L, 64);
        const int rr = rk - __shfl(excl_b, L, 64);
        int32_t rs = 0, deg = 0, u = 0;
        int64_t b = 0, ul = 0, gstart = 0;
        if (rk < tot_b) {
            const int64_t wi = w0 + L;
            b = wi / a.W;
            const int64_t q = wi - b * a.W;
            const int32_t j = (int32_t)(b - (int64_t)r * a.P);
            ul = (q << 6) + select_bit(wb, rr);
            const int32_t *rp = a.row_ptr + b * (a.R + 1) + ul;
            rs = rp[0];
            deg = rp[1] - rs;
            gstart = a.col_base[b] + rs;
            u = (int32_t)(j * a.R + ul);
        }
        const int32_t items = deg > kBigRow ? (deg + kBigChunk - 1) / kBigChunk : 0;
        const int32_t items_incl = wave_incl_scan_i32(items);
        const int32_t items_total = __shfl(items_incl, 63, 64);
        if (items_total) {
            uint32_t qbase = 0;
            if (lane == 63) qbase = atomicAdd(qcount, (uint32_t)items_total);
            qbase = __shfl(qbase, 63, 64);
            if (items) {
                const int64_t pos = (int64_t)qbase + items_incl - items;
                if (pos + items > qcap) {
                    *a.status = 2;  // cannot happen: the capacity bounds every row at once
                } else {
                    for (int32_t c = 0; c < items; ++c) {
                        BigItem it;
                        it.block = (int32_t)b;
                        it.u_local = (int32_t)ul;
                        it.start = rs + c * kBigChunk;
                        it.end = min(rs + deg, rs + (c + 1) * kBigChunk);
                        queue[pos + c] = it;
                    }
                }
                deg = 0;
            }
        }
        const int32_t incl = wave_incl_scan_i32(deg);
        const int32_t total = __shfl(incl, 63, 64);
        const int32_t excl = incl - deg;
        edges += (unsigned long long)total;
        const int64_t vbase = (int64_t)r * a.R;
        for (int32_t e0 = 0; e0 < total; e0 += 64 * kUnroll) {
            int64_t v[kUnroll];
            int32_t uu[kUnroll];
            bool ok[kUnroll];
            uint32_t c[kUnroll];
#pragma unroll
            for (int k = 0; k < kUnroll; ++k) {
                const int32_t e = e0 + 64 * k + lane;
                ok[k] = e < total;
                const int o = owner_lane(excl, ok[k] ? e : total - 1);
                const int64_t gs = shfl64(gstart, o);
                const int32_t ex = __shfl(excl, o, 64);
                uu[k] = __shfl(u, o, 64);
                c[k] = ok[k] ? a.col[gs + (e - ex)] : 0u;
            }
#pragma unroll
            for (int k = 0; k < kUnroll; ++k) v[k] = vbase + c[k];
            relax_batch<kDense>(a, v, uu, ok);
        }
    }
}

// A wavefront takes tiles of tile_words view words (lane = word), strided
// over the grid. The set bits of a tile are ranked and taken 64 at a time
// (lane = source u). Rows longer than kBigRow go to the processor's chunk
// queue (one wave-aggregated reservation); the remaining edges of the 64
// sources are spread evenly over the lanes, kUnroll edges per lane per step.
template <bool kDense>
__device__ __forceinline__ void expand_body(const ExpandArgs &a) {
    const int64_t wave = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) >> 6;
    const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
    const int64_t ntiles = (a.rank_words + a.tile_words - 1) / a.tile_words;
    unsigned long long edges = 0;
    for (int64_t gt = wave; gt < ntiles * a.P; gt += nwaves) {
        const int32_t r = (int32_t)(gt / ntiles);
        expand_tile<kDense>(a, r, gt - (int64_t)r * ntiles, edges);
    }
    // `total` is wave-uniform, so every lane holds the wave's edge count
    block_add<kExpThreads / 64>(edges, a.edges);
}

template <bool kDense>
__global__ __launch_bounds__(kExpThreads) void expand_kernel(ExpandArgs a) {
    const int32_t d = *a.dir;
    if (d == kDirBU || d == kDirIdle) return;
    a.tile_words = *a.tile;
    expand_body<kDense>(a);
}

// Chunk-queue items (<= kBigChunk entries of one long row) of every
// processor, strided over the grid.
template <bool kDense>
__global__ __launch_bounds__(kExpThreads) void expand_big_kernel(ExpandArgs a) {
    const int32_t d = *a.dir;
    if (d == kDirBU || d == kDirIdle) return;
    const int lane = threadIdx.x & 63;
    const int64_t wave = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) >> 6;
    const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
    unsigned long long edges = 0;
    int64_t before = 0;  // items of the processors before r, for a grid-wide stride
    for (int32_t r = 0; r < a.P; ++r) {
        const int64_t cap = a.qoff[r + 1] - a.qoff[r];
        const int64_t queued = a.queue_count[r];
        const int64_t count = queued < cap ? queued : cap;
        const BigItem *queue = a.queue + a.qoff[r];
        const int64_t vbase = (int64_t)r * a.R;
        int64_t first = (wave - before) % nwaves;
        if (first < 0) first += nwaves;
        before += count;
        for (int64_t kk = first; kk < count; kk += nwaves) {
            const BigItem it = queue[kk];
            const int64_t b = it.block;
            const int32_t j = (int32_t)(b - (int64_t)r * a.P);
            const int32_t u = (int32_t)(j * a.R + it.u_local);
            const uint32_t *colb = a.col + a.col_base[b];
            for (int32_t e0 = it.start; e0 < it.end; e0 += 64 * kUnroll) {
                int64_t v[kUnroll];
                int32_t uu[kUnroll];
                bool ok[kUnroll];
#pragma unroll
                for (int k = 0; k < kUnroll; ++k) {
                    const int32_t e = e0 + 64 * k + lane;
                    ok[k] = e < it.end;
                    v[k] = vbase + (ok[k] ? colb[e] : 0u);
                    uu[k] = u;
                }
                relax_batch<kDense>(a, v, uu, ok);
            }
            edges += (unsigned long long)(it.end - it.start);
        }
    }
    block_add<kExpThreads / 64>(edges, a.edges);
}

struct PullArgs {
    uint64_t *S;
    const uint64_t *pi;
    const uint64_t *live;  // vertices with at least one adjacency entry
    const uint64_t *view;
    const int64_t *pull_off;   // merged rows (global ids, decreasing) of every vertex
    const uint32_t *pull_col;
    int32_t *parent;
    int64_t words;  // n / 64
    int64_t R;
    int64_t W;
    int32_t P;
    int32_t tile_words;  // bitmap words per wave tile (<= 64)
    int32_t *status;
    const int32_t *dir;
    unsigned long long *edges;   // bottom-up: entries read
    unsigned long long *pulled;  // bottom-up: candidates examined
};

// Pull: a vertex v of R_i reads its merged row (the rows of v in blocks
// (j, i), j = P-1 down to 0, as global ids in decreasing order) and stops at
// the first entry set in its views: the highest-labelled frontier neighbour.
// P_i's views (i, 0..P-1) are consecutive R-bit pieces, so together they are
// one n-bit map indexed by the global id.
//   dense (second half of the dense evaluation): the candidates are the
//       vertices discovered in this level (S & ~pi); each has a frontier
//       neighbour.
//   bottom-up: the candidates are the unvisited vertices with at least one
//       adjacency entry (~pi & live); one that finds no frontier neighbour
//       stays unvisited. The found ones are gathered per bitmap word in LDS
//       and set in S by the wave that owns the word.
// A wavefront takes tile_words bitmap words at a time and ranks their
// candidates, 64 at a time (lane = v). Each lane reads kUnroll entries per
// step; lanes still searching after kPullRounds steps are finished by the
// whole wave, 64 entries per step.
template <bool kBottomUp>
__device__ __forceinline__ void pull_body(const PullArgs &a) {
    __shared__ unsigned long long found_bits[kPullThreads / 64][kPullTileBU];
    const int lane = threadIdx.x & 63;
    const int wid = threadIdx.x >> 6;
    const int64_t wave = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) >> 6;
    const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
    const int64_t tw_n = a.tile_words;  // <= kPullTileBU in bottom-up
    const int64_t ntiles = (a.words + tw_n - 1) / tw_n;
    unsigned long long read = 0, examined = 0;
    if (kBottomUp && lane < kPullTileBU) found_bits[wid][lane] = 0;
    for (int64_t tile = wave; tile < ntiles; tile += nwaves) {
        const int64_t wq = tile * tw_n + lane;
        uint64_t t = 0;
        if (lane < tw_n && wq < a.words)
            t = kBottomUp ? (a.live[wq] & ~a.pi[wq]) : (a.S[wq] & ~a.pi[wq]);
        const int cnt = __popcll(t);
        const int incl_b = wave_incl_scan_i32(cnt);
        const int tot_b = __shfl(incl_b, 63, 64);
        const int excl_b = incl_b - cnt;
        examined += (unsigned long long)tot_b;
        for (int base = 0; base < tot_b; base += 64) {
            const int r = base + lane;
            const int L = owner_lane(excl_b, r < tot_b ? r : tot_b - 1);
            const uint64_t tw = __shfl(t, L, 64);
            const int rr = r - __shfl(excl_b, L, 64);
            const bool mine = r < tot_b;
            int64_t v = 0, e = 0, re = 0;
            int bitpos = 0;
            int32_t found = -1;
            if (mine) {
                bitpos = select_bit(tw, rr);
                v = ((tile * tw_n + L) << 6) + bitpos;
                e = a.pull_off[v];
                re = a.pull_off[v + 1];
            }
            const int64_t i = v / a.R;
            const uint64_t *vw = a.view + i * a.P * a.W;  // P_i's views as one n-bit map
            bool busy = mine && e < re;
            for (int round = 0; round < kPullRounds; ++round) {
                if (busy) {
                    // every lane reads kUnroll entries, positions past the row end
                    // clamped to its last entry and masked out of the hits: the
                    // loads need no per-entry branch
                    const int32_t nk = re - e < kUnroll ? (int32_t)(re - e) : kUnroll;
                    const uint32_t *cp = a.pull_col + e;
                    uint32_t c[kUnroll];
                    uint64_t x[kUnroll];
#pragma unroll
                    for (int k = 0; k < kUnroll; ++k) c[k] = cp[k < nk ? k : nk - 1];
#pragma unroll
                    for (int k = 0; k < kUnroll; ++k) x[k] = vw[c[k] >> 6];
                    uint32_t hm = 0;
#pragma unroll
                    for (int k = 0; k < kUnroll; ++k) hm |= (uint32_t)((x[k] >> (c[k] & 63)) & 1) << k;
                    hm &= (1u << nk) - 1u;
                    if (hm) {
                        const int hit = __builtin_ctz(hm);
                        found = (int32_t)c[hit];
                        busy = false;
                        read += (unsigned long long)(hit + 1);
                    } else {
                        read += (unsigned long long)nk;
                        e += nk;
                        if (e >= re) busy = false;  // row exhausted: no frontier neighbour
                    }
                }
                if (!__ballot(busy)) break;
            }
            uint64_t slow = __ballot(busy);
            while (slow) {
                const int Ls = __ffsll((unsigned long long)slow) - 1;
                slow &= slow - 1;
                int64_t ee = shfl64(e, Ls);
                const int64_t rr2 = shfl64(re, Ls);
                const int64_t ii = shfl64(i, Ls);
                const uint64_t *vws = a.view + ii * a.P * a.W;
                int32_t got = -1;
                for (; ee < rr2; ee += 64) {
                    const int64_t pos = ee + lane;
                    bool hit = false;
                    uint32_t u = 0;
                    if (pos < rr2) {
                        u = a.pull_col[pos];
                        hit = (vws[u >> 6] >> (u & 63)) & 1;
                    }
                    const uint64_t hits = __ballot(hit);
                    if (hits) {
                        const int first = __ffsll((unsigned long long)hits) - 1;
                        got = (int32_t)__shfl((int32_t)u, first, 64);
                        if (lane == 0) read += (unsigned long long)(first + 1);
                        break;
                    }
                    if (lane == 0) read += (unsigned long long)(rr2 - ee < 64 ? rr2 - ee : 64);
                }
                if (lane == Ls) found = got;
            }
            if (mine) {
                if (found >= 0) {
                    a.parent[v] = found;
                    if (kBottomUp) atomicOr(&found_bits[wid][L], 1ull << bitpos);
                } else if (!kBottomUp) {
                    *a.status = 3;  // a vertex seen in this level has a frontier neighbour
                }
            }
        }
        if (kBottomUp) {
            // this wave owns the tile's words of S: merge the found vertices
            wave_lds_sync();
            if (lane < tw_n && wq < a.words) {
                const unsigned long long fb = found_bits[wid][lane];
                if (fb) {
                    a.S[wq] |= fb;
                    found_bits[wid][lane] = 0;
                }
            }
            wave_lds_sync();
        }
    }
    if (kBottomUp) {
        for (int d = 32; d > 0; d >>= 1) read += (unsigned long long)shfl64((int64_t)read, lane ^ d);
        block_add<kPullThreads / 64>(read, a.edges, examined, a.pulled);
    }
}

template <bool kBottomUp>
__global__ __launch_bounds__(kPullThreads) void pull_kernel(PullArgs a) {
    const int32_t d = *a.dir;
    if (kBottomUp ? d != kDirBU : d == kDirIdle) return;
    pull_body<kBottomUp>(a);
}

// One launch per level for the default (direction-optimizing) search: the
// top-down push or the bottom-up pull, as the level's direction says.
static_assert(kExpThreads == kPullThreads, "one block size for both directions");
__global__ __launch_bounds__(kExpThreads) void level_kernel(ExpandArgs ea, PullArgs pa) {
    const int32_t d = *ea.dir;
    if (d == kDirBU) {
        pull_body<true>(pa);
    } else if (d != kDirIdle) {
        ea.tile_words = *ea.tile;
        expand_body<false>(ea);
    }
}

// Direction state carried from level to level on the device.
struct DirState {
    int32_t cur;              // direction of the level expanded next
    int32_t tile;             // view words per top-down tile of that level: 64, or
                              // 16 when the frontier holds n/64 vertices or more
    unsigned long long vdeg;  // adjacency entries of the visited vertices
    unsigned long long prev;  // size of the newest frontier (compared with the next one)
};

struct DirArgs {
    DirState *st;
    int32_t *rec;   // direction recorded for level k + 1
    int64_t n;
    int64_t nnz;
    float alpha;
    float beta;
    int32_t force;  // < 0: choose by the rule; else this direction at every level
};

// Beamer's rule (Sec. VIII names direction optimization as the next step):
// m_f = entries of the new frontier, m_u = entries of unvisited vertices.
// Top-down turns bottom-up when m_f * alpha > m_u; bottom-up turns top-down
// when the frontier is below n / beta and shrinking. One thread.
__device__ void choose_direction(const DirArgs &a, unsigned long long nf, unsigned long long mf) {
    DirState s = *a.st;
    s.vdeg += mf;
    const double mu = (double)a.nnz - (double)s.vdeg;
    int32_t next = s.cur;
    if (nf == 0) {
        next = kDirIdle;
    } else if (a.force >= 0) {
        next = a.force;
    } else if (s.cur == kDirTD) {
        // only while the frontier does not shrink: near the end the unvisited
        // entries are mostly other components', and m_u alone would pull
        // (scanning those components' rows) on a frontier of a few vertices
        if (a.alpha > 0.f && (double)mf * (double)a.alpha > mu && nf >= s.prev) next = kDirBU;
    } else if ((double)nf * (double)a.beta < (double)a.n && nf < s.prev) {
        next = kDirTD;
    }
    s.prev = nf;
    s.cur = next;
    s.tile = (double)nf * 64.0 >= (double)a.n ? 16 : 64;
    *a.st = s;
    *a.rec = next;
}

constexpr int kUpdWords = 8;  // bitmap words per wavefront step of the update (8 beat 4, 16, 32)
// Groups per encoder thread of a search: 2 (segments of 1024 groups) when
// segments of 2048 would leave fewer than two workgroups per CU, else 4.
int search_enc_gpt(int64_t R, int64_t streams) {
    return streams * enc_segments(R, 4) < 2 * 256 ? 2 : 4;
}
static_assert((kEncThreads * 2 * kGroupBits) % 64 == 0, "encoder segments end on word boundaries");

// Per-workgroup sums of the update: new vertices, their adjacency entries.
__device__ __forceinline__ unsigned long long *update_sums() {
    __shared__ unsigned long long sums[2];
    return sums;
}

// The update of Alg. 3 (t = S and not pi, pi = pi or t, f = t, levels of
// the new vertices) done inside the encoder of f. The words the encoder
// stages are S & ~pi_old, so f is never stored. Beside the look-back, the
// workgroup of stream i -> j clears view (j, i) at the segment's words (the
// view that stream decodes into) and, with the other p - 1 workgroups of
// sender i's segment, takes the segment's 8-word steps round-robin: pi for
// the next level (pi_new = S), then level and adjacency-entry count of every
// new vertex (lane = vertex; all masked loads of a step in flight before
// any is summed). pi is double-buffered because every receiver's workgroup
// reads pi_old while the words are being written.
struct FrontierHook {
    const uint64_t *S;
    const uint64_t *pi_old;  // visited before level k
    uint64_t *pi_new;        // visited through level k
    uint64_t *view;
    int32_t *level;
    const int32_t *deg;
    unsigned long long *part;  // [streams * nseg][2] per-workgroup sums
    int64_t W;
    int64_t seg_words;  // bitmap words per encoder segment
    int32_t P;
    int32_t lvl;  // k

    __device__ __forceinline__ uint64_t load(const WahBatch &, int64_t, int64_t i, int64_t w) const {
        const int64_t q = i * W + w;
        return S[q] & ~pi_old[q];
    }
    __device__ __forceinline__ void init() {
        if (threadIdx.x < 2) update_sums()[threadIdx.x] = 0;
    }
    // waves 1.. of the workgroup
    __device__ void side(const WahBatch &b, int64_t s, int64_t seg, const StreamIdx &x) {
        const int t = (int)threadIdx.x - 64, nt = (int)blockDim.x - 64;
        const int lane = threadIdx.x & 63;
        const int64_t q0 = seg * seg_words;
        const int64_t q1 = seg == b.nseg - 1 ? W : (q0 + seg_words < W ? q0 + seg_words : W);
        uint64_t *vw = view + (x.j * P + x.i) * W;
        for (int64_t q = q0 + t; q < q1; q += nt) vw[q] = 0;
        const int64_t base = x.i * W;
        const int64_t nsteps = (q1 - q0 + kUpdWords - 1) / kUpdWords;
        unsigned long long cnt = 0, dsum = 0;
        for (int64_t c = x.j + (int64_t)P * (t >> 6); c < nsteps; c += (int64_t)P * (nt >> 6)) {
            const int64_t qa = q0 + c * kUpdWords;
            const int64_t qk = qa + lane;
            uint64_t tk = 0;
            if (lane < kUpdWords && qk < q1) {
                const uint64_t sq = S[base + qk];
                tk = sq & ~pi_old[base + qk];
                pi_new[base + qk] = sq;
                cnt += (unsigned long long)__popcll(tk);
            }
            int32_t d[kUpdWords];
#pragma unroll
            for (int k = 0; k < kUpdWords; ++k) {
                d[k] = 0;
                const uint64_t tw = readlane64(tk, k);
                if ((tw >> lane) & 1) {
                    const int64_t v = ((base + qa + k) << 6) + lane;
                    d[k] = deg[v];
                    level[v] = lvl;
                }
            }
#pragma unroll
            for (int k = 0; k < kUpdWords; ++k) dsum += (unsigned long long)d[k];
        }
        for (int dd = 32; dd > 0; dd >>= 1) {
            cnt += (unsigned long long)shfl64((int64_t)cnt, lane ^ dd);
            dsum += (unsigned long long)shfl64((int64_t)dsum, lane ^ dd);
        }
        if (lane == 0 && (cnt | dsum)) {
            atomicAdd(&update_sums()[0], cnt);
            atomicAdd(&update_sums()[1], dsum);
        }
    }
    // thread 0, after the workgroup's last barrier
    __device__ __forceinline__ void finish(const WahBatch &b, int64_t s, int64_t seg) {
        part[2 * (s * b.nseg + seg)] = update_sums()[0];
        part[2 * (s * b.nseg + seg) + 1] = update_sums()[1];
    }
};

// Update + sieve + compress of level k (k >= 1): one workgroup per (stream,
// segment). Returns at once once the search has ended.
template <int kGpt>
__global__ __launch_bounds__(kEncThreads) void frontier_encode_kernel(WahBatch b, FrontierHook h,
                                                                      const DirState *st) {
    if (st->cur == kDirIdle) return;
    encode_segment<kGpt>(b, h);
}

struct ReduceArgs {
    const unsigned long long *part;  // [nparts][2] sums of the update's workgroups
    int64_t nparts;
    unsigned long long *total;       // [2]: |f^k| and its adjacency entries (level counters)
    unsigned long long *host;        // pinned [2]: the same, for the host
    uint32_t *ctrs;                  // [P]: chunk-queue counts, cleared for the expansion
    int32_t P;
    DirArgs dir;
};

// Decode of level k into the views; workgroup (0, 0) first reduces the
// update's sums, stores the level's counters, writes |f^k| for the host and
// chooses the direction of the expansion of f^k. A workgroup that starts
// after that choice and finds the idle direction has an empty frontier's
// streams to decode, which set no bit: returning is the same.
__global__ __launch_bounds__(kDecThreads) void search_decode_kernel(WahBatch b, ReduceArgs r) {
    if (r.dir.st->cur == kDirIdle) return;
    if (blockIdx.x == 0 && blockIdx.y == 0) {
        unsigned long long nf = 0, mf = 0;
        for (int64_t k = threadIdx.x; k < r.nparts; k += blockDim.x) {
            nf += r.part[2 * k];
            mf += r.part[2 * k + 1];
        }
        nf = (unsigned long long)block_reduce((long long)nf, SumI64(), 0LL);
        mf = (unsigned long long)block_reduce((long long)mf, SumI64(), 0LL);
        if (threadIdx.x < r.P) r.ctrs[threadIdx.x] = 0;
        if (threadIdx.x == 0) {
            r.total[0] = nf;
            r.total[1] = mf;
            r.host[0] = nf;
            r.host[1] = mf;
            choose_direction(r.dir, nf, mf);
        }
    }
    dec_scatter_body(b);
}

// Vertices with at least one adjacency entry, one bit each.
__global__ void live_kernel(const int32_t *deg, int64_t n, uint64_t *live) {
    const int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    const uint64_t b = __ballot(v < n && deg[v] > 0);
    if ((threadIdx.x & 63) == 0 && v < n) live[v >> 6] = b;
}

struct SeedArgs {
    int32_t *level;
    int32_t *parent;
    uint64_t *pi;
    uint64_t *S;
    uint64_t *view;
    int64_t n;
    int64_t words;
    int64_t view_words;
    uint32_t *zero;      // the search's counters, flags and tickets
    int64_t zero_words;
};

__global__ void seed_fill_kernel(SeedArgs a) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    int64_t top = a.n > a.view_words ? a.n : a.view_words;
    top = top > a.zero_words ? top : a.zero_words;
    for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < top; k += stride) {
        if (k < a.zero_words) a.zero[k] = 0;
        if (k < a.n) {
            a.level[k] = -1;
            a.parent[k] = -1;
        }
        if (k < a.words) {
            a.pi[k] = 0;
            a.S[k] = 0;
        }
        if (k < a.view_words) a.view[k] = 0;
    }
}

// f(s) <- s: the source is known to every processor without a message.
__global__ void seed_root_kernel(SeedArgs a, int64_t root, int64_t R, int64_t W, int32_t P,
                                 unsigned long long *ctl0, unsigned long long *rank0,
                                 const int32_t *deg, DirState *ds, int32_t *rec0, int32_t dir0) {
    const int64_t own = root / R, rl = root - own * R;
    DirState s;
    s.cur = dir0;
    s.tile = 64;
    s.vdeg = (unsigned long long)deg[root];
    s.prev = 1;
    *ds = s;
    *rec0 = dir0;
    a.level[root] = 0;
    a.parent[root] = (int32_t)root;
    a.pi[root >> 6] |= 1ull << (root & 63);
    a.S[root >> 6] |= 1ull << (root & 63);
    for (int32_t i = 0; i < P; ++i) a.view[((int64_t)i * P + own) * W + (rl >> 6)] |= 1ull << (rl & 63);
    ctl0[0] = 1;
    rank0[own] = 1;
}


}  // namespace
}  // namespace csbfs

using namespace csbfs;

// Per-level device counters, slot k for k < L and slot L for levels past the
// engine's capacity (reset before each use).
struct LevelCounters {
    unsigned long long *ctl;     // [L+1][2]: |f^k|, sum of degrees over f^k
    unsigned long long *rank;    // [L+1][P]
    unsigned long long *edges;   // [L+1]
    unsigned long long *pulled;  // [L+1]
    unsigned long long *sbits;   // [L+1][S]
    unsigned long long *uwords;  // [L+1][P]
    int64_t *words;              // [L+1][S]
    int32_t *dir;                // [L+1]: direction used to expand f^k
};

struct csbfs_engine {
    const csbfs_graph *g = nullptr;
    int device = -1;
    int32_t L = 0;
    uint32_t flags = 0;
    int64_t S = 0, cap = 0, nseg = 0, nchunk = 0;
    int enc_gpt = 4;  // groups per encoder thread (segment size)
    uint64_t *pi[2] = {nullptr, nullptr};  // visited vertices, by level parity
    uint64_t *seen = nullptr, *view = nullptr, *arena = nullptr;
    unsigned long long *look = nullptr;  // encoder look-back words [S * nseg]
    uint32_t *enc_ticket = nullptr;      // [kTicketStride * S], after look
    size_t look_bytes = 0;
    int64_t *chunk_groups = nullptr;
    BigItem *queue = nullptr;
    uint32_t *ctrs = nullptr;     // [P]: chunk-queue items pushed
    int64_t *qoff = nullptr;      // [P + 1] chunk queue regions
    int64_t queue_cap = 0;
    void *counters_mem = nullptr;
    size_t counters_bytes = 0;
    LevelCounters lc{};
    int32_t *status = nullptr;
    unsigned long long *host_ctl = nullptr;  // pinned [2][2]: frontier counts, double-buffered
    unsigned long long *host_ctl_dev = nullptr;  // its device address
    hipEvent_t count_ev[2] = {nullptr, nullptr};
    std::vector<hipEvent_t> events;
    int32_t last_levels = 0;
    uint64_t *live = nullptr;    // [n / 64]: vertices with adjacency entries
    unsigned long long *part = nullptr;  // [S * nseg][2]: sums of the update's workgroups
    DirState *dstate = nullptr;
    // Beamer's parameters of the per-level direction choice, measured best
    // on R-MAT graphs of scale 22 (4 x 4) and 26 (8 x 8)
    float alpha = 8.0f, beta = 24.0f;
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
    if (e->host_ctl) (void)hipHostFree(e->host_ctl);
    for (hipEvent_t ev : e->count_ev)
        if (ev) (void)hipEventDestroy(ev);
    for (hipEvent_t ev : e->events)
        if (ev) (void)hipEventDestroy(ev);
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
    if (flags & ~(CSBFS_FLAG_TIMING | CSBFS_FLAG_KEEP_STREAMS | CSBFS_FLAG_NO_SIEVE |
                  CSBFS_FLAG_SPARSE_ONLY | CSBFS_FLAG_DENSE_ONLY | CSBFS_FLAG_BOTTOM_UP_ONLY))
        return fail(CSBFS_EINVAL, "csbfs_engine_create: unknown flag");
    const uint32_t modes = flags & (CSBFS_FLAG_SPARSE_ONLY | CSBFS_FLAG_DENSE_ONLY | CSBFS_FLAG_BOTTOM_UP_ONLY);
    if (modes & (modes - 1))
        return fail(CSBFS_EINVAL, "csbfs_engine_create: SPARSE_ONLY, DENSE_ONLY and BOTTOM_UP_ONLY exclude each other");
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
    e->enc_gpt = search_enc_gpt(g->R, e->S);
    if (const char *ev = std::getenv("CSBFS_ENC_GPT")) {  // fixed segment size (tests, tuning)
        if (ev[0] == '2' && ev[1] == 0) e->enc_gpt = 2;
        if (ev[0] == '4' && ev[1] == 0) e->enc_gpt = 4;
    }
    e->nseg = enc_segments(g->R, e->enc_gpt);
    e->nchunk = dec_chunks(g->R);
    const int64_t words = n / 64;
    const int64_t arena_slots = (flags & CSBFS_FLAG_KEEP_STREAMS) ? (int64_t)max_levels + 1 : 1;
    std::vector<int64_t> qoff(P + 1, 0);
    for (int64_t r = 0; r < P; ++r) qoff[r + 1] = qoff[r] + g->big_items[r];
    e->queue_cap = qoff[P] > 0 ? qoff[P] : 1;
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
    ALLOC(e->pi[0], sizeof(uint64_t) * words);
    ALLOC(e->pi[1], sizeof(uint64_t) * words);
    ALLOC(e->seen, sizeof(uint64_t) * words);
    ALLOC(e->view, sizeof(uint64_t) * P * words);
    ALLOC(e->arena, sizeof(uint64_t) * e->S * e->cap * arena_slots);
    // encoder look-back words, then its tickets: zero before the first encode
    e->look_bytes = sizeof(unsigned long long) * e->S * e->nseg + sizeof(uint32_t) * kTicketStride * e->S;
    ALLOC(e->look, e->look_bytes);
    e->enc_ticket = reinterpret_cast<uint32_t *>(e->look + e->S * e->nseg);
    ALLOC(e->chunk_groups, sizeof(int64_t) * e->S * e->nchunk);
    ALLOC(e->queue, sizeof(BigItem) * e->queue_cap);
    ALLOC(e->qoff, sizeof(int64_t) * (P + 1));
    ALLOC(e->live, sizeof(uint64_t) * words);
    ALLOC(e->part, sizeof(unsigned long long) * 2 * e->S * e->nseg);
    ALLOC(e->dstate, sizeof(DirState));
    // everything a search starts from zero, in one block the seed clears:
    // per-level counters, then the status flag, queue counts and update ticket
    const int64_t slots = (int64_t)max_levels + 1;
    const size_t cnt_bytes = sizeof(unsigned long long) * slots * (2 + P + 1 + 1 + e->S + P) +
                             sizeof(int64_t) * slots * e->S + sizeof(int32_t) * slots +
                             sizeof(int32_t) * (2 + P);
    ALLOC(e->counters_mem, cnt_bytes);
#undef ALLOC
    e->counters_bytes = cnt_bytes;
    const hipError_t zerr = hipMemset(e->look, 0, e->look_bytes);
    if (zerr != hipSuccess) {
        engine_release(e);
        return hip_fail(zerr, "hipMemset(look)", __FILE__, __LINE__);
    }
    unsigned long long *c = (unsigned long long *)e->counters_mem;
    e->lc.ctl = c;
    c += slots * 2;
    e->lc.rank = c;
    c += slots * P;
    e->lc.edges = c;
    c += slots;
    e->lc.pulled = c;
    c += slots;
    e->lc.sbits = c;
    c += slots * e->S;
    e->lc.uwords = c;
    c += slots * P;
    e->lc.words = (int64_t *)c;
    e->lc.dir = (int32_t *)(e->lc.words + slots * e->S);
    e->status = e->lc.dir + slots;
    e->ctrs = reinterpret_cast<uint32_t *>(e->status + 1);
    hipError_t herr = hipMemcpy(e->qoff, qoff.data(), sizeof(int64_t) * (P + 1), hipMemcpyHostToDevice);
    if (herr != hipSuccess) {
        engine_release(e);
        return hip_fail(herr, "hipMemcpy(qoff)", __FILE__, __LINE__);
    }
    hipLaunchKernelGGL(live_kernel, dim3(grid_for(n, 256, 1u << 30)), dim3(256), 0, 0, g->deg, n, e->live);
    herr = hipGetLastError();
    if (herr == hipSuccess) herr = hipDeviceSynchronize();
    if (herr != hipSuccess) {
        engine_release(e);
        return hip_fail(herr, "live_kernel", __FILE__, __LINE__);
    }
    herr = hipHostMalloc((void **)&e->host_ctl, 4 * sizeof(unsigned long long));
    if (herr != hipSuccess) {
        e->host_ctl = nullptr;
        engine_release(e);
        return hip_fail(herr, "hipHostMalloc", __FILE__, __LINE__);
    }
    herr = hipHostGetDevicePointer((void **)&e->host_ctl_dev, e->host_ctl, 0);
    if (herr != hipSuccess) {
        engine_release(e);
        return hip_fail(herr, "hipHostGetDevicePointer", __FILE__, __LINE__);
    }
    for (auto &ev : e->count_ev) {
        herr = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
        if (herr != hipSuccess) {
            ev = nullptr;
            engine_release(e);
            return hip_fail(herr, "hipEventCreate", __FILE__, __LINE__);
        }
    }
    if (flags & CSBFS_FLAG_TIMING) {
        e->events.assign((size_t)max_levels * kEvPerLevel, nullptr);
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

extern "C" int csbfs_engine_set_direction(csbfs_engine *e, float alpha, float beta) {
    if (!e) return fail(CSBFS_EINVAL, "csbfs_engine_set_direction: engine is NULL");
    if (!(beta > 0.f) || alpha != alpha)
        return fail(CSBFS_EINVAL, "csbfs_engine_set_direction: beta must be > 0 and alpha a number");
    e->alpha = alpha;
    e->beta = beta;
    return CSBFS_OK;
}

extern "C" int csbfs_engine_free(csbfs_engine *e) {
    if (!e) return CSBFS_OK;
    engine_release(e);
    return CSBFS_OK;
}

namespace {

inline int64_t slot_of(const csbfs_engine *e, int64_t k) { return k < e->L ? k : e->L; }

int reset_overflow_slot(csbfs_engine *e, hipStream_t st) {
    const int64_t L = e->L, P = e->g->P, S = e->S;
    CSBFS_HIP(hipMemsetAsync(e->lc.ctl + 2 * L, 0, 2 * sizeof(unsigned long long), st));
    CSBFS_HIP(hipMemsetAsync(e->lc.rank + L * P, 0, sizeof(unsigned long long) * P, st));
    CSBFS_HIP(hipMemsetAsync(e->lc.edges + L, 0, sizeof(unsigned long long), st));
    CSBFS_HIP(hipMemsetAsync(e->lc.pulled + L, 0, sizeof(unsigned long long), st));
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

    // evaluation of the product: dense, or top-down / bottom-up per level
    // (forced by a flag, or chosen on the device after every update)
    const bool dense = (e->flags & CSBFS_FLAG_DENSE_ONLY) != 0;
    const bool td_only = (e->flags & CSBFS_FLAG_SPARSE_ONLY) != 0 || (!dense && !(e->alpha > 0.f) &&
                                                                      !(e->flags & CSBFS_FLAG_BOTTOM_UP_ONLY));
    const bool bu_only = (e->flags & CSBFS_FLAG_BOTTOM_UP_ONLY) != 0;
    const int32_t force = dense ? kDirDense : td_only ? kDirTD : bu_only ? kDirBU : -1;
    const int32_t dir0 = dense ? kDirDense : bu_only ? kDirBU : kDirTD;

    // a0: seed
    SeedArgs sa{level, parent, e->pi[0], e->seen, e->view, n, words, view_words,
                (uint32_t *)e->counters_mem, (int64_t)(e->counters_bytes / sizeof(uint32_t))};
    const int64_t fill_items = n > view_words ? n : view_words;
    hipLaunchKernelGGL(seed_fill_kernel, dim3(grid_for(fill_items, 256, 8192)), dim3(256), 0, st, sa);
    CSBFS_HIP(hipGetLastError());
    hipLaunchKernelGGL(seed_root_kernel, dim3(1), dim3(1), 0, st, sa, root, R, W, (int32_t)P,
                       e->lc.ctl, e->lc.rank, (const int32_t *)g->deg, e->dstate, e->lc.dir, dir0);
    CSBFS_HIP(hipGetLastError());

    ExpandArgs ea{};
    ea.view = e->view;
    ea.rank_words = P * W;
    ea.row_ptr = g->row_ptr;
    ea.col_base = g->col_base;
    ea.col = g->col;
    ea.S = e->seen;
    ea.parent = parent;
    ea.queue = e->queue;
    ea.qoff = e->qoff;
    ea.queue_count = e->ctrs;
    ea.R = R;
    ea.W = W;
    ea.P = (int32_t)P;
    ea.status = e->status;
    ea.dir = &e->dstate->cur;
    ea.tile = &e->dstate->tile;
    ea.tile_words = 64;
    PullArgs pa{};
    pa.S = e->seen;
    pa.live = e->live;
    pa.view = e->view;
    pa.pull_off = g->pull_off;
    pa.pull_col = g->pull_col;
    pa.parent = parent;
    pa.words = words;
    pa.R = R;
    pa.W = W;
    pa.P = (int32_t)P;
    pa.status = e->status;
    pa.dir = &e->dstate->cur;
    PullArgs pb = pa;
    pa.tile_words = kPullTileDense;
    pb.tile_words = kPullTileBU;
    // grids (multiples of the XCD count) from sweeps at scales 22 and 26:
    // 512 expansion workgroups of 8 waves and 256 for the long rows (the
    // same waves as 1024 and 512 of 4, which beat 512-4096 and 512-2048)
    const unsigned exp_grid = 512, big_grid = 256;
    const unsigned pull_grid = grid_for((words + kPullTileDense - 1) / kPullTileDense, kPullThreads / 64, 16384);
    const unsigned bu_grid = grid_for((words + kPullTileBU - 1) / kPullTileBU, kPullThreads / 64, 2048);
    DirArgs da{};
    da.st = e->dstate;
    da.n = n;
    da.nnz = g->nnz;
    da.alpha = e->alpha;
    da.beta = e->beta;
    da.force = force;

    WahBatch wb{};  // the words come from FrontierHook, not from a bits buffer
    wb.mask_base = (e->flags & CSBFS_FLAG_NO_SIEVE) ? nullptr : g->dir;
    wb.nbits = R;
    wb.words_per_piece = W;
    wb.cap = e->cap;
    wb.P = (int32_t)P;
    wb.look = e->look;
    wb.ticket = e->enc_ticket;
    wb.nseg = e->nseg;
    wb.chunk_groups = e->chunk_groups;
    wb.nchunk = e->nchunk;
    wb.chunk_starts = 1;  // the decode reads the chunk starts the encode records
    wb.dst_base = e->view;
    wb.status = e->status;
    const dim3 enc_grid((unsigned)e->nseg, (unsigned)S), dec_grid((unsigned)e->nchunk, (unsigned)S);

    // Iteration j: for j >= 1 the update that forms f^j together with the
    // sieve and compression of its messages, then their decode into the views
    // (whose first workgroup reduces |f^j|, writes it to host slot j & 1 and
    // chooses the direction); then the expansion of f^j. pi[j & 1] holds the
    // vertices visited through level j.
    auto enqueue_iter = [&](int64_t j) -> int {
        const int64_t sj = slot_of(e, j);
        if (j >= e->L) {
            const int r2 = reset_overflow_slot(e, st);
            if (r2) return r2;
        }
        hipEvent_t *ev = (timing && j < e->L) ? &e->events[(size_t)j * kEvPerLevel] : nullptr;
        uint64_t *pi_j = e->pi[j & 1];
        if (ev) CSBFS_HIP(hipEventRecord(ev[0], st));
        if (j >= 1) {
            // a2 + a4 + a5: t = S & ~pi, levels, sieve and compress every stream i -> j
            const int64_t arena_slot = keep ? sj : 0;
            wb.out_base = e->arena + arena_slot * S * e->cap;
            wb.n_words = e->lc.words + sj * S;
            wb.stat_sieved_bits = e->lc.sbits + sj * S;
            wb.stat_unsieved_words = e->lc.uwords + sj * P;
            FrontierHook fh{e->seen, e->pi[(j + 1) & 1], pi_j, e->view, level, g->deg, e->part, W,
                            (int64_t)kEncThreads * e->enc_gpt * kGroupBits / 64, (int32_t)P, (int32_t)j};
            if (e->enc_gpt == 2)
                hipLaunchKernelGGL(frontier_encode_kernel<2>, enc_grid, dim3(kEncThreads), 0, st, wb, fh,
                                   (const DirState *)e->dstate);
            else
                hipLaunchKernelGGL(frontier_encode_kernel<4>, enc_grid, dim3(kEncThreads), 0, st, wb, fh,
                                   (const DirState *)e->dstate);
            CSBFS_HIP(hipGetLastError());
            if (ev) CSBFS_HIP(hipEventRecord(ev[1], st));
            // a6: the stream slots are the receive buffers; a7: decode into the
            // views; a3: reduction of |f^j|, direction of its expansion
            da.rec = e->lc.dir + sj;
            ReduceArgs ra{e->part, S * e->nseg, e->lc.ctl + 2 * sj, e->host_ctl_dev + 2 * (j & 1), e->ctrs,
                          (int32_t)P, da};
            hipLaunchKernelGGL(search_decode_kernel, dec_grid, dim3(kDecThreads), 0, st, wb, ra);
            CSBFS_HIP(hipGetLastError());
            CSBFS_HIP(hipEventRecord(e->count_ev[j & 1], st));
        } else if (ev) {
            CSBFS_HIP(hipEventRecord(ev[1], st));
        }
        if (ev) CSBFS_HIP(hipEventRecord(ev[2], st));
        ea.pi = pi_j;
        pa.pi = pi_j;
        pb.pi = pi_j;
        // a1: expand f^j (tile width and direction chosen on the device)
        ea.edges = e->lc.edges + sj;
        if (dense) {
            hipLaunchKernelGGL(expand_kernel<true>, dim3(exp_grid), dim3(kExpThreads), 0, st, ea);
            CSBFS_HIP(hipGetLastError());
            hipLaunchKernelGGL(expand_big_kernel<true>, dim3(big_grid), dim3(kExpThreads), 0, st, ea);
            CSBFS_HIP(hipGetLastError());
            hipLaunchKernelGGL(pull_kernel<false>, dim3(pull_grid), dim3(kPullThreads), 0, st, pa);
            CSBFS_HIP(hipGetLastError());
        } else if (td_only) {
            hipLaunchKernelGGL(expand_kernel<false>, dim3(exp_grid), dim3(kExpThreads), 0, st, ea);
            CSBFS_HIP(hipGetLastError());
            hipLaunchKernelGGL(expand_big_kernel<false>, dim3(big_grid), dim3(kExpThreads), 0, st, ea);
            CSBFS_HIP(hipGetLastError());
        } else {
            pb.edges = e->lc.edges + sj;
            pb.pulled = e->lc.pulled + sj;
            if (bu_only) {
                hipLaunchKernelGGL(pull_kernel<true>, dim3(bu_grid), dim3(kPullThreads), 0, st, pb);
                CSBFS_HIP(hipGetLastError());
            } else {
                // one launch: the push or the pull, as the level's direction
                // says; the long-row pass returns at once on bottom-up levels
                hipLaunchKernelGGL(level_kernel, dim3(exp_grid), dim3(kExpThreads), 0, st, ea, pb);
                CSBFS_HIP(hipGetLastError());
                hipLaunchKernelGGL(expand_big_kernel<false>, dim3(big_grid), dim3(kExpThreads), 0, st, ea);
                CSBFS_HIP(hipGetLastError());
            }
        }
        if (ev) CSBFS_HIP(hipEventRecord(ev[3], st));
        return CSBFS_OK;
    };

    // The host reads |f^k| (written by the decode of level k) while the
    // expansion of level k and iteration k + 1 are already queued. When f^k
    // is empty the decode chose the idle direction: the expansion of level k
    // and every kernel of iteration k + 1 return at once, and their counters
    // lie past the last reported level.
    rc = enqueue_iter(0);
    if (rc) return rc;
    rc = enqueue_iter(1);
    if (rc) return rc;
    int64_t k = 1;
    for (;;) {
        rc = enqueue_iter(k + 1);
        if (rc) return rc;
        CSBFS_HIP(hipEventSynchronize(e->count_ev[k & 1]));
        const unsigned long long cnt = e->host_ctl[2 * (k & 1)];
        if (cnt == 0) break;
        if (++k > n) {  // every level visits a vertex: more than n levels is a broken count
            CSBFS_HIP(hipStreamSynchronize(st));
            return fail(CSBFS_ECORRUPT, "csbfs_bfs: frontier counts did not reach zero");
        }
    }
    const int64_t nl = k;  // levels 0..k-1
    *n_levels = (int32_t)(nl < INT32_MAX ? nl : INT32_MAX);
    e->last_levels = *n_levels;

    // statistics
    int32_t hstatus = 0;
    CSBFS_HIP(hipMemcpyAsync(&hstatus, e->status, sizeof(hstatus), hipMemcpyDeviceToHost, st));
    const int64_t have = nl < e->L ? nl : e->L;
    const int64_t want = stats_cap < have ? stats_cap : have;
    std::vector<unsigned long long> ctl, ed, sb, uw, pl;
    std::vector<int64_t> wd;
    std::vector<int32_t> dr;
    if (want > 0) {
        ctl.resize(2 * want);
        ed.resize(want);
        pl.resize(want);
        dr.resize(want);
        CSBFS_HIP(hipMemcpyAsync(pl.data(), e->lc.pulled, sizeof(unsigned long long) * want,
                                 hipMemcpyDeviceToHost, st));
        CSBFS_HIP(hipMemcpyAsync(dr.data(), e->lc.dir, sizeof(int32_t) * want, hipMemcpyDeviceToHost, st));
        sb.resize(want * S);
        uw.resize(want * P);
        wd.resize(want * S);
        CSBFS_HIP(hipMemcpyAsync(ctl.data(), e->lc.ctl, sizeof(unsigned long long) * 2 * want,
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
    if (hstatus != 0) {
        // an encode that gave up waiting may have left look-back state behind
        CSBFS_HIP(hipMemsetAsync(e->look, 0, e->look_bytes, st));
        CSBFS_HIP(hipStreamSynchronize(st));
        if (hstatus == 1) return fail(CSBFS_ECORRUPT, "csbfs_bfs: a stream failed validation while decoding");
        return fail(CSBFS_ECORRUPT, "csbfs_bfs: internal consistency check failed");
    }
    for (int64_t lv = 0; lv < want; ++lv) {
        csbfs_level_stats &s = stats[lv];
        s = csbfs_level_stats{};
        s.frontier = (int64_t)ctl[2 * lv];
        s.edges = (int64_t)ed[lv];
        s.pulled = (int64_t)pl[lv];
        s.direction = dr[lv];
        s.view_bits = P;  // the source is set in every view at level 0
        if (lv > 0) {
            int64_t sieved = 0, sent = 0, self = 0, uws = 0, maxr = 0;
            s.view_bits = 0;
            for (int64_t q = 0; q < S; ++q) s.view_bits += (int64_t)sb[lv * S + q];
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
        // the update of f^k runs inside its encoder: ms_update stays 0 and
        // ms_compress holds update + sieve + compress of level k
        for (int64_t lv = 0; lv < want; ++lv) {
            hipEvent_t *ev = &e->events[(size_t)lv * kEvPerLevel];
            float c = 0, d = 0, x = 0;
            CSBFS_HIP(hipEventElapsedTime(&c, ev[0], ev[1]));
            CSBFS_HIP(hipEventElapsedTime(&d, ev[1], ev[2]));
            CSBFS_HIP(hipEventElapsedTime(&x, ev[2], ev[3]));
            stats[lv].ms_compress = c;
            stats[lv].ms_decode = d;
            stats[lv].ms_expand = x;
            stats[lv].ms_update = 0.f;
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
