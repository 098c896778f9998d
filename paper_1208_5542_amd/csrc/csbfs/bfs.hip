// The level loop of Algorithm 3 (Sec. V.B) over P virtual processors on one
// GPU. Processor i's state lives in slices of device arrays: visited bits
// pi_i (R bits), the bits N_i of the vertices discovered during the current
// expansion (two copies by level parity: one is the frontier f_i being sent
// while the other collects the next one), and its P incoming frontier
// pieces f_{i,j}, the "views" (bits of R_j as received from P_j).
// Level k (launch order: update + sieve + compress, decode + reduction,
// expansion):
//
//   expand   t_i = sum_j A_{i,j} (x) f_{i,j} over the (select, max) semiring
//            (Sec. III.A: the highest-labelled frontier neighbour wins).
//            Three exact evaluations of the same product:
//              top-down (sparse): every set bit u of view (i, j) is a source
//                      whose row in block (i, j) is pushed to its targets v
//                      in R_i; an unvisited v takes u by atomicMax into
//                      parent[v], and its first discoverer sets its N bit
//                      (atomic push); on wide levels the (v, u) pairs of
//                      the long rows are instead written into bins of 2^15
//                      targets, each resolved in LDS (binned push);
//              bottom-up: every unvisited v of R_i reads its merged row
//                      (global ids in decreasing order) and stops at the
//                      first neighbour set in P_i's views: the maximum;
//              dense:  a top-down push that only sets N bits, then every
//                      new v pulls its parent as in bottom-up.
//            By default each level is top-down or bottom-up: the
//            reduction applies Beamer's rule to the frontier's size and
//            adjacency entries and stores the direction (and the top-down
//            tile width) on the device, where the expansion reads it.
//   update   f_i = N_i (the copy the last expansion filled), staged by the
//            encoder; pi_i |= f_i; level[v] = k; the other copy of N_i
//            (the frontier before) is cleared for the next expansion; the
//            views are cleared for this level's messages.
//   sieve + compress   stream i -> j = WAH-64(f_i AND V_{j,i})
//   exchange           stream slot (i, j) is P_j's receive buffer from P_i
//   decode/merge       view (j, i) |= WAH^-1(stream i -> j); the decode's
//                      first workgroup reduces |f| (read by the host) and
//                      chooses the direction.
//
// Processor i's pull reads the column of v in its block-row A_{i,*}; by the
// symmetry of A that is the row of v in blocks (j, i), which the graph keeps
// merged per vertex (the pull layout) next to the blocks.
#include <algorithm>
#include <memory>
#include <vector>

#include "wah_device.hpp"
#include "graph.hpp"

namespace csbfs {
namespace {

constexpr int kExpThreads = 512;
constexpr int kPullThreads = 512;
constexpr int kPullRounds = 16;  // per-lane steps (kPullUnroll entries each) before the wave helps
constexpr int kPullUnroll = 2;   // entries per lane step of the pull
constexpr int kPullWindow = 4;   // row entries a lane loads at once (a multiple of kPullUnroll; 4 beat 8 and 16)
constexpr int kEvPerLevel = 5;  // before/after the update + encode, after the decode, after the
                                // main expansion kernel, after the long rows
constexpr int kPullTileDense = 64;  // bitmap words per wave tile of the dense pull
constexpr int kPullTileBU = 8;      // ... and of the bottom-up pull (many more candidates; 8 beat 2 and 4)
constexpr int32_t kDirTD = CSBFS_DIR_TOP_DOWN, kDirBU = CSBFS_DIR_BOTTOM_UP, kDirDense = CSBFS_DIR_DENSE;
// No frontier left: every kernel of the iteration returns at once (the
// host learns of it one iteration late, and that iteration costs nothing).
constexpr int32_t kDirIdle = 3;

// One chunk of a long row: its entries col[gcol, gcol + len) are the
// targets (ids local to R_r) of source u.
struct BigItem {
    int64_t gcol;
    int32_t u;      // global id of the row's source
    uint32_t rlen;  // r << 16 | len (len <= kBigChunk, r < 64)
};

// Binned push (propagation blocking: Beamer, Asanovic and Patterson, IPDPS
// 2017), for top-down levels whose frontier has many long rows. The short
// rows are relaxed by the atomic push as usual; the long-row kernel takes its
// chunk items kBinGrab at a time, turns their entries into (target v, source
// u) pairs, sorts them in LDS by bin (2^kBinShift targets per bin) and
// appends each run to its own segment of the bin (one segment per
// workgroup: no global atomics). bin_resolve_kernel then takes one bin at a
// time: the highest u per target in LDS, merged with what the atomic push
// found, and each new vertex's parent and bitmap word written once. Random
// atomics to the memory side become streamed pairs.
constexpr int kBinShift = 15;
constexpr int kBinVerts = 1 << kBinShift;
constexpr int kBinMax = 2048;                  // bins of one graph (n <= 2^26)
constexpr int kBinGrid = 512;                  // workgroups of the long-row kernel: segments per bin
constexpr int kBinGrab = 16;                   // items sorted together
constexpr int kBinBuf = kBinGrab * kBigChunk;  // their entries, at most
constexpr int kResolveThreads = 1024;
constexpr unsigned long long kBinMinEdges = 1ull << 23;  // default: bin levels with this many entries
constexpr unsigned long long kBinMinDegree = 64;         // ... and this many per frontier vertex
constexpr unsigned long long kBinNever = ~0ull;

// Block marks: one uint32 per 64 words (4096 vertices) of an n-bit map
// tells whether a level's bitmap may have a vertex there, so that the
// encoder, the top-down view scan and the clearing of old state skip the
// blocks that are all zero. Marked with plain stores of 1 (idempotent; a
// stale read only costs a repeated store). Block of global word q: q >> 6;
// view (r, j) word q holds bits of global word j * W + q, the index of that
// word within processor r's views, so one index serves both.
constexpr int kMarkShift = 6;
struct BlockMarks {
    uint32_t *m;  // [ceil(n / 4096)]
    __device__ __forceinline__ void mark_word(int64_t q) const {
        const int64_t k = q >> kMarkShift;
        if (!m[k]) m[k] = 1u;
    }
    __device__ __forceinline__ bool word_marked(int64_t q) const { return m[q >> kMarkShift] != 0; }
};

// Workgroups of a launch are dealt to the 8 XCDs round-robin (workgroup b
// runs on XCD b % 8, as a probe of the XCC id register showed), and each XCD
// has its own L2. When p divides 8, a kernel whose workgroups on XCD x all
// work for processor x % p keeps that processor's data (its n-bit view, its
// piece of the frontier) in the L2 of 8 / p XCDs instead of spreading every
// processor's data over all eight.
constexpr int kXcds = 8;
inline bool xcd_split(int64_t P, int64_t grid) { return P >= 1 && P <= kXcds && kXcds % P == 0 && grid % kXcds == 0; }

// Stream of encoder workgroup b of a one-dimensional grid of S * nseg: with
// the split, the p streams i -> 0..p-1 of sender i run on the XCDs x with
// x % p == i, taking turns, so the p workgroups that stage one segment of
// f_i (one per receiver) find its words in one L2; without it the streams
// lie one after another. `first` marks one workgroup per stream.
__device__ __forceinline__ void enc_stream_of(int64_t b, int32_t P, int64_t nseg, bool split, int64_t &s,
                                              bool &first) {
    if (!split) {
        s = b / nseg;
        first = b - s * nseg == 0;
        return;
    }
    const int x = (int)(b % kXcds);
    const int64_t kk = (b / kXcds) * (kXcds / P) + x / P;  // turn among sender x % p's workgroups
    s = (int64_t)(x % P) * P + kk % P;
    first = kk < P;
}

struct ExpandArgs {
    const uint64_t *view;
    uint64_t *view_clear;      // the same views: the push zeroes each non-zero word it takes
    BlockMarks marks_next;     // blocks of the vertices this expansion discovers
    BlockMarks marks_view;     // blocks of the frontier being expanded (its view words)
    int64_t rank_words;        // view words per processor: P * W
    const int32_t *row_ptr;
    const int64_t *col_base;
    const uint32_t *col;
    const uint64_t *pi;        // visited through the level being expanded
    uint64_t *N;               // vertices discovered by this expansion (zero at its start)
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
    // binned push (when the level's *bin is set): the long-row kernel writes
    // the pairs of the queued rows into the bins instead of relaxing them
    const int32_t *bin;        // device: this level's push is binned
    int32_t nbins;
    uint64_t *bpairs;          // [nbins][kBinGrid][cseg]: (u << 32) | (v mod 2^kBinShift)
    uint32_t *bseg;            // [nbins][kBinGrid]: pairs each workgroup wrote (may pass cseg)
    int64_t cseg;
};


constexpr int kUnroll = 2;  // independent edges in flight per lane (2 beat 4 and 8: scale 26 237 -> 253 GTEPS)
constexpr int kTilesAhead = 4;  // view tiles whose words are loaded together
constexpr int kBigUnroll = 2;   // edges in flight per lane in the long-row kernel

// Relax kUnroll (target v, source u) pairs; every load is issued before any
// result is used, so their latencies overlap.
//   sparse: an unvisited v takes u by atomicMax into parent[v]; the lane
//           that finds it still without a parent also sets its N bit.
//   dense:  an unvisited v is only marked in N.
template <bool kDense, int U>
__device__ __forceinline__ void relax_batch(const ExpandArgs &a, const int64_t (&v)[U], const int32_t (&u)[U],
                                            const bool (&ok)[U]) {
    if (kDense) {
        uint64_t w[U];
#pragma unroll
        for (int k = 0; k < U; ++k)
            w[k] = ok[k] ? (a.pi[v[k] >> 6] | __hip_atomic_load(&a.N[v[k] >> 6], __ATOMIC_RELAXED,
                                                                 __HIP_MEMORY_SCOPE_AGENT))
                         : ~0ull;
#pragma unroll
        for (int k = 0; k < U; ++k) {
            const uint64_t bit = 1ull << (v[k] & 63);
            if (!(w[k] & bit)) {
                atomicOr((unsigned long long *)&a.N[v[k] >> 6], (unsigned long long)bit);
                a.marks_next.mark_word(v[k] >> 6);
            }
        }
    } else {
        uint64_t pw[U];
#pragma unroll
        for (int k = 0; k < U; ++k) pw[k] = ok[k] ? a.pi[v[k] >> 6] : ~0ull;
        int32_t old[U];
#pragma unroll
        for (int k = 0; k < U; ++k) {
            const bool need = !((pw[k] >> (v[k] & 63)) & 1);
            old[k] = need ? __hip_atomic_load(&a.parent[v[k]], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)
                          : INT32_MAX;
        }
        // The first atomicMax on a vertex comes from a lane whose load still
        // saw no parent: that lane also sets its N bit, so N is exactly this
        // level's new vertices.
#pragma unroll
        for (int k = 0; k < U; ++k) {
            if (old[k] < u[k]) atomicMax(&a.parent[v[k]], u[k]);
            if (old[k] < 0) {
                atomicOr((unsigned long long *)&a.N[v[k] >> 6], (unsigned long long)(1ull << (v[k] & 63)));
                a.marks_next.mark_word(v[k] >> 6);
            }
        }
    }
}

// A wavefront takes 64 view words at a time (lane = word). Their set bits
// are ranked across the tile and taken 64 at a time (lane = source u). Rows
// longer than kBigRow go to the chunk queue (one wave-aggregated
// reservation); the remaining edges of the 64 sources are spread evenly over
// the lanes, kUnroll edges per lane per step.
// The view word of this lane in tile `tile` of processor r (0 past the end,
// and 0 without a load where the frontier's block mark is clear).
__device__ __forceinline__ uint64_t tile_word(const ExpandArgs &a, int32_t r, int64_t tile) {
    const int lane = threadIdx.x & 63;
    const int64_t wl = tile * a.tile_words + lane;
    const bool in = lane < a.tile_words && wl < a.rank_words && a.marks_view.word_marked(wl);
    return in ? a.view[(int64_t)r * a.rank_words + wl] : 0;
}

template <bool kDense>
__device__ __forceinline__ void expand_tile(const ExpandArgs &a, int32_t r, int64_t tile, uint64_t bits,
                                            unsigned long long &edges) {
    const int lane = threadIdx.x & 63;
    const int64_t w0 = (int64_t)r * a.rank_words + tile * a.tile_words;  // word of lane 0
    // the push reads each view word once: zero it for the next level's
    // decode (the dense evaluation's pull still reads the views after this)
    if (!kDense && bits) a.view_clear[w0 + lane] = 0;
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
                        it.gcol = gstart + (int64_t)c * kBigChunk;
                        it.u = u;
                        it.rlen = ((uint32_t)r << 16) | (uint32_t)min(deg - c * kBigChunk, kBigChunk);
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
            relax_batch<kDense, kUnroll>(a, v, uu, ok);
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
    const int lane = threadIdx.x & 63;
    const int64_t wave = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) >> 6;
    const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
    const int64_t ntiles = (a.rank_words + a.tile_words - 1) / a.tile_words;
    unsigned long long edges = 0;
    // The wave's tiles are gt = wave + i * nwaves (tile gt % ntiles of
    // processor gt / ntiles; both below 2^31). Lane i reads the block mark of
    // the wave's i-th tile of a batch of 64, so only marked tiles are read:
    // most tiles of a small frontier are empty. kTilesAhead marked tiles'
    // words are loaded before any is looked at, so their loads overlap.
    const int64_t total = ntiles * a.P;
    for (int64_t g0 = wave; g0 < total; g0 += nwaves * 64) {
        const int64_t mine = g0 + (int64_t)lane * nwaves;
        bool marked = false;
        if (mine < total) {
            const uint32_t r = (uint32_t)mine / (uint32_t)ntiles;
            const int64_t t = mine - (int64_t)r * ntiles;
            marked = a.marks_view.m[(t * a.tile_words) >> kMarkShift] != 0;
        }
        uint64_t todo = __ballot(marked);
        while (todo) {
            int32_t rs[kTilesAhead];
            int64_t ts[kTilesAhead];
            uint64_t bits[kTilesAhead];
#pragma unroll
            for (int k = 0; k < kTilesAhead; ++k) {
                rs[k] = -1;
                ts[k] = 0;
                bits[k] = 0;
                if (todo) {
                    const int idx = __ffsll((unsigned long long)todo) - 1;
                    todo &= todo - 1;
                    const int64_t gt = g0 + (int64_t)idx * nwaves;
                    const uint32_t r = (uint32_t)gt / (uint32_t)ntiles;
                    rs[k] = (int32_t)r;
                    ts[k] = gt - (int64_t)r * ntiles;
                    bits[k] = tile_word(a, (int32_t)r, ts[k]);
                }
            }
#pragma unroll
            for (int k = 0; k < kTilesAhead; ++k)
                if (rs[k] >= 0 && __ballot(bits[k] != 0)) expand_tile<kDense>(a, rs[k], ts[k], bits[k], edges);
        }
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

// Binned push, first half, in the long-row kernel (kBinGrid workgroups):
// grab g of all processors' chunk items (kBinGrab items each, in processor
// order) goes to workgroup g mod kBinGrid. A grab's entries (at most kBinBuf,
// 16 per lane) are loaded together and each pair gets its rank in its bin
// from an LDS counter; after a scan of the counts every pair is placed in
// bin order in LDS as a 32-bit key (bin, item, v mod 2^15) and written out,
// consecutive lanes to consecutive slots of this workgroup's segment of the
// bin. Pairs past a segment's capacity are relaxed by the atomic push. The
// next grab's items are loaded while the current one is sorted. At the end
// every workgroup records how many pairs it put in each bin.
__device__ void bin_emit(const ExpandArgs &a) {
    static_assert(kBinGrab <= 16 && kBinMax <= 2048 && kBinShift == 15, "key: 11 + 4 + 15 bits");
    static_assert(kBinBuf <= 65535, "16-bit offsets");
    constexpr int kPerLane = kBinBuf / kExpThreads;
    constexpr int kPer = kBinMax / kExpThreads;  // bins per thread in the scan
    __shared__ uint32_t sorted[kBinBuf];
    __shared__ uint32_t cnt[kBinMax];
    __shared__ uint16_t off[kBinMax], seg_fill[kBinMax];
    __shared__ int64_t it_col[kBinGrab];
    __shared__ int32_t it_pre[kBinGrab + 1];
    __shared__ int32_t it_u[kBinGrab];
    __shared__ uint32_t it_vb[kBinGrab];
    __shared__ int64_t qbase[64];
    __shared__ int32_t qcnt[64], gpre[65];
    __shared__ uint32_t wsum[kExpThreads / 64];
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    const int64_t G = gridDim.x;
    for (int b = tid; b < a.nbins; b += kExpThreads) {
        cnt[b] = 0;
        seg_fill[b] = 0;
    }
    if (wid == 0) {
        // per processor: where its items are, how many, and the grabs before it
        int32_t c = 0, ng = 0;
        if (lane < a.P) {
            const int64_t cap = a.qoff[lane + 1] - a.qoff[lane];
            const int64_t queued = a.queue_count[lane];
            c = (int32_t)(queued < cap ? queued : cap);
            ng = (c + kBinGrab - 1) / kBinGrab;
            qbase[lane] = a.qoff[lane];
            qcnt[lane] = c;
        }
        const int32_t inc = wave_incl_scan_i32(ng);
        gpre[lane + 1] = inc;
        if (lane == 0) gpre[0] = 0;
    }
    __syncthreads();
    const int64_t total = gpre[a.P];
    // item `lane` of grab g, for lanes below kBinGrab of wave 0
    auto fetch = [&](int64_t g, BigItem &it) -> bool {
        if (g >= total) return false;
        int32_t r = 0;
        while (gpre[r + 1] <= g) ++r;
        const int64_t idx = (g - gpre[r]) * kBinGrab + lane;
        if (idx >= qcnt[r]) return false;
        it = a.queue[qbase[r] + idx];
        return true;
    };
    BigItem nx{};
    bool nok = false;
    if (wid == 0 && lane < kBinGrab) nok = fetch(blockIdx.x, nx);
    unsigned long long edges = 0;
    for (int64_t g = blockIdx.x; g < total; g += G) {
        if (wid == 0) {
            int32_t len = 0;
            if (lane < kBinGrab && nok) {
                it_col[lane] = nx.gcol;
                it_u[lane] = nx.u;
                it_vb[lane] = (nx.rlen >> 16) * (uint32_t)a.R;
                len = (int32_t)(nx.rlen & 0xFFFFu);
            }
            const int32_t inc = wave_incl_scan_i32(len);
            if (lane < kBinGrab) it_pre[lane + 1] = inc;
            if (lane == 0) it_pre[0] = 0;
            nok = false;
            if (lane < kBinGrab) nok = fetch(g + G, nx);
        }
        __syncthreads();
        const int32_t tot = it_pre[kBinGrab];
        if (tid == 0) edges += (unsigned long long)tot;
        uint32_t c[kPerLane], key[kPerLane], rank[kPerLane];
        int32_t ix[kPerLane];
#pragma unroll
        for (int k = 0; k < kPerLane; ++k) {
            const int32_t e = tid + k * kExpThreads;
            ix[k] = -1;
            c[k] = 0;
            if (e < tot) {
                int32_t it = 0;
#pragma unroll
                for (int step = kBinGrab / 2; step > 0; step >>= 1)
                    if (it_pre[it + step] <= e) it += step;
                ix[k] = it;
                c[k] = a.col[it_col[it] + (e - it_pre[it])];
            }
        }
#pragma unroll
        for (int k = 0; k < kPerLane; ++k) {
            key[k] = 0;
            rank[k] = 0;
            if (ix[k] >= 0) {
                const uint32_t v = it_vb[ix[k]] + c[k];
                key[k] = ((v >> kBinShift) << 19) | ((uint32_t)ix[k] << 15) | (v & (uint32_t)(kBinVerts - 1));
                rank[k] = atomicAdd(&cnt[v >> kBinShift], 1u);
            }
        }
        __syncthreads();
        uint32_t loc[kPer], sum = 0;
#pragma unroll
        for (int q = 0; q < kPer; ++q) {
            const int b = tid * kPer + q;
            loc[q] = b < a.nbins ? cnt[b] : 0u;
            sum += loc[q];
        }
        const int incl = wave_incl_scan_i32((int)sum);
        if (lane == 63) wsum[wid] = (uint32_t)incl;
        __syncthreads();
        uint32_t base = (uint32_t)incl - sum;
        for (int w = 0; w < wid; ++w) base += wsum[w];
#pragma unroll
        for (int q = 0; q < kPer; ++q) {
            const int b = tid * kPer + q;
            if (b < a.nbins) off[b] = (uint16_t)base;
            base += loc[q];
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < kPerLane; ++k)
            if (ix[k] >= 0) sorted[off[key[k] >> 19] + rank[k]] = key[k];
        __syncthreads();
        for (int i = tid; i < tot; i += kExpThreads) {
            const uint32_t kk = sorted[i], b = kk >> 19;
            const int32_t it = (int32_t)((kk >> 15) & 15u);
            const uint32_t vl = kk & (uint32_t)(kBinVerts - 1);
            const int64_t slot = (int64_t)seg_fill[b] + (i - (int64_t)off[b]);
            if (slot < a.cseg) {
                a.bpairs[((int64_t)b * kBinGrid + blockIdx.x) * a.cseg + slot] = ((uint64_t)(uint32_t)it_u[it] << 32) | vl;
            } else {
                const int64_t vv[1] = {(int64_t)((b << kBinShift) | vl)};
                const int32_t uu[1] = {it_u[it]};
                const bool ok[1] = {true};
                relax_batch<false, 1>(a, vv, uu, ok);
            }
        }
        __syncthreads();  // sorted, off, seg_fill and the item table read
#pragma unroll
        for (int q = 0; q < kPer; ++q) {
            const int b = tid * kPer + q;
            if (b < a.nbins) {
                const uint32_t f = seg_fill[b] + loc[q];
                seg_fill[b] = (uint16_t)(f < 65535u ? f : 65535u);  // only compared with cseg
                cnt[b] = 0;
            }
        }
    }
    __syncthreads();
    for (int b = tid; b < a.nbins; b += kExpThreads) a.bseg[(int64_t)b * kBinGrid + blockIdx.x] = seg_fill[b];
    block_add<kExpThreads / 64>(edges, a.edges);
}

// Chunk-queue items (<= kBigChunk entries of one long row) of every
// processor, strided over the grid; with the binned push,
// their pairs go into the bins.
template <bool kDense>
__global__ __launch_bounds__(kExpThreads) void expand_big_kernel(ExpandArgs a) {
    const int32_t d = *a.dir;
    if (d == kDirBU || d == kDirIdle) return;
    if constexpr (!kDense) {
        if (*a.bin) {
            bin_emit(a);
            return;
        }
    }
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
            const int32_t len = (int32_t)(it.rlen & 0xFFFFu);
            const uint32_t *colb = a.col + it.gcol;
            for (int32_t e0 = 0; e0 < len; e0 += 64 * kBigUnroll) {
                int64_t v[kBigUnroll];
                int32_t uu[kBigUnroll];
                bool ok[kBigUnroll];
#pragma unroll
                for (int k = 0; k < kBigUnroll; ++k) {
                    const int32_t e = e0 + 64 * k + lane;
                    ok[k] = e < len;
                    v[k] = vbase + (ok[k] ? colb[e] : 0u);
                    uu[k] = it.u;
                }
                relax_batch<kDense, kBigUnroll>(a, v, uu, ok);
            }
            edges += (unsigned long long)len;
        }
    }
    block_add<kExpThreads / 64>(edges, a.edges);
}

struct PullArgs {
    uint64_t *N;           // vertices discovered in this level
    BlockMarks marks_next;  // their blocks (bottom-up)
    const uint64_t *pi;
    const uint64_t *live;  // vertices with at least one adjacency entry
    const uint64_t *view;
    const int64_t *pull_off;   // merged rows (global ids, decreasing) of every vertex
    const uint32_t *pull_col;
    const uint32_t *head;      // [2n]: the first two ids of each merged row
    int32_t *parent;
    int32_t *level;            // the found vertices' level (next_level); their
    unsigned long long *mf;    // adjacency entries (merged row lengths) are summed here
    int32_t next_level;
    int64_t words;  // n / 64
    int64_t R;
    int64_t W;
    int32_t P;
    int32_t tile_words;  // bitmap words per wave tile (<= 64)
    int32_t xcd;         // tiles of processor x % p on XCD x (p divides 8, the grid is a
                         // multiple of 8 and a processor's words a multiple of the tile)
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
//       vertices discovered in this level (N); each has a frontier
//       neighbour.
//   bottom-up: the candidates are the unvisited vertices with at least one
//       adjacency entry (~pi & live); one that finds no frontier neighbour
//       stays unvisited. The found ones are gathered per bitmap word in LDS
//       and set in N by the wave that owns the word.
// Either way the lane that finds v's parent also writes v's level and adds
// v's adjacency entries (its merged row's length) to the level's sum, so
// the update of f^(k+1) does not visit v again.
// A wavefront takes tile_words bitmap words at a time and ranks their
// candidates, 64 at a time (lane = v). Each lane reads kPullUnroll entries per
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
    // tiles tbase + u for u = u0, u0 + ustep, ... < uend: all tiles, or those of
    // processor x % p (x = this workgroup's XCD) spread over its 8 / p XCDs, so
    // that each XCD reads one processor's view (P_i's n-bit map)
    int64_t tbase = 0, u0 = wave, ustep = nwaves, uend = (a.words + tw_n - 1) / tw_n;
    if (a.xcd) {
        const int x = (int)(blockIdx.x % kXcds), c = kXcds / a.P;
        const int64_t wpw = blockDim.x >> 6;
        uend = a.W / tw_n;
        tbase = (int64_t)(x % a.P) * uend;
        u0 = ((int64_t)(blockIdx.x / kXcds) * c + x / a.P) * wpw + wid;
        ustep = (int64_t)(gridDim.x / kXcds) * c * wpw;
    }
    unsigned long long read = 0, examined = 0, mf = 0;
    if (kBottomUp && lane < kPullTileBU) found_bits[wid][lane] = 0;
    for (int64_t u = u0; u < uend; u += ustep) {
        const int64_t tile = tbase + u;
        const int64_t wq = tile * tw_n + lane;
        uint64_t t = 0;
        if (lane < tw_n && wq < a.words)
            t = kBottomUp ? (a.live[wq] & ~a.pi[wq]) : a.N[wq];
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
            uint2 hd = make_uint2(0u, 0u);
            int bitpos = 0;
            int32_t found = -1;
            if (mine) {
                bitpos = select_bit(tw, rr);
                v = ((tile * tw_n + L) << 6) + bitpos;
                e = a.pull_off[v];
                re = a.pull_off[v + 1];
                hd = *reinterpret_cast<const uint2 *>(a.head + 2 * v);
            }
            const int64_t dv = re - e;  // v's adjacency entries: its merged row is all of them
            const int64_t i = v / a.R;
            const uint64_t *vw = a.view + i * a.P * a.W;  // P_i's views as one n-bit map
            bool busy = mine && e < re;
            // the row's first two ids come from head (no row access): most
            // vertices of a wide frontier find their parent among them
            if (busy) {
                const int32_t nk = re - e < 2 ? (int32_t)(re - e) : 2;
                const uint32_t c0 = hd.x, c1 = nk > 1 ? hd.y : hd.x;
                const uint64_t x0 = vw[c0 >> 6], x1 = vw[c1 >> 6];
                uint32_t hm = (uint32_t)((x0 >> (c0 & 63)) & 1) | ((uint32_t)((x1 >> (c1 & 63)) & 1) << 1);
                hm &= (1u << nk) - 1u;
                if (hm) {
                    const int hit = __builtin_ctz(hm);
                    found = (int32_t)(hit ? c1 : c0);
                    busy = false;
                    read += (unsigned long long)(hit + 1);
                } else {
                    read += (unsigned long long)nk;
                    e += nk;
                    if (e >= re) busy = false;
                }
            }
            // kPullWindow entries of the row are loaded at once (positions past
            // the row end clamped to its last entry) and tested kPullUnroll at a
            // time, hits past the end masked out: the loads need no per-entry
            // branch, and a row's cache line is fetched once per window instead
            // of once per step
            for (int wr = 0; wr < kPullRounds * kPullUnroll / kPullWindow; ++wr) {
                uint32_t win[kPullWindow];
                if (busy) {
                    const int32_t wn = re - e < kPullWindow ? (int32_t)(re - e) : kPullWindow;
                    const uint32_t *cp = a.pull_col + e;
#pragma unroll
                    for (int k = 0; k < kPullWindow; ++k) win[k] = cp[k < wn ? k : wn - 1];
                }
#pragma unroll
                for (int h = 0; h < kPullWindow / kPullUnroll; ++h) {
                    if (busy) {
                        const int32_t nk = re - e < kPullUnroll ? (int32_t)(re - e) : kPullUnroll;
                        uint32_t c[kPullUnroll];
                        uint64_t x[kPullUnroll];
#pragma unroll
                        for (int k = 0; k < kPullUnroll; ++k) c[k] = win[h * kPullUnroll + k];
#pragma unroll
                        for (int k = 0; k < kPullUnroll; ++k) x[k] = vw[c[k] >> 6];
                        uint32_t hm = 0;
#pragma unroll
                        for (int k = 0; k < kPullUnroll; ++k) hm |= (uint32_t)((x[k] >> (c[k] & 63)) & 1) << k;
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
                    a.level[v] = a.next_level;
                    mf += (unsigned long long)dv;
                    if (kBottomUp) atomicOr(&found_bits[wid][L], 1ull << bitpos);
                } else if (!kBottomUp) {
                    *a.status = 3;  // a vertex seen in this level has a frontier neighbour
                }
            }
        }
        if (kBottomUp) {
            // this wave owns the tile's words of N: merge the found vertices
            wave_lds_sync();
            if (lane < tw_n && wq < a.words) {
                const unsigned long long fb = found_bits[wid][lane];
                if (fb) {
                    a.N[wq] |= fb;
                    a.marks_next.mark_word(wq);
                    found_bits[wid][lane] = 0;
                }
            }
            wave_lds_sync();
        }
    }
    for (int d = 32; d > 0; d >>= 1) mf += (unsigned long long)shfl64((int64_t)mf, lane ^ d);
    if (kBottomUp) {
        for (int d = 32; d > 0; d >>= 1) read += (unsigned long long)shfl64((int64_t)read, lane ^ d);
        block_add<kPullThreads / 64>(read, a.edges, examined, a.pulled);
        __syncthreads();  // block_add's LDS is used again below
    }
    block_add<kPullThreads / 64>(mf, a.mf);
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
__device__ __forceinline__ void level_body(ExpandArgs ea, const PullArgs &pa) {
    const int32_t d = *ea.dir;
    if (d == kDirBU) {
        pull_body<true>(pa);
    } else if (d != kDirIdle) {
        ea.tile_words = *ea.tile;
        expand_body<false>(ea);
    }
}

__global__ __launch_bounds__(kExpThreads) void level_kernel(ExpandArgs ea, PullArgs pa) { level_body(ea, pa); }

// The same for large graphs (kWideWords bitmap words or more): a register
// budget of 80 (6 waves per SIMD, at the price of a few spills) so that three
// workgroups share a CU, launched as kWideGrid workgroups. Scale 26: 350.4 ->
// 363.3 GTEPS (top-down push 0.25 -> 0.19 ms per search, pull 1.60 -> 1.57);
// scale 24: 276.5 -> 280.7; scale 22 loses 2-3% with it and keeps
// level_kernel.
constexpr int64_t kWideWords = int64_t(1) << 18;  // n >= 2^24
constexpr unsigned kWideGrid = 768;
__global__ __launch_bounds__(kExpThreads) __attribute__((amdgpu_waves_per_eu(6))) void level_kernel_wide(
    ExpandArgs ea, PullArgs pa) {
    level_body(ea, pa);
}

// Binned push, second half: bin b takes the highest source of each target
// from the pairs of its kBinGrid segments, in LDS. A target that is
// unvisited is new if it has such a source or the atomic push (short rows,
// and pairs past a segment) already found it (its bit in N); then its parent
// is the larger of the two, and its bitmap word is written once, by the wave
// that owns the word. A bin without pairs is already complete.
struct ResolveArgs {
    const int32_t *dir;
    const int32_t *bin;
    const uint64_t *bpairs;
    const uint32_t *bseg;
    int64_t cseg;
    int32_t nbins;
    const uint64_t *pi;
    uint64_t *N;
    BlockMarks marks_next;
    int32_t *parent;
    int64_t words;
};

__global__ __launch_bounds__(kResolveThreads) void bin_resolve_kernel(ResolveArgs a) {
    if (*a.dir != kDirTD || !*a.bin) return;
    __shared__ int32_t best[kBinVerts];
    __shared__ int32_t spre[kBinGrid + 1];
    __shared__ int32_t wtot[kResolveThreads / 64];
    constexpr int kBinMarks = kBinVerts / 64 >> kMarkShift;  // block marks of one bin (8)
    __shared__ uint32_t bmark[kBinMarks];
    constexpr int kWaves = kResolveThreads / 64;
    constexpr int kWordsPerWave = kBinVerts / 64 / kWaves;  // 32: word wid + kWaves * k of the bin
    constexpr int kPairUnroll = 8;
    static_assert(kWordsPerWave <= 64, "one word per lane");
    static_assert(kBinGrid <= kResolveThreads, "one segment count per thread");
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    // segment sizes of bin b (loaded one bin ahead)
    auto seg_size = [&](int64_t b) -> int32_t {
        if (b >= a.nbins || tid >= kBinGrid) return 0;
        const int64_t sz = a.bseg[b * kBinGrid + tid];
        return (int32_t)(sz < a.cseg ? sz : a.cseg);
    };
    int32_t cnext = seg_size(blockIdx.x);
    for (int64_t b = blockIdx.x; b < a.nbins; b += gridDim.x) {
        // segment sizes and their prefix sums
        const int32_t c = cnext;
        cnext = seg_size(b + gridDim.x);
        const int32_t incl = wave_incl_scan_i32(c);
        if (lane == 63) wtot[wid] = incl;
        __syncthreads();
        int32_t before = 0;
        for (int w = 0; w < wid; ++w) before += wtot[w];
        if (tid < kBinGrid) spre[tid + 1] = before + incl;
        if (tid == 0) spre[0] = 0;
        __syncthreads();
        const int32_t total = spre[kBinGrid];
        if (total == 0) continue;  // no pair: the atomic push did all of this bin
        const int64_t w0 = b * (kBinVerts / 64);
        // this wave's visited and atomic-push words, one per lane
        const int64_t myw = w0 + wid + (int64_t)kWaves * lane;
        const bool mine = lane < kWordsPerWave && myw < a.words;
        const uint64_t visv = mine ? a.pi[myw] : ~0ull;
        const uint64_t nv = mine ? a.N[myw] : 0ull;
        for (int i = tid; i < kBinVerts; i += kResolveThreads) best[i] = -1;
        if (tid < kBinMarks) bmark[tid] = 0;
        __syncthreads();
        const uint64_t *pb = a.bpairs + b * kBinGrid * a.cseg;
        for (int32_t i0 = 0; i0 < total; i0 += kPairUnroll * kResolveThreads) {
            uint64_t q[kPairUnroll];
            bool ok[kPairUnroll];
#pragma unroll
            for (int k = 0; k < kPairUnroll; ++k) {
                const int32_t i = i0 + k * kResolveThreads + tid;
                ok[k] = i < total;
                q[k] = 0ull;
                if (ok[k]) {
                    int32_t sg = 0;
#pragma unroll
                    for (int step = kBinGrid / 2; step > 0; step >>= 1)
                        if (spre[sg + step] <= i) sg += step;
                    q[k] = pb[sg * a.cseg + (i - spre[sg])];
                }
            }
#pragma unroll
            for (int k = 0; k < kPairUnroll; ++k)
                if (ok[k]) atomicMax(&best[q[k] & (uint64_t)(kBinVerts - 1)], (int32_t)(q[k] >> 32));
        }
        __syncthreads();
        // targets both paths reached: the atomic push's parent, all loaded first
        int32_t pk[kWordsPerWave];
#pragma unroll
        for (int k = 0; k < kWordsPerWave; ++k) {
            pk[k] = -1;
            const int64_t gw = w0 + wid + (int64_t)kWaves * k;
            const bool both = gw < a.words && ((readlane64(nv, k) >> lane) & 1) &&
                              best[(wid + kWaves * k) * 64 + lane] >= 0;
            if (both) pk[k] = a.parent[gw * 64 + lane];
        }
#pragma unroll
        for (int k = 0; k < kWordsPerWave; ++k) {
            const int64_t wl = wid + (int64_t)kWaves * k;
            const int64_t gw = w0 + wl;
            if (gw < a.words) {
                const uint64_t vis = readlane64(visv, k), old = readlane64(nv, k);
                const int32_t m = best[wl * 64 + lane];
                const bool open = !((vis >> lane) & 1);
                if (open && m >= 0) a.parent[gw * 64 + lane] = m > pk[k] ? m : pk[k];
                const uint64_t bits = __ballot(open && m >= 0) | old;
                if (lane == 0 && bits != old) {
                    a.N[gw] = bits;
                    bmark[wl >> kMarkShift] = 1u;
                }
            }
        }
        __syncthreads();  // best, spre, wtot and bmark are used again
        // the bin's block marks, one store each (no read: a set mark stays set)
        if (tid < kBinMarks && bmark[tid]) a.marks_next.m[(w0 >> kMarkShift) + tid] = 1u;
    }
}

// Direction state carried from level to level on the device.
struct DirState {
    int32_t cur;              // direction of the level expanded next
    int32_t tile;             // view words per top-down tile of that level: 64, or
                              // 16 when the frontier holds n/64 vertices or more
    int32_t bin;              // 1: that level is top-down with the binned push
    int32_t spare;
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
    // a top-down level is binned when its entries are at least bin_min
    // (kBinNever: never) and bin_deg per frontier vertex, and at most bin_cap
    unsigned long long bin_min;
    unsigned long long bin_deg;
    unsigned long long bin_cap;
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
    s.bin = next == kDirTD && a.bin_min != kBinNever && mf >= a.bin_min && mf >= a.bin_deg * nf &&
            mf <= a.bin_cap;
    *a.st = s;
    *a.rec = next | (s.bin << 8);  // direction, and the binned push in bit 8
}

// decode workgroups per stream, each looping over chunks: 12, with a register
// budget of 80 (three workgroups per CU; 97 registers gave two): scale 26
// 362.0 -> 368.3 GTEPS (decode 0.272 -> 0.233 ms per search), scale 22
// 158.5 -> 160.2; at two per CU 8 had beaten 16, 32 and 64
constexpr int64_t kDecGridChunks = 12;
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

// The update of Alg. 3 (t = the new vertices, pi = pi or t, f = t, levels
// of the new vertices) done inside the encoder of f. The words the encoder
// stages are N_cur, filled by the last expansion; segments whose mark says
// N_cur is zero there are not staged at all (the encoder's clean path).
// Beside the look-back, the workgroup of stream i -> j clears view (j, i)
// at the segment's words (the view that stream decodes into) if they can
// hold bits of f^(k-1) that the last expansion did not zero, and, with the
// other p - 1 workgroups of sender i's segment, takes the segment's 8-word
// steps round-robin: pi |= f, the other copy N_old (the previous frontier)
// cleared for the next expansion, then, if f came from a push (a pull did it
// already), level and adjacency-entry count of every new vertex (lane =
// vertex; all masked loads of a step in flight before any is summed). Each word is taken by one lane, and no workgroup
// of this launch reads pi or N_old, so the plain read-modify-writes need no
// atomics.
struct FrontierHook {
    const uint64_t *N_cur;   // f^k: vertices discovered while expanding f^(k-1)
    uint64_t *N_old;         // f^(k-1): cleared here, refilled by the next expansion
    uint64_t *pi;            // visited; pi |= f^k
    uint64_t *view;
    int32_t *level;
    const int32_t *deg;
    unsigned long long *part;  // [streams * nseg][2] per-workgroup sums
    BlockMarks mark_cur;       // blocks where f^k may have a vertex
    BlockMarks mark_old;       // blocks where f^(k-1) may have had one
    int64_t W;
    int64_t seg_words;  // bitmap words per encoder segment
    int32_t P;
    int32_t lvl;  // k
    int32_t clear_views;  // the expansion of f^(k-1) left its view words in place
    int32_t write_levels;  // the expansion of f^(k-1) was a push: levels and entries of f^k here

    __device__ __forceinline__ uint64_t load(const WahBatch &, int64_t, int64_t i, int64_t w) const {
        return N_cur[i * W + w];
    }
    __device__ __forceinline__ int64_t seg_end(const WahBatch &b, int64_t seg) const {
        const int64_t q0 = seg * seg_words;
        return seg == b.nseg - 1 ? W : (q0 + seg_words < W ? q0 + seg_words : W);
    }
    // the whole workgroup: is every block of sender i's segment unmarked?
    __device__ __forceinline__ bool clean(const WahBatch &b, int64_t seg, const StreamIdx &x) const {
        const int64_t g0 = x.i * W + seg * seg_words, g1 = x.i * W + seg_end(b, seg);
        const int64_t k0 = g0 >> kMarkShift, k1 = (g1 - 1) >> kMarkShift;
        int any = 0;
        for (int64_t k = k0 + threadIdx.x; k <= k1; k += blockDim.x) any |= mark_cur.m[k] != 0;
        return !__syncthreads_or(any);
    }
    // thread 0: is the group before the segment (its last bits) surely zero?
    __device__ __forceinline__ bool prev_clean(const WahBatch &b, int64_t seg, const StreamIdx &x) const {
        if (seg == 0) return false;
        const int64_t gx = seg * (seg_words * 64 / kGroupBits) - 1;  // the segment's first group, minus one
        const int64_t w0 = x.i * W + (gx * kGroupBits >> 6), w1 = x.i * W + ((gx * kGroupBits + kGroupBits - 1) >> 6);
        return !mark_cur.word_marked(w0) && !mark_cur.word_marked(w1);
    }
    __device__ __forceinline__ void init() {
        if (threadIdx.x < 2) update_sums()[threadIdx.x] = 0;
    }
    // waves 1.. of the workgroup
    __device__ void side(const WahBatch &b, int64_t s, int64_t seg, const StreamIdx &x) {
        const int t = (int)threadIdx.x - 64, nt = (int)blockDim.x - 64;
        const int lane = threadIdx.x & 63;
        const int64_t q0 = seg * seg_words;
        const int64_t q1 = seg_end(b, seg);
        const int64_t base = x.i * W;
        if (clear_views) {
            // one 64-word block per wave at a time (lane = word); the marks of
            // 64 of the wave's blocks are loaded at once first
            uint64_t *vw = view + (x.j * P + x.i) * W;
            const int wv = t >> 6, nwv = nt >> 6;
            const int64_t k0 = (base + q0) >> kMarkShift, k1 = (base + q1 - 1) >> kMarkShift;
            for (int64_t kb = k0 + wv; kb <= k1; kb += (int64_t)nwv * 64) {
                const int64_t mk = kb + (int64_t)lane * nwv;
                uint64_t todo = __ballot(mk <= k1 && mark_old.m[mk] != 0);
                while (todo) {
                    const int sl = __ffsll((unsigned long long)todo) - 1;
                    todo &= todo - 1;
                    const int64_t q = ((kb + (int64_t)sl * nwv) << kMarkShift) + lane - base;
                    if (q >= q0 && q < q1) vw[q] = 0;
                }
            }
        }
        const int64_t nsteps = (q1 - q0 + kUpdWords - 1) / kUpdWords;
        const int64_t wstride = (int64_t)P * (nt >> 6);  // steps between one wave's consecutive steps
        constexpr int kSlots = 64 / kUpdWords;           // the wave's steps taken at once
        unsigned long long cnt = 0, dsum = 0;
        // lane = step slot * kUpdWords + word: all of a wave's loads of
        // kSlots steps are issued together rather than step after step
        for (int64_t cb = x.j + (int64_t)P * (t >> 6); cb < nsteps; cb += wstride * kSlots) {
            const int64_t c = cb + (int64_t)(lane / kUpdWords) * wstride;
            const int64_t qk = q0 + c * kUpdWords + (lane % kUpdWords);
            uint64_t tk = 0;
            if (c < nsteps && qk < q1) {
                if (mark_cur.word_marked(base + qk)) {
                    tk = N_cur[base + qk];
                    if (tk) pi[base + qk] |= tk;
                }
                if (mark_old.word_marked(base + qk) && N_old[base + qk]) N_old[base + qk] = 0;
                cnt += (unsigned long long)__popcll(tk);
            }
            if (!write_levels || !__ballot(tk != 0)) continue;
            // levels and adjacency entries of the new vertices, kUpdWords
            // words at a time (lane = vertex of the word)
            for (int gs = 0; gs < kSlots; ++gs) {
                uint64_t tw[kUpdWords];
                uint64_t any = 0;
#pragma unroll
                for (int k = 0; k < kUpdWords; ++k) {
                    tw[k] = readlane64(tk, gs * kUpdWords + k);
                    any |= tw[k];
                }
                if (!any) continue;
                int32_t d[kUpdWords];
#pragma unroll
                for (int k = 0; k < kUpdWords; ++k) {
                    d[k] = 0;
                    if ((tw[k] >> lane) & 1) {
                        const int64_t qw = (int64_t)readlane64((uint64_t)qk, gs * kUpdWords + k);
                        const int64_t v = ((base + qw) << 6) + lane;
                        d[k] = deg[v];
                        level[v] = lvl;
                    }
                }
#pragma unroll
                for (int k = 0; k < kUpdWords; ++k) dsum += (unsigned long long)d[k];
            }
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
__device__ __forceinline__ void frontier_encode_body(const WahBatch &b, FrontierHook &h, const DirState *st,
                                                     int32_t split) {
    const int32_t d = st->cur;  // the direction f^(k-1) was expanded in
    if (d == kDirIdle) return;
    h.clear_views = d != kDirTD;  // the sparse push zeroes the view words it reads
    h.write_levels = d == kDirTD;  // a pull wrote the levels of the vertices it found
    int64_t s;
    bool first;
    enc_stream_of(blockIdx.x, b.P, b.nseg, split != 0, s, first);
    encode_segment<kGpt>(b, h, s, first);
}

// Segments of 1024 groups: the grids of smaller graphs (fewer workgroups than
// the GPU holds), where the register budget below only costs spills.
__global__ __launch_bounds__(kEncThreads) void frontier_encode_kernel_g2(WahBatch b, FrontierHook h,
                                                                      const DirState *st, int32_t split) {
    frontier_encode_body<2>(b, h, st, split);
}

// Segments of 2048 groups, for large graphs: 8 waves per SIMD (the 106
// scalar registers it would take allow 7; the spilled ones go to vector
// lanes) so that four workgroups share a CU, their 37 KiB of LDS each
// fitting. Scale 26, 16 roots: encoder 0.532 -> 0.497 ms per search, 367.6
// -> 373.1 GTEPS.
__global__ __launch_bounds__(kEncThreads) __attribute__((amdgpu_waves_per_eu(8))) void frontier_encode_kernel_g4(
    WahBatch b, FrontierHook h, const DirState *st, int32_t split) {
    frontier_encode_body<4>(b, h, st, split);
}

struct ReduceArgs {
    const unsigned long long *part;  // [nparts][2] sums of the update's workgroups
    int64_t nparts;
    unsigned long long *total;       // [2]: |f^k| and its adjacency entries (level counters)
    unsigned long long *host;        // pinned host word (level k << 32 | |f^k|), or null
    uint32_t *ctrs;                  // [P]: chunk-queue counts, cleared for the expansion
    int32_t P;
    int32_t level;                   // k
    uint32_t *marks_clear;           // [nmarks]: the marks of f^(k-1), cleared for the next expansion
    int64_t nmarks;
    unsigned long long *exp_mf;      // entries of the vertices a pull found, cleared here
    DirArgs dir;
};

// Decode of level k into the views; workgroup (0, 0) first reduces the
// update's sums, stores the level's counters, writes |f^k| for the host and
// chooses the direction of the expansion of f^k. A workgroup that starts
// after that choice and finds the idle direction has an empty frontier's
// streams to decode, which set no bit: returning is the same.
__global__ __launch_bounds__(kDecThreads) __attribute__((amdgpu_waves_per_eu(6))) void search_decode_kernel(WahBatch b, ReduceArgs r) {
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
        for (int64_t k = threadIdx.x; k < r.nmarks; k += blockDim.x) r.marks_clear[k] = 0;
        if (threadIdx.x == 0) {
            mf += *r.exp_mf;  // f^k came from a pull: its entries were summed there
            *r.exp_mf = 0;
            r.total[0] = nf;
            r.total[1] = mf;
            // one 64-bit word (level tag, |f^k|) so the host sees both or neither
            if (r.host)
                __hip_atomic_store(r.host, ((unsigned long long)r.level << 32) | nf, __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_SYSTEM);
            choose_direction(r.dir, nf, mf);
        }
    }
    // the grid holds at most kDecGridChunks workgroups per stream, each
    // taking every kDecGridChunks-th chunk up to the stream's end (a small
    // frontier's streams are a few words: most chunk slots hold nothing)
    const int64_t nw = b.n_words[blockIdx.y];
    for (int64_t c = blockIdx.x; c < b.nchunk; c += gridDim.x) {
        if (c > 0 && c * kDecChunk >= nw) break;
        dec_scatter_body(b, c);
    }
}

struct SeedArgs {
    int32_t *level;
    int32_t *parent;
    uint64_t *pi;
    uint64_t *N0;
    uint64_t *N1;
    uint64_t *view;
    int64_t n;
    int64_t words;
    int64_t view_words;
    uint32_t *zero;      // the search's counters and flags
    int64_t zero_words;
    uint32_t *look;      // encoder look-back words and tickets (any contents in a new workspace)
    int64_t look_words;
    uint32_t *marks;     // both levels' segment marks [2 * nmarks]
    int64_t mark_words;
};

__global__ void seed_fill_kernel(SeedArgs a) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    int64_t top = a.n > a.view_words ? a.n : a.view_words;
    top = top > a.zero_words ? top : a.zero_words;
    top = top > a.look_words ? top : a.look_words;
    top = top > a.mark_words ? top : a.mark_words;
    for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < top; k += stride) {
        if (k < a.zero_words) a.zero[k] = 0;
        if (k < a.look_words) a.look[k] = 0;
        if (k < a.mark_words) a.marks[k] = 0;
        if (k < a.n) {
            a.level[k] = -1;
            a.parent[k] = -1;
        }
        if (k < a.words) {
            a.pi[k] = 0;
            a.N0[k] = 0;
            a.N1[k] = 0;
        }
        if (k < a.view_words) a.view[k] = 0;
    }
}

// f(s) <- s: the source is known to every processor without a message.
__global__ void seed_root_kernel(SeedArgs a, int64_t root, int64_t R, int64_t W, int32_t P,
                                 unsigned long long *ctl0, unsigned long long *rank0,
                                 const int32_t *deg, DirState *ds, int32_t *rec0, int32_t dir0,
                                 BlockMarks marks0) {
    const int64_t own = root / R, rl = root - own * R;
    DirState s;
    s.cur = dir0;
    s.tile = 64;
    s.bin = 0;
    s.spare = 0;
    s.vdeg = (unsigned long long)deg[root];
    s.prev = 1;
    *ds = s;
    *rec0 = dir0;
    a.level[root] = 0;
    a.parent[root] = (int32_t)root;
    a.pi[root >> 6] |= 1ull << (root & 63);
    for (int32_t i = 0; i < P; ++i) a.view[((int64_t)i * P + own) * W + (rl >> 6)] |= 1ull << (rl & 63);
    marks0.mark_word(root >> 6);  // f^0's block, so its views are scanned and later cleared
    ctl0[0] = 1;
    rank0[own] = 1;
}


}  // namespace
}  // namespace csbfs

using namespace csbfs;


namespace csbfs {
namespace {

// Per-level device counters, slot k for k < L and slot L for levels past the
// workspace's capacity (reset before each use).
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

// Where every buffer of one search lives inside its workspace, and the
// search's parameters; a function of (n, p, adjacency total, config) only.
struct SearchLayout {
    int64_t n, P, R, W, S, cap, nseg, nchunk, words, L, arena_slots, queue_cap;
    int64_t nbins, cseg, bin_cap;  // binned push: bins, pairs per segment, pairs in all
    unsigned long long bin_min, bin_deg, bin_limit;  // a level's entries: at least, per frontier vertex, at most
    int enc_gpt;  // groups per encoder thread: segments of 512 * enc_gpt groups
    uint32_t flags;
    float alpha, beta;
    // byte offsets
    int64_t seg_words, nmarks;  // bitmap words per encoder segment; block marks per level
    int64_t pi, nb0, nb1, view, arena, look, look_bytes, chunk_groups, queue, part, dstate, marks, bpairs, bseg,
        counters, counters_bytes, total;
};

// Pointers into one workspace.
struct SearchState {
    uint64_t *pi;    // visited
    uint64_t *nb[2];  // new vertices, by level parity: nb[k & 1] holds f^k
    uint64_t *view, *arena;
    unsigned long long *look;  // look-back words [S * nseg], then tickets [kTicketStride * S]
    uint32_t *enc_ticket;
    int64_t *chunk_groups;
    BigItem *queue;
    unsigned long long *part;  // [S * nseg][2]: sums of the update's workgroups
    DirState *dstate;
    void *counters_mem;
    LevelCounters lc;
    int32_t *status;
    uint32_t *ctrs;  // [P]: chunk-queue items pushed
    uint64_t *bpairs;
    uint32_t *bseg;
    uint32_t *marks[2];  // block marks by level parity: marks[k & 1] for f^k
    unsigned long long *exp_mf;  // adjacency entries of the vertices a pull found (one level)
};

constexpr uint32_t kSearchFlags = CSBFS_FLAG_KEEP_STREAMS | CSBFS_FLAG_NO_SIEVE | CSBFS_FLAG_SPARSE_ONLY |
                                  CSBFS_FLAG_DENSE_ONLY | CSBFS_FLAG_BOTTOM_UP_ONLY | CSBFS_FLAG_BINNED_PUSH |
                                  CSBFS_FLAG_ATOMIC_PUSH;

int search_layout(int64_t n, int32_t p, int64_t nnz, const csbfs_search_config *cfg, SearchLayout *out) {
    csbfs_search_config c{};
    if (cfg) c = *cfg;
    if (c.flags & ~kSearchFlags) return fail(CSBFS_EINVAL, "search config: unknown or unsupported flag");
    const uint32_t modes = c.flags & (CSBFS_FLAG_SPARSE_ONLY | CSBFS_FLAG_DENSE_ONLY | CSBFS_FLAG_BOTTOM_UP_ONLY);
    if (modes & (modes - 1))
        return fail(CSBFS_EINVAL, "search config: SPARSE_ONLY, DENSE_ONLY and BOTTOM_UP_ONLY exclude each other");
    if (c.max_levels == 0) c.max_levels = 64;
    if (c.max_levels < 1 || c.max_levels > 65536)
        return fail(CSBFS_EINVAL, "search config: max_levels outside [1, 65536]");
    if (c.alpha != c.alpha || c.beta != c.beta || c.beta < 0.f)
        return fail(CSBFS_EINVAL, "search config: alpha must be a number and beta >= 0");
    if (c.segment_groups != 0 && c.segment_groups != 1024 && c.segment_groups != 2048)
        return fail(CSBFS_EINVAL, "search config: segment_groups must be 0, 1024 or 2048");
    if ((c.flags & CSBFS_FLAG_BINNED_PUSH) && (c.flags & CSBFS_FLAG_ATOMIC_PUSH))
        return fail(CSBFS_EINVAL, "search config: BINNED_PUSH and ATOMIC_PUSH exclude each other");
    if (c.push_bin_pairs < 0) return fail(CSBFS_EINVAL, "search config: push_bin_pairs must be >= 0");
    SearchLayout y{};
    y.n = n;
    y.P = p;
    y.R = n / p;
    y.W = y.R / 64;
    y.S = (int64_t)p * p;
    y.cap = wah_cap(y.R);
    y.enc_gpt = c.segment_groups == 1024 ? 2 : c.segment_groups == 2048 ? 4 : search_enc_gpt(y.R, y.S);
    y.nseg = enc_segments(y.R, y.enc_gpt);
    y.seg_words = (int64_t)kEncThreads * y.enc_gpt * kGroupBits / 64;
    y.nchunk = dec_chunks(y.R);
    y.words = n / 64;
    y.nmarks = (y.words + 63) >> kMarkShift;
    y.L = c.max_levels;
    y.arena_slots = (c.flags & CSBFS_FLAG_KEEP_STREAMS) ? y.L + 1 : 1;
    y.queue_cap = big_items_bound(nnz);
    // binned push: bins of 2^kBinShift targets, kBinGrid segments per bin, the
    // capacity split evenly (64-byte segments). By default a level is binned
    // only with half the capacity to spare, and only on graphs where such a
    // level can pass the entry threshold twice over (else there are no bins,
    // and no resolve launches); BINNED_PUSH bins any top-down level that fits.
    // No bins with ATOMIC_PUSH or above kBinMax bins.
    const bool forced = (c.flags & CSBFS_FLAG_BINNED_PUSH) != 0;
    const int64_t cap0 = c.push_bin_pairs > 0 ? c.push_bin_pairs : nnz / 8 + 65536;
    y.nbins = (n + kBinVerts - 1) >> kBinShift;
    if ((c.flags & CSBFS_FLAG_ATOMIC_PUSH) || y.nbins > kBinMax) y.nbins = 0;
    if (!forced && (unsigned long long)cap0 / 2 < 2 * kBinMinEdges) y.nbins = 0;
    if (y.nbins) {
        y.bin_cap = cap0;
        y.cseg = ((y.bin_cap + y.nbins * kBinGrid - 1) / (y.nbins * kBinGrid) + 7) / 8 * 8;
        // a workgroup counts its pairs per bin in 16 bits, saturating at
        // 65535: segments stay below that, so every pair counted past a
        // segment's end goes to the atomic push
        y.cseg = std::min<int64_t>(y.cseg, 65528);
        y.bin_min = forced ? 0ull : kBinMinEdges;
        y.bin_deg = forced ? 0ull : kBinMinDegree;
        y.bin_limit = (unsigned long long)(forced ? y.bin_cap : y.bin_cap / 2);
    } else {
        y.bin_cap = y.cseg = 0;
        y.bin_min = kBinNever;
        y.bin_deg = y.bin_limit = 0;
    }
    y.flags = c.flags;
    // Beamer's parameters of the per-level direction choice, measured best
    // on R-MAT graphs of scale 22 (4 x 4) and 26 (8 x 8): beta 48 keeps a
    // shrinking frontier of a few million low-degree vertices bottom-up,
    // where the pull finds the few remaining vertices cheaply
    y.alpha = c.alpha == 0.f && c.beta == 0.f ? 16.0f : c.alpha;
    y.beta = c.beta == 0.f ? 48.0f : c.beta;
    int64_t o = 0;
    auto take = [&o](int64_t bytes) {
        const int64_t at = o;
        o += align_up(bytes > 0 ? bytes : 1);
        return at;
    };
    y.pi = take(8 * y.words);
    y.nb0 = take(8 * y.words);
    y.nb1 = take(8 * y.words);
    y.view = take(8 * y.P * y.words);
    y.arena = take(8 * y.S * y.cap * y.arena_slots);
    y.look_bytes = 8 * y.S * y.nseg + 4 * kTicketStride * y.S;
    y.look = take(y.look_bytes);
    y.chunk_groups = take(8 * y.S * y.nchunk);
    y.queue = take((int64_t)sizeof(BigItem) * y.queue_cap);
    y.part = take(16 * y.S * y.nseg);
    y.dstate = take((int64_t)sizeof(DirState));
    y.marks = take(4 * 2 * y.nmarks);
    y.bpairs = take(8 * y.nbins * kBinGrid * y.cseg);
    y.bseg = take(4 * y.nbins * kBinGrid);
    // everything a search starts from zero, in one block the seed clears:
    // per-level counters, then the status flag and the queue counts
    const int64_t slots = y.L + 1;
    y.counters_bytes = 8 + 8 * slots * (2 + y.P + 1 + 1 + y.S + y.P) + 8 * slots * y.S + 4 * slots + 4 * (2 + y.P);
    y.counters_bytes = (y.counters_bytes + 3) / 4 * 4;
    y.counters = take(y.counters_bytes);
    y.total = o;
    *out = y;
    return CSBFS_OK;
}

SearchState bind_workspace(const SearchLayout &y, void *ws) {
    char *b = (char *)ws;
    SearchState w{};
    w.pi = (uint64_t *)(b + y.pi);
    w.nb[0] = (uint64_t *)(b + y.nb0);
    w.nb[1] = (uint64_t *)(b + y.nb1);
    w.view = (uint64_t *)(b + y.view);
    w.arena = (uint64_t *)(b + y.arena);
    w.look = (unsigned long long *)(b + y.look);
    w.enc_ticket = reinterpret_cast<uint32_t *>(w.look + y.S * y.nseg);
    w.chunk_groups = (int64_t *)(b + y.chunk_groups);
    w.queue = (BigItem *)(b + y.queue);
    w.part = (unsigned long long *)(b + y.part);
    w.dstate = (DirState *)(b + y.dstate);
    w.marks[0] = (uint32_t *)(b + y.marks);
    w.marks[1] = w.marks[0] + y.nmarks;
    w.counters_mem = b + y.counters;
    const int64_t slots = y.L + 1, P = y.P, S = y.S;
    unsigned long long *c = (unsigned long long *)w.counters_mem;
    w.exp_mf = c++;
    w.lc.ctl = c;
    c += slots * 2;
    w.lc.rank = c;
    c += slots * P;
    w.lc.edges = c;
    c += slots;
    w.lc.pulled = c;
    c += slots;
    w.lc.sbits = c;
    c += slots * S;
    w.lc.uwords = c;
    c += slots * P;
    w.lc.words = (int64_t *)c;
    w.lc.dir = (int32_t *)(w.lc.words + slots * S);
    w.status = w.lc.dir + slots;
    w.ctrs = reinterpret_cast<uint32_t *>(w.status + 1);
    w.bpairs = (uint64_t *)(b + y.bpairs);
    w.bseg = (uint32_t *)(b + y.bseg);
    return w;
}

inline int64_t slot_of(const SearchLayout &y, int64_t k) { return k < y.L ? k : y.L; }

int reset_overflow_slot(const SearchLayout &y, const SearchState &w, hipStream_t st) {
    const int64_t L = y.L, P = y.P, S = y.S;
    CSBFS_HIP(hipMemsetAsync(w.lc.ctl + 2 * L, 0, 2 * sizeof(unsigned long long), st));
    CSBFS_HIP(hipMemsetAsync(w.lc.rank + L * P, 0, sizeof(unsigned long long) * P, st));
    CSBFS_HIP(hipMemsetAsync(w.lc.edges + L, 0, sizeof(unsigned long long), st));
    CSBFS_HIP(hipMemsetAsync(w.lc.pulled + L, 0, sizeof(unsigned long long), st));
    CSBFS_HIP(hipMemsetAsync(w.lc.sbits + L * S, 0, sizeof(unsigned long long) * S, st));
    CSBFS_HIP(hipMemsetAsync(w.lc.uwords + L * P, 0, sizeof(unsigned long long) * P, st));
    return CSBFS_OK;
}

// Host side of the frontier-size readback. With a pinned mailbox the decode
// of level k stores (k << 32 | |f^k|) in word k & 1 and the host polls it;
// without one the host copies the level's counter back after the stream has
// drained (one round trip per level).
struct Mailbox {
    volatile unsigned long long *host = nullptr;  // pinned, two words, or null
    unsigned long long *dev = nullptr;            // its device address
};

int wait_count(const Mailbox &mb, const SearchLayout &y, const SearchState &w, int64_t k, hipStream_t st,
               unsigned long long *cnt) {
    if (mb.host) {
        const unsigned long long want = (unsigned long long)k & 0xffffffffull;
        uint64_t spins = 0;
        for (;;) {
            const unsigned long long v = mb.host[k & 1];
            if ((v >> 32) == want) {
                *cnt = v & 0xffffffffull;
                return CSBFS_OK;
            }
            if ((++spins & 0x3ff) == 0) {
                // a failed launch never writes the word: ask the stream
                const hipError_t q = hipStreamQuery(st);
                if (q != hipSuccess && q != hipErrorNotReady) return hip_fail(q, "search stream", __FILE__, __LINE__);
                if (q == hipSuccess) {
                    // the stream drained: the word must be there now
                    const unsigned long long v2 = mb.host[k & 1];
                    if ((v2 >> 32) != want)
                        return fail(CSBFS_ECORRUPT, "csbfs_bfs: frontier count of a level never arrived");
                    *cnt = v2 & 0xffffffffull;
                    return CSBFS_OK;
                }
            }
        }
    }
    unsigned long long v = 0;
    CSBFS_HIP(hipMemcpyAsync(&v, w.lc.ctl + 2 * slot_of(y, k), sizeof(v), hipMemcpyDeviceToHost, st));
    CSBFS_HIP(hipStreamSynchronize(st));
    *cnt = v;
    return CSBFS_OK;
}

constexpr int kEvPerLevel2 = kEvPerLevel;

// One search from root on workspace state w (Algorithm 3 level loop).
int run_search(const csbfs_graph *g, const SearchLayout &y, const SearchState &w, int64_t root, int32_t *level,
               int32_t *parent, csbfs_level_stats *stats, int32_t stats_cap, int32_t *n_levels, const Mailbox &mb,
               hipEvent_t *events, hipStream_t st) {
    const int64_t P = g->P, n = g->n, R = g->R, W = g->W, S = y.S;
    const int64_t words = n / 64, view_words = P * words;
    const bool timing = events != nullptr;
    const bool keep = (y.flags & CSBFS_FLAG_KEEP_STREAMS) != 0;

    // evaluation of the product: dense, or top-down / bottom-up per level
    // (forced by a flag, or chosen on the device after every update)
    const bool dense = (y.flags & CSBFS_FLAG_DENSE_ONLY) != 0;
    const bool td_only = (y.flags & CSBFS_FLAG_SPARSE_ONLY) != 0 ||
                         (!dense && !(y.alpha > 0.f) && !(y.flags & CSBFS_FLAG_BOTTOM_UP_ONLY));
    const bool bu_only = (y.flags & CSBFS_FLAG_BOTTOM_UP_ONLY) != 0;
    const int32_t force = dense ? kDirDense : td_only ? kDirTD : bu_only ? kDirBU : -1;
    const int32_t dir0 = dense ? kDirDense : bu_only ? kDirBU : kDirTD;

    if (mb.host) {
        mb.host[0] = 0;  // level tags start at 1
        mb.host[1] = 0;
    }
    // a0: seed (also clears the counters and the encoder's look-back state)
    SeedArgs sa{level, parent, w.pi, w.nb[0], w.nb[1], w.view, n, words, view_words,
                (uint32_t *)w.counters_mem, y.counters_bytes / 4, (uint32_t *)w.look, y.look_bytes / 4,
                w.marks[0], 2 * y.nmarks};
    auto marks_of = [&](int64_t k) { return BlockMarks{w.marks[k & 1]}; };
    int64_t fill_items = n > view_words ? n : view_words;
    fill_items = fill_items > y.look_bytes / 4 ? fill_items : y.look_bytes / 4;
    hipLaunchKernelGGL(seed_fill_kernel, dim3(grid_for(fill_items, 256, 8192)), dim3(256), 0, st, sa);
    CSBFS_HIP(hipGetLastError());
    hipLaunchKernelGGL(seed_root_kernel, dim3(1), dim3(1), 0, st, sa, root, R, W, (int32_t)P, w.lc.ctl, w.lc.rank,
                       (const int32_t *)g->deg, w.dstate, w.lc.dir, dir0, marks_of(0));
    CSBFS_HIP(hipGetLastError());

    ExpandArgs ea{};
    ea.view = w.view;
    ea.view_clear = w.view;
    ea.rank_words = P * W;
    ea.row_ptr = g->row_ptr;
    ea.col_base = g->col_base;
    ea.col = g->col;
    ea.pi = w.pi;
    ea.parent = parent;
    ea.queue = w.queue;
    ea.qoff = g->qoff;
    ea.queue_count = w.ctrs;
    ea.R = R;
    ea.W = W;
    ea.P = (int32_t)P;
    ea.status = w.status;
    ea.dir = &w.dstate->cur;
    ea.tile = &w.dstate->tile;
    ea.tile_words = 64;
    ea.bin = &w.dstate->bin;
    ea.nbins = (int32_t)y.nbins;
    ea.bpairs = w.bpairs;
    ea.bseg = w.bseg;
    ea.cseg = y.cseg;
    ResolveArgs rsa{&w.dstate->cur, &w.dstate->bin, w.bpairs, w.bseg, y.cseg, (int32_t)y.nbins,
                    w.pi, nullptr, BlockMarks{nullptr}, parent, words};
    const unsigned resolve_grid = (unsigned)std::min<int64_t>(std::max<int64_t>(y.nbins, 1), 256);
    PullArgs pa{};
    pa.pi = w.pi;
    pa.live = g->live;
    pa.view = w.view;
    pa.pull_off = g->pull_off;
    pa.pull_col = g->pull_col;
    pa.head = g->head;
    pa.level = level;
    pa.mf = w.exp_mf;
    pa.parent = parent;
    pa.words = words;
    pa.R = R;
    pa.W = W;
    pa.P = (int32_t)P;
    pa.status = w.status;
    pa.dir = &w.dstate->cur;
    PullArgs pb = pa;
    pa.tile_words = kPullTileDense;
    pb.tile_words = kPullTileBU;
    // grids (multiples of the XCD count) from sweeps at scales 22 and 26:
    // 512 expansion workgroups of 8 waves (the same waves as 1024 of 4,
    // which beat 512-4096; 768 for the wide level kernel) and kBinGrid for
    // the long rows
    const unsigned exp_grid = 512, big_grid = kBinGrid;
    const bool wide = words >= kWideWords;
    const unsigned level_grid = wide ? kWideGrid : exp_grid;
    const unsigned pull_grid = grid_for((words + kPullTileDense - 1) / kPullTileDense, kPullThreads / 64, 16384);
    const unsigned bu_grid = grid_for((words + kPullTileBU - 1) / kPullTileBU, kPullThreads / 64, 2048);
    pa.xcd = xcd_split(P, pull_grid) && W % kPullTileDense == 0;
    pb.xcd = xcd_split(P, exp_grid) && xcd_split(P, level_grid) && W % kPullTileBU == 0;
    const int32_t bu_xcd = xcd_split(P, bu_grid) && W % kPullTileBU == 0;
    DirArgs da{};
    da.st = w.dstate;
    da.n = n;
    da.nnz = g->nnz;
    da.alpha = y.alpha;
    da.beta = y.beta;
    da.force = force;
    da.bin_min = y.bin_min;
    da.bin_deg = y.bin_deg;
    da.bin_cap = y.bin_limit;

    WahBatch wb{};  // the words come from FrontierHook, not from a bits buffer
    wb.mask_base = (y.flags & CSBFS_FLAG_NO_SIEVE) ? nullptr : g->dir;
    wb.nbits = R;
    wb.words_per_piece = W;
    wb.cap = y.cap;
    wb.P = (int32_t)P;
    wb.look = w.look;
    wb.ticket = w.enc_ticket;
    wb.nseg = y.nseg;
    wb.chunk_groups = w.chunk_groups;
    wb.nchunk = y.nchunk;
    wb.chunk_starts = 1;  // the decode reads the chunk starts the encode records
    wb.dst_base = w.view;
    wb.status = w.status;
    const int32_t enc_split = xcd_split(P, S * y.nseg);
    const dim3 enc_grid((unsigned)(S * y.nseg)),
        dec_grid((unsigned)std::min<int64_t>(y.nchunk, kDecGridChunks), (unsigned)S);

    // Iteration j: for j >= 1 the update that forms f^j together with the
    // sieve and compression of its messages, then their decode into the views
    // (whose first workgroup reduces |f^j|, posts it for the host and
    // chooses the direction); then the expansion of f^j, which collects the
    // vertices of level j + 1 in nb[(j + 1) & 1]. pi holds the vertices
    // visited through level j once the update of iteration j is done.
    auto enqueue_iter = [&](int64_t j) -> int {
        const int64_t sj = slot_of(y, j);
        if (j >= y.L) {
            const int r2 = reset_overflow_slot(y, w, st);
            if (r2) return r2;
        }
        hipEvent_t *ev = (timing && j < y.L) ? &events[(size_t)j * kEvPerLevel2] : nullptr;
        if (ev) CSBFS_HIP(hipEventRecord(ev[0], st));
        if (j >= 1) {
            // a2 + a4 + a5: t = S & ~pi, levels, sieve and compress every stream i -> j
            const int64_t arena_slot = keep ? sj : 0;
            wb.out_base = w.arena + arena_slot * S * y.cap;
            wb.n_words = w.lc.words + sj * S;
            wb.stat_sieved_bits = w.lc.sbits + sj * S;
            wb.stat_unsieved_words = w.lc.uwords + sj * P;
            FrontierHook fh{w.nb[j & 1], w.nb[(j + 1) & 1], w.pi, w.view, level, g->deg, w.part,
                            marks_of(j), marks_of(j + 1), W, y.seg_words, (int32_t)P, (int32_t)j, 1, 1};
            if (y.enc_gpt == 2)
                hipLaunchKernelGGL(frontier_encode_kernel_g2, enc_grid, dim3(kEncThreads), 0, st, wb, fh,
                                   (const DirState *)w.dstate, enc_split);
            else
                hipLaunchKernelGGL(frontier_encode_kernel_g4, enc_grid, dim3(kEncThreads), 0, st, wb, fh,
                                   (const DirState *)w.dstate, enc_split);
            CSBFS_HIP(hipGetLastError());
            if (ev) CSBFS_HIP(hipEventRecord(ev[1], st));
            // a6: the stream slots are the receive buffers; a7: decode into the
            // views; a3: reduction of |f^j|, direction of its expansion
            da.rec = w.lc.dir + sj;
            ReduceArgs ra{w.part, S * y.nseg, w.lc.ctl + 2 * sj, mb.dev ? mb.dev + (j & 1) : nullptr, w.ctrs,
                          (int32_t)P, (int32_t)j, w.marks[(j + 1) & 1], y.nmarks, w.exp_mf, da};
            hipLaunchKernelGGL(search_decode_kernel, dec_grid, dim3(kDecThreads), 0, st, wb, ra);
            CSBFS_HIP(hipGetLastError());
        } else if (ev) {
            CSBFS_HIP(hipEventRecord(ev[1], st));
        }
        if (ev) CSBFS_HIP(hipEventRecord(ev[2], st));
        ea.N = w.nb[(j + 1) & 1];
        pa.N = w.nb[(j + 1) & 1];
        pb.N = w.nb[(j + 1) & 1];
        pa.next_level = (int32_t)(j + 1);
        pb.next_level = (int32_t)(j + 1);
        ea.marks_next = marks_of(j + 1);
        ea.marks_view = marks_of(j);
        rsa.N = w.nb[(j + 1) & 1];
        rsa.marks_next = marks_of(j + 1);
        pa.marks_next = marks_of(j + 1);
        pb.marks_next = marks_of(j + 1);
        // a1: expand f^j (tile width and direction chosen on the device)
        ea.edges = w.lc.edges + sj;
        if (dense) {
            hipLaunchKernelGGL(expand_kernel<true>, dim3(exp_grid), dim3(kExpThreads), 0, st, ea);
            CSBFS_HIP(hipGetLastError());
            if (ev) CSBFS_HIP(hipEventRecord(ev[3], st));
            hipLaunchKernelGGL(expand_big_kernel<true>, dim3(big_grid), dim3(kExpThreads), 0, st, ea);
            CSBFS_HIP(hipGetLastError());
            hipLaunchKernelGGL(pull_kernel<false>, dim3(pull_grid), dim3(kPullThreads), 0, st, pa);
            CSBFS_HIP(hipGetLastError());
        } else if (td_only) {
            hipLaunchKernelGGL(expand_kernel<false>, dim3(exp_grid), dim3(kExpThreads), 0, st, ea);
            CSBFS_HIP(hipGetLastError());
            if (ev) CSBFS_HIP(hipEventRecord(ev[3], st));
            hipLaunchKernelGGL(expand_big_kernel<false>, dim3(big_grid), dim3(kExpThreads), 0, st, ea);
            CSBFS_HIP(hipGetLastError());
            if (y.nbins) {
                hipLaunchKernelGGL(bin_resolve_kernel, dim3(resolve_grid), dim3(kResolveThreads), 0, st, rsa);
                CSBFS_HIP(hipGetLastError());
            }
        } else {
            pb.edges = w.lc.edges + sj;
            pb.pulled = w.lc.pulled + sj;
            if (bu_only) {
                PullArgs pbu = pb;
                pbu.xcd = bu_xcd;
                hipLaunchKernelGGL(pull_kernel<true>, dim3(bu_grid), dim3(kPullThreads), 0, st, pbu);
                CSBFS_HIP(hipGetLastError());
                if (ev) CSBFS_HIP(hipEventRecord(ev[3], st));
            } else {
                // one launch: the push or the pull, as the level's direction
                // says; the long-row pass returns at once on bottom-up levels
                if (wide)
                    hipLaunchKernelGGL(level_kernel_wide, dim3(level_grid), dim3(kExpThreads), 0, st, ea, pb);
                else
                    hipLaunchKernelGGL(level_kernel, dim3(level_grid), dim3(kExpThreads), 0, st, ea, pb);
                CSBFS_HIP(hipGetLastError());
                if (ev) CSBFS_HIP(hipEventRecord(ev[3], st));
                hipLaunchKernelGGL(expand_big_kernel<false>, dim3(big_grid), dim3(kExpThreads), 0, st, ea);
                CSBFS_HIP(hipGetLastError());
                if (y.nbins) {
                    hipLaunchKernelGGL(bin_resolve_kernel, dim3(resolve_grid), dim3(kResolveThreads), 0, st, rsa);
                    CSBFS_HIP(hipGetLastError());
                }
            }
        }
        if (ev) CSBFS_HIP(hipEventRecord(ev[4], st));
        return CSBFS_OK;
    };

    // The host reads |f^k| (posted by the decode of level k) while the
    // expansion of level k and iteration k + 1 are already queued. When f^k
    // is empty the decode chose the idle direction: the expansion of level k
    // and every kernel of iteration k + 1 return at once, and their counters
    // lie past the last reported level.
    int rc = enqueue_iter(0);
    if (rc) return rc;
    rc = enqueue_iter(1);
    if (rc) return rc;
    int64_t k = 1;
    for (;;) {
        rc = enqueue_iter(k + 1);
        if (rc) return rc;
        unsigned long long cnt = 0;
        rc = wait_count(mb, y, w, k, st, &cnt);
        if (rc) {
            (void)hipStreamSynchronize(st);
            return rc;
        }
        if (cnt == 0) break;
        if (++k > n) {  // every level visits a vertex: more than n levels is a broken count
            CSBFS_HIP(hipStreamSynchronize(st));
            return fail(CSBFS_ECORRUPT, "csbfs_bfs: frontier counts did not reach zero");
        }
    }
    const int64_t nl = k;  // levels 0..k-1
    *n_levels = (int32_t)(nl < INT32_MAX ? nl : INT32_MAX);

    // statistics
    int32_t hstatus = 0;
    CSBFS_HIP(hipMemcpyAsync(&hstatus, w.status, sizeof(hstatus), hipMemcpyDeviceToHost, st));
    const int64_t have = nl < y.L ? nl : y.L;
    const int64_t want = stats_cap < have ? stats_cap : have;
    std::vector<unsigned long long> ctl, ed, sb, uw, pl;
    std::vector<int64_t> wd;
    std::vector<int32_t> dr;
    if (want > 0) {
        ctl.resize(2 * want);
        ed.resize(want);
        pl.resize(want);
        dr.resize(want);
        sb.resize(want * S);
        uw.resize(want * P);
        wd.resize(want * S);
        CSBFS_HIP(hipMemcpyAsync(pl.data(), w.lc.pulled, sizeof(unsigned long long) * want,
                                 hipMemcpyDeviceToHost, st));
        CSBFS_HIP(hipMemcpyAsync(dr.data(), w.lc.dir, sizeof(int32_t) * want, hipMemcpyDeviceToHost, st));
        CSBFS_HIP(hipMemcpyAsync(ctl.data(), w.lc.ctl, sizeof(unsigned long long) * 2 * want,
                                 hipMemcpyDeviceToHost, st));
        CSBFS_HIP(hipMemcpyAsync(ed.data(), w.lc.edges, sizeof(unsigned long long) * want,
                                 hipMemcpyDeviceToHost, st));
        CSBFS_HIP(hipMemcpyAsync(sb.data(), w.lc.sbits, sizeof(unsigned long long) * want * S,
                                 hipMemcpyDeviceToHost, st));
        CSBFS_HIP(hipMemcpyAsync(uw.data(), w.lc.uwords, sizeof(unsigned long long) * want * P,
                                 hipMemcpyDeviceToHost, st));
        CSBFS_HIP(hipMemcpyAsync(wd.data(), w.lc.words, sizeof(int64_t) * want * S,
                                 hipMemcpyDeviceToHost, st));
    }
    CSBFS_HIP(hipStreamSynchronize(st));
    if (hstatus != 0) {
        if (hstatus == 1) return fail(CSBFS_ECORRUPT, "csbfs_bfs: a stream failed validation while decoding");
        return fail(CSBFS_ECORRUPT, "csbfs_bfs: internal consistency check failed");
    }
    for (int64_t lv = 0; lv < want; ++lv) {
        csbfs_level_stats &s = stats[lv];
        s = csbfs_level_stats{};
        s.frontier = (int64_t)ctl[2 * lv];
        s.edges = (int64_t)ed[lv];
        s.pulled = (int64_t)pl[lv];
        s.direction = dr[lv] & 0xFF;
        s.push = dr[lv] >> 8;
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
            hipEvent_t *ev = &events[(size_t)lv * kEvPerLevel2];
            float c = 0, d = 0, x = 0, b = 0;
            CSBFS_HIP(hipEventElapsedTime(&c, ev[0], ev[1]));
            CSBFS_HIP(hipEventElapsedTime(&d, ev[1], ev[2]));
            CSBFS_HIP(hipEventElapsedTime(&x, ev[2], ev[3]));
            CSBFS_HIP(hipEventElapsedTime(&b, ev[3], ev[4]));
            stats[lv].ms_compress = c;
            stats[lv].ms_decode = d;
            stats[lv].ms_expand = x;
            stats[lv].ms_long_rows = b;
            stats[lv].ms_update = 0.f;
        }
    }
    return CSBFS_OK;
}

int stream_words_of(const SearchLayout &y, const SearchState &w, int32_t last_levels, int32_t *words,
                    int32_t cap_levels, hipStream_t st) {
    const int64_t S = y.S;
    const int64_t have = std::min<int64_t>(std::min<int64_t>(cap_levels, last_levels), y.L);
    std::vector<int64_t> wd((size_t)(have > 0 ? have : 1) * S);
    if (have > 0) {
        CSBFS_HIP(hipMemcpyAsync(wd.data(), w.lc.words, sizeof(int64_t) * have * S, hipMemcpyDeviceToHost, st));
        CSBFS_HIP(hipStreamSynchronize(st));
    }
    for (int64_t lv = 0; lv < cap_levels; ++lv)
        for (int64_t s = 0; s < S; ++s) words[lv * S + s] = lv < have ? (int32_t)wd[lv * S + s] : 0;
    return CSBFS_OK;
}

int copy_stream_of(const SearchLayout &y, const SearchState &w, int32_t last_levels, int32_t k, int32_t i,
                   int32_t j, uint64_t *dst, int64_t cap_words, int64_t *n_words_out, hipStream_t st) {
    if (!(y.flags & CSBFS_FLAG_KEEP_STREAMS))
        return fail(CSBFS_EINVAL, "copy stream: the search did not keep its streams (CSBFS_FLAG_KEEP_STREAMS)");
    if (k < 0 || k >= y.L || k >= last_levels || i < 0 || i >= y.P || j < 0 || j >= y.P)
        return fail(CSBFS_EINVAL, "copy stream: level or processor out of range");
    const int64_t s = (int64_t)i * y.P + j;
    int64_t nw = 0;
    CSBFS_HIP(hipMemcpyAsync(&nw, w.lc.words + (int64_t)k * y.S + s, sizeof(int64_t), hipMemcpyDeviceToHost, st));
    CSBFS_HIP(hipStreamSynchronize(st));
    *n_words_out = nw;
    if (nw > cap_words) return fail(CSBFS_ENOSPACE, "copy stream: dst too small");
    if (nw > 0)
        CSBFS_HIP(hipMemcpyAsync(dst, w.arena + ((int64_t)k * y.S + s) * y.cap, sizeof(uint64_t) * nw,
                                 hipMemcpyDeviceToDevice, st));
    CSBFS_HIP(hipStreamSynchronize(st));
    return CSBFS_OK;
}

int check_workspace(const csbfs_graph *g, const csbfs_search_config *cfg, void *ws, size_t ws_bytes,
                    SearchLayout *y, const char *who) {
    if (!g || !ws) return fail(CSBFS_EINVAL, std::string(who) + ": null graph or workspace");
    int rc = search_layout(g->n, g->P, g->nnz, cfg, y);
    if (rc) return rc;
    if ((uintptr_t)ws % kAlign) return fail(CSBFS_EINVAL, std::string(who) + ": workspace must be 256-byte aligned");
    if ((int64_t)ws_bytes < y->total)
        return fail(CSBFS_ENOSPACE, std::string(who) + ": workspace smaller than csbfs_layout_query gives");
    return CSBFS_OK;
}

}  // namespace
}  // namespace csbfs

using namespace csbfs;

extern "C" int csbfs_layout_query(int64_t n, int64_t n_tuples, int32_t p, const csbfs_search_config *cfg,
                                  csbfs_sizes *out) {
    if (!out) return fail(CSBFS_EINVAL, "csbfs_layout_query: out is NULL");
    GraphLayout gl;
    int rc = graph_layout(n, n_tuples, p, &gl);
    if (rc) return rc;
    SearchLayout y;
    rc = search_layout(n, p, 2 * n_tuples, cfg, &y);
    if (rc) return rc;
    out->graph_bytes = gl.graph_bytes;
    out->build_scratch_bytes = gl.scratch_bytes;
    out->workspace_bytes = y.total;
    out->alignment = kAlign;
    return CSBFS_OK;
}

extern "C" int csbfs_bfs_ws(const csbfs_graph *g, int64_t root, const csbfs_search_config *cfg, int32_t *level,
                            int32_t *parent, csbfs_level_stats *stats, int32_t stats_cap, int32_t *n_levels,
                            void *workspace, size_t ws_bytes, uint64_t *host_mailbox, void *stream) {
    if (!g || !level || !parent || !n_levels || stats_cap < 0 || (stats_cap > 0 && !stats))
        return fail(CSBFS_EINVAL, "csbfs_bfs_ws: null argument or negative stats_cap");
    SearchLayout y;
    int rc = check_workspace(g, cfg, workspace, ws_bytes, &y, "csbfs_bfs_ws");
    if (rc) return rc;
    if (root < 0 || root >= g->n) return fail(CSBFS_ERANGE, "csbfs_bfs_ws: root outside [0, n)");
    rc = graph_device_check(g);
    if (rc) return rc;
    Mailbox mb;
    if (host_mailbox) {
        void *dev = nullptr;
        const hipError_t e = hipHostGetDevicePointer(&dev, host_mailbox, 0);
        if (e != hipSuccess || !dev) {
            (void)hipGetLastError();  // the refusal must not surface at the next launch check
            return fail(CSBFS_EINVAL, "csbfs_bfs_ws: host_mailbox is not pinned host memory");
        }
        mb.host = reinterpret_cast<volatile unsigned long long *>(host_mailbox);
        mb.dev = (unsigned long long *)dev;
    }
    const SearchState w = bind_workspace(y, workspace);
    return run_search(g, y, w, root, level, parent, stats, stats_cap, n_levels, mb, nullptr, as_stream(stream));
}

extern "C" int csbfs_ws_stream_words(const csbfs_graph *g, const csbfs_search_config *cfg, const void *workspace,
                                     size_t ws_bytes, int32_t n_levels, int32_t *words, int32_t cap_levels,
                                     void *stream) {
    if (!words || cap_levels < 0 || n_levels < 0) return fail(CSBFS_EINVAL, "csbfs_ws_stream_words: bad argument");
    SearchLayout y;
    int rc = check_workspace(g, cfg, (void *)workspace, ws_bytes, &y, "csbfs_ws_stream_words");
    if (rc) return rc;
    return stream_words_of(y, bind_workspace(y, (void *)workspace), n_levels, words, cap_levels, as_stream(stream));
}

extern "C" int csbfs_ws_copy_stream(const csbfs_graph *g, const csbfs_search_config *cfg, const void *workspace,
                                    size_t ws_bytes, int32_t n_levels, int32_t k, int32_t i, int32_t j,
                                    uint64_t *dst, int64_t cap_words, int64_t *n_words_out, void *stream) {
    if (!dst || !n_words_out) return fail(CSBFS_EINVAL, "csbfs_ws_copy_stream: null argument");
    SearchLayout y;
    int rc = check_workspace(g, cfg, (void *)workspace, ws_bytes, &y, "csbfs_ws_copy_stream");
    if (rc) return rc;
    return copy_stream_of(y, bind_workspace(y, (void *)workspace), n_levels, k, i, j, dst, cap_words, n_words_out,
                          as_stream(stream));
}

// ------------------------------------------------------------------ engine --
// A convenience owner of one workspace (device memory from hipMalloc), a
// pinned mailbox and, with CSBFS_FLAG_TIMING, per-level events.

struct csbfs_engine {
    const csbfs_graph *g = nullptr;
    csbfs_search_config cfg{};
    SearchLayout y{};
    void *ws = nullptr;
    SearchState w{};
    unsigned long long *mbox = nullptr;  // pinned [2]
    Mailbox mb;
    std::vector<hipEvent_t> events;
    int32_t last_levels = 0;
};

namespace {

void engine_release(csbfs_engine *e) {
    if (e->ws) (void)hipFree(e->ws);
    if (e->mbox) (void)hipHostFree(e->mbox);
    for (hipEvent_t ev : e->events)
        if (ev) (void)hipEventDestroy(ev);
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
    if (flags & ~(kSearchFlags | CSBFS_FLAG_TIMING)) return fail(CSBFS_EINVAL, "csbfs_engine_create: unknown flag");
    int rc = graph_device_check(g);
    if (rc) return rc;
    std::unique_ptr<csbfs_engine> e(new csbfs_engine());
    e->g = g;
    e->cfg.flags = flags & kSearchFlags;
    e->cfg.max_levels = max_levels;
    rc = search_layout(g->n, g->P, g->nnz, &e->cfg, &e->y);
    if (rc) return rc;
    CSBFS_HIP(hipMalloc(&e->ws, (size_t)e->y.total));
    e->w = bind_workspace(e->y, e->ws);
    hipError_t herr = hipHostMalloc((void **)&e->mbox, 2 * sizeof(unsigned long long));
    if (herr != hipSuccess) {
        e->mbox = nullptr;
        engine_release(e.release());
        return hip_fail(herr, "hipHostMalloc", __FILE__, __LINE__);
    }
    void *dev = nullptr;
    herr = hipHostGetDevicePointer(&dev, e->mbox, 0);
    if (herr != hipSuccess) {
        engine_release(e.release());
        return hip_fail(herr, "hipHostGetDevicePointer", __FILE__, __LINE__);
    }
    e->mb.host = e->mbox;
    e->mb.dev = (unsigned long long *)dev;
    if (flags & CSBFS_FLAG_TIMING) {
        e->events.assign((size_t)max_levels * kEvPerLevel2, nullptr);
        // timestamps only: no system-scope fence at each record, which would
        // write the caches back between the kernels being timed
        for (auto &ev : e->events) {
            herr = hipEventCreateWithFlags(&ev, hipEventDisableSystemFence);
            if (herr != hipSuccess) {
                ev = nullptr;
                engine_release(e.release());
                return hip_fail(herr, "hipEventCreate", __FILE__, __LINE__);
            }
        }
    }
    *out = e.release();
    return CSBFS_OK;
}

extern "C" int csbfs_engine_set_direction(csbfs_engine *e, float alpha, float beta) {
    if (!e) return fail(CSBFS_EINVAL, "csbfs_engine_set_direction: engine is NULL");
    if (!(beta > 0.f) || alpha != alpha)
        return fail(CSBFS_EINVAL, "csbfs_engine_set_direction: beta must be > 0 and alpha a number");
    e->y.alpha = alpha;
    e->y.beta = beta;
    return CSBFS_OK;
}

extern "C" int csbfs_engine_free(csbfs_engine *e) {
    if (!e) return CSBFS_OK;
    engine_release(e);
    return CSBFS_OK;
}

extern "C" int csbfs_bfs(csbfs_engine *e, int64_t root, int32_t *level, int32_t *parent,
                         csbfs_level_stats *stats, int32_t stats_cap, int32_t *n_levels,
                         void *stream) {
    if (!e || !level || !parent || !n_levels || stats_cap < 0 || (stats_cap > 0 && !stats))
        return fail(CSBFS_EINVAL, "csbfs_bfs: null argument or negative stats_cap");
    const csbfs_graph *g = e->g;
    if (root < 0 || root >= g->n) return fail(CSBFS_ERANGE, "csbfs_bfs: root outside [0, n)");
    int rc = graph_device_check(g);
    if (rc) return rc;
    rc = run_search(g, e->y, e->w, root, level, parent, stats, stats_cap, n_levels, e->mb,
                    e->events.empty() ? nullptr : e->events.data(), as_stream(stream));
    e->last_levels = rc == CSBFS_OK ? *n_levels : 0;
    return rc;
}

extern "C" int csbfs_engine_stream_words(const csbfs_engine *e, int32_t *words, int32_t cap_levels) {
    if (!e || !words || cap_levels < 0) return fail(CSBFS_EINVAL, "csbfs_engine_stream_words: bad argument");
    return stream_words_of(e->y, e->w, e->last_levels, words, cap_levels, nullptr);
}

extern "C" int csbfs_engine_copy_stream(const csbfs_engine *e, int32_t k, int32_t i, int32_t j,
                                        uint64_t *dst, int64_t cap_words, int64_t *n_words_out,
                                        void *stream) {
    if (!e || !dst || !n_words_out) return fail(CSBFS_EINVAL, "csbfs_engine_copy_stream: null argument");
    return copy_stream_of(e->y, e->w, e->last_levels, k, i, j, dst, cap_words, n_words_out, as_stream(stream));
}
