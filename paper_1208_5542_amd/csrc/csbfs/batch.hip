// Batched searches: Algorithm 3 (Sec. V.B) for up to 64 roots at once.
//
// Vertex v carries a visit mask vis[v] (bit r: reached by root r) and, during
// a level, a mask nx[v] of the roots that discovered it; the two are stored
// side by side (vn[2v], vn[2v+1]) so that one 16-byte access serves the
// push's check of both. Each root keeps its
// own frontier bitmap: plane r of `f` holds f_r, and plane r of the views
// holds the pieces P_i received for root r. One level:
//
//   expand   top-down: every view word position (i, j, q) is read in all
//            planes at once (lane = root) and transposed with ballots into
//            the masks of its 64 sources (lane = source); a source's mask
//            travels along its row of block (i, j) once, for all its roots:
//            nx[v] |= m & ~vis[v]. Long rows go to per-processor chunk queues.
//            bottom-up: every vertex v still missing some roots whose
//            frontier is not empty reads its merged row and ORs its
//            neighbours' frontier masks fm[u] (bit r: u is in root r's
//            frontier) until every missing root is found or the row ends;
//            nx[v] = the roots found (one writer per vertex, no atomics). A
//            neighbour u of v in R_i has V_{i,j}[u] = 1 (Eq. dir-vec), so
//            u's bit in P_i's view equals its frontier bit (Lemma 1): the
//            masks stand for the views, which this level then clears.
//            Chosen per level on the device by Beamer's rule over the union
//            of the roots' frontiers, as in the single-root search.
//   update   new = nx & ~vis; vis |= new; fm[v] = new; level[r][v] = k + 1
//            for each new bit r; the new masks are transposed back into the
//            planes of f^{k+1}; per-root frontier sizes and the direction
//            rule's sums (union frontier, its adjacency entries, entries of
//            vertices still missing a root) are reduced.
//   messages plane r of f^{k+1} is sieved, WAH-64 compressed, exchanged and
//            decoded exactly as in the single-root search (wah.hip, one
//            launch for all planes), so every root's streams equal those of
//            its own search.
//
// Levels only: the (select, max) parents would need one 32-bit slot per
// (vertex, root) and a max-reduction per root and edge.
#include <memory>
#include <vector>

#include "device.hpp"
#include "graph.hpp"

namespace csbfs {
namespace {

constexpr int kBThreads = 256;
constexpr int kBUnroll = 4;
constexpr int kBEvPerLevel = 5;
constexpr int kMaxRoots = 64;

struct BItem {
    uint64_t mask;  // roots whose frontier holds the source
    int32_t block;
    int32_t u_local;
    int32_t start;  // offsets within the block's col
    int32_t end;
};

struct BArgs {
    uint64_t *view;  // [B][P * P * W] planes of views
    int64_t vplane;  // words per view plane
    int32_t B;
    const int32_t *row_ptr;
    const int64_t *col_base;
    const uint32_t *col;
    uint64_t *vn;         // [n][2]: visit mask, discovery mask
    BItem *queue;
    const int64_t *qoff;     // [P + 1]
    uint32_t *queue_count;   // [P]
    int64_t R;
    int64_t W;
    int32_t P;
    unsigned long long *edges;
    int32_t *status;
    // nullable: |f^j| summed over the roots; 0 leaves nothing to expand
    const unsigned long long *fcount;
    const int32_t *dir;  // direction of this level (CSBFS_DIR_*); the push runs if top-down
};

// Push kBUnroll (target v, root mask m) pairs; loads first, then atomics.
// Every load is issued unconditionally: the callers clamp the positions of
// lanes past a row's end to its last entry (an in-bounds address), and ok
// masks those lanes' results out.
__device__ __forceinline__ void brelax(const BArgs &a, const int64_t (&v)[kBUnroll],
                                       const uint64_t (&m)[kBUnroll], const bool (&ok)[kBUnroll]) {
    // one 16-byte load per target: its visit mask and a (possibly stale)
    // view of its discovery mask, which only saves redundant atomics
    ulonglong2 w[kBUnroll];
#pragma unroll
    for (int k = 0; k < kBUnroll; ++k) w[k] = *reinterpret_cast<const ulonglong2 *>(a.vn + 2 * v[k]);
#pragma unroll
    for (int k = 0; k < kBUnroll; ++k) {
        const uint64_t add = ok[k] ? m[k] & ~w[k].x : 0ull;
        if (add & ~w[k].y) atomicOr((unsigned long long *)(a.vn + 2 * v[k] + 1), (unsigned long long)add);
    }
}

// A wave's tile: kBTile consecutive words of every root plane. Loads and
// stores of a tile move 4 roots x kBTile words (four 128-byte lines) per
// instruction; LDS turns them around so that lane r holds root r's word.
constexpr int kBTile = 16;
constexpr int kBRootsPerOp = 64 / kBTile;

__global__ __launch_bounds__(kBThreads) void bexpand_kernel(BArgs a) {
    __shared__ uint64_t tile[kBThreads / 64][kBTile][kMaxRoots];
    if (a.fcount && *a.fcount == 0) return;
    if (*a.dir != CSBFS_DIR_TOP_DOWN) return;
    const int lane = threadIdx.x & 63;
    uint64_t(*tw)[kMaxRoots] = tile[threadIdx.x >> 6];
    const int64_t wave = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) >> 6;
    const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
    const int64_t npos = (int64_t)a.P * a.P * a.W;
    const int64_t ntiles = (npos + kBTile - 1) / kBTile;
    const int t_ld = lane % kBTile, r_ld = lane / kBTile;
    const int nsteps = (a.B + kBRootsPerOp - 1) / kBRootsPerOp;
    unsigned long long edges = 0;
    for (int64_t tl = wave; tl < ntiles; tl += nwaves) {
        const int64_t pos0 = tl * kBTile;
        uint64_t anyw = 0;
        for (int s = 0; s < nsteps; ++s) {
            const int r = r_ld + kBRootsPerOp * s;
            const int64_t p = pos0 + t_ld;
            uint64_t w = 0;
            if (r < a.B && p < npos) {
                uint64_t *src = a.view + r * a.vplane + p;
                w = *src;
                if (w) *src = 0;  // the views are empty again when the level ends
            }
            tw[t_ld][r] = w;
            anyw |= w;
        }
        wave_lds_sync();
        if (__ballot(anyw != 0)) {
            for (int t = 0; t < kBTile; ++t) {
                // lane r: root r's view word at this position
                const uint64_t w = lane < a.B ? tw[t][lane] : 0ull;
                if (!__ballot(w != 0)) continue;
                const int64_t pos = pos0 + t;
                // transpose: lane b gets the roots in whose frontier source b is
                const uint64_t any = wave_or64(w);
                uint64_t mymask = 0;
                for (uint64_t it = any; it; it &= it - 1) {
                    const int b = __ffsll((unsigned long long)it) - 1;
                    const uint64_t m = __ballot((w >> b) & 1);
                    if (lane == b) mymask = m;
                }
                const int64_t blk = pos / a.W;
                const int64_t q = pos - blk * a.W;
                const int32_t i = (int32_t)(blk / a.P);
                const int64_t ul = (q << 6) + lane;
                int32_t rs = 0, deg = 0;
                if (mymask) {
                    const int32_t *rp = a.row_ptr + blk * (a.R + 1) + ul;
                    rs = rp[0];
                    deg = rp[1] - rs;
                }
                const int32_t items = deg > kBigRow ? (deg + kBigChunk - 1) / kBigChunk : 0;
                const int32_t items_incl = wave_incl_scan_i32(items);
                const int32_t items_total = __shfl(items_incl, 63, 64);
                if (items_total) {
                    uint32_t qbase = 0;
                    if (lane == 63) qbase = atomicAdd(&a.queue_count[i], (uint32_t)items_total);
                    qbase = __shfl(qbase, 63, 64);
                    if (items) {
                        const int64_t qpos = (int64_t)qbase + items_incl - items;
                        const int64_t qcap = a.qoff[i + 1] - a.qoff[i];
                        if (qpos + items > qcap) {
                            *a.status = 2;  // a row is queued at most once per level: unreachable
                        } else {
                            for (int32_t c = 0; c < items; ++c) {
                                BItem it;
                                it.mask = mymask;
                                it.block = (int32_t)blk;
                                it.u_local = (int32_t)ul;
                                it.start = rs + c * kBigChunk;
                                it.end = min(rs + deg, rs + (c + 1) * kBigChunk);
                                a.queue[a.qoff[i] + qpos + c] = it;
                            }
                        }
                        deg = 0;
                    }
                }
                const int32_t incl = wave_incl_scan_i32(deg);
                const int32_t total = __shfl(incl, 63, 64);
                const int32_t excl = incl - deg;
                edges += (unsigned long long)total;
                const uint32_t *colb = a.col + a.col_base[blk];
                const int64_t vbase = (int64_t)i * a.R;
                for (int32_t e0 = 0; e0 < total; e0 += 64 * kBUnroll) {
                    int64_t v[kBUnroll];
                    uint64_t m[kBUnroll];
                    bool ok[kBUnroll];
#pragma unroll
                    for (int k = 0; k < kBUnroll; ++k) {
                        const int32_t e = e0 + 64 * k + lane;
                        ok[k] = e < total;
                        const int o = owner_lane(excl, ok[k] ? e : total - 1);
                        const int32_t ex = __shfl(excl, o, 64);
                        const int32_t r0 = __shfl(rs, o, 64);
                        m[k] = (uint64_t)shfl64((int64_t)mymask, o);
                        const int32_t ec = ok[k] ? e : total - 1;  // clamped: an entry of the last row
                        v[k] = vbase + colb[r0 + (ec - ex)];
                    }
                    brelax(a, v, m, ok);
                }
            }
        }
        wave_lds_sync();
    }
    block_add<kBThreads / 64>(edges, a.edges);
}

__global__ __launch_bounds__(kBThreads) void bexpand_big_kernel(BArgs a) {
    if (a.fcount && *a.fcount == 0) return;
    if (*a.dir != CSBFS_DIR_TOP_DOWN) return;
    const int lane = threadIdx.x & 63;
    const int64_t wave = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) >> 6;
    const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
    unsigned long long edges = 0;
    int64_t before = 0;  // items of the processors before r, for a grid-wide stride
    for (int32_t r = 0; r < a.P; ++r) {
        const int64_t cap = a.qoff[r + 1] - a.qoff[r];
        const int64_t queued = a.queue_count[r];
        const int64_t count = queued < cap ? queued : cap;
        const BItem *queue = a.queue + a.qoff[r];
        const int64_t vbase = (int64_t)r * a.R;
        int64_t first = (wave - before) % nwaves;
        if (first < 0) first += nwaves;
        before += count;
        for (int64_t kk = first; kk < count; kk += nwaves) {
            const BItem it = queue[kk];
            const uint32_t *colb = a.col + a.col_base[it.block];
            for (int32_t e0 = it.start; e0 < it.end; e0 += 64 * kBUnroll) {
                int64_t v[kBUnroll];
                uint64_t m[kBUnroll];
                bool ok[kBUnroll];
#pragma unroll
                for (int k = 0; k < kBUnroll; ++k) {
                    const int32_t e = e0 + 64 * k + lane;
                    ok[k] = e < it.end;
                    v[k] = vbase + colb[ok[k] ? e : it.end - 1];  // clamped to the item's last entry
                    m[k] = it.mask;
                }
                brelax(a, v, m, ok);
            }
            edges += (unsigned long long)(it.end - it.start);
        }
    }
    block_add<kBThreads / 64>(edges, a.edges);
}

// ---------------------------------------------------------------- pull ---

constexpr int kBPullUnroll = 2;   // entries per lane step
// Direction rule of batched searches (Beamer's alpha and beta over the union
// of the roots' frontiers)
constexpr float kBatchAlpha = 16.0f, kBatchBeta = 24.0f;
constexpr int kBPullRounds = 16;  // lane steps before the wave takes over slow lanes

struct BPullArgs {
    uint64_t *vn;              // [n][2]: visit mask, discovery mask
    const uint64_t *fm;        // [n]: frontier masks of the level
    const int64_t *pull_off;   // merged rows (global ids) of every vertex
    const uint32_t *pull_col;
    const uint32_t *head;      // [2n]: the first two ids of each merged row
    uint64_t *view;            // every view plane, zeroed here (the decode ORs into zeroed views)
    int64_t view_words;
    int64_t n;
    const unsigned long long *rootc;  // [B]: frontier size of each root at this level
    int32_t B;
    const int32_t *dir;
    unsigned long long *edges;
    const unsigned long long *fcount;
};

__global__ __launch_bounds__(kBThreads) void bpull_kernel(BPullArgs a) {
    if (a.fcount && *a.fcount == 0) return;
    if (*a.dir != CSBFS_DIR_BOTTOM_UP) return;
    const int lane = threadIdx.x & 63;
    const int64_t tid = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    const int64_t nthreads = (int64_t)gridDim.x * blockDim.x;
    for (int64_t k = tid; k < a.view_words; k += nthreads) a.view[k] = 0;
    // roots whose frontier is not empty: only they can find anything
    const uint64_t active = __ballot(lane < a.B && (!a.rootc || a.rootc[lane] > 0));
    const int64_t wave = tid >> 6, nwaves = nthreads >> 6;
    unsigned long long read = 0;
    for (int64_t v0 = wave * 64; v0 < a.n; v0 += nwaves * 64) {
        const int64_t v = v0 + lane;
        uint64_t missing = 0, found = 0;
        int64_t e = 0, re = 0;
        uint2 hd = make_uint2(0u, 0u);
        if (v < a.n) {
            missing = active & ~a.vn[2 * v];
            if (missing) {
                e = a.pull_off[v];
                re = a.pull_off[v + 1];
                hd = *reinterpret_cast<const uint2 *>(a.head + 2 * v);
            }
        }
        bool busy = missing && e < re;
        // the row's first two ids come from head, without the row itself
        if (busy) {
            const int32_t nk = re - e < 2 ? (int32_t)(re - e) : 2;
            const uint64_t m0 = a.fm[hd.x], m1 = a.fm[nk > 1 ? hd.y : hd.x];
            found |= (m0 | m1) & missing;
            read += (unsigned long long)nk;
            e += nk;
            if (found == missing || e >= re) busy = false;
        }
        for (int round = 0; round < kBPullRounds; ++round) {
            if (busy) {
                // every lane reads kBPullUnroll entries, positions past the row end
                // clamped to its last entry and masked out
                const int32_t nk = re - e < kBPullUnroll ? (int32_t)(re - e) : kBPullUnroll;
                uint32_t c[kBPullUnroll];
                uint64_t m[kBPullUnroll];
#pragma unroll
                for (int q = 0; q < kBPullUnroll; ++q) c[q] = a.pull_col[e + (q < nk ? q : nk - 1)];
#pragma unroll
                for (int q = 0; q < kBPullUnroll; ++q) m[q] = a.fm[c[q]];
#pragma unroll
                for (int q = 0; q < kBPullUnroll; ++q)
                    if (q < nk) found |= m[q] & missing;
                read += (unsigned long long)nk;
                e += nk;
                if (found == missing || e >= re) busy = false;
            }
            if (!__ballot(busy)) break;
        }
        // rows still being read: the whole wave takes them one at a time
        uint64_t slow = __ballot(busy);
        while (slow) {
            const int Ls = __ffsll((unsigned long long)slow) - 1;
            slow &= slow - 1;
            int64_t ee = shfl64(e, Ls);
            const int64_t rr = shfl64(re, Ls);
            const uint64_t miss = (uint64_t)shfl64((int64_t)missing, Ls);
            uint64_t got = (uint64_t)shfl64((int64_t)found, Ls);
            for (; ee < rr && got != miss; ee += 64) {
                const int64_t pos = ee + lane;
                const uint64_t f = pos < rr ? a.fm[a.pull_col[pos]] & miss : 0ull;
                got |= wave_or64(f);
                if (lane == 0) read += (unsigned long long)(rr - ee < 64 ? rr - ee : 64);
            }
            if (lane == Ls) found = got;
        }
        if (found) a.vn[2 * v + 1] = found;  // this lane's vertex: no other writer
    }
    for (int d = 32; d > 0; d >>= 1) read += (unsigned long long)shfl64((int64_t)read, lane ^ d);
    block_add<kBThreads / 64>(read, a.edges);
}

// Direction state of a batched search, carried from level to level.
struct BDirState {
    int32_t cur;              // direction of the level expanded next
    int32_t force;            // < 0: chosen by the rule; else this direction every level
    unsigned long long prev;  // union frontier size of the level before
    unsigned long long sums[3];  // union frontier, its adjacency entries, entries still missing a root
};

// Beamer's rule over the union of the roots' frontiers (one thread, after the
// update): top-down turns bottom-up when the frontier's entries times alpha
// exceed the entries of vertices some root has not reached and the frontier
// did not shrink; bottom-up turns top-down when the frontier is below
// n / beta and shrinking. The sums are cleared for the next update.
__global__ void bdir_kernel(BDirState *st, int32_t *rec, int64_t n, float alpha, float beta) {
    BDirState s = *st;
    const unsigned long long nf = s.sums[0], mf = s.sums[1], mu = s.sums[2];
    int32_t next = s.cur;
    if (s.force >= 0) {
        next = s.force;
    } else if (s.cur == CSBFS_DIR_TOP_DOWN) {
        if ((double)mf * alpha > (double)mu && nf >= s.prev) next = CSBFS_DIR_BOTTOM_UP;
    } else if ((double)nf * beta < (double)n && nf < s.prev) {
        next = CSBFS_DIR_TOP_DOWN;
    }
    s.prev = nf;
    s.cur = next;
    s.sums[0] = s.sums[1] = s.sums[2] = 0;
    *st = s;
    if (rec) *rec = next;
}

struct BUpdateArgs {
    uint64_t *vn;      // [n][2]
    uint64_t *f;       // [B][n / 64] planes of the new frontier
    int32_t *level;    // [B][n]
    int32_t next_level;
    int32_t B;
    int64_t n;
    unsigned long long *root_count;  // [B]
    unsigned long long *total;       // [1]
    uint32_t *queue_count;           // [P], cleared for the next level
    int32_t P;
    const unsigned long long *fcount;  // as in BArgs: 0 visits nothing
    uint64_t *fm;                      // [n]: frontier mask of every vertex (written for all)
    const int32_t *deg;                // [n]: adjacency entries
    unsigned long long *dsums;         // [3]: union frontier, its entries, entries still missing a root
};

__global__ __launch_bounds__(kBThreads) void bupdate_kernel(BUpdateArgs a) {
    __shared__ uint64_t tile[kBThreads / 64][kBTile][kMaxRoots];
    __shared__ unsigned long long cnt[kMaxRoots];
    __shared__ unsigned long long dsum[3];
    const int lane = threadIdx.x & 63;
    uint64_t(*tw)[kMaxRoots] = tile[threadIdx.x >> 6];
    if (a.fcount && *a.fcount == 0) return;
    if (threadIdx.x < kMaxRoots) cnt[threadIdx.x] = 0;
    if (threadIdx.x < 3) dsum[threadIdx.x] = 0;
    if (blockIdx.x == 0)
        for (int q = threadIdx.x; q < a.P; q += blockDim.x) a.queue_count[q] = 0;
    __syncthreads();
    const int64_t words = a.n / 64;
    const int64_t ntiles = (words + kBTile - 1) / kBTile;
    const int64_t wave = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) >> 6;
    const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
    const int t_st = lane % kBTile, r_st = lane / kBTile;
    const int nsteps = (a.B + kBRootsPerOp - 1) / kBRootsPerOp;
    unsigned long long mine = 0;  // lane r: new vertices of root r seen by this wave
    unsigned long long u_nf = 0, u_mf = 0, u_mu = 0;  // the direction rule's sums, this lane
    for (int64_t tl = wave; tl < ntiles; tl += nwaves) {
        const int64_t q0 = tl * kBTile;
        for (int t = 0; t < kBTile; ++t) {
            const int64_t q = q0 + t;
            uint64_t plane = 0;
            if (q < words) {
                const int64_t v = (q << 6) + lane;
                ulonglong2 *pv = reinterpret_cast<ulonglong2 *>(a.vn + 2 * v);
                const ulonglong2 w = *pv;
                uint64_t nw = 0;
                if (w.y) {
                    nw = w.y & ~w.x;
                    *pv = make_ulonglong2(w.x | nw, 0ull);
                }
                a.fm[v] = nw;
                const uint64_t all = a.B == 64 ? ~0ull : ((1ull << a.B) - 1);
                if (nw || (all & ~(w.x | nw))) {
                    const unsigned long long dg = (unsigned long long)a.deg[v];
                    if (nw) {
                        u_nf += 1;
                        u_mf += dg;
                    }
                    if (all & ~(w.x | nw)) u_mu += dg;
                }
                // lane r collects root r's frontier word: bit b = vertex q*64+b is new for r
                for (uint64_t it = wave_or64(nw); it; it &= it - 1) {
                    const int r = __ffsll((unsigned long long)it) - 1;
                    const bool mine_r = (nw >> r) & 1;
                    if (mine_r) a.level[(int64_t)r * a.n + v] = a.next_level;
                    const uint64_t bal = __ballot(mine_r);
                    if (lane == r) plane = bal;
                }
            }
            tw[t][lane] = plane;
            mine += (unsigned long long)__popcll(plane);
        }
        wave_lds_sync();
        for (int s = 0; s < nsteps; ++s) {
            const int r = r_st + kBRootsPerOp * s;
            const int64_t q = q0 + t_st;
            if (r < a.B && q < words) a.f[r * words + q] = tw[t_st][r];
        }
        wave_lds_sync();
    }
    if (lane < a.B && mine) atomicAdd(&cnt[lane], mine);
    for (int d = 32; d > 0; d >>= 1) {
        u_nf += (unsigned long long)shfl64((int64_t)u_nf, lane ^ d);
        u_mf += (unsigned long long)shfl64((int64_t)u_mf, lane ^ d);
        u_mu += (unsigned long long)shfl64((int64_t)u_mu, lane ^ d);
    }
    if (lane == 0 && (u_nf | u_mf | u_mu)) {
        atomicAdd(&dsum[0], u_nf);
        atomicAdd(&dsum[1], u_mf);
        atomicAdd(&dsum[2], u_mu);
    }
    __syncthreads();
    if (threadIdx.x < 3 && dsum[threadIdx.x]) atomicAdd(&a.dsums[threadIdx.x], dsum[threadIdx.x]);
    if (threadIdx.x < a.B && cnt[threadIdx.x]) atomicAdd(&a.root_count[threadIdx.x], cnt[threadIdx.x]);
    if (threadIdx.x == 0) {
        unsigned long long sum = 0;
        for (int r = 0; r < a.B; ++r) sum += cnt[r];
        if (sum) atomicAdd(a.total, sum);
    }
}

struct BSeedArgs {
    uint64_t *vn;      // [n][2]
    uint64_t *fm;      // [n]
    uint64_t *view;
    int64_t view_words;  // all planes
    int32_t *level;
    int64_t level_words;  // n_roots * n
    int64_t n;
};

__global__ void bseed_fill_kernel(BSeedArgs a) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const int64_t top = a.view_words > a.level_words ? a.view_words : a.level_words;
    for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < top; k += stride) {
        if (k < a.n) {
            reinterpret_cast<ulonglong2 *>(a.vn)[k] = make_ulonglong2(0ull, 0ull);
            a.fm[k] = 0;
        }
        if (k < a.view_words) a.view[k] = 0;
        if (k < a.level_words) a.level[k] = -1;
    }
}

// f(s) <- s for every root: known to every processor without a message.
__global__ void bseed_root_kernel(BSeedArgs a, const int64_t *roots, int32_t B, int64_t R, int64_t W,
                                  int32_t P, int64_t vplane, unsigned long long *root_count0,
                                  unsigned long long *total0, BDirState *ds, int32_t dir0, int32_t force,
                                  int32_t *rec0) {
    const int r = threadIdx.x;
    if (r == 0) {
        BDirState d{};
        d.cur = dir0;
        d.force = force;
        d.prev = (unsigned long long)B;
        *ds = d;
        if (rec0) *rec0 = dir0;
    }
    if (r >= B) return;
    const int64_t s = roots[r];
    const int64_t own = s / R, sl = s - own * R;
    atomicOr((unsigned long long *)(a.vn + 2 * s), 1ull << r);
    atomicOr((unsigned long long *)(a.fm + s), 1ull << r);
    a.level[(int64_t)r * a.n + s] = 0;
    for (int32_t i = 0; i < P; ++i)
        a.view[r * vplane + ((int64_t)i * P + own) * W + (sl >> 6)] = 1ull << (sl & 63);
    root_count0[r] = 1;
    atomicAdd(total0, 1ull);
}

}  // namespace
}  // namespace csbfs

using namespace csbfs;

struct csbfs_batch_engine {
    const csbfs_graph *g = nullptr;
    int32_t Bmax = 0, L = 0;
    uint32_t flags = 0;
    int64_t cap = 0, nseg = 0, nchunk = 0, Smax = 0;
    uint64_t *vn = nullptr, *f = nullptr, *view = nullptr, *arena = nullptr;
    uint64_t *fm = nullptr;           // [n] frontier mask of every vertex (bottom-up levels)
    BDirState *dstate = nullptr;
    int32_t *dirs = nullptr;          // [L + 1] direction used to expand each level
    unsigned long long *look = nullptr;  // encoder look-back words [Smax * nseg]
    uint32_t *enc_ticket = nullptr;      // [kTicketStride * Smax], after look
    size_t look_bytes = 0;
    int64_t *chunk_groups = nullptr;
    BItem *queue = nullptr;
    int64_t *qoff = nullptr;
    uint32_t *qcount = nullptr;
    int64_t *roots_dev = nullptr;
    int32_t *status = nullptr;
    void *counters_mem = nullptr;
    size_t counters_bytes = 0;
    unsigned long long *ctl = nullptr;    // [L+1] total frontier
    unsigned long long *rootc = nullptr;  // [L+1][Bmax]
    unsigned long long *edges = nullptr;  // [L+1]
    unsigned long long *sbits = nullptr;  // [L+1][Smax]
    unsigned long long *uwords = nullptr; // [L+1][Bmax * P]
    int64_t *words = nullptr;             // [L+1][Smax]
    unsigned long long *host_ctl = nullptr;  // pinned [2]
    hipEvent_t count_ev[2] = {nullptr, nullptr};
    std::vector<hipEvent_t> events;
    void *mem = nullptr;     // every device buffer, carved from one block
    bool owns_mem = false;   // hipMalloc'd here (else the caller's, e.g. the server's pool)
    bool owns_host = false;  // host_ctl hipHostMalloc'd here
    int32_t last_levels = 0, last_roots = 0;
};

namespace {

// Releases what the engine itself allocated (hipFree orders itself after
// work still using the block; a caller-provided block stays the caller's).
void bengine_release(csbfs_batch_engine *e) {
    if (e->owns_mem && e->mem) (void)hipFree(e->mem);
    if (e->owns_host && e->host_ctl) (void)hipHostFree(e->host_ctl);
    for (hipEvent_t ev : e->count_ev)
        if (ev) (void)hipEventDestroy(ev);
    for (hipEvent_t ev : e->events)
        if (ev) (void)hipEventDestroy(ev);
    delete e;
}

}  // namespace

namespace {

// Device bytes of every buffer of a batch engine; total() is the size of
// the one block they are carved from (each buffer 256-byte aligned).
struct BatchSizes {
    int64_t vis, nx, f, view, arena, look, ticket, chunk, queue, qoff, qcount, roots, status, counters;
    int64_t fm, dstate, dirs;
    int64_t total() const {
        int64_t t = 0;
        for (int64_t b : {vis, f, view, arena, look + ticket, chunk, queue, qoff, qcount, roots, status, counters, fm,
                          dstate, dirs})
            t += align_up(b > 0 ? b : 1);
        return t;
    }
};

BatchSizes batch_sizes(const csbfs_graph *g, int64_t B, int64_t L, uint32_t flags) {
    const int64_t P = g->P, n = g->n;
    const int64_t Smax = B * P * P, slots = L + 1;
    const int64_t arena_slots = (flags & CSBFS_FLAG_KEEP_STREAMS) ? slots : 1;
    int64_t items = 0;
    for (int64_t r = 0; r < P; ++r) items += g->big_items[r];
    BatchSizes z{};
    z.vis = 16 * n;
    z.nx = 0;
    z.f = 8 * B * (n / 64);
    z.view = 8 * B * P * (n / 64);
    z.arena = 8 * Smax * wah_cap(g->R) * arena_slots;
    z.look = 8 * Smax * enc_segments(g->R);
    z.ticket = 4 * kTicketStride * Smax;
    z.chunk = 8 * Smax * dec_chunks(g->R);
    z.queue = (int64_t)sizeof(BItem) * (items > 0 ? items : 1);
    z.qoff = 8 * (P + 1);
    z.qcount = 4 * P;
    z.roots = 8 * B;
    z.status = 4;
    z.counters = 8 * slots * (1 + B + 1 + Smax + B * P) + 8 * slots * Smax;
    z.fm = 8 * n;
    z.dstate = (int64_t)sizeof(BDirState);
    z.dirs = 4 * slots;
    return z;
}

}  // namespace

extern "C" int64_t csbfs_batch_engine_bytes(const csbfs_graph *g, int32_t max_roots, int32_t max_levels,
                                            uint32_t flags) {
    if (!g || max_roots < 1 || max_roots > kMaxRoots || max_levels < 1 || max_levels > 65536) return -1;
    return batch_sizes(g, max_roots, max_levels, flags).total();
}

namespace csbfs {

// A batch engine on a device block `mem` of csbfs_batch_engine_bytes bytes
// and a pinned two-word host buffer, both owned by the caller (null: the
// engine allocates them itself). Zeroing runs on `st` and is awaited with a
// synchronization of `st` alone.
int batch_engine_make(const csbfs_graph *g, int32_t max_roots, int32_t max_levels, uint32_t flags, void *mem,
                      unsigned long long *host_ctl, hipStream_t st, csbfs_batch_engine **out) {
    if (!out) return fail(CSBFS_EINVAL, "csbfs_batch_engine_create: out is NULL");
    *out = nullptr;
    if (!g) return fail(CSBFS_EINVAL, "csbfs_batch_engine_create: graph is NULL");
    if (max_roots < 1 || max_roots > kMaxRoots)
        return fail(CSBFS_EINVAL, "csbfs_batch_engine_create: max_roots outside [1, 64]");
    if (max_levels < 1 || max_levels > 65536)
        return fail(CSBFS_EINVAL, "csbfs_batch_engine_create: max_levels outside [1, 65536]");
    if (flags & ~(CSBFS_FLAG_TIMING | CSBFS_FLAG_KEEP_STREAMS | CSBFS_FLAG_NO_SIEVE | CSBFS_FLAG_SPARSE_ONLY |
                  CSBFS_FLAG_BOTTOM_UP_ONLY))
        return fail(CSBFS_EINVAL, "csbfs_batch_engine_create: unsupported flag");
    if ((flags & CSBFS_FLAG_SPARSE_ONLY) && (flags & CSBFS_FLAG_BOTTOM_UP_ONLY))
        return fail(CSBFS_EINVAL, "csbfs_batch_engine_create: SPARSE_ONLY and BOTTOM_UP_ONLY exclude each other");
    int rc = graph_device_check(g);
    if (rc) return rc;
    std::unique_ptr<csbfs_batch_engine> e(new csbfs_batch_engine());
    e->g = g;
    e->Bmax = max_roots;
    e->L = max_levels;
    e->flags = flags;
    const int64_t P = g->P, n = g->n, B = max_roots;
    e->cap = wah_cap(g->R);
    e->nseg = enc_segments(g->R);
    e->nchunk = dec_chunks(g->R);
    e->Smax = B * P * P;
    const int64_t slots = (int64_t)max_levels + 1;
    std::vector<int64_t> qoff(P + 1, 0);
    for (int64_t r = 0; r < P; ++r) qoff[r + 1] = qoff[r] + g->big_items[r];
    const BatchSizes z = batch_sizes(g, B, max_levels, flags);
    if (!mem) {
        CSBFS_HIP(hipMalloc(&e->mem, (size_t)z.total()));
        e->owns_mem = true;
    } else {
        e->mem = mem;
    }
    if (!host_ctl) {
        const hipError_t herr = hipHostMalloc((void **)&e->host_ctl, 2 * sizeof(unsigned long long));
        if (herr != hipSuccess) {
            e->host_ctl = nullptr;
            bengine_release(e.release());
            return hip_fail(herr, "hipHostMalloc", __FILE__, __LINE__);
        }
        e->owns_host = true;
    } else {
        e->host_ctl = host_ctl;
    }
    char *at = (char *)e->mem;
    auto carve = [&at](int64_t bytes) {
        void *p = at;
        at += align_up(bytes > 0 ? bytes : 1);
        return p;
    };
    e->vn = (uint64_t *)carve(z.vis);
    e->f = (uint64_t *)carve(z.f);
    e->view = (uint64_t *)carve(z.view);
    e->arena = (uint64_t *)carve(z.arena);
    // encoder look-back words, then its tickets: zero before the first encode
    e->look = (unsigned long long *)carve(z.look + z.ticket);
    e->enc_ticket = reinterpret_cast<uint32_t *>(e->look + e->Smax * e->nseg);
    e->chunk_groups = (int64_t *)carve(z.chunk);
    e->queue = (BItem *)carve(z.queue);
    e->qoff = (int64_t *)carve(z.qoff);
    e->qcount = (uint32_t *)carve(z.qcount);
    e->roots_dev = (int64_t *)carve(z.roots);
    e->status = (int32_t *)carve(z.status);
    e->fm = (uint64_t *)carve(z.fm);
    e->dstate = (BDirState *)carve(z.dstate);
    e->dirs = (int32_t *)carve(z.dirs);
    e->counters_mem = carve(z.counters);
    e->counters_bytes = (size_t)z.counters;
    e->look_bytes = (size_t)(z.look + z.ticket);
    unsigned long long *c = (unsigned long long *)e->counters_mem;
    e->ctl = c;
    c += slots;
    e->rootc = c;
    c += slots * B;
    e->edges = c;
    c += slots;
    e->sbits = c;
    c += slots * e->Smax;
    e->uwords = c;
    c += slots * B * P;
    e->words = (int64_t *)c;
    hipError_t herr = hipMemsetAsync(e->look, 0, e->look_bytes, st);
    if (herr == hipSuccess)
        herr = hipMemcpyAsync(e->qoff, qoff.data(), sizeof(int64_t) * (P + 1), hipMemcpyHostToDevice, st);
    if (herr == hipSuccess) herr = hipMemsetAsync(e->view, 0, sizeof(uint64_t) * B * P * (n / 64), st);
    if (herr == hipSuccess) herr = hipStreamSynchronize(st);  // qoff is read from host memory
    for (auto &ev : e->count_ev)
        if (herr == hipSuccess) herr = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
    if (herr == hipSuccess && (flags & CSBFS_FLAG_TIMING)) {
        e->events.assign((size_t)max_levels * kBEvPerLevel, nullptr);
        for (auto &ev : e->events)  // timestamps only: no system-scope fence at each record
            if (herr == hipSuccess) herr = hipEventCreateWithFlags(&ev, hipEventDisableSystemFence);
    }
    if (herr != hipSuccess) {
        bengine_release(e.release());
        return hip_fail(herr, "csbfs_batch_engine_create", __FILE__, __LINE__);
    }
    *out = e.release();
    return CSBFS_OK;
}

void batch_engine_release(csbfs_batch_engine *e) {
    if (e) bengine_release(e);
}

}  // namespace csbfs

extern "C" int csbfs_batch_engine_create(const csbfs_graph *g, int32_t max_roots, int32_t max_levels,
                                         uint32_t flags, csbfs_batch_engine **out) {
    return batch_engine_make(g, max_roots, max_levels, flags, nullptr, nullptr, nullptr, out);
}

extern "C" int csbfs_batch_engine_free(csbfs_batch_engine *e) {
    if (!e) return CSBFS_OK;
    bengine_release(e);
    return CSBFS_OK;
}

extern "C" int csbfs_batch_bfs(csbfs_batch_engine *e, const int64_t *roots, int32_t n_roots,
                               int32_t *level, csbfs_level_stats *stats, int32_t stats_cap,
                               int32_t *n_levels, void *stream) {
    if (!e || !roots || !level || !n_levels || stats_cap < 0 || (stats_cap > 0 && !stats))
        return fail(CSBFS_EINVAL, "csbfs_batch_bfs: null argument or negative stats_cap");
    if (n_roots < 1 || n_roots > e->Bmax)
        return fail(CSBFS_EINVAL, "csbfs_batch_bfs: n_roots outside [1, max_roots]");
    const csbfs_graph *g = e->g;
    for (int32_t r = 0; r < n_roots; ++r)
        if (roots[r] < 0 || roots[r] >= g->n) return fail(CSBFS_ERANGE, "csbfs_batch_bfs: root outside [0, n)");
    int rc = graph_device_check(g);
    if (rc) return rc;
    hipStream_t st = as_stream(stream);
    const int64_t P = g->P, n = g->n, R = g->R, W = g->W, B = n_roots, Bm = e->Bmax;
    const int64_t words = n / 64, vplane = P * words;
    const bool timing = (e->flags & CSBFS_FLAG_TIMING) != 0;
    const bool keep = (e->flags & CSBFS_FLAG_KEEP_STREAMS) != 0;

    // a0: seed every root
    CSBFS_HIP(hipMemsetAsync(e->counters_mem, 0, e->counters_bytes, st));
    CSBFS_HIP(hipMemsetAsync(e->status, 0, sizeof(int32_t), st));
    CSBFS_HIP(hipMemsetAsync(e->qcount, 0, sizeof(uint32_t) * P, st));
    // the encoder's tickets count on over the batch's levels: start them at zero
    CSBFS_HIP(hipMemsetAsync(e->look, 0, e->look_bytes, st));
    CSBFS_HIP(hipMemcpyAsync(e->roots_dev, roots, sizeof(int64_t) * B, hipMemcpyHostToDevice, st));
    BSeedArgs sa{e->vn, e->fm, e->view, B * vplane, level, B * n, n};
    // evaluation of each level: top-down, bottom-up, or chosen on the device
    const int32_t force = (e->flags & CSBFS_FLAG_SPARSE_ONLY)      ? CSBFS_DIR_TOP_DOWN
                          : (e->flags & CSBFS_FLAG_BOTTOM_UP_ONLY) ? CSBFS_DIR_BOTTOM_UP
                                                                   : -1;
    const int32_t dir0 = force == CSBFS_DIR_BOTTOM_UP ? CSBFS_DIR_BOTTOM_UP : CSBFS_DIR_TOP_DOWN;
    const int64_t fill = B * n > B * vplane ? B * n : B * vplane;
    hipLaunchKernelGGL(bseed_fill_kernel, dim3(grid_for(fill, 256, 16384)), dim3(256), 0, st, sa);
    CSBFS_HIP(hipGetLastError());
    hipLaunchKernelGGL(bseed_root_kernel, dim3(1), dim3(64), 0, st, sa, (const int64_t *)e->roots_dev,
                       (int32_t)B, R, W, (int32_t)P, vplane, e->rootc, e->ctl, e->dstate, dir0, force, e->dirs);
    CSBFS_HIP(hipGetLastError());

    BArgs ea{};
    ea.view = e->view;
    ea.vplane = vplane;
    ea.B = (int32_t)B;
    ea.row_ptr = g->row_ptr;
    ea.col_base = g->col_base;
    ea.col = g->col;
    ea.vn = e->vn;
    ea.queue = e->queue;
    ea.qoff = e->qoff;
    ea.queue_count = e->qcount;
    ea.R = R;
    ea.W = W;
    ea.P = (int32_t)P;
    ea.status = e->status;
    ea.dir = &e->dstate->cur;
    const unsigned grid = 2048;
    BPullArgs pa{};
    pa.vn = e->vn;
    pa.fm = e->fm;
    pa.pull_off = g->pull_off;
    pa.pull_col = g->pull_col;
    pa.head = g->head;
    pa.view = e->view;
    pa.view_words = B * vplane;
    pa.n = n;
    pa.B = (int32_t)B;
    pa.dir = &e->dstate->cur;

    WahBatch wb{};
    wb.bits_base = e->f;
    wb.mask_base = (e->flags & CSBFS_FLAG_NO_SIEVE) ? nullptr : g->dir;
    wb.nbits = R;
    wb.words_per_piece = W;
    wb.cap = e->cap;
    wb.P = (int32_t)P;
    wb.planes = (int32_t)B;
    wb.bits_plane_stride = words;
    wb.dst_plane_stride = vplane;
    wb.look = e->look;
    wb.ticket = e->enc_ticket;
    wb.nseg = e->nseg;
    wb.chunk_groups = e->chunk_groups;
    wb.nchunk = e->nchunk;
    wb.chunk_starts = 1;  // the decode reads the chunk starts the encode records
    wb.dst_base = e->view;
    wb.status = e->status;

    auto slot = [&](int64_t k) { return k < e->L ? k : (int64_t)e->L; };
    auto enqueue_iter = [&](int64_t j) -> int {
        const int64_t sj = slot(j), sn = slot(j + 1);
        if (j + 1 >= e->L) {
            const int64_t Lz = e->L;
            CSBFS_HIP(hipMemsetAsync(e->ctl + Lz, 0, sizeof(unsigned long long), st));
            CSBFS_HIP(hipMemsetAsync(e->rootc + Lz * Bm, 0, sizeof(unsigned long long) * Bm, st));
            CSBFS_HIP(hipMemsetAsync(e->edges + Lz, 0, sizeof(unsigned long long), st));
            CSBFS_HIP(hipMemsetAsync(e->sbits + Lz * e->Smax, 0, sizeof(unsigned long long) * e->Smax, st));
            CSBFS_HIP(hipMemsetAsync(e->uwords + Lz * Bm * P, 0, sizeof(unsigned long long) * Bm * P, st));
        }
        hipEvent_t *evp = (timing && j >= 1 && j - 1 < e->L) ? &e->events[(size_t)(j - 1) * kBEvPerLevel] : nullptr;
        hipEvent_t *ev = (timing && j < e->L) ? &e->events[(size_t)j * kBEvPerLevel] : nullptr;
        if (j >= 1) {
            wb.out_base = e->arena + (keep ? sj : 0) * e->Smax * e->cap;
            wb.n_words = e->words + sj * e->Smax;
            wb.stat_sieved_bits = e->sbits + sj * e->Smax;
            wb.stat_unsieved_words = e->uwords + sj * Bm * P;
            // roots whose level-j frontier is empty send nothing (the counter
            // slot past max_levels is reset before this encode: no skipping)
            wb.plane_count = j < e->L ? e->rootc + sj * Bm : nullptr;
            int r2 = launch_wah_encode(wb, st);
            if (r2) return r2;
            if (evp) CSBFS_HIP(hipEventRecord(evp[3], st));
            r2 = launch_wah_decode(wb, st);
            if (r2) return r2;
            if (evp) CSBFS_HIP(hipEventRecord(evp[4], st));
        }
        if (ev) CSBFS_HIP(hipEventRecord(ev[0], st));
        // the iteration after the last level (one of look-ahead) does nothing
        const unsigned long long *fc = j < e->L ? e->ctl + sj : nullptr;
        ea.edges = e->edges + sj;
        ea.fcount = fc;
        hipLaunchKernelGGL(bexpand_kernel, dim3(grid), dim3(kBThreads), 0, st, ea);
        CSBFS_HIP(hipGetLastError());
        // long rows: 1024 workgroups beat 512, 2048 and 4096 (a sweep, within 2%)
        hipLaunchKernelGGL(bexpand_big_kernel, dim3(1024), dim3(kBThreads), 0, st, ea);
        CSBFS_HIP(hipGetLastError());
        // the bottom-up evaluation (returns at once on top-down levels); past
        // the kept counters every root counts as active
        pa.rootc = j < e->L ? e->rootc + sj * Bm : nullptr;
        pa.edges = e->edges + sj;
        pa.fcount = fc;
        hipLaunchKernelGGL(bpull_kernel, dim3(grid), dim3(kBThreads), 0, st, pa);
        CSBFS_HIP(hipGetLastError());
        if (ev) CSBFS_HIP(hipEventRecord(ev[1], st));
        BUpdateArgs ua{e->vn, e->f, level, (int32_t)(j + 1), (int32_t)B, n,
                       e->rootc + sn * Bm, e->ctl + sn, e->qcount, (int32_t)P, fc,
                       e->fm, g->deg, e->dstate->sums};
        hipLaunchKernelGGL(bupdate_kernel, dim3(grid_for((words + kBTile - 1) / kBTile, kBThreads / 64, 2048)), dim3(kBThreads), 0, st, ua);
        CSBFS_HIP(hipGetLastError());
        // direction of the next level's expansion, from the update's sums
        hipLaunchKernelGGL(bdir_kernel, dim3(1), dim3(1), 0, st, e->dstate, j + 1 < e->L ? e->dirs + j + 1 : nullptr,
                           n, kBatchAlpha, kBatchBeta);
        CSBFS_HIP(hipGetLastError());
        if (ev) CSBFS_HIP(hipEventRecord(ev[2], st));
        const int hs = (int)((j + 1) & 1);
        CSBFS_HIP(hipMemcpyAsync(e->host_ctl + hs, e->ctl + sn, sizeof(unsigned long long),
                                 hipMemcpyDeviceToHost, st));
        CSBFS_HIP(hipEventRecord(e->count_ev[hs], st));
        return CSBFS_OK;
    };

    rc = enqueue_iter(0);
    if (rc) return rc;
    int64_t k = 0;
    for (;; ++k) {
        rc = enqueue_iter(k + 1);
        if (rc) return rc;
        const int hs = (int)((k + 1) & 1);
        CSBFS_HIP(hipEventSynchronize(e->count_ev[hs]));
        if (e->host_ctl[hs] == 0) break;
    }
    const int64_t nl = k + 1;
    *n_levels = (int32_t)(nl < INT32_MAX ? nl : INT32_MAX);
    e->last_levels = *n_levels;
    e->last_roots = (int32_t)B;

    int32_t hstatus = 0;
    CSBFS_HIP(hipMemcpyAsync(&hstatus, e->status, sizeof(hstatus), hipMemcpyDeviceToHost, st));
    const int64_t have = nl < e->L ? nl : e->L;
    const int64_t want = stats_cap < have ? stats_cap : have;
    std::vector<unsigned long long> rootc, ed, sb, uw;
    std::vector<int64_t> wd;
    std::vector<int32_t> dr;
    if (want > 0) {
        dr.resize(want);
        CSBFS_HIP(hipMemcpyAsync(dr.data(), e->dirs, sizeof(int32_t) * want, hipMemcpyDeviceToHost, st));
        rootc.resize(want * Bm);
        ed.resize(want);
        sb.resize(want * e->Smax);
        uw.resize(want * Bm * P);
        wd.resize(want * e->Smax);
        CSBFS_HIP(hipMemcpyAsync(rootc.data(), e->rootc, sizeof(unsigned long long) * want * Bm, hipMemcpyDeviceToHost, st));
        CSBFS_HIP(hipMemcpyAsync(ed.data(), e->edges, sizeof(unsigned long long) * want, hipMemcpyDeviceToHost, st));
        CSBFS_HIP(hipMemcpyAsync(sb.data(), e->sbits, sizeof(unsigned long long) * want * e->Smax, hipMemcpyDeviceToHost, st));
        CSBFS_HIP(hipMemcpyAsync(uw.data(), e->uwords, sizeof(unsigned long long) * want * Bm * P, hipMemcpyDeviceToHost, st));
        CSBFS_HIP(hipMemcpyAsync(wd.data(), e->words, sizeof(int64_t) * want * e->Smax, hipMemcpyDeviceToHost, st));
    }
    CSBFS_HIP(hipStreamSynchronize(st));
    if (hstatus != 0) {
        // an encode that gave up waiting may have left look-back state behind
        CSBFS_HIP(hipMemsetAsync(e->look, 0, e->look_bytes, st));
        CSBFS_HIP(hipStreamSynchronize(st));
        if (hstatus == 1) return fail(CSBFS_ECORRUPT, "csbfs_batch_bfs: a stream failed validation while decoding");
        return fail(CSBFS_ECORRUPT, "csbfs_batch_bfs: internal consistency check failed");
    }
    for (int64_t lv = 0; lv < want; ++lv) {
        csbfs_level_stats &s = stats[lv];
        s = csbfs_level_stats{};
        s.edges = (int64_t)ed[lv];
        s.direction = dr[lv];
        std::vector<int64_t> send(P, 0), recv(P, 0);
        for (int64_t r = 0; r < B; ++r) {
            const int64_t fr = (int64_t)rootc[lv * Bm + r];
            if (fr == 0) continue;
            s.frontier += fr;
            if (lv == 0) {
                s.view_bits += P;
                continue;
            }
            s.unsieved_bits += (P - 1) * fr;
            s.raw_bytes += P * (P - 1) * 8 * W;
            for (int64_t i = 0; i < P; ++i) {
                s.wah_unsieved_bytes += 8 * (P - 1) * (int64_t)uw[lv * Bm * P + r * P + i];
                for (int64_t j = 0; j < P; ++j) {
                    const int64_t sidx = lv * e->Smax + (r * P + i) * P + j;
                    s.view_bits += (int64_t)sb[sidx];
                    if (i == j) {
                        s.self_bytes += 8 * wd[sidx];
                        continue;
                    }
                    s.sieved_bits += (int64_t)sb[sidx];
                    s.wah_sieved_bytes += 8 * wd[sidx];
                    send[i] += 8 * wd[sidx];
                    recv[j] += 8 * wd[sidx];
                }
            }
        }
        for (int64_t i = 0; i < P; ++i) s.max_rank_bytes = std::max(s.max_rank_bytes, send[i] + recv[i]);
    }
    if (timing) {
        for (int64_t lv = 0; lv < nl && lv < e->L; ++lv) {
            hipEvent_t *ev = &e->events[(size_t)lv * kBEvPerLevel];
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

extern "C" int csbfs_batch_stream_words(const csbfs_batch_engine *e, int32_t *words, int32_t cap_levels) {
    if (!e || !words || cap_levels < 0) return fail(CSBFS_EINVAL, "csbfs_batch_stream_words: bad argument");
    const int64_t P = e->g->P, B = e->last_roots, Bm = e->Bmax;
    const int64_t lv_have = std::min<int64_t>(e->L, e->last_levels);
    std::vector<int64_t> wd((size_t)(lv_have > 0 ? lv_have : 1) * e->Smax);
    std::vector<unsigned long long> rc((size_t)(lv_have > 0 ? lv_have : 1) * Bm);
    if (lv_have > 0) {
        CSBFS_HIP(hipMemcpy(wd.data(), e->words, sizeof(int64_t) * lv_have * e->Smax, hipMemcpyDeviceToHost));
        CSBFS_HIP(hipMemcpy(rc.data(), e->rootc, sizeof(unsigned long long) * lv_have * Bm, hipMemcpyDeviceToHost));
    }
    for (int64_t lv = 0; lv < cap_levels; ++lv)
        for (int64_t r = 0; r < B; ++r)
            for (int64_t s = 0; s < P * P; ++s) {
                const bool live = lv > 0 && lv < lv_have && rc[lv * Bm + r] > 0;
                words[(lv * B + r) * P * P + s] = live ? (int32_t)wd[lv * e->Smax + r * P * P + s] : 0;
            }
    return CSBFS_OK;
}

extern "C" int csbfs_batch_copy_stream(const csbfs_batch_engine *e, int32_t k, int32_t r, int32_t i,
                                       int32_t j, uint64_t *dst, int64_t cap_words, int64_t *n_words_out,
                                       void *stream) {
    if (!e || !dst || !n_words_out) return fail(CSBFS_EINVAL, "csbfs_batch_copy_stream: null argument");
    if (!(e->flags & CSBFS_FLAG_KEEP_STREAMS))
        return fail(CSBFS_EINVAL, "csbfs_batch_copy_stream: engine lacks CSBFS_FLAG_KEEP_STREAMS");
    const int64_t P = e->g->P;
    if (k < 0 || k >= e->L || k >= e->last_levels || r < 0 || r >= e->last_roots || i < 0 || i >= P ||
        j < 0 || j >= P)
        return fail(CSBFS_EINVAL, "csbfs_batch_copy_stream: level, root or processor out of range");
    const int64_t s = ((int64_t)r * P + i) * P + j;
    hipStream_t st = as_stream(stream);
    int64_t nw = 0;
    unsigned long long fr = 0;
    CSBFS_HIP(hipMemcpyAsync(&fr, e->rootc + (int64_t)k * e->Bmax + r, sizeof(fr), hipMemcpyDeviceToHost, st));
    CSBFS_HIP(hipMemcpyAsync(&nw, e->words + (int64_t)k * e->Smax + s, sizeof(int64_t), hipMemcpyDeviceToHost, st));
    CSBFS_HIP(hipStreamSynchronize(st));
    if (k == 0 || fr == 0) nw = 0;  // no message carries level 0 or an empty frontier
    *n_words_out = nw;
    if (nw > cap_words) return fail(CSBFS_ENOSPACE, "csbfs_batch_copy_stream: dst too small");
    if (nw > 0)
        CSBFS_HIP(hipMemcpyAsync(dst, e->arena + ((int64_t)k * e->Smax + s) * e->cap, sizeof(uint64_t) * nw,
                                 hipMemcpyDeviceToDevice, st));
    CSBFS_HIP(hipStreamSynchronize(st));
    return CSBFS_OK;
}
