#pragma once
// Device side of the WAH-64 codec, shared by the codec's kernels and the
// search's fused kernels (internal linkage in each file that includes it).
//
// Sieve + compress and decompress (Sec. IV, Table 3; Alg. 3
// sieve, Compress and Uncompress), batched over the p * p streams of a level.
//
// Encoder. Group x of a piece is bits [63x, 63x + 63). A group is Z (all 0),
// O (all 1) or L (mixed). Group x starts a word iff it is L, or x = 0, or its
// class differs from group x - 1's; a run-starting fill group x covers the
// groups up to the next word-starting group. One pass (encode_segment): a
// workgroup per segment of kEncThreads x kGpt groups ranks the word-starting
// groups with a block scan, finds the count of those before the segment by
// a decoupled look-back over the earlier segments' published counts, and
// writes its words; a fill that runs past the segment's end is written by
// the segment where the run ends. The sieve (AND with the directory vector)
// is applied while the segment is staged into LDS, so the sieved piece is
// never written to memory.
//
// Decoder. dec_scatter_body gives every word its first group by a block scan
// from its chunk's first group, and ORs literal and 1-fill
// bits into the destination (0-fills write nothing: the destination starts
// zeroed). A chunk of kDecChunk words learns its first group from the
// encoder, which records it while writing the chunk's first word (searches),
// or from a first pass (dec_count_body) that sums the groups of every chunk
// (streams from elsewhere). Every stream is validated: zero-length fills,
// group totals that do not match floor(N/63), chunks that do not meet, or
// active-word bits above r set the status flag.
#include "device.hpp"

namespace csbfs {
namespace {

// LDS words that stage a segment of seg groups and the group before it
constexpr int enc_lds_words(int seg) { return ((seg + 2) * kGroupBits) / 64 + 4; }

__device__ __forceinline__ int wave_incl_scan(int v) {
    const int lane = threadIdx.x & (kWave - 1);
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
        int t = __shfl_up(v, d, kWave);
        if (lane >= d) v += t;
    }
    return v;
}

__device__ __forceinline__ long long wave_incl_scan64(long long v) {
    const int lane = threadIdx.x & (kWave - 1);
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
        long long t = __shfl_up(v, d, kWave);
        if (lane >= d) v += t;
    }
    return v;
}

// Exclusive scan over the block (blockDim.x a multiple of 64, at most 1024);
// returns the exclusive prefix and writes the block total to *total.
__device__ int block_excl_scan(int v, int *total) {
    __shared__ int wsum[16];
    const int lane = threadIdx.x & (kWave - 1);
    const int wid = threadIdx.x / kWave;
    const int nw = blockDim.x / kWave;
    int incl = wave_incl_scan(v);
    if (lane == kWave - 1) wsum[wid] = incl;
    __syncthreads();
    if (wid == 0) {
        int s = lane < nw ? wsum[lane] : 0;
        s = wave_incl_scan(s);
        if (lane < nw) wsum[lane] = s;
    }
    __syncthreads();
    int before = wid > 0 ? wsum[wid - 1] : 0;
    *total = wsum[nw - 1];
    __syncthreads();
    return before + incl - v;
}

__device__ long long block_excl_scan64(long long v, long long *total) {
    __shared__ long long wsum64[16];
    const int lane = threadIdx.x & (kWave - 1);
    const int wid = threadIdx.x / kWave;
    const int nw = blockDim.x / kWave;
    long long incl = wave_incl_scan64(v);
    if (lane == kWave - 1) wsum64[wid] = incl;
    __syncthreads();
    if (wid == 0) {
        long long s = lane < nw ? wsum64[lane] : 0;
        s = wave_incl_scan64(s);
        if (lane < nw) wsum64[lane] = s;
    }
    __syncthreads();
    long long before = wid > 0 ? wsum64[wid - 1] : 0;
    *total = wsum64[nw - 1];
    __syncthreads();
    return before + incl - v;
}

template <typename T, typename Op>
__device__ T block_reduce(T v, Op op, T identity) {
    __shared__ T red[16];
    const int lane = threadIdx.x & (kWave - 1);
    const int wid = threadIdx.x / kWave;
    const int nw = blockDim.x / kWave;
#pragma unroll
    for (int d = kWave / 2; d > 0; d >>= 1) v = op(v, __shfl_xor(v, d, kWave));
    if (lane == 0) red[wid] = v;
    __syncthreads();
    T r = identity;
    for (int k = 0; k < nw; ++k) r = op(r, red[k]);
    __syncthreads();
    return r;
}

struct SumI64 {
    __device__ long long operator()(long long a, long long b) const { return a + b; }
};
struct MinI32 {
    __device__ int operator()(int a, int b) const { return a < b ? a : b; }
};
struct SumI32 {
    __device__ int operator()(int a, int b) const { return a + b; }
};

// 63 bits of group x from words staged in LDS; word 0 of `arr` is piece word wlo.
__device__ __forceinline__ uint64_t group_bits(const uint64_t *arr, int64_t x, int64_t wlo) {
    const int64_t sb = x * kGroupBits - wlo * 64;
    const int64_t a = sb >> 6;
    const int off = (int)(sb & 63);
    uint64_t v = arr[a] >> off;
    if (off > 1) v |= arr[a + 1] << (64 - off);
    return v & kMask63;
}

__device__ __forceinline__ int group_class(uint64_t v) {
    return v == 0 ? 0 : (v == kMask63 ? 1 : 2);
}

struct SegGeom {
    int64_t G, r, x0, x1, wlo, nload;
    bool last;
};

template <int kSeg>
__device__ __forceinline__ SegGeom seg_geom(const WahBatch &b, int64_t seg) {
    SegGeom g;
    g.G = b.nbits / kGroupBits;
    g.r = b.nbits - g.G * kGroupBits;
    g.x0 = seg * kSeg;
    g.x1 = g.x0 + kSeg < g.G ? g.x0 + kSeg : g.G;
    g.last = seg == b.nseg - 1;
    const int64_t bit_lo = (g.x0 > 0 ? g.x0 - 1 : 0) * kGroupBits;
    const int64_t bit_hi = g.last ? b.nbits : g.x1 * kGroupBits;  // exclusive
    g.wlo = bit_lo >> 6;
    g.nload = bit_hi > bit_lo ? ((bit_hi - 1) >> 6) - g.wlo + 1 : 0;
    return g;
}

// Stage the segment's words (sieved, and optionally unsieved) into LDS; the
// hook gives word w of sender i's piece in plane r before the sieve. A thread
// loads all its words (at most kIt) and their directory words before it
// uses any, so the loads of a segment overlap instead of forming a chain.
template <int kIt, class Hook>
__device__ __forceinline__ void stage(const WahBatch &b, int64_t s, const SegGeom &g, uint64_t *sw,
                                      uint64_t *su, const Hook &h) {
    const StreamIdx x = stream_idx(s, b.P);
    const int64_t i = x.i, j = x.j;
    const uint64_t *mask = b.mask_base ? b.mask_base + (j * b.P + i) * b.words_per_piece : nullptr;
    const int tail = (int)(b.nbits & 63);
    uint64_t v[kIt], m[kIt];
#pragma unroll
    for (int it = 0; it < kIt; ++it) {
        const int64_t k = threadIdx.x + (int64_t)it * blockDim.x;
        const int64_t w = g.wlo + k;
        v[it] = k < g.nload ? h.load(b, x.r, i, w) : 0;
        m[it] = (mask && k < g.nload) ? mask[w] : ~0ull;
    }
#pragma unroll
    for (int it = 0; it < kIt; ++it) {
        const int64_t k = threadIdx.x + (int64_t)it * blockDim.x;
        if (k < g.nload) {
            const int64_t w = g.wlo + k;
            uint64_t vv = v[it];
            if (tail && w == b.words_per_piece - 1) vv &= (1ull << tail) - 1;
            if (su) su[k] = vv;
            sw[k] = vv & m[it];
        }
    }
    __syncthreads();
}

// The codec's own words: the bits buffer of the batch.
struct PlainWords {
    __device__ __forceinline__ uint64_t load(const WahBatch &b, int64_t r, int64_t i, int64_t w) const {
        return b.bits_base[r * b.bits_plane_stride + i * b.words_per_piece + w];
    }
    // no segment is known to be all zero without reading it
    __device__ __forceinline__ bool clean(const WahBatch &, int64_t, const StreamIdx &) const { return false; }
    __device__ __forceinline__ bool prev_clean(const WahBatch &, int64_t, const StreamIdx &) const { return false; }
    __device__ __forceinline__ void init() {}
    __device__ __forceinline__ void side(const WahBatch &, int64_t, int64_t, const StreamIdx &) {}
    __device__ __forceinline__ void finish(const WahBatch &, int64_t, int64_t) {}
};

// Class of group gx read straight from memory (sieved or not): the clean
// segment's look at the group before it.
template <class Hook>
__device__ int group_class_direct(const WahBatch &b, const StreamIdx &x, int64_t gx, const Hook &h, bool sieved) {
    const uint64_t *mask = sieved && b.mask_base ? b.mask_base + (x.j * b.P + x.i) * b.words_per_piece : nullptr;
    const int tail = (int)(b.nbits & 63);
    auto word = [&](int64_t w) {
        uint64_t v = h.load(b, x.r, x.i, w);
        if (tail && w == b.words_per_piece - 1) v &= (1ull << tail) - 1;
        if (mask && v) v &= mask[w];
        return v;
    };
    const int64_t sb = gx * kGroupBits;
    const int64_t w0 = sb >> 6;
    const int off = (int)(sb & 63);
    uint64_t v = word(w0) >> off;
    if (off > 1) v |= word(w0 + 1) << (64 - off);
    return group_class(v & kMask63);
}

// r trailing bits, right-aligned, first bit most significant.
__device__ __forceinline__ uint64_t active_word(const uint64_t *arr, const SegGeom &g) {
    const int64_t sb = g.G * kGroupBits - g.wlo * 64;
    const int64_t a = sb >> 6;
    const int off = (int)(sb & 63);
    uint64_t v = arr[a] >> off;
    if (off + g.r > 64) v |= arr[a + 1] << (64 - off);
    v &= (1ull << g.r) - 1;
    return __builtin_bitreverse64(v) >> (64 - g.r);
}

// Count word-starting groups of a thread's groups [xa, xb).
__device__ __forceinline__ void classify(const uint64_t *arr, const SegGeom &g, int64_t xa,
                                         int64_t xb, int &flags, int &first, long long &ones) {
    int prev = xa > 0 ? group_class(group_bits(arr, xa - 1, g.wlo)) : -1;
    flags = 0;
    first = INT32_MAX;
    ones = 0;
    for (int64_t x = xa; x < xb; ++x) {
        const uint64_t v = group_bits(arr, x, g.wlo);
        const int c = group_class(v);
        ones += __popcll(v);
        if (c == 2 || c != prev) {
            ++flags;
            if (first == INT32_MAX) first = (int)x;
        }
        prev = c;
    }
}

// A plane whose frontier is empty sends no message (batched searches).
__device__ __forceinline__ bool plane_skipped(const WahBatch &b, int64_t s) {
    return b.plane_count && b.plane_count[s / ((int64_t)b.P * b.P)] == 0;
}

// Look-back words of the encoder, one per (stream, segment): a segment's
// state and value sit in one 64-bit word written by one atomic store, so a
// reader sees both or neither. State 1 holds the segment's own aggregate,
// state 2 the inclusive prefix through it. A value is (count of word-starting
// groups, the last of them, its class) and prefixes combine by adding the
// counts and keeping the later last group.
//
// Launches of one stream's encoder follow each other without clearing
// anything: its ticket counts on (every launch takes nseg tickets, so ticket
// t is segment t % nseg of the stream's launch t / nseg), and every word
// carries the parity of that launch number. Each launch rewrites all of its
// stream's words, so a word of the other parity is the last launch's and
// reads as not yet published.
constexpr int kLbBits = 29;  // count and group-index fields: at most 2^29 - 1 groups
constexpr uint64_t kLbField = (1ull << kLbBits) - 1;
constexpr uint64_t kLbAgg = 1ull << 62, kLbInc = 2ull << 62;
constexpr uint64_t kLbHasLast = 1ull << 60;
constexpr uint64_t kLbEpoch = 1ull << 61;  // parity of the stream's launch
constexpr uint64_t kLbLastMask = (kLbField << kLbBits) | (3ull << (2 * kLbBits)) | kLbHasLast;
constexpr uint32_t kLbSpinLimit = 1u << 22;  // polls of one look-back window

__device__ __forceinline__ uint64_t lb_value(int64_t cnt, int64_t last, int cls) {
    return (uint64_t)cnt | (cnt ? ((uint64_t)last << kLbBits) | ((uint64_t)cls << (2 * kLbBits)) | kLbHasLast : 0);
}

// Exclusive prefix of segment seg (> 0) of one stream, by wave 0: windows of
// up to 64 earlier segments are read at once, each lane waiting for its
// segment to publish in this launch (parity ep), until a window holds an
// inclusive prefix.
__device__ uint64_t lb_prefix(const WahBatch &b, unsigned long long *look, int64_t seg, uint64_t ep) {
    const int lane = threadIdx.x & 63;
    int64_t cnt = 0;
    uint64_t last = 0;
    auto ready = [ep](uint64_t v) { return (v >> 62) != 0 && (v & kLbEpoch) == ep; };
    for (int64_t k0 = seg - 1;; k0 -= 64) {
        const int64_t k = k0 - lane;
        // lanes before segment 0 hold an empty inclusive prefix
        uint64_t v = k >= 0 ? __hip_atomic_load(&look[k], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)
                            : (kLbInc | ep);
        uint32_t polls = 0;
        while (__ballot(!ready(v))) {
            if (++polls == kLbSpinLimit) {  // a lost publication: flag the stream, stop waiting
                if (lane == 0 && b.status) *b.status = 1;
                if (!ready(v)) v = kLbInc | ep;
                break;
            }
            if (!ready(v)) v = __hip_atomic_load(&look[k], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        const uint64_t inc = __ballot((v >> 62) == 2);
        const int stop = inc ? __ffsll((unsigned long long)inc) - 1 : 63;
        long long c = lane <= stop ? (long long)(v & kLbField) : 0;
#pragma unroll
        for (int d = 32; d > 0; d >>= 1) c += __shfl_xor(c, d, 64);
        cnt += c;
        const uint64_t has = __ballot(lane <= stop && (v & kLbHasLast));
        if (!last && has) last = readlane64(v, __ffsll((unsigned long long)has) - 1) & kLbLastMask;
        if (inc) break;
    }
    return (uint64_t)cnt | last;
}

// One pass per stream segment: stage, classify, publish the segment's count,
// look back for the counts before it, write its words. The trailing fill of
// a segment ends at a later segment's first word-starting group, so the
// segment holding that group (or the last segment, which ends every run)
// writes the fill word; the look-back carries its start and class. The last
// workgroup's ticket gives its segment and the parity of this launch of the
// stream (see the look-back words above).
//
// The hook stages the words (Hook::load), may do other work with waves 1..
// while wave 0 looks back (Hook::side), and finishes that work with thread 0
// (Hook::finish) once the workgroup's sums are in. The workgroup encodes a
// segment of stream s; `first` marks one workgroup per stream (it reports
// the empty stream of a skipped plane).
template <int kGpt, class Hook>
__device__ __forceinline__ void encode_segment(const WahBatch &b, Hook &hook, int64_t s, bool first) {
    constexpr int kSeg = kEncThreads * kGpt;  // groups per segment
    constexpr int kLds = enc_lds_words(kSeg);
    __shared__ uint64_t sw[kLds];
    __shared__ uint64_t su[kLds];
    // groups that start a word, relative to the segment's first group (16
    // bits, so that four workgroups of the encoder fit a CU's LDS)
    static_assert(kSeg <= 65536, "16-bit group offsets");
    __shared__ uint16_t starts[kSeg];
    __shared__ int sh_last_cls;
    __shared__ uint64_t sh_prefix;
    __shared__ uint32_t sh_ticket;
    __shared__ int sh_clean_words;
    if (plane_skipped(b, s)) {
        if (first && threadIdx.x == 0) b.n_words[s] = 0;
        return;
    }
    // segments in the order the workgroups start, so every awaited one runs
    uint32_t *ticket = b.ticket + s * kTicketStride;  // segments started, over all launches
    if (threadIdx.x == 0) sh_ticket = atomicAdd(&ticket[0], 1u);
    hook.init();
    __syncthreads();
    const uint32_t tk = sh_ticket;
    const int64_t seg = (int64_t)(tk % (uint32_t)b.nseg);
    const uint64_t ep = ((tk / (uint32_t)b.nseg) & 1u) ? kLbEpoch : 0;
    const StreamIdx x = stream_idx(s, b.P);
    const bool unsieved = b.stat_unsieved_words && x.i == x.j;
    const SegGeom g = seg_geom<kSeg>(b, seg);
    // A clean segment (all zero, known from the hook without reading it) is
    // a run of 0-groups: it starts a word only at group 0 or after a group
    // of another class, which it reads from memory if the segment before is
    // not clean too. Nothing is staged.
    const bool clean = hook.clean(b, seg, x);
    int clean_uflag = 0;
    if (!clean) stage<(kLds + kEncThreads - 1) / kEncThreads>(b, s, g, sw, unsieved ? su : nullptr, hook);

    const int64_t xa = g.x0 + (int64_t)threadIdx.x * kGpt;
    const int64_t xb = xa + kGpt < g.x1 ? xa + kGpt : g.x1;
    int cls[kGpt];
    uint64_t val[kGpt];
    int nflag = 0;
    long long ones = 0;
#pragma unroll
    for (int k = 0; k < kGpt; ++k) cls[k] = -1;
    if (clean) {
        if (threadIdx.x == 0 && g.x0 < g.x1) {
            const bool first = seg == 0;
            const bool look = !first && !hook.prev_clean(b, seg, x);
            if (first || (look && group_class_direct(b, x, g.x0 - 1, hook, true) != 0)) {
                cls[0] = 0;
                nflag = 1;
            }
            if (unsieved && (first || (look && group_class_direct(b, x, g.x0 - 1, hook, false) != 0)))
                clean_uflag = 1;
        }
    } else if (xa < g.x1) {
        int prev = xa > 0 ? group_class(group_bits(sw, xa - 1, g.wlo)) : -1;
        for (int k = 0; k < kGpt; ++k) {
            const int64_t gx = xa + k;
            if (gx >= xb) break;
            val[k] = group_bits(sw, gx, g.wlo);
            ones += __popcll(val[k]);
            const int c = group_class(val[k]);
            if (c == 2 || c != prev) {
                cls[k] = c;
                ++nflag;
            }
            prev = c;
        }
    }
    int seg_words = 0, base = 0;
    if (clean) {
        // only thread 0 can start a word (at the segment's first group)
        if (threadIdx.x == 0) {
            sh_clean_words = nflag;
            if (nflag) {
                sh_last_cls = cls[0];
                starts[0] = (uint16_t)(xa - g.x0);
            }
        }
        __syncthreads();
        seg_words = sh_clean_words;
    } else {
        base = block_excl_scan(nflag, &seg_words);
        int pos = base;
        for (int k = 0; k < kGpt; ++k) {
            if (cls[k] < 0) continue;
            if (pos == seg_words - 1) sh_last_cls = cls[k];
            starts[pos++] = (uint16_t)(xa + k - g.x0);
        }
        __syncthreads();
    }

    unsigned long long *look = b.look + s * b.nseg;
    // a clean segment that starts no word and is not the last writes nothing:
    // it publishes its (empty) aggregate and needs no prefix
    const bool quiet = clean && seg_words == 0 && !g.last && seg > 0;
    if (threadIdx.x < 64) {
        const uint64_t mine = lb_value(seg_words, seg_words ? g.x0 + starts[seg_words - 1] : 0, sh_last_cls);
        if (quiet) {
            if (threadIdx.x == 0) {
                __hip_atomic_store(&look[seg], mine | kLbAgg | ep, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                sh_prefix = 0;
            }
        } else if (seg == 0) {
            if (threadIdx.x == 0) {
                __hip_atomic_store(&look[0], mine | kLbInc | ep, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                sh_prefix = 0;
            }
        } else {
            if (threadIdx.x == 0)
                __hip_atomic_store(&look[seg], mine | kLbAgg | ep, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            const uint64_t pre = lb_prefix(b, look, seg, ep);
            if (threadIdx.x == 0) {
                const uint64_t inc = ((pre & kLbField) + seg_words) | (seg_words ? (mine & kLbLastMask) : (pre & kLbLastMask));
                __hip_atomic_store(&look[seg], inc | kLbInc | ep, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                sh_prefix = pre;
            }
        }
    } else {
        hook.side(b, s, seg, x);
    }
    __syncthreads();
    const uint64_t pre = sh_prefix;
    const int64_t offset = (int64_t)(pre & kLbField);

    // every index is below the stream's capacity unless the look-back failed
    uint64_t *out = b.out_base + s * b.cap;
    int64_t *cstart = b.chunk_starts ? b.chunk_groups + s * b.nchunk : nullptr;
    const bool fits = offset + seg_words + 1 <= b.cap;
    int pos = base;
    for (int k = 0; k < kGpt && fits; ++k) {
        if (cls[k] < 0) continue;
        const int64_t gx = xa + k;
        if (cstart && (offset + pos) % kDecChunk == 0) cstart[(offset + pos) / kDecChunk] = gx;
        if (cls[k] == 2) {
            out[offset + pos] = __builtin_bitreverse64(val[k]) >> 1;  // bit (62 - t) = group bit t
        } else if (pos + 1 < seg_words || g.last) {
            const int64_t end = pos + 1 < seg_words ? g.x0 + starts[pos + 1] : g.G;
            out[offset + pos] = kFillFlag | (cls[k] == 1 ? kFillBit : 0) | (uint64_t)(end - gx);
        }
        ++pos;
    }
    if (threadIdx.x == 0) {
        if (!fits && b.status) *b.status = 1;
        // the fill that began at the last word-starting group before this segment
        const int prev_cls = (int)((pre >> (2 * kLbBits)) & 3);
        if (fits && offset >= 1 && (pre & kLbHasLast) && prev_cls != 2 && (seg_words > 0 || g.last)) {
            const int64_t begin = (int64_t)((pre >> kLbBits) & kLbField);
            const int64_t end = seg_words > 0 ? g.x0 + starts[0] : g.G;
            out[offset - 1] = kFillFlag | (prev_cls == 1 ? kFillBit : 0) | (uint64_t)(end - begin);
            if (cstart && (offset - 1) % kDecChunk == 0) cstart[(offset - 1) / kDecChunk] = begin;
        }
        if (g.last) {
            int64_t total = offset + seg_words;
            if (g.r > 0 && fits) out[total++] = clean ? 0ull : active_word(sw, g);
            b.n_words[s] = fits ? total : 0;
        }
    }

    // statistics: set bits after the sieve, words of the unsieved piece
    // (a clean segment has no ones, and only thread 0 may count an unsieved word)
    long long tot = 0;
    int ucnt = clean_uflag;
    if (!clean) {
        tot = block_reduce(ones, SumI64(), 0LL);
        if (unsieved) {
            int uf = 0, ufirst;
            long long uones;
            if (xa < g.x1) classify(su, g, xa, xb, uf, ufirst, uones);
            ucnt = block_reduce(uf, SumI32(), 0);
        }
    }
    if (threadIdx.x == 0) {
        if (g.last && g.r > 0 && !clean) tot += __popcll(active_word(sw, g));
        if (b.stat_sieved_bits && tot) atomicAdd(&b.stat_sieved_bits[s], (unsigned long long)tot);
        if (unsieved) {
            const int words = ucnt + (g.last && g.r > 0 ? 1 : 0);
            if (words) atomicAdd(&b.stat_unsieved_words[x.r * b.P + x.i], (unsigned long long)words);
        }
        hook.finish(b, s, seg);
    }
}

__device__ __forceinline__ int64_t stream_words(const WahBatch &b, int64_t s) {
    return b.n_words[s];
}

__device__ __forceinline__ void or_bits(uint64_t *dst, int64_t bit, uint64_t v, int nbits) {
    // OR nbits (<= 63) bits of v, bit t of v to bit (bit + t) of dst.
    const int64_t q = bit >> 6;
    const int sh = (int)(bit & 63);
    const uint64_t lo = v << sh;
    if (lo) atomicOr((unsigned long long *)&dst[q], (unsigned long long)lo);
    if (sh + nbits > 64) {
        const uint64_t hi = v >> (64 - sh);
        if (hi) atomicOr((unsigned long long *)&dst[q + 1], (unsigned long long)hi);
    }
}

__device__ void fill_ones(uint64_t *dst, int64_t lo, int64_t hi) {
    // set bits [lo, hi) of dst
    int64_t q0 = lo >> 6, q1 = (hi - 1) >> 6;
    for (int64_t q = q0; q <= q1; ++q) {
        const int64_t a = lo > q * 64 ? lo - q * 64 : 0;
        const int64_t e = hi < q * 64 + 64 ? hi - q * 64 : 64;
        if (a == 0 && e == 64) {
            dst[q] = ~0ull;
        } else {
            const uint64_t m = (e == 64 ? ~0ull : ((1ull << e) - 1)) & ~((1ull << a) - 1);
            atomicOr((unsigned long long *)&dst[q], (unsigned long long)m);
        }
    }
}

// The same two helpers on a workgroup's LDS copy of a range of words.
constexpr int kDecLdsWords = 2048;

__device__ __forceinline__ void or_bits_lds(unsigned long long *buf, int64_t bit, uint64_t v, int nbits) {
    const int64_t q = bit >> 6;
    const int sh = (int)(bit & 63);
    const uint64_t lo = v << sh;
    if (lo) atomicOr(&buf[q], (unsigned long long)lo);
    if (sh + nbits > 64) {
        const uint64_t hi = v >> (64 - sh);
        if (hi) atomicOr(&buf[q + 1], (unsigned long long)hi);
    }
}

__device__ void fill_ones_lds(unsigned long long *buf, int64_t lo, int64_t hi) {
    int64_t q0 = lo >> 6, q1 = (hi - 1) >> 6;
    for (int64_t q = q0; q <= q1; ++q) {
        const int64_t a = lo > q * 64 ? lo - q * 64 : 0;
        const int64_t e = hi < q * 64 + 64 ? hi - q * 64 : 64;
        if (a == 0 && e == 64) {
            buf[q] = ~0ull;  // a whole word inside one fill has no other writer
        } else {
            const uint64_t m = (e == 64 ? ~0ull : ((1ull << e) - 1)) & ~((1ull << a) - 1);
            atomicOr(&buf[q], (unsigned long long)m);
        }
    }
}

__device__ __forceinline__ void dec_count_body(const WahBatch &b) {
    const int64_t c = blockIdx.x;
    const int64_t s = blockIdx.y;
    if (plane_skipped(b, s)) return;
    const int64_t G = b.nbits / kGroupBits;
    const int64_t r = b.nbits - G * kGroupBits;
    const int64_t nw = stream_words(b, s);
    const int64_t nreg = nw - (r > 0 ? 1 : 0);
    const uint64_t *words = b.out_base + s * b.cap;
    long long groups = 0;
    bool bad = false;
    const int64_t w0 = c * kDecChunk;
    for (int64_t w = w0 + threadIdx.x; w < w0 + kDecChunk && w < nreg; w += blockDim.x) {
        const uint64_t v = words[w];
        if (v & kFillFlag) {
            const uint64_t cnt = v & kCountMask;
            if (cnt == 0 || cnt > (uint64_t)G) bad = true;
            groups += (long long)cnt;
        } else {
            groups += 1;
        }
    }
    groups = block_reduce(groups, SumI64(), 0LL);
    if (bad) *b.status = 1;
    if (threadIdx.x == 0) b.chunk_groups[s * b.nchunk + c] = groups;
}

__device__ __forceinline__ void dec_scatter_body(const WahBatch &b, int64_t c = -1) {
    if (c < 0) c = blockIdx.x;
    const int64_t s = blockIdx.y;
    if (plane_skipped(b, s)) return;
    const StreamIdx si = stream_idx(s, b.P);
    const int64_t i = si.i, j = si.j;
    const int64_t G = b.nbits / kGroupBits;
    const int64_t r = b.nbits - G * kGroupBits;
    const int64_t nw = stream_words(b, s);
    const int64_t nreg = nw - (r > 0 ? 1 : 0);
    const uint64_t *words = b.out_base + s * b.cap;
    uint64_t *dst = b.dst_base + si.r * b.dst_plane_stride + (j * b.P + i) * b.words_per_piece;
    const int64_t w0 = c * kDecChunk;

    if (c == 0 && threadIdx.x == 0) {
        if (nw < 0 || nreg < 0 || (nw == 0 && b.nbits > 0) || nw > b.cap) {
            *b.status = 1;
        } else if (r > 0) {
            const uint64_t a = words[nw - 1];
            if (a >> r) {
                *b.status = 1;
            } else if (a) {
                const uint64_t v = __builtin_bitreverse64(a) >> (64 - r);
                or_bits(dst, G * kGroupBits, v, (int)r);
            }
        }
        if (nreg == 0 && G != 0) *b.status = 1;
    }
    if (nw < 0 || nw > b.cap || w0 >= nreg) return;

    long long before = 0;
    if (b.chunk_starts) {
        before = c > 0 ? b.chunk_groups[s * b.nchunk + c] : 0;
        if (before < 0 || before > G) {
            if (threadIdx.x == 0) *b.status = 1;
            return;
        }
    } else {
        for (int64_t k = threadIdx.x; k < c; k += blockDim.x) before += b.chunk_groups[s * b.nchunk + k];
        before = block_reduce(before, SumI64(), 0LL);
    }

    uint64_t v[kDecWpt];
    long long g[kDecWpt];
    long long mine = 0;
    const int64_t wa = w0 + (int64_t)threadIdx.x * kDecWpt;
    for (int k = 0; k < kDecWpt; ++k) {
        const int64_t w = wa + k;
        g[k] = 0;
        if (w < nreg) {
            v[k] = words[w];
            g[k] = (v[k] & kFillFlag) ? (long long)(v[k] & kCountMask) : 1;
            mine += g[k];
        }
    }
    long long chunk_total;
    long long x = before + block_excl_scan64(mine, &chunk_total);
    // recorded starts: this chunk must end where the next one starts
    if (b.chunk_starts && threadIdx.x == 0 && w0 + kDecChunk < nreg &&
        before + chunk_total != b.chunk_groups[s * b.nchunk + c + 1])
        *b.status = 1;

    // The chunk's groups [g0, g1) fill output words [q0, q1]. When those fit
    // in LDS (always for literal words: 1024 groups span 1008 words) the
    // chunk is assembled there and written with one store per word; only
    // the two end words, which neighbouring chunks also touch, need global
    // atomics. Chunks whose fills span more words OR straight into dst.
    __shared__ unsigned long long lbuf[kDecLdsWords];
    const long long g0 = before, g1 = before + chunk_total;
    const int64_t q0 = (g0 * kGroupBits) >> 6;
    const int64_t q1 = g1 > g0 ? (g1 * kGroupBits - 1) >> 6 : q0;
    const bool staged = g1 > g0 && g1 <= G && q1 - q0 + 1 <= kDecLdsWords;
    if (staged) {
        for (int64_t k = threadIdx.x; k <= q1 - q0; k += blockDim.x) lbuf[k] = 0;
        __syncthreads();
    }
    const int64_t base_bit = q0 * 64;
    bool bad = false;
    for (int k = 0; k < kDecWpt; ++k) {
        const int64_t w = wa + k;
        if (w >= nreg) break;
        if (g[k] == 0 || x + g[k] > G) {
            bad = true;
            break;
        }
        if (!(v[k] & kFillFlag)) {
            const uint64_t bits = __builtin_bitreverse64(v[k]) >> 1;
            if (bits) {
                if (staged)
                    or_bits_lds(lbuf, x * kGroupBits - base_bit, bits, kGroupBits);
                else
                    or_bits(dst, x * kGroupBits, bits, kGroupBits);
            }
        } else if (v[k] & kFillBit) {
            if (staged)
                fill_ones_lds(lbuf, x * kGroupBits - base_bit, (x + g[k]) * kGroupBits - base_bit);
            else
                fill_ones(dst, x * kGroupBits, (x + g[k]) * kGroupBits);
        }
        x += g[k];
        if (w == nreg - 1 && x != G) bad = true;
    }
    if (bad) *b.status = 1;
    if (staged) {
        __syncthreads();
        for (int64_t k = threadIdx.x; k <= q1 - q0; k += blockDim.x) {
            const unsigned long long val = lbuf[k];
            if (!val) continue;
            const int64_t q = q0 + k;
            if (q == q0 || q == q1)
                atomicOr((unsigned long long *)&dst[q], val);
            else
                dst[q] |= val;  // no other workgroup writes an inner word
        }
    }
}

}  // namespace
}  // namespace csbfs
