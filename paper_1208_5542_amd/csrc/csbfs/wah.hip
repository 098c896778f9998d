// WAH-64 sieve + compress and decompress kernels (Sec. IV, Table 3; Alg. 3
// sieve, Compress and Uncompress), batched over the p * p streams of a level.
//
// Encoder. Group x of a piece is bits [63x, 63x + 63). A group is Z (all 0),
// O (all 1) or L (mixed). Group x starts a word iff it is L, or x = 0, or its
// class differs from group x - 1's; a run-starting fill group x covers the
// groups up to the next word-starting group. Pass 1 (wah_enc_count) counts
// word-starting groups per segment of kEncSeg groups and records the first
// one; pass 2 (wah_enc_emit) turns the counts of earlier segments into the
// segment's output offset, ranks the word-starting groups with a block scan,
// and writes every word, reading the end of a trailing run from the first
// word-starting group of the later segments. The sieve (AND with the
// directory vector) is applied while the segment is staged into LDS, so the
// sieved piece is never written to memory.
//
// Decoder. Pass 1 (wah_dec_count) sums the groups each chunk of kDecChunk
// words covers; pass 2 (wah_dec_scatter) gives every word its first group by a
// block scan plus the totals of earlier chunks, and ORs literal and 1-fill
// bits into the destination (0-fills write nothing: the destination starts
// zeroed). Every stream is validated: zero-length fills, group totals that do
// not match floor(N/63), or active-word bits above r set the status flag.
#include "common.hpp"

namespace csbfs {
namespace {

constexpr int kEncLds = ((kEncSeg + 2) * kGroupBits) / 64 + 4;

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

__device__ __forceinline__ SegGeom seg_geom(const WahBatch &b, int64_t seg) {
    SegGeom g;
    g.G = b.nbits / kGroupBits;
    g.r = b.nbits - g.G * kGroupBits;
    g.x0 = seg * kEncSeg;
    g.x1 = g.x0 + kEncSeg < g.G ? g.x0 + kEncSeg : g.G;
    g.last = seg == b.nseg - 1;
    const int64_t bit_lo = (g.x0 > 0 ? g.x0 - 1 : 0) * kGroupBits;
    const int64_t bit_hi = g.last ? b.nbits : g.x1 * kGroupBits;  // exclusive
    g.wlo = bit_lo >> 6;
    g.nload = bit_hi > bit_lo ? ((bit_hi - 1) >> 6) - g.wlo + 1 : 0;
    return g;
}

// Stage the segment's words (sieved, and optionally unsieved) into LDS.
__device__ __forceinline__ void stage(const WahBatch &b, int64_t s, const SegGeom &g, uint64_t *sw,
                                      uint64_t *su) {
    const StreamIdx x = stream_idx(s, b.P);
    const int64_t i = x.i, j = x.j;
    const uint64_t *bits = b.bits_base + x.r * b.bits_plane_stride + i * b.words_per_piece;
    const uint64_t *mask = b.mask_base ? b.mask_base + (j * b.P + i) * b.words_per_piece : nullptr;
    const int tail = (int)(b.nbits & 63);
    for (int64_t k = threadIdx.x; k < g.nload; k += blockDim.x) {
        const int64_t w = g.wlo + k;
        uint64_t v = bits[w];
        if (tail && w == b.words_per_piece - 1) v &= (1ull << tail) - 1;
        if (su) su[k] = v;
        if (mask) v &= mask[w];
        sw[k] = v;
    }
    __syncthreads();
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

// Count word-starting groups of a thread's kEncGpt groups.
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

__global__ __launch_bounds__(kEncThreads) void wah_enc_count(WahBatch b) {
    __shared__ uint64_t sw[kEncLds];
    __shared__ uint64_t su[kEncLds];
    const int64_t seg = blockIdx.x;
    const int64_t s = blockIdx.y;
    if (plane_skipped(b, s)) {
        if (seg == 0 && threadIdx.x == 0) b.n_words[s] = 0;
        return;
    }
    const StreamIdx x = stream_idx(s, b.P);
    const int64_t i = x.i, j = x.j;
    const bool unsieved = b.stat_unsieved_words && i == j;
    const SegGeom g = seg_geom(b, seg);
    stage(b, s, g, sw, unsieved ? su : nullptr);

    const int64_t xa = g.x0 + (int64_t)threadIdx.x * kEncGpt;
    const int64_t xb = xa + kEncGpt < g.x1 ? xa + kEncGpt : g.x1;
    int flags = 0, first = INT32_MAX;
    long long ones = 0;
    if (xa < g.x1) classify(sw, g, xa, xb, flags, first, ones);
    const int cnt = block_reduce(flags, SumI32(), 0);
    const int fst = block_reduce(first, MinI32(), INT32_MAX);
    long long tot = block_reduce(ones, SumI64(), 0LL);
    int ucnt = 0;
    if (unsieved) {
        int uf = 0, ufirst;
        long long uones;
        if (xa < g.x1) classify(su, g, xa, xb, uf, ufirst, uones);
        ucnt = block_reduce(uf, SumI32(), 0);
    }
    if (threadIdx.x == 0) {
        b.seg_count[s * b.nseg + seg] = cnt;
        b.seg_first[s * b.nseg + seg] = fst;
        if (g.last && g.r > 0) tot += __popcll(active_word(sw, g));
        if (b.stat_sieved_bits && tot) atomicAdd(&b.stat_sieved_bits[s], (unsigned long long)tot);
        if (unsieved) {
            const int words = ucnt + (g.last && g.r > 0 ? 1 : 0);
            if (words) atomicAdd(&b.stat_unsieved_words[x.r * b.P + i], (unsigned long long)words);
        }
    }
}

__global__ __launch_bounds__(kEncThreads) void wah_enc_emit(WahBatch b) {
    __shared__ uint64_t sw[kEncLds];
    __shared__ int starts[kEncSeg + 1];
    const int64_t seg = blockIdx.x;
    const int64_t s = blockIdx.y;
    if (plane_skipped(b, s)) return;
    const SegGeom g = seg_geom(b, seg);

    // Output offset and the first word-starting group after this segment.
    int before = 0, after = INT32_MAX;
    for (int64_t k = threadIdx.x; k < b.nseg; k += blockDim.x) {
        if (k < seg) before += b.seg_count[s * b.nseg + k];
        else if (k > seg) after = min(after, b.seg_first[s * b.nseg + k]);
    }
    const int offset = block_reduce(before, SumI32(), 0);
    after = block_reduce(after, MinI32(), INT32_MAX);
    const int64_t next_after = after == INT32_MAX ? g.G : after;

    stage(b, s, g, sw, nullptr);
    const int64_t xa = g.x0 + (int64_t)threadIdx.x * kEncGpt;
    const int64_t xb = xa + kEncGpt < g.x1 ? xa + kEncGpt : g.x1;
    int cls[kEncGpt];
    uint64_t val[kEncGpt];
    int nflag = 0;
    if (xa < g.x1) {
        int prev = xa > 0 ? group_class(group_bits(sw, xa - 1, g.wlo)) : -1;
        for (int k = 0; k < kEncGpt; ++k) {
            const int64_t x = xa + k;
            cls[k] = -1;
            if (x >= xb) continue;
            val[k] = group_bits(sw, x, g.wlo);
            const int c = group_class(val[k]);
            if (c == 2 || c != prev) {
                cls[k] = c;
                ++nflag;
            }
            prev = c;
        }
    } else {
        for (int k = 0; k < kEncGpt; ++k) cls[k] = -1;
    }
    int seg_words = 0;
    const int base = block_excl_scan(nflag, &seg_words);
    {
        int pos = base;
        for (int k = 0; k < kEncGpt; ++k)
            if (cls[k] >= 0) starts[pos++] = (int)(xa + k);
    }
    if (threadIdx.x == 0) starts[seg_words] = (int)next_after;
    __syncthreads();

    uint64_t *out = b.out_base + s * b.cap;
    int pos = base;
    for (int k = 0; k < kEncGpt; ++k) {
        if (cls[k] < 0) continue;
        const int64_t x = xa + k;
        uint64_t word;
        if (cls[k] == 2) {
            word = __builtin_bitreverse64(val[k]) >> 1;  // bit (62 - t) = group bit t
        } else {
            const uint64_t c = (uint64_t)(starts[pos + 1] - x);
            word = kFillFlag | (cls[k] == 1 ? kFillBit : 0) | c;
        }
        out[offset + pos] = word;
        ++pos;
    }
    if (g.last && threadIdx.x == 0) {
        int64_t total = offset + seg_words;
        if (g.r > 0) out[total++] = active_word(sw, g);
        b.n_words[s] = total;
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

__global__ __launch_bounds__(kDecThreads) void wah_dec_count(WahBatch b) {
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

__global__ __launch_bounds__(kDecThreads) void wah_dec_scatter(WahBatch b) {
    const int64_t c = blockIdx.x;
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
    for (int64_t k = threadIdx.x; k < c; k += blockDim.x) before += b.chunk_groups[s * b.nchunk + k];
    before = block_reduce(before, SumI64(), 0LL);

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

int launch_wah_encode(const WahBatch &b, hipStream_t stream) {
    const int64_t S = batch_streams(b);
    dim3 grid((unsigned)b.nseg, (unsigned)S);
    hipLaunchKernelGGL(wah_enc_count, grid, dim3(kEncThreads), 0, stream, b);
    CSBFS_HIP(hipGetLastError());
    hipLaunchKernelGGL(wah_enc_emit, grid, dim3(kEncThreads), 0, stream, b);
    CSBFS_HIP(hipGetLastError());
    return CSBFS_OK;
}

int launch_wah_decode(const WahBatch &b, hipStream_t stream) {
    const int64_t S = batch_streams(b);
    dim3 grid((unsigned)b.nchunk, (unsigned)S);
    hipLaunchKernelGGL(wah_dec_count, grid, dim3(kDecThreads), 0, stream, b);
    CSBFS_HIP(hipGetLastError());
    hipLaunchKernelGGL(wah_dec_scatter, grid, dim3(kDecThreads), 0, stream, b);
    CSBFS_HIP(hipGetLastError());
    return CSBFS_OK;
}

}  // namespace csbfs

// ------------------------------------------------------------ C ABI ---

using namespace csbfs;

namespace {
constexpr size_t kAlign = 256;
size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }
struct WsLayout {
    size_t seg_count, seg_first, chunk_groups, n_words, total;
};
WsLayout ws_layout(int64_t nbits) {
    WsLayout l;
    const int64_t nseg = enc_segments(nbits);
    const int64_t nchunk = dec_chunks(nbits);
    l.seg_count = 0;
    l.seg_first = l.seg_count + align_up(sizeof(int32_t) * nseg);
    l.chunk_groups = l.seg_first + align_up(sizeof(int32_t) * nseg);
    l.n_words = l.chunk_groups + align_up(sizeof(int64_t) * nchunk);
    l.total = l.n_words + align_up(sizeof(int64_t));
    return l;
}
}  // namespace

extern "C" int64_t csbfs_wah_capacity(int64_t nbits) { return nbits < 0 ? -1 : wah_cap(nbits); }

extern "C" size_t csbfs_wah_workspace_bytes(int64_t nbits) {
    return nbits < 0 ? 0 : ws_layout(nbits).total;
}

extern "C" int csbfs_wah_encode(const uint64_t *bits, const uint64_t *mask, int64_t nbits,
                                uint64_t *out, int64_t cap_words, int64_t *n_words,
                                void *workspace, size_t ws_bytes, void *stream) {
    if (nbits < 0 || !out || !n_words || !workspace || (nbits > 0 && !bits))
        return fail(CSBFS_EINVAL, "csbfs_wah_encode: null pointer or negative size");
    if (nbits >= ((int64_t)1 << 37))
        return fail(CSBFS_EINVAL, "csbfs_wah_encode: nbits too large");
    if (cap_words < wah_cap(nbits))
        return fail(CSBFS_ENOSPACE, "csbfs_wah_encode: output capacity below floor(nbits/63)+1");
    const WsLayout l = ws_layout(nbits);
    if (ws_bytes < l.total) return fail(CSBFS_ENOSPACE, "csbfs_wah_encode: workspace too small");
    char *ws = (char *)workspace;
    WahBatch b{};
    b.bits_base = bits;
    b.mask_base = mask;
    b.out_base = out;
    b.n_words = n_words;
    b.nbits = nbits;
    b.words_per_piece = (nbits + 63) / 64;
    b.cap = cap_words;
    b.P = 1;
    b.seg_count = (int32_t *)(ws + l.seg_count);
    b.seg_first = (int32_t *)(ws + l.seg_first);
    b.nseg = enc_segments(nbits);
    if (nbits == 0) {
        CSBFS_HIP(hipMemsetAsync(n_words, 0, sizeof(int64_t), as_stream(stream)));
        return CSBFS_OK;
    }
    return launch_wah_encode(b, as_stream(stream));
}

extern "C" int csbfs_wah_decode_or(const uint64_t *words, int64_t n_words, int64_t nbits,
                                   uint64_t *dst, int32_t *status, void *workspace,
                                   size_t ws_bytes, void *stream) {
    if (nbits < 0 || n_words < 0 || !status || !workspace || (nbits > 0 && !dst) ||
        (n_words > 0 && !words))
        return fail(CSBFS_EINVAL, "csbfs_wah_decode_or: null pointer or negative size");
    if (nbits >= ((int64_t)1 << 37))
        return fail(CSBFS_EINVAL, "csbfs_wah_decode_or: nbits too large");
    const WsLayout l = ws_layout(nbits);
    if (ws_bytes < l.total) return fail(CSBFS_ENOSPACE, "csbfs_wah_decode_or: workspace too small");
    hipStream_t st = as_stream(stream);
    CSBFS_HIP(hipMemsetAsync(status, 0, sizeof(int32_t), st));
    if (n_words > wah_cap(nbits)) {
        const int32_t one = 1;
        CSBFS_HIP(hipMemcpyAsync(status, &one, sizeof(one), hipMemcpyHostToDevice, st));
        CSBFS_HIP(hipStreamSynchronize(st));
        return CSBFS_OK;
    }
    if (nbits == 0) {
        if (n_words != 0) {
            const int32_t one = 1;
            CSBFS_HIP(hipMemcpyAsync(status, &one, sizeof(one), hipMemcpyHostToDevice, st));
            CSBFS_HIP(hipStreamSynchronize(st));
        }
        return CSBFS_OK;
    }
    char *ws = (char *)workspace;
    int64_t *nw_dev = (int64_t *)(ws + l.n_words);
    CSBFS_HIP(hipMemcpyAsync(nw_dev, &n_words, sizeof(int64_t), hipMemcpyHostToDevice, st));
    WahBatch b{};
    b.out_base = const_cast<uint64_t *>(words);
    b.n_words = nw_dev;
    b.nbits = nbits;
    b.words_per_piece = (nbits + 63) / 64;
    b.cap = n_words > 0 ? n_words : 1;
    b.P = 1;
    b.chunk_groups = (int64_t *)(ws + l.chunk_groups);
    b.nchunk = dec_chunks(nbits);
    b.dst_base = dst;
    b.status = status;
    int rc = launch_wah_decode(b, st);
    if (rc != CSBFS_OK) return rc;
    // the host-to-device copies above read stack memory: finish before returning
    CSBFS_HIP(hipStreamSynchronize(st));
    return CSBFS_OK;
}
