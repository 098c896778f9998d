// WAH-64 sieve + compress and decompress kernels (Sec. IV, Table 3; Alg. 3
// sieve, Compress and Uncompress), batched over the p * p streams of a level;
// the device code is in wah_device.hpp.
#include <mutex>

#include "wah_device.hpp"

namespace csbfs {
namespace {

__global__ __launch_bounds__(kEncThreads) void wah_encode_kernel(WahBatch b) {
    PlainWords h;
    encode_segment<kEncGpt>(b, h, blockIdx.y, blockIdx.x == 0);
}

__global__ __launch_bounds__(kDecThreads) void wah_dec_count(WahBatch b) { dec_count_body(b); }

__global__ __launch_bounds__(kDecThreads) void wah_dec_scatter(WahBatch b) { dec_scatter_body(b); }

// Zero `words` 32-bit words (a kernel rather than a memset node, so that the
// allocation-free entry point can be captured into a HIP graph).
__global__ void zero_words_kernel(uint32_t *p, int64_t words) {
    for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < words;
         k += (int64_t)gridDim.x * blockDim.x)
        p[k] = 0;
}

__global__ void store_i64_kernel(int64_t *p, int64_t v) { *p = v; }

}  // namespace

int launch_wah_encode(const WahBatch &b, hipStream_t stream) {
    const int64_t S = batch_streams(b);
    if (b.nbits / kGroupBits > kLbField) return fail(CSBFS_EINVAL, "WAH encode: more than 2^29 - 1 groups");
    dim3 grid((unsigned)b.nseg, (unsigned)S);
    hipLaunchKernelGGL(wah_encode_kernel, grid, dim3(kEncThreads), 0, stream, b);
    CSBFS_HIP(hipGetLastError());
    return CSBFS_OK;
}

int launch_wah_decode(const WahBatch &b, hipStream_t stream) {
    const int64_t S = batch_streams(b);
    dim3 grid((unsigned)b.nchunk, (unsigned)S);
    if (!b.chunk_starts) {
        hipLaunchKernelGGL(wah_dec_count, grid, dim3(kDecThreads), 0, stream, b);
        CSBFS_HIP(hipGetLastError());
    }
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
    size_t look, ticket, chunk_groups, n_words, total;
};
WsLayout ws_layout(int64_t nbits) {
    WsLayout l;
    const int64_t nseg = enc_segments(nbits);
    const int64_t nchunk = dec_chunks(nbits);
    l.look = 0;
    l.ticket = l.look + align_up(sizeof(unsigned long long) * nseg);
    l.chunk_groups = l.ticket + align_up(sizeof(uint32_t) * kTicketStride);
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
    if (nbits / kGroupBits > (int64_t)kLbField)
        return fail(CSBFS_EINVAL, "csbfs_wah_encode: nbits above 63 * (2^29 - 1)");
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
    b.look = (unsigned long long *)(ws + l.look);
    b.ticket = (uint32_t *)(ws + l.ticket);
    b.nseg = enc_segments(nbits);
    if (nbits == 0) {
        CSBFS_HIP(hipMemsetAsync(n_words, 0, sizeof(int64_t), as_stream(stream)));
        return CSBFS_OK;
    }
    // the look-back words and tickets start at zero (the caller's workspace
    // may hold anything)
    CSBFS_HIP(hipMemsetAsync(ws + l.look, 0, l.chunk_groups - l.look, as_stream(stream)));
    return launch_wah_encode(b, as_stream(stream));
}

// ------------------------------------------- allocation-free encoder ---
//
// Scratch of csbfs_wah_encode_noalloc: the encoder's look-back words and
// segment tickets, in a file-scope device array. Each GPU the library runs
// on holds its own copy until the process ends. Host code never passes the
// array's name to a kernel (on the host it is only a stand-in symbol): the
// device address is looked up once per device with hipGetSymbolAddress and
// that pointer is used everywhere.
namespace {
constexpr size_t kNoAllocScratchBytes = 256 * 1024;
__device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

int scratch_ptr(void **out) {
    int dev = -1;
    CSBFS_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return fail(CSBFS_EINVAL, "csbfs_wah_encode_noalloc: device id out of range");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) return hip_fail(e, "hipGetSymbolAddress(scratch)", __FILE__, __LINE__);
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return CSBFS_OK;
}
}  // namespace

extern "C" int64_t csbfs_wah_noalloc_max_bits(void) {
    // the largest nbits whose look-back words and tickets fit the scratch
    int64_t lo = 0, hi = 63 * (int64_t)kLbField;
    while (lo < hi) {
        const int64_t mid = lo + (hi - lo + 1) / 2;
        const WsLayout l = ws_layout(mid);
        if (l.chunk_groups <= kNoAllocScratchBytes)
            lo = mid;
        else
            hi = mid - 1;
    }
    return lo;
}

extern "C" int csbfs_wah_encode_noalloc(const uint64_t *bits, const uint64_t *mask, int64_t nbits, uint64_t *out,
                                        int64_t cap_words, int64_t *n_words, void *stream) {
    if (nbits < 0 || !out || !n_words || (nbits > 0 && !bits))
        return fail(CSBFS_EINVAL, "csbfs_wah_encode_noalloc: null pointer or negative size");
    if (nbits > csbfs_wah_noalloc_max_bits())
        return fail(CSBFS_EINVAL, "csbfs_wah_encode_noalloc: nbits above csbfs_wah_noalloc_max_bits() (the "
                                  "encoder's scratch is a fixed 256 KiB device array)");
    if (cap_words < wah_cap(nbits))
        return fail(CSBFS_ENOSPACE, "csbfs_wah_encode_noalloc: output capacity below floor(nbits/63)+1");
    void *ptr = nullptr;
    int rc = scratch_ptr(&ptr);
    if (rc) return rc;
    hipStream_t st = as_stream(stream);
    if (nbits == 0) {
        hipLaunchKernelGGL(store_i64_kernel, dim3(1), dim3(1), 0, st, n_words, (int64_t)0);
        CSBFS_HIP(hipGetLastError());
        return CSBFS_OK;
    }
    const WsLayout l = ws_layout(nbits);
    char *ws = (char *)ptr;
    // look-back words and tickets start at zero; the previous call on this
    // device left them zero unless it failed, so clear them every time
    const int64_t words = (int64_t)((l.chunk_groups - l.look) / 4);
    hipLaunchKernelGGL(zero_words_kernel, dim3((unsigned)((words + 255) / 256)), dim3(256), 0, st,
                       (uint32_t *)(ws + l.look), words);
    CSBFS_HIP(hipGetLastError());
    WahBatch b{};
    b.bits_base = bits;
    b.mask_base = mask;
    b.out_base = out;
    b.n_words = n_words;
    b.nbits = nbits;
    b.words_per_piece = (nbits + 63) / 64;
    b.cap = cap_words;
    b.P = 1;
    b.look = (unsigned long long *)(ws + l.look);
    b.ticket = (uint32_t *)(ws + l.ticket);
    b.nseg = enc_segments(nbits);
    return launch_wah_encode(b, st);
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
