// Internal declarations shared by the csbfs translation units (not installed).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <string>

#include "csbfs.h"

namespace csbfs {

// ---------------------------------------------------------------- errors ---

void set_error(const std::string &msg);
int fail(int status, const std::string &msg);
int hip_fail(hipError_t err, const char *what, const char *file, int line);

#define CSBFS_HIP(call)                                                     \
    do {                                                                    \
        hipError_t _e = (call);                                             \
        if (_e != hipSuccess)                                               \
            return ::csbfs::hip_fail(_e, #call, __FILE__, __LINE__);        \
    } while (0)

inline hipStream_t as_stream(void *s) { return reinterpret_cast<hipStream_t>(s); }

// ------------------------------------------------------------- constants ---

constexpr int kWave = 64;             // gfx950 wavefront
constexpr int kGroupBits = 63;        // WAH-64 group
constexpr uint64_t kFillFlag = 1ull << 63;
constexpr uint64_t kFillBit = 1ull << 62;
constexpr uint64_t kCountMask = (1ull << 62) - 1;
constexpr uint64_t kMask63 = (1ull << 63) - 1;

// Encoder tiling: a workgroup of kEncThreads threads classifies one segment
// of kEncSeg groups, kEncGpt consecutive groups per thread.
constexpr int kEncThreads = 512;
// Encoder tickets of a stream: its own 128-byte line (atomics on one line
// are serialized).
constexpr int kTicketStride = 32;
constexpr int kEncGpt = 4;
constexpr int kEncSeg = kEncThreads * kEncGpt;
// Decoder tiling: a workgroup reads one chunk of kDecChunk stream words.
constexpr int kDecThreads = 512;  // 512 x 2 beat 256 x 4 for the same chunk (scale 22)
constexpr int kDecWpt = 2;
constexpr int kDecChunk = kDecThreads * kDecWpt;

inline int64_t wah_cap(int64_t nbits) { return nbits / kGroupBits + 1; }
// Segments of an encoder with gpt groups per thread (kEncGpt by default;
// searches on small pieces take 2 to get more workgroups).
inline int64_t enc_segments(int64_t nbits, int gpt = kEncGpt) {
    int64_t G = nbits / kGroupBits;
    const int64_t seg = (int64_t)kEncThreads * gpt;
    return G == 0 ? 1 : (G + seg - 1) / seg;
}
inline int64_t dec_chunks(int64_t nbits) { return (wah_cap(nbits) + kDecChunk - 1) / kDecChunk; }

// ---------------------------------------------------------- WAH batches ---
//
// A batch holds S = planes * P * P streams (one plane per search root; one
// plane for a single search). Stream s = (r * P + i) * P + j carries the
// piece of processor i in plane r (bits_base + r * bits_plane_stride + i *
// words_per_piece) sieved with the directory vector V_{j,i} (mask_base +
// (j * P + i) * words_per_piece, or no mask), is written to out_base + s *
// cap, and is decoded into dst_base + r * dst_plane_stride + (j * P + i) *
// words_per_piece (receiver j's view of the range of i, plane r).

struct WahBatch {
    const uint64_t *bits_base;
    const uint64_t *mask_base;  // nullable
    uint64_t *out_base;
    int64_t *n_words;           // device [S]
    int64_t nbits;              // bits per piece
    int64_t words_per_piece;    // ceil(nbits / 64)
    int64_t cap;                // words per stream slot
    int32_t P;
    int32_t planes;             // 0 or 1 for one search
    int64_t bits_plane_stride;
    int64_t dst_plane_stride;
    // encoder scratch, zero between launches (each launch leaves it zero):
    // per (stream, segment) look-back words; per stream a segment ticket and
    // a count of finished segments
    unsigned long long *look;   // device [S * nseg]
    uint32_t *ticket;           // device [kTicketStride * S]
    int64_t nseg;
    // decoder scratch: per (stream, chunk) group totals, or (chunk_starts)
    // the first group of each chunk, recorded by the encoder: the decoder
    // then runs one pass and checks that consecutive chunks meet
    int64_t *chunk_groups;      // device [S * nchunk]
    int64_t nchunk;
    int32_t chunk_starts;
    uint64_t *dst_base;         // decoder output
    int32_t *status;            // device [1], non-zero on a corrupt stream
    // optional statistics (device, nullable)
    unsigned long long *stat_sieved_bits;    // [S]
    unsigned long long *stat_unsieved_words; // [planes * P]: words of WAH(piece_i), no mask
    // optional (device, nullable): frontier size of each plane; the streams
    // of a plane whose frontier is empty get 0 words and decode nothing
    const unsigned long long *plane_count;   // [planes]
};

// Stream s of a batch: plane r, sender i, receiver j.
struct StreamIdx {
    int64_t r, i, j;
};
__host__ __device__ inline StreamIdx stream_idx(int64_t s, int32_t P) {
    const int64_t pp = (int64_t)P * P, s2 = s % pp;
    return StreamIdx{s / pp, s2 / P, s2 % P};
}
inline int64_t batch_streams(const WahBatch &b) {
    return (int64_t)(b.planes > 1 ? b.planes : 1) * b.P * b.P;
}

int launch_wah_encode(const WahBatch &b, hipStream_t stream);
int launch_wah_decode(const WahBatch &b, hipStream_t stream);

}  // namespace csbfs
