// rtm_codec.h -- launch parameters of the block-transform codec kernels
// (rtm_codec.hip), shared with the host runtime (rtm_runtime.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace rtm {

constexpr int kZcChunk = 256;              // blocks per chunk = threads per workgroup
constexpr uint32_t kZcMagic = 0x315A5452;  // "RTZ1"
constexpr int kZcHeaderWords = 8;
constexpr int64_t kZcMaxBlocks = (1LL << 26) - 1;  // keeps payload offsets below 2^32 words

// error bits the kernels raise in ZcParams::flags
constexpr uint32_t kZcRange = 1u;     // a value is non-finite or beyond the tolerance's range
constexpr uint32_t kZcCapacity = 2u;  // the stream did not fit the caller's buffer
constexpr uint32_t kZcSpin = 4u;      // a chunk prefix did not arrive within the wait bound
constexpr uint32_t kZcCorrupt = 8u;   // decode: widths, chunk table or length inconsistent

struct ZcParams {
  const float* x;       // encode input [count][rows][cols]
  float* y;             // decode output, same layout
  uint32_t* out;        // encode: stream words
  const uint32_t* in;   // decode: stream words
  uint64_t* status;     // encode: [nchunks] look-back state, zeroed before launch
  uint32_t* ticket;     // encode: chunk ticket counter, zeroed before launch
  uint32_t* flags;      // error bits, zeroed before launch
  uint32_t* result;     // encode: [0] total payload words
  int32_t count, rows, cols, mode;
  int32_t bz, bx, nblocks, nchunks;
  int64_t hdr_base;     // word index of the block headers
  int64_t pay_base;     // word index of the payload
  int64_t cap_words;    // encode: capacity of out; decode: words available in
  double r;             // 1 / (2 tol)
  double step;          // 2 tol
  uint32_t head[8];     // encode: the stream's first eight words
};

hipError_t launch_zc_encode(const ZcParams& p, hipStream_t s);
hipError_t launch_zc_decode(const ZcParams& p, hipStream_t s);

// Device scratch of the encoder that allocates nothing (rtm_codec_encode_noalloc):
// the look-back state of up to kZcNoAllocChunks chunks (8 bytes each) and
// 64 bytes of ticket, flags and result words, in a file-scope device array
// each device holds until the process ends.
constexpr size_t kZcNoAllocBytes = size_t(1) << 20;
constexpr int64_t kZcNoAllocChunks = (int64_t)(kZcNoAllocBytes - 256) / 8;
// Looks up the array's address on `device` (which must be current) once and
// keeps it; later calls return the kept address.
hipError_t zc_noalloc_scratch_init(int device);
// The kept address of the array on `device`, or null before a successful init.
void* zc_noalloc_scratch(int device);

}  // namespace rtm
