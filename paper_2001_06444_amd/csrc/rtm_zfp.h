// rtm_zfp.h -- launch parameters of the fixed-accuracy ZFP-method coder
// (rtm_zfp.hip), shared with the host runtime (rtm_runtime.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace rtm {

constexpr uint32_t kZfMagic = 0x465A5452;  // "RTZF"
constexpr int kZfMode = 2;                 // the stream's mode word (RTM_CODEC_ZFP)
constexpr int kZfChunk = 16;               // 4 x 4 blocks per chunk
constexpr int kZfThreads = 64;             // decoder: lanes (chunks) per workgroup
constexpr int kZfEncThreads = 256;         // encoder: lanes (blocks) per workgroup
constexpr int kZfHeaderWords = 8;
constexpr int64_t kZfMaxBlocks = int64_t(1) << 27;  // keeps payload word offsets below 2^32
// Longest block code: 1 + 8 header bits, at most 16 verbatim bits per plane
// over 32 planes, at most 32 failed and 16 successful group tests and 16
// scan bits: 585 bits.
constexpr int kZfMaxBlockBits = 585;
constexpr int kZfBlockWords = (kZfMaxBlockBits + 31) / 32;              // 19
constexpr int kZfChunkWords = (kZfChunk * kZfMaxBlockBits + 31) / 32;   // 293
constexpr int64_t kZfMaxStageBytes = 65536;  // decoder: LDS budget per workgroup, at most

// error bits the kernels raise in ZfParams::flags
constexpr uint32_t kZfRange = 1u;    // a value is non-finite or |x| >= 2^100
constexpr uint32_t kZfCorrupt = 8u;  // decode: chunk table or block codes inconsistent
constexpr uint32_t kZfSpin = 16u;    // encode: a look-back wait exceeded its bound

struct ZfParams {
  const float* x;      // encode input [count][rows][cols]
  float* y;            // decode output, same layout
  uint32_t* out;       // encode: stream words
  const uint32_t* in;  // decode: stream words
  uint32_t* flags;     // error bits, zeroed before launch
  uint32_t* result;    // encode: [0..1] total payload words (64-bit)
  uint64_t* status;    // encode: look-back state, one word per workgroup, zeroed before launch
  uint32_t* ticket;    // encode: workgroup order, zeroed before launch
  int32_t count, rows, cols, minexp;
  int32_t bz, bx;
  int64_t nblocks, nchunks;
  int64_t hdr_base;    // word index of the chunk table
  int64_t pay_base;    // word index of the payload
  int64_t cap_words;   // encode: capacity of out; decode: words in the stream
  uint32_t head[8];    // encode: the stream's first eight words
};

// Encoder: p.status [(nblocks + kZfEncThreads - 1) / kZfEncThreads] and
// p.ticket are device scratch, zeroed before the launch.
hipError_t launch_zf_encode(const ZfParams& p, hipStream_t s);
// Decoder: stage_bytes is the LDS budget per workgroup for the staged
// payload (0: every lane reads global memory; negative: chosen from the
// stream's mean payload per workgroup); at most kZfMaxStageBytes.
hipError_t launch_zf_decode(const ZfParams& p, int64_t stage_bytes, hipStream_t s);

}  // namespace rtm
