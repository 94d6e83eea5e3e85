// rtm_zfp.hip -- fixed-accuracy coder of the published ZFP method for 2-D
// float32 arrays (the data-compression stage of the workflow: Sec. 3,
// data-compression paragraph; Sec. 4.2, Tables 1-2, which use ZFP's
// fixed-accuracy mode at absolute error bounds 1e-4 and 1e-1).
//
// The method (Lindstrom, IEEE TVCG 20(12), 2014), per 4 x 4 block, edges
// repeated:
//   1. block floating point: e = exponent of the largest |x| (f 2^e, f in
//      [1/2, 1)), q = trunc(x 2^(30 - e)) as int32 (two guard bits);
//   2. the non-orthogonal decorrelating transform
//        T = 1/16 [[4, 4, 4, 4], [5, 1, -1, -5], [-4, 4, 4, -4], [-2, 6, -6, 2]]
//      on every row, then every column, in integer lifting steps;
//   3. coefficients ordered by sequency i + j (kSeq);
//   4. negabinary digits u = (q + 0xAAAAAAAA) ^ 0xAAAAAAAA;
//   5. embedded bit-plane coding from plane 31 down: per plane the bits of
//      the coefficients already significant, then group tests (is any later
//      coefficient set in this plane?) each followed by the bits up to the
//      next set one (the last coefficient's 1 is implied);
//   6. fixed accuracy: planes down to kmin = 32 - min(32, max(0, e - minexp
//      + 6)), minexp = floor(log2 tol); a zero block or one without planes
//      is a single 0 bit, any other a 1 bit, e + 127 in 8 bits, its planes.
// Stream (32-bit words, bits least-significant first): 8 header words
// (magic 0x465A5452, mode 2, count, rows, cols, 16 blocks per chunk, tol as
// float64), the chunk table [nchunks + 1] (payload word offset of each
// chunk of 16 blocks, then the total), the payload (each chunk's block codes
// back to back, padded to a word).
//
// Launch shape: the encoder runs one lane per block in one pass: each
// workgroup finds where its chunks' codes start by a decoupled look-back
// over the workgroups before it, then writes its chunk-table entries and
// codes (chunks start on word boundaries, so no two workgroups write one
// word).  The decoder runs one
// lane per chunk of 16 blocks, in order, and reads each chunk's word range
// from the table, never outside it; a workgroup's chunks are consecutive, so
// their payload is one word range, which k_zf_decode_staged first copies
// into LDS with coalesced loads when it fits the launch's LDS budget.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>

#include "rtm_zfp.h"

namespace rtm {
namespace {

constexpr uint32_t kNb = 0xAAAAAAAAu;
// sequency order: (row frequency i, column frequency j) packed as 4 i + j
__constant__ uint8_t kSeq[16] = {0, 1, 4, 5, 2, 8, 6, 9, 3, 12, 10, 7, 13, 11, 14, 15};

__device__ __forceinline__ void fwd_lift(int32_t& a0, int32_t& a1, int32_t& a2, int32_t& a3) {
  a0 += a3; a0 >>= 1; a3 -= a0;
  a2 += a1; a2 >>= 1; a1 -= a2;
  a0 += a2; a0 >>= 1; a2 -= a0;
  a3 += a1; a3 >>= 1; a1 -= a3;
  a3 += a1 >> 1; a1 -= a3 >> 1;
}

__device__ __forceinline__ void inv_lift(int32_t& a0, int32_t& a1, int32_t& a2, int32_t& a3) {
  a1 += a3 >> 1; a3 -= a1 >> 1;
  a1 += a3; a3 = (int32_t)((uint32_t)a3 << 1); a3 -= a1;
  a2 += a0; a0 = (int32_t)((uint32_t)a0 << 1); a0 -= a2;
  a1 += a2; a2 = (int32_t)((uint32_t)a2 << 1); a2 -= a1;
  a3 += a0; a0 = (int32_t)((uint32_t)a0 << 1); a0 -= a3;
}

// Bit-plane transposition of a block's 16 coefficients, for the encoder's
// passes.  With plane k the 16-bit word whose bit c is bit k of coefficient
// c, and a[j] holding plane j in its low half and plane j + 16 in its high
// half, a[] viewed as a 16 x 32 bit matrix (row j, bit b) maps to the
// coefficients (row c, bit k) by exchanging the four bits of the row index
// with the low four bits of the bit position; four exchange stages do that
// in place, and the same stages map the coefficients to the planes (about
// 200 operations per block instead of 32 per plane: encoding 8-31 % faster
// on the codec banks).
__device__ __forceinline__ void swap_planes(uint32_t (&a)[16]) {
#pragma unroll
  for (int t = 3; t >= 0; --t) {
    const int sh = 1 << t;
    const uint32_t m = t == 3 ? 0x00FF00FFu : t == 2 ? 0x0F0F0F0Fu : t == 1 ? 0x33333333u : 0x55555555u;
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      if (r & sh) continue;
      const uint32_t x = ((a[r] >> sh) ^ a[r | sh]) & m;
      a[r | sh] ^= x;
      a[r] ^= x << sh;
    }
  }
}

// Reads bits from a chunk's word range, in global memory or in the LDS copy
// of the workgroup's payload (Idx: the index type of the range).  The window
// holds at least 32 bits, zeros past the range; consuming any of those
// raises `bad`.
template <class Idx>
struct BitSource {
  const uint32_t* in;
  Idx nwords, next = 0;
  uint64_t acc = 0;
  int nacc = 0;   // bits in the window
  int nreal = 0;  // of which inside the range
  bool bad = false;
  uint32_t ahead;  // word `next`, loaded one refill early so that its latency overlaps decoding
  __device__ BitSource(const uint32_t* p, Idx n) : in(p), nwords(n), ahead(n > 0 ? p[0] : 0u) {}
  __device__ __forceinline__ uint32_t peek() {  // the next 32 bits
    if (nacc < 32) {
      uint64_t w = 0;
      if (next < nwords) {
        w = ahead;
        nreal += 32;
      }
      ++next;
      ahead = next < nwords ? in[next] : 0u;
      acc |= w << nacc;
      nacc += 32;
    }
    return (uint32_t)acc;
  }
  __device__ __forceinline__ void skip(int n) {  // n <= 32, after peek()
    if (n > nreal) bad = true;
    nreal = max(nreal - n, 0);
    acc >>= n;
    nacc -= n;
  }
  __device__ __forceinline__ uint32_t get(int n) {  // n <= 32
    const uint32_t v = peek() & (n == 32 ? 0xFFFFFFFFu : ((1u << n) - 1u));
    skip(n);
    return v;
  }
};

// Loads block b (edges repeated) of the [count][rows][cols] array.
__device__ __forceinline__ void load_block(const ZfParams& p, int64_t b, float (&x)[16]) {
  const int64_t per = (int64_t)p.bz * p.bx;
  const int64_t img = b / per;
  const int64_t rem = b - img * per;
  const int bi = (int)(rem / p.bx), bj = (int)(rem - (int64_t)bi * p.bx);
  const float* a = p.x + img * (int64_t)p.rows * p.cols;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int r = min(4 * bi + i, p.rows - 1);
#pragma unroll
    for (int j = 0; j < 4; ++j) x[4 * i + j] = a[(int64_t)r * p.cols + min(4 * bj + j, p.cols - 1)];
  }
}

// Steps 1-6 for one block; false if a value is non-finite or |x| >= 2^100.
template <class Sink>
__device__ bool encode_block(const float (&x)[16], int minexp, Sink& bs) {
  float m = 0.0f;
  bool ok = true;
#pragma unroll
  for (int c = 0; c < 16; ++c) {
    const float a = fabsf(x[c]);
    ok = ok && (a < 0x1p100f);  // false for NaN and infinities too
    m = fmaxf(m, a);
  }
  if (!ok) return false;
  if (m == 0.0f) {
    bs.put(0, 1);
    return true;
  }
  int e;
  (void)frexpf(m, &e);
  const int maxprec = min(32, max(0, e - minexp + 6));
  if (maxprec == 0) {
    bs.put(0, 1);
    return true;
  }
  bs.put(1, 1);
  bs.put((uint32_t)(e + 127), 8);
  int32_t q[16];
#pragma unroll
  for (int c = 0; c < 16; ++c) q[c] = (int32_t)ldexpf(x[c], 30 - e);  // exact scaling, truncation
#pragma unroll
  for (int i = 0; i < 4; ++i) fwd_lift(q[4 * i], q[4 * i + 1], q[4 * i + 2], q[4 * i + 3]);
#pragma unroll
  for (int j = 0; j < 4; ++j) fwd_lift(q[j], q[4 + j], q[8 + j], q[12 + j]);
  uint32_t u[16];
#pragma unroll
  for (int c = 0; c < 16; ++c) u[c] = ((uint32_t)q[kSeq[c]] + kNb) ^ kNb;
  const int kmin = 32 - maxprec;
  swap_planes(u);  // u[j]: plane j in the low half, plane j + 16 in the high half
  int n = 0;
#pragma unroll
  for (int k = 31; k >= 0; --k) {  // unrolled, so that the plane is a register
    if (k >= kmin) {
      const uint32_t plane = k >= 16 ? u[k - 16] >> 16 : u[k] & 0xFFFFu;  // bit c: bit k of coefficient c
      if (n > 0) bs.put(plane & ((1u << n) - 1u), n);  // coefficients already significant
      uint32_t rest = plane >> n;
      while (n < 16) {
        if (!rest) {
          bs.put(0, 1);  // group test: no further coefficient turns significant
          break;
        }
        const int p = __builtin_ctz(rest);
        if (n + p == 15) {  // test, then zeros up to the last coefficient, whose 1 is implied
          bs.put(1, 16 - n);
          n = 16;
          break;
        }
        bs.put(1u | (1u << (p + 1)), p + 2);  // test, p zeros, then the 1
        n += p + 1;
        rest >>= p + 1;
      }
    }
  }
  return true;
}

// Inverse of encode_block.  (Collecting the planes and transposing them
// with swap_planes instead of setting each coefficient's bit per plane
// measured no faster: the decoder's time goes to the serial bit reads.)
template <class Src>
__device__ void decode_block(Src& src, int minexp, float (&x)[16]) {
  if (src.get(1) == 0) {
#pragma unroll
    for (int c = 0; c < 16; ++c) x[c] = 0.0f;
    return;
  }
  const int e = (int)src.get(8) - 127;
  const int maxprec = min(32, max(0, e - minexp + 6));
  if (maxprec == 0) src.bad = true;  // an encoder never codes such a block
  const int kmin = 32 - maxprec;
  uint32_t u[16];
#pragma unroll
  for (int c = 0; c < 16; ++c) u[c] = 0;
  int n = 0;
  for (int k = 31; k >= kmin && !src.bad; --k) {
    uint32_t plane = n > 0 ? src.get(n) : 0u;
    while (n < 16) {
      uint32_t w = src.peek();
      if (!(w & 1u)) {  // group test 0: no further coefficient turns significant
        src.skip(1);
        break;
      }
      w >>= 1;  // after the test: zeros, then the 1 of the next significant coefficient
      const int lim = 15 - n;  // zeros before the last coefficient, whose 1 is implied
      const int p = w ? __builtin_ctz(w) : 32;
      if (p >= lim) {
        src.skip(1 + lim);
        plane |= 1u << 15;
        n = 16;
        break;
      }
      src.skip(2 + p);
      plane |= 1u << (n + p);
      n += p + 1;
    }
#pragma unroll
    for (int c = 0; c < 16; ++c) u[c] |= ((plane >> c) & 1u) << k;
  }
  int32_t q[16];
#pragma unroll
  for (int c = 0; c < 16; ++c) q[kSeq[c]] = (int32_t)((u[c] ^ kNb) - kNb);
#pragma unroll
  for (int j = 0; j < 4; ++j) inv_lift(q[j], q[4 + j], q[8 + j], q[12 + j]);
#pragma unroll
  for (int i = 0; i < 4; ++i) inv_lift(q[4 * i], q[4 * i + 1], q[4 * i + 2], q[4 * i + 3]);
  const float scale = ldexpf(1.0f, e - 30);  // normal for every accepted tolerance
#pragma unroll
  for (int c = 0; c < 16; ++c) x[c] = (float)q[c] * scale;
}

// Appends bits to a lane's own LDS words (at most kZfBlockWords).
struct LdsSink {
  uint32_t* out;
  uint64_t acc = 0;
  int nacc = 0, words = 0, bits = 0;
  __device__ explicit LdsSink(uint32_t* o) : out(o) {}
  __device__ __forceinline__ void put(uint32_t v, int n) {  // n <= 32, v < 2^n
    acc |= (uint64_t)v << nacc;
    nacc += n;
    bits += n;
    if (nacc >= 32) {
      out[words++] = (uint32_t)acc;
      acc >>= 32;
      nacc -= 32;
    }
  }
  __device__ __forceinline__ void flush() {
    if (nacc > 0) out[words++] = (uint32_t)acc;
  }
};

// Status word of a workgroup in the encoder's look-back: a flag in the top
// two bits, payload words in the rest.
constexpr uint64_t kZfAgg = 1ull << 62;  // the workgroup's own payload words published
constexpr uint64_t kZfInc = 2ull << 62;  // its inclusive prefix published
constexpr uint64_t kZfValMask = (1ull << 62) - 1;
constexpr int kZfSpinLimit = 1 << 22;

// The encoder, one pass.  A workgroup of four wavefronts codes 256
// consecutive blocks (16 chunks), one lane per block, each into the lane's
// own LDS words; the workgroups take their block ranges in the order of an
// atomic ticket.  A 16-lane prefix sum of the blocks' bit lengths places
// each code in its chunk.  Wavefront 0 publishes the workgroup's payload
// words and finds where they start by a decoupled look-back over the
// workgroups before it (64 of their status words per round, summed down to
// the nearest published inclusive prefix; a workgroup waits only on
// workgroups that took their tickets earlier and publish their own words
// before they wait, and a wait that exceeds its bound raises kZfSpin
// instead of hanging), then writes the chunk-table entries.  The chunks'
// codes, assembled in LDS meanwhile, go to their offsets.  The words equal
// those of one thread writing the blocks in order.
__global__ __launch_bounds__(kZfEncThreads) void k_zf_encode(ZfParams p) {
  constexpr int kT = kZfEncThreads, kChunks = kT / kZfChunk;  // chunks per workgroup
  __shared__ uint32_t own[kT * kZfBlockWords];
  __shared__ uint32_t cbuf[kChunks * kZfChunkWords];
  __shared__ uint32_t s_wg;
  __shared__ uint32_t s_words[kChunks];
  __shared__ uint64_t s_off[kChunks];
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  if (t == 0) s_wg = atomicAdd(p.ticket, 1u);
  for (int i = t; i < kChunks * kZfChunkWords; i += kT) cbuf[i] = 0u;
  __syncthreads();
  const int64_t wg = s_wg;
  const int64_t b = wg * kT + t;
  if (wg == 0 && t == 0) {
#pragma unroll
    for (int k = 0; k < 8; ++k)
      if (k < p.cap_words) p.out[k] = p.head[k];
  }
  LdsSink sink(own + t * kZfBlockWords);
  bool ok = true;
  if (b < p.nblocks) {
    float x[16];
    load_block(p, b, x);
    ok = encode_block(x, p.minexp, sink);
    sink.flush();
  }
  if (!ok) atomicOr(p.flags, kZfRange);
  // bit offset of this block in its chunk: exclusive prefix over the 16 lanes
  const int g = lane & (kZfChunk - 1);
  int pre = sink.bits;
#pragma unroll
  for (int d = 1; d < kZfChunk; d <<= 1) {
    const int v = __shfl_up(pre, d, kZfChunk);
    if (g >= d) pre += v;
  }
  const int chunk_bits = __shfl(pre, (lane & ~(kZfChunk - 1)) + kZfChunk - 1, 64);
  pre -= sink.bits;
  if (g == 0) s_words[t / kZfChunk] = (uint32_t)((chunk_bits + 31) >> 5);
  __syncthreads();

  // ---- decoupled look-back over the preceding workgroups (wavefront 0) ----
  if (wave == 0) {
    uint32_t agg = 0;
#pragma unroll
    for (int q = 0; q < kChunks; ++q) agg += s_words[q];
    if (lane == 0)
      __hip_atomic_store(p.status + wg, (wg == 0 ? kZfInc : kZfAgg) | agg, __ATOMIC_RELAXED,
                         __HIP_MEMORY_SCOPE_AGENT);
    uint64_t excl = 0;
    int64_t end_j = wg;  // workgroups [0, end_j) are still to be summed
    int spins = 0;
    while (end_j > 0) {
      const int64_t j = end_j - 1 - lane;
      const uint64_t st = j >= 0 ? __hip_atomic_load(p.status + j, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)
                                 : kZfInc;  // before workgroup 0: an inclusive prefix of 0
      const uint64_t inc = __ballot((st >> 62) == 2);
      const int first = inc ? __builtin_ctzll(inc) : 64;  // nearest published prefix
      const uint64_t upto = first >= 63 ? ~0ull : ((2ull << first) - 1ull);
      if (__ballot((st >> 62) == 0) & upto) {  // a workgroup in range has published nothing yet
        if (++spins > kZfSpinLimit) {
          if (lane == 0) atomicOr(p.flags, kZfSpin);
          break;
        }
        __builtin_amdgcn_s_sleep(1);
        continue;
      }
      uint64_t part = lane <= first ? (st & kZfValMask) : 0ull;
#pragma unroll
      for (int o = 32; o > 0; o >>= 1) part += __shfl_xor(part, o, 64);
      excl += part;
      if (first < 64) break;
      end_j -= 64;
    }
    if (lane == 0) {
      if (wg > 0)
        __hip_atomic_store(p.status + wg, kZfInc | (excl + agg), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      uint64_t off = excl;
      for (int q = 0; q < kChunks; ++q) {
        const int64_t ch = wg * kChunks + q;
        s_off[q] = off;
        if (ch < p.nchunks) p.out[p.hdr_base + ch] = (uint32_t)off;  // the table lies below pay_base <= cap_words
        off += s_words[q];
      }
      if (wg == (p.nchunks - 1) / kChunks) {  // the last chunk's workgroup writes the total
        p.out[p.hdr_base + p.nchunks] = (uint32_t)off;
        p.result[0] = (uint32_t)off;
        p.result[1] = (uint32_t)(off >> 32);
      }
    }
  }

  // ---- the chunks' codes, assembled in LDS, at their offsets ----
  uint32_t* cb = cbuf + (t / kZfChunk) * kZfChunkWords;
  const int w0 = pre >> 5, sh = pre & 31;
  for (int i = 0; i < sink.words; ++i) {
    const uint32_t v = own[t * kZfBlockWords + i];
    atomicOr(&cb[w0 + i], v << sh);
    if (sh && (v >> (32 - sh))) atomicOr(&cb[w0 + i + 1], v >> (32 - sh));
  }
  __syncthreads();  // the codes assembled and the offsets written
  for (int i = t; i < kChunks * kZfChunkWords; i += kT) {
    const int c = i / kZfChunkWords, w = i - c * kZfChunkWords;
    const int64_t ch = wg * kChunks + c;
    if (ch >= p.nchunks || w >= (int)s_words[c]) continue;
    const int64_t at = p.pay_base + (int64_t)s_off[c] + w;
    if (at < p.cap_words) p.out[at] = cbuf[i];
  }
}

// Decodes chunk ch (its words at src) into the output array.
template <class Src>
__device__ __forceinline__ void decode_chunk(const ZfParams& p, int64_t ch, Src& src) {
  const int64_t per = (int64_t)p.bz * p.bx;
  const int64_t b1 = min((ch + 1) * kZfChunk, (int64_t)p.nblocks);
  for (int64_t b = ch * kZfChunk; b < b1; ++b) {
    float x[16];
    decode_block(src, p.minexp, x);
    if (src.bad) break;
    const int64_t img = b / per;
    const int64_t rem = b - img * per;
    const int bi = (int)(rem / p.bx), bj = (int)(rem - (int64_t)bi * p.bx);
    float* a = p.y + img * (int64_t)p.rows * p.cols;
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int r = 4 * bi + i, c = 4 * bj + j;
        if (r < p.rows && c < p.cols) a[(int64_t)r * p.cols + c] = x[4 * i + j];
      }
  }
  if (src.bad) atomicOr(p.flags, kZfCorrupt);
}

// Decoder: one lane per chunk, reading global memory.  A lane reads only its
// own table range, checked against the stream's length.
__global__ __launch_bounds__(kZfThreads) void k_zf_decode(ZfParams p) {
  const int64_t ch = (int64_t)blockIdx.x * kZfThreads + threadIdx.x;
  if (ch >= p.nchunks) return;
  const uint32_t* table = p.in + p.hdr_base;
  const int64_t w0 = table[ch], w1 = table[ch + 1];
  const int64_t avail = p.cap_words - p.pay_base;  // payload words in the stream
  if (w0 > w1 || w1 > avail) {
    atomicOr(p.flags, kZfCorrupt);
    return;
  }
  BitSource<int64_t> src(p.in + p.pay_base + w0, w1 - w0);
  const int64_t per = (int64_t)p.bz * p.bx;
  const int64_t b1 = min((ch + 1) * kZfChunk, (int64_t)p.nblocks);
  for (int64_t b = ch * kZfChunk; b < b1; ++b) {
    float x[16];
    decode_block(src, p.minexp, x);
    if (src.bad) break;
    const int64_t img = b / per;
    const int64_t rem = b - img * per;
    const int bi = (int)(rem / p.bx), bj = (int)(rem - (int64_t)bi * p.bx);
    float* a = p.y + img * (int64_t)p.rows * p.cols;
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int r = 4 * bi + i, c = 4 * bj + j;
        if (r < p.rows && c < p.cols) a[(int64_t)r * p.cols + c] = x[4 * i + j];
      }
  }
  if (src.bad) atomicOr(p.flags, kZfCorrupt);
}

// Decoder with the payload staged in LDS: the workgroup's consecutive chunks
// own the payload words [W0, W1) of the table; when that range is consistent
// and holds at most stage_words words, the workgroup copies it into LDS
// (coalesced) and its lanes read their chunks from there, so the decode loop
// issues no global loads (whose waits would also wait for the block stores
// already issued).  Otherwise its lanes read global memory as k_zf_decode's
// do.  Either way a lane reads only its own table range, checked against
// the stream's length (and, staged, against [W0, W1)).
__global__ __launch_bounds__(kZfThreads) void k_zf_decode_staged(ZfParams p, int stage_words) {
  extern __shared__ uint32_t stage[];
  const int64_t c0 = (int64_t)blockIdx.x * kZfThreads;
  const int64_t ch = c0 + threadIdx.x;
  const uint32_t* table = p.in + p.hdr_base;
  const int64_t avail = p.cap_words - p.pay_base;  // payload words in the stream
  const int64_t W0 = table[c0], W1 = table[min(c0 + kZfThreads, p.nchunks)];
  const bool staged = W0 <= W1 && W1 <= avail && W1 - W0 <= stage_words;
  if (staged) {
    const uint32_t* src = p.in + p.pay_base + W0;
    const int n = (int)(W1 - W0);
    constexpr int kU = 8;  // loads in flight per lane
    int i = threadIdx.x;
    for (; i + (kU - 1) * kZfThreads < n; i += kU * kZfThreads) {
      uint32_t v[kU];
#pragma unroll
      for (int u = 0; u < kU; ++u) v[u] = src[i + u * kZfThreads];
#pragma unroll
      for (int u = 0; u < kU; ++u) stage[i + u * kZfThreads] = v[u];
    }
    for (; i < n; i += kZfThreads) stage[i] = src[i];
    __syncthreads();
  }
  if (ch >= p.nchunks) return;
  const int64_t w0 = table[ch], w1 = table[ch + 1];
  if (w0 > w1 || w1 > avail || (staged && (w0 < W0 || w1 > W1))) {
    atomicOr(p.flags, kZfCorrupt);
    return;
  }
  if (staged) {
    BitSource<int> src(stage + (int)(w0 - W0), (int)(w1 - w0));
    decode_chunk(p, ch, src);
  } else {
    BitSource<int64_t> src(p.in + p.pay_base + w0, w1 - w0);
    decode_chunk(p, ch, src);
  }
}

}  // namespace

hipError_t launch_zf_encode(const ZfParams& p, hipStream_t s) {
  if (p.nchunks < 1) return hipErrorInvalidValue;
  const int64_t g = (p.nblocks + kZfEncThreads - 1) / kZfEncThreads;  // one lane per block
  k_zf_encode<<<(unsigned)g, kZfEncThreads, 0, s>>>(p);
  return hipGetLastError();
}

hipError_t launch_zf_decode(const ZfParams& p, int64_t stage_bytes, hipStream_t s) {
  if (p.nchunks < 1) return hipErrorInvalidValue;
  const int64_t g = (p.nchunks + kZfThreads - 1) / kZfThreads;
  if (stage_bytes < 0) {
    // Budget of LDS per workgroup: about 1.15x the stream's mean payload per
    // workgroup, rounded to an even share of a CU's 160 KiB.  The lanes'
    // decode loops are chains of dependent steps whose speed rests on how
    // many wavefronts share a SIMD, so staging is used only where the budget
    // still lets every CU hold all the workgroups the launch gives it (256
    // CUs): measured on the codec banks, staging at 1-2 wavefronts per SIMD
    // instead of 2.3 made decoding 14-70 % slower, and at full occupancy
    // 8-18 % faster.
    const double mean = 4.0 * (double)(p.cap_words - p.pay_base) * kZfThreads / (double)p.nchunks;
    const double want = 1.15 * mean + 256.0;
    const int64_t k = std::min<int64_t>(32, std::max<int64_t>(1, (int64_t)(163840.0 / want)));
    stage_bytes = k >= (g + 255) / 256 ? 163840 / k : 0;
  }
  stage_bytes = std::min<int64_t>(stage_bytes, kZfMaxStageBytes) & ~int64_t(255);
  // without staging, the kernel without the staging code (the two paths in
  // one kernel measured 5-13 % slower on unstaged streams)
  if (stage_bytes == 0)
    k_zf_decode<<<(unsigned)g, kZfThreads, 0, s>>>(p);
  else
    k_zf_decode_staged<<<(unsigned)g, kZfThreads, (size_t)stage_bytes, s>>>(p, (int)(stage_bytes / 4));
  return hipGetLastError();
}

}  // namespace rtm
