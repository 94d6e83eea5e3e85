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
// Launch shape: the encoder runs one lane per block, twice: a pass that only
// counts each chunk's words, a scan of the counts into the chunk table, and
// a pass that writes the codes at their offsets (chunks start on word
// boundaries, so no two workgroups write one word).  The decoder runs one
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

// Bits encode_block emits for a block (the same steps, no stream): per bit
// plane the verbatim bits of the significant coefficients, then one group
// test per coefficient that turns significant plus the run up to it, and a
// closing test unless the last coefficient was reached (its 1 implied).
__device__ int count_block(const float (&x)[16], int minexp, bool& ok) {
  float m = 0.0f;
  bool fin = true;
#pragma unroll
  for (int c = 0; c < 16; ++c) {
    const float a = fabsf(x[c]);
    fin = fin && (a < 0x1p100f);
    m = fmaxf(m, a);
  }
  if (!fin) {
    ok = false;
    return 0;
  }
  if (m == 0.0f) return 1;
  int e;
  (void)frexpf(m, &e);
  const int maxprec = min(32, max(0, e - minexp + 6));
  if (maxprec == 0) return 1;
  int32_t q[16];
#pragma unroll
  for (int c = 0; c < 16; ++c) q[c] = (int32_t)ldexpf(x[c], 30 - e);
#pragma unroll
  for (int i = 0; i < 4; ++i) fwd_lift(q[4 * i], q[4 * i + 1], q[4 * i + 2], q[4 * i + 3]);
#pragma unroll
  for (int j = 0; j < 4; ++j) fwd_lift(q[j], q[4 + j], q[8 + j], q[12 + j]);
  uint32_t u[16];
#pragma unroll
  for (int c = 0; c < 16; ++c) u[c] = ((uint32_t)q[kSeq[c]] + kNb) ^ kNb;
  const int kmin = 32 - maxprec;
  swap_planes(u);  // u[j]: plane j in the low half, plane j + 16 in the high half
  int bits = 9, n = 0;
#pragma unroll
  for (int k = 31; k >= 0; --k) {  // unrolled, so that the plane is a register
    if (k >= kmin && n < 16) {
      const uint32_t plane = k >= 16 ? u[k - 16] >> 16 : u[k] & 0xFFFFu;
      const uint32_t rest = plane >> n;
      bits += n;
      if (!rest) {
        bits += 1;
      } else {
        const int ones = __builtin_popcount(rest);
        const int nf = n + 32 - __builtin_clz(rest);  // one past the highest new significant coefficient
        bits += nf == 16 ? ones + 15 - n : ones + nf - n + 1;
        n = nf;
      }
    } else if (k >= kmin) {
      bits += 16;  // every coefficient significant: verbatim planes from here on
    }
  }
  return bits;
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

// Pass 1: payload words of every chunk -> counts[chunk].  One lane per
// block: the 64 lanes of a workgroup read 64 neighbouring blocks (row by
// row, 1 KB contiguous), and each 16-lane group sums the bits of one chunk.
__global__ __launch_bounds__(kZfThreads) void k_zf_count(ZfParams p, uint32_t* counts) {
  const int lane = threadIdx.x;
  const int64_t b = (int64_t)blockIdx.x * kZfThreads + lane;
  bool ok = true;
  int bits = 0;
  if (b < p.nblocks) {
    float x[16];
    load_block(p, b, x);
    bits = count_block(x, p.minexp, ok);
  }
#pragma unroll
  for (int d = kZfChunk / 2; d > 0; d >>= 1) bits += __shfl_xor(bits, d, kZfChunk);
  const int64_t ch = b / kZfChunk;
  if ((lane & (kZfChunk - 1)) == 0 && ch < p.nchunks) counts[ch] = (uint32_t)((bits + 31) >> 5);  // words written
  if (!ok) atomicOr(p.flags, kZfRange);
}

// Exclusive scan of the counts into the stream's chunk table, in three
// launches: per-workgroup totals, a scan of the totals (one workgroup), and
// the table entries.
__global__ __launch_bounds__(kZfScan) void k_zf_scan_totals(const uint32_t* counts, int64_t n, uint64_t* totals) {
  __shared__ uint64_t red[kZfScan];
  const int64_t i = (int64_t)blockIdx.x * kZfScan + threadIdx.x;
  red[threadIdx.x] = i < n ? counts[i] : 0;
  __syncthreads();
  for (int s = kZfScan / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) totals[blockIdx.x] = red[0];
}

__global__ __launch_bounds__(kZfScan) void k_zf_scan_base(uint64_t* totals, int64_t ngroups) {
  // exclusive scan of ngroups totals, in place, kZfScan at a time
  __shared__ uint64_t buf[kZfScan];
  uint64_t carry = 0;
  for (int64_t base = 0; base < ngroups; base += kZfScan) {
    const int64_t i = base + threadIdx.x;
    const uint64_t v = i < ngroups ? totals[i] : 0;
    buf[threadIdx.x] = v;
    __syncthreads();
    for (int s = 1; s < kZfScan; s <<= 1) {  // inclusive Hillis-Steele scan
      const uint64_t t = (int)threadIdx.x >= s ? buf[threadIdx.x - s] : 0;
      __syncthreads();
      buf[threadIdx.x] += t;
      __syncthreads();
    }
    if (i < ngroups) totals[i] = carry + buf[threadIdx.x] - v;
    const uint64_t sum = buf[kZfScan - 1];
    __syncthreads();
    carry += sum;
  }
  if (threadIdx.x == 0) totals[ngroups] = carry;
}

__global__ __launch_bounds__(kZfScan) void k_zf_scan_table(const uint32_t* counts, int64_t n, const uint64_t* base,
                                                           ZfParams p) {
  __shared__ uint64_t buf[kZfScan];
  const int64_t i = (int64_t)blockIdx.x * kZfScan + threadIdx.x;
  const uint64_t v = i < n ? counts[i] : 0;
  buf[threadIdx.x] = v;
  __syncthreads();
  for (int s = 1; s < kZfScan; s <<= 1) {
    const uint64_t t = (int)threadIdx.x >= s ? buf[threadIdx.x - s] : 0;
    __syncthreads();
    buf[threadIdx.x] += t;
    __syncthreads();
  }
  const uint64_t off = base[blockIdx.x] + buf[threadIdx.x] - v;  // exclusive prefix
  if (i < n && p.hdr_base + i < p.cap_words) p.out[p.hdr_base + i] = (uint32_t)off;
  if (i == n - 1) {
    const uint64_t total = off + v;
    if (p.hdr_base + n < p.cap_words) p.out[p.hdr_base + n] = (uint32_t)total;
    p.result[0] = (uint32_t)total;
    p.result[1] = (uint32_t)(total >> 32);
  }
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

// Pass 2: the block codes of every chunk at its table offset.  One lane per
// block: each lane codes its block into its own LDS words; a 16-lane prefix
// sum of the block lengths places the codes in their chunk, which is
// assembled in LDS and copied to the stream.  The words equal those of one
// thread writing the chunk's blocks in order.
__global__ __launch_bounds__(kZfThreads) void k_zf_encode(ZfParams p) {
  constexpr int kChunks = kZfThreads / kZfChunk;  // chunks per workgroup
  __shared__ uint32_t own[kZfThreads * kZfBlockWords];
  __shared__ uint32_t cbuf[kChunks * kZfChunkWords];
  const int lane = threadIdx.x;
  const int64_t b = (int64_t)blockIdx.x * kZfThreads + lane;
  if (blockIdx.x == 0 && lane == 0) {
#pragma unroll
    for (int k = 0; k < 8; ++k)
      if (k < p.cap_words) p.out[k] = p.head[k];
  }
  for (int i = lane; i < kChunks * kZfChunkWords; i += kZfThreads) cbuf[i] = 0u;
  LdsSink sink(own + lane * kZfBlockWords);
  if (b < p.nblocks) {
    float x[16];
    load_block(p, b, x);
    (void)encode_block(x, p.minexp, sink);
    sink.flush();
  }
  // bit offset of this block in its chunk: exclusive prefix over the 16 lanes
  const int g = lane & (kZfChunk - 1);
  int pre = sink.bits;
#pragma unroll
  for (int d = 1; d < kZfChunk; d <<= 1) {
    const int t = __shfl_up(pre, d, kZfChunk);
    if (g >= d) pre += t;
  }
  pre -= sink.bits;
  __syncthreads();  // chunk buffers zeroed, own words written
  uint32_t* cb = cbuf + (lane / kZfChunk) * kZfChunkWords;
  const int w0 = pre >> 5, sh = pre & 31;
  for (int i = 0; i < sink.words; ++i) {
    const uint32_t v = own[lane * kZfBlockWords + i];
    atomicOr(&cb[w0 + i], v << sh);
    if (sh && (v >> (32 - sh))) atomicOr(&cb[w0 + i + 1], v >> (32 - sh));
  }
  __syncthreads();
  const uint32_t* table = p.out + p.hdr_base;  // written by the scan
  for (int i = lane; i < kChunks * kZfChunkWords; i += kZfThreads) {
    const int c = i / kZfChunkWords, w = i - c * kZfChunkWords;
    const int64_t ch = (int64_t)blockIdx.x * kChunks + c;
    if (ch >= p.nchunks) continue;
    const int64_t off = table[ch], nw = (int64_t)table[ch + 1] - off;
    const int64_t at = p.pay_base + off + w;
    if (w < nw && at < p.cap_words) p.out[at] = cbuf[i];
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

hipError_t launch_zf_encode(const ZfParams& p, uint32_t* counts, uint64_t* totals, hipStream_t s) {
  if (p.nchunks < 1) return hipErrorInvalidValue;
  const int64_t gb = (p.nblocks + kZfThreads - 1) / kZfThreads;  // one lane per block
  k_zf_count<<<(unsigned)gb, kZfThreads, 0, s>>>(p, counts);
  const int64_t ng = (p.nchunks + kZfScan - 1) / kZfScan;
  k_zf_scan_totals<<<(unsigned)ng, kZfScan, 0, s>>>(counts, p.nchunks, totals);
  k_zf_scan_base<<<1, kZfScan, 0, s>>>(totals, ng);
  k_zf_scan_table<<<(unsigned)ng, kZfScan, 0, s>>>(counts, p.nchunks, totals, p);
  k_zf_encode<<<(unsigned)gb, kZfThreads, 0, s>>>(p);
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
