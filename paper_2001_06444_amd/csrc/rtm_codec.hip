// rtm_codec.hip -- block-transform codec for float32 arrays (fixed accuracy or
// lossless), the data-compression stage of the workflow (Sec. 3, data
// compression; Sec. 4.2, Tables 1-2).
//
// Stream format and arithmetic (the host runtime writes nothing but the
// launch parameters; every word of the stream is written here):
//   words [0..7]   magic, mode, count, rows, cols, blocks per chunk, tol (f64)
//   chunk table    [nchunks + 1] payload word offset of each chunk, then the total
//   block headers  [nblocks] five 6-bit sub-band widths
//   payload        per block, its 64 coefficients in their sub-band widths,
//                  least-significant bit first, padded to a 32-bit word
// Per block: 8 x 8 values (edge rows/columns repeated) -> int32 (fixed
// accuracy: rint(x / (2 tol)); lossless: order-preserving bit key) -> three
// levels of the 2-D integer Haar lifting (d = a - b, s = b + (d >> 1), modulo
// 2^32) -> zig-zag -> widths of the five sub-bands -> packed bits.
//
// Launch shape: one 64-lane wavefront handles 64 blocks, one block per lane,
// with the block's 64 values in registers; a 256-thread workgroup is one
// chunk of 256 blocks.  Array rows move between HBM and a row buffer in LDS
// in runs of 64 consecutive floats, and payload words through the same LDS
// area in runs of 64 consecutive words, so every global load and store is
// coalesced (a decoder wave whose payload exceeds the area reads it from
// the stream directly).  The encoder finds each chunk's payload offset with a
// single-pass decoupled look-back over the chunks (chunk order taken from an
// atomic ticket, so every chunk waits only on chunks that are already
// running); the wait is bounded and reports an error instead of hanging.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <mutex>

#include "rtm_codec.h"

namespace rtm {
namespace {

constexpr int kB = 8;
constexpr uint64_t kAgg = 1ull << 62;   // status: chunk aggregate published
constexpr uint64_t kInc = 2ull << 62;   // status: inclusive prefix published
constexpr uint64_t kValMask = (1ull << 62) - 1;
constexpr int kSpinLimit = 1 << 22;

#ifndef RTM_ZC_NT_LOAD
#define RTM_ZC_NT_LOAD 0
#endif
#ifndef RTM_ZC_NT_STORE
#define RTM_ZC_NT_STORE 0
#endif
template <typename T>
__device__ inline T ld(const T* p) {
  if (RTM_ZC_NT_LOAD) return __builtin_nontemporal_load(p);
  return *p;
}
template <typename T>
__device__ inline void st(T v, T* p) {
  if (RTM_ZC_NT_STORE)
    __builtin_nontemporal_store(v, p);
  else
    *p = v;
}

// sub-band of position (z, x) of the 8 x 8 coefficient layout
__host__ __device__ constexpr int band_of(int z, int x) {
  return (z < 2 && x < 2) ? 0 : (z < 4 && x < 4) ? 1 : (z < 4) ? 2 : (x < 4) ? 3 : 4;
}

// number of positions before c (row-major) that belong to sub-band g: the bit
// offset of coefficient c in its block is sum_g count_before(c, g) * w_g
__host__ __device__ constexpr int count_before(int c, int g) {
  int n = 0;
  for (int i = 0; i < c; ++i) n += band_of(i / 8, i % 8) == g ? 1 : 0;
  return n;
}

__device__ inline int32_t wsub(int32_t a, int32_t b) { return (int32_t)((uint32_t)a - (uint32_t)b); }
__device__ inline int32_t wadd(int32_t a, int32_t b) { return (int32_t)((uint32_t)a + (uint32_t)b); }

// One level of the forward lifting on the top-left n x n corner.
template <int N>
__device__ inline void lift_level(int32_t (&v)[64]) {
  constexpr int H = N / 2;
  int32_t t[N * N];
#pragma unroll
  for (int z = 0; z < N; ++z)
#pragma unroll
    for (int k = 0; k < H; ++k) {
      const int32_t d = wsub(v[z * kB + 2 * k], v[z * kB + 2 * k + 1]);
      t[z * N + k] = wadd(v[z * kB + 2 * k + 1], d >> 1);
      t[z * N + H + k] = d;
    }
#pragma unroll
  for (int k = 0; k < H; ++k)
#pragma unroll
    for (int x = 0; x < N; ++x) {
      const int32_t d = wsub(t[(2 * k) * N + x], t[(2 * k + 1) * N + x]);
      v[k * kB + x] = wadd(t[(2 * k + 1) * N + x], d >> 1);
      v[(H + k) * kB + x] = d;
    }
}

// Inverse of lift_level<N>.
template <int N>
__device__ inline void unlift_level(int32_t (&v)[64]) {
  constexpr int H = N / 2;
  int32_t t[N * N];
#pragma unroll
  for (int k = 0; k < H; ++k)
#pragma unroll
    for (int x = 0; x < N; ++x) {
      const int32_t s = v[k * kB + x], d = v[(H + k) * kB + x];
      const int32_t b = wsub(s, d >> 1);
      t[(2 * k) * N + x] = wadd(d, b);
      t[(2 * k + 1) * N + x] = b;
    }
#pragma unroll
  for (int z = 0; z < N; ++z)
#pragma unroll
    for (int k = 0; k < H; ++k) {
      const int32_t s = t[z * N + k], d = t[z * N + H + k];
      const int32_t b = wsub(s, d >> 1);
      v[z * kB + 2 * k] = wadd(d, b);
      v[z * kB + 2 * k + 1] = b;
    }
}

__device__ inline uint32_t zigzag(int32_t v) { return ((uint32_t)v << 1) ^ (uint32_t)(v >> 31); }
__device__ inline int32_t unzigzag(uint32_t u) { return (int32_t)(u >> 1) ^ -(int32_t)(u & 1u); }
__device__ inline int32_t float_key(float f) {
  const int32_t k = __float_as_int(f);
  return k ^ ((k >> 31) & 0x7fffffff);
}
__device__ inline float key_float(int32_t k) { return __int_as_float(k ^ ((k >> 31) & 0x7fffffff)); }
__device__ inline int bitlen(uint32_t u) { return 32 - __clz(u); }

// Orders the LDS accesses of one wave around this point (each wave owns its
// own LDS area, so the other waves need not wait).
__device__ inline void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Exclusive scan of one value per thread over a 256-thread workgroup;
// returns the exclusive prefix and writes the workgroup total to *total.
__device__ inline uint32_t wg_exclusive_scan(uint32_t v, uint32_t* lds4, uint32_t* total) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  uint32_t inc = v;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const uint32_t y = __shfl_up(inc, o, 64);
    if (lane >= o) inc += y;
  }
  if (lane == 63) lds4[wave] = inc;
  __syncthreads();
  uint32_t base = 0;
#pragma unroll
  for (int w = 0; w < 4; ++w) base += (w < wave) ? lds4[w] : 0u;
  *total = lds4[0] + lds4[1] + lds4[2] + lds4[3];
  return base + inc - v;
}

// Grid position of the first value of block b.
struct BlockPos {
  int32_t a, z0, x0;
};
__device__ inline BlockPos block_pos(int32_t b, int32_t bz, int32_t bx) {
  const int32_t per = bz * bx;
  const int32_t a = b / per, rem = b - a * per;
  const int32_t r = rem / bx;
  return {a, r * kB, (rem - r * bx) * kB};
}

}  // namespace

// Array rows move through a 512-word LDS row buffer per wave: one row of
// the wave's 64 blocks (64 x 8 consecutive floats when the blocks share a
// block row).  Element m of the buffer is column m % 8 of block m / 8, so the
// wave's global loads and stores of a row touch 64 consecutive floats per
// instruction and a lane finds its block's eight values at [8 lane, 8 lane + 8).
constexpr int kRowWords = 64 * kB;
// Each wave owns kStageWords of LDS: its row buffer while array rows move,
// and the staging area of its payload words.  Three 256-thread workgroups
// (the register limit) fit the 160 KB of LDS per CU.
constexpr int kStageWords = 3328;
static_assert(kStageWords >= kRowWords, "the LDS area must hold one row of the wave's blocks");

// Element offsets of the eight blocks a lane touches in the wave's
// cooperative row loads / stores: block 8 k + lane / 8, k = 0..7.
struct WaveBlocks {
  int64_t img[8];
  int32_t z0[8], x0[8];
  bool live[8];
};
__device__ inline void wave_blocks(const ZcParams& p, int32_t b0, int lane, WaveBlocks& wb) {
  // the first block by division, the next seven by stepping 8 blocks along the
  // block order; blocks past the end take the last block's position
  const int32_t first = b0 + (lane >> 3);
  const BlockPos last = block_pos(p.nblocks - 1, p.bz, p.bx);
  const int32_t per = p.bz * p.bx, bf = min(first, p.nblocks - 1);
  int32_t a = bf / per, rem = bf - a * per, r = rem / p.bx, c = rem - r * p.bx;
  const int64_t plane = (int64_t)p.rows * p.cols;
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    const bool live = first + 8 * k < p.nblocks;
    wb.live[k] = live;
    wb.img[k] = (int64_t)(live ? a : last.a) * plane;
    wb.z0[k] = live ? r * kB : last.z0;
    wb.x0[k] = live ? c * kB : last.x0;
    c += 8;
    while (c >= p.bx) {
      c -= p.bx;
      if (++r == p.bz) {
        r = 0;
        ++a;
      }
    }
  }
}

template <int MODE>
__global__ __launch_bounds__(kZcChunk, 3) void k_zc_encode(ZcParams p) {
  __shared__ __attribute__((aligned(16))) uint32_t s_stage[4][kStageWords];
  __shared__ uint32_t s_scan[4];
  __shared__ uint32_t s_chunk;
  __shared__ uint64_t s_excl;
  if (threadIdx.x == 0) s_chunk = atomicAdd(p.ticket, 1u);
  __syncthreads();
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  uint32_t* row = s_stage[wave];
  const int32_t chunk = (int32_t)s_chunk;
  const int32_t b0 = chunk * kZcChunk + wave * 64;  // first block of this wave
  const int32_t b = b0 + lane;                       // this lane's block
  const bool active = b < p.nblocks;

  // rows of the wave's 64 blocks, one at a time, into this lane's block values
  int32_t v[64];
  bool bad = false;
  {
    // all 64 loads are issued before the first row goes through LDS, so the
    // workgroup waits for memory once
    uint32_t lv[kB][8];
    {
      WaveBlocks wb;
      wave_blocks(p, b0, lane, wb);
      const int j = lane & 7;
#pragma unroll
      for (int i = 0; i < kB; ++i)
#pragma unroll
        for (int k = 0; k < 8; ++k)
          lv[i][k] = __float_as_uint(ld(p.x + wb.img[k] + (int64_t)min(wb.z0[k] + i, p.rows - 1) * p.cols +
                                        min(wb.x0[k] + j, p.cols - 1)));
    }
#pragma unroll
    for (int i = 0; i < kB; ++i) {
#pragma unroll
      for (int k = 0; k < 8; ++k) row[64 * k + lane] = lv[i][k];
      wave_sync();
      const uint4 r0 = reinterpret_cast<const uint4*>(row)[2 * lane];
      const uint4 r1 = reinterpret_cast<const uint4*>(row)[2 * lane + 1];
      const uint32_t e[8] = {r0.x, r0.y, r0.z, r0.w, r1.x, r1.y, r1.z, r1.w};
#pragma unroll
      for (int jj = 0; jj < kB; ++jj) {
        const float f = __uint_as_float(e[jj]);
        if (MODE == 0) {
          const double q = __builtin_rint((double)f * p.r);
          const bool ok = fabs(q) <= 2147483647.0;
          bad |= !ok;
          v[i * kB + jj] = ok ? (int32_t)q : 0;
        } else {
          v[i * kB + jj] = float_key(f);
        }
      }
      wave_sync();
    }
  }
  lift_level<8>(v);
  lift_level<4>(v);
  lift_level<2>(v);

  uint32_t u[64];
  uint32_t orb[5] = {0, 0, 0, 0, 0};
#pragma unroll
  for (int c = 0; c < 64; ++c) {
    u[c] = zigzag(v[c]);
    orb[band_of(c / kB, c % kB)] |= u[c];
  }
  int w[5];
#pragma unroll
  for (int g = 0; g < 5; ++g) w[g] = bitlen(orb[g]);
  const uint32_t header = (uint32_t)(w[0] | w[1] << 6 | w[2] << 12 | w[3] << 18 | w[4] << 24);
  const uint32_t bits = 4u * w[0] + 12u * w[1] + 16u * (w[2] + w[3] + w[4]);
  const uint32_t nwords = active ? (bits + 31u) >> 5 : 0u;
  if (active && bad) atomicOr(p.flags, kZcRange);

  uint32_t agg;
  const uint32_t local = wg_exclusive_scan(nwords, s_scan, &agg);
  const uint32_t wave_base = __shfl(local, 0, 64);
  const uint32_t wave_total = __shfl(local + nwords, 63, 64) - wave_base;
  const uint32_t my_rounds = (wave_total + kStageWords - 1) / kStageWords;

  // payload words are packed into the wave's LDS area kStageWords at a time
  // (more than one round only for nearly incompressible blocks) and stored
  // 64 consecutive words per instruction.  The first round is packed before
  // the look-back: it needs only offsets within the wave.
  const uint32_t my0 = local - wave_base;  // this block's first word, wave-relative
  auto pack = [&](uint32_t r) __attribute__((always_inline)) {
    const uint32_t w0 = r * kStageWords, w1 = w0 + kStageWords;
    if (active && my0 < w1 && my0 + nwords > w0) {
      uint32_t wo = my0;
      uint64_t acc = 0;
      int nb = 0;
#pragma unroll
      for (int c = 0; c < 64; ++c) {
        const int wc = w[band_of(c / kB, c % kB)];
        acc |= (uint64_t)u[c] << nb;
        nb += wc;
        if (nb >= 32) {
          if (wo >= w0 && wo < w1) row[wo - w0] = (uint32_t)acc;
          ++wo;
          acc >>= 32;
          nb -= 32;
        }
      }
      if (nb > 0 && wo >= w0 && wo < w1) row[wo - w0] = (uint32_t)acc;
    }
    wave_sync();
  };
  if (wave == 0 && lane == 0)
    __hip_atomic_store(p.status + chunk, (chunk == 0 ? kInc : kAgg) | agg, __ATOMIC_RELAXED,
                       __HIP_MEMORY_SCOPE_AGENT);
  pack(0);

  // decoupled look-back, one wave wide: wave 0 reads the status of up to 64
  // preceding chunks per round, sums them down to the nearest one whose
  // inclusive prefix is published, and repeats further back if none is
  if (wave == 0) {
    uint64_t excl = 0;
    int32_t end_j = chunk;  // chunks [0, end_j) are still to be summed
    int spins = 0;
    while (end_j > 0) {
      const int32_t j = end_j - 1 - lane;
      const uint64_t st = j >= 0 ? __hip_atomic_load(p.status + j, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)
                                 : kInc;  // before chunk 0: an inclusive prefix of 0
      const uint64_t inc = __ballot((st >> 62) == 2);
      const int first = inc ? __builtin_ctzll(inc) : 64;  // nearest published prefix
      const uint64_t upto = first >= 63 ? ~0ull : ((2ull << first) - 1ull);
      if (__ballot((st >> 62) == 0) & upto) {  // a chunk in range has published nothing yet
        if (++spins > kSpinLimit) {
          if (lane == 0) atomicOr(p.flags, kZcSpin);
          break;
        }
        __builtin_amdgcn_s_sleep(1);
        continue;
      }
      uint64_t part = lane <= first ? (st & kValMask) : 0ull;
#pragma unroll
      for (int o = 32; o > 0; o >>= 1) part += __shfl_xor(part, o, 64);
      excl += part;
      if (first < 64) break;
      end_j -= 64;
    }
    if (lane == 0) {
      if (chunk > 0)
        __hip_atomic_store(p.status + chunk, kInc | (excl + agg), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      s_excl = excl;
      p.out[8 + chunk] = (uint32_t)excl;
      if (chunk == p.nchunks - 1) {
        p.out[8 + p.nchunks] = (uint32_t)(excl + agg);
        p.result[0] = (uint32_t)(excl + agg);
      }
      if (chunk == 0) {
#pragma unroll
        for (int k = 0; k < 8; ++k) p.out[k] = p.head[k];
      }
      if ((int64_t)(p.pay_base + excl + agg) > p.cap_words) atomicOr(p.flags, kZcCapacity);
    }
  }
  __syncthreads();
  if (active) p.out[p.hdr_base + b] = header;

  const int64_t dst0 = p.pay_base + (int64_t)s_excl + wave_base;
  for (uint32_t r = 0; r < my_rounds; ++r) {
    if (r > 0) pack(r);
    const uint32_t w0 = r * kStageWords;
    const uint32_t n = wave_total > w0 ? min(wave_total - w0, (uint32_t)kStageWords) : 0u;
    for (uint32_t k0 = 0; k0 < n; k0 += 8 * 64) {
      uint32_t t[8];
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        const uint32_t k = k0 + q * 64 + lane;
        t[q] = k < n ? row[k] : 0u;
      }
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        const uint32_t k = k0 + q * 64 + lane;
        const int64_t d = dst0 + w0 + k;
        if (k < n && d < p.cap_words) st(t[q], p.out + d);
      }
    }
    wave_sync();
  }
}

// Word i of a decoder wave's payload: from the LDS area when staged, else
// from the stream; 0 past the block's own words (end) or the stream.
__device__ __attribute__((always_inline)) inline uint32_t payload_word(const uint32_t* row, const uint32_t* in,
                                                                      uint32_t i, uint32_t end, uint32_t nstaged,
                                                                      int64_t src0, int64_t cap_words) {
  if (i >= end) return 0u;
  if (i < nstaged) return row[i];
  return src0 + i < cap_words ? ld(in + src0 + i) : 0u;
}

// STAGE words of LDS per wave at MINW waves per SIMD: the host takes the
// smaller area and a fourth wave when the stream's payload mostly fits it.
template <int MODE, int STAGE, int MINW>
__global__ __launch_bounds__(kZcChunk, MINW) void k_zc_decode(ZcParams p) {
  static_assert(STAGE >= kRowWords && STAGE % 64 == 0, "the LDS area must hold one row of the wave's blocks");
  __shared__ __attribute__((aligned(16))) uint32_t s_stage[4][STAGE];
  __shared__ uint32_t s_scan[4];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  uint32_t* row = s_stage[wave];
  const int32_t chunk = blockIdx.x;
  const int32_t b0 = chunk * kZcChunk + wave * 64;
  const int32_t b = b0 + lane;
  const bool active = b < p.nblocks;
  const uint32_t* __restrict__ in = p.in;
  const uint32_t header = active ? in[p.hdr_base + b] : 0u;
  int w[5];
  bool bad = false;
#pragma unroll
  for (int g = 0; g < 5; ++g) {
    const int wg = (header >> (6 * g)) & 63;
    bad |= wg > 32;
    w[g] = min(wg, 32);
  }
  if (bad) atomicOr(p.flags, kZcCorrupt);
  const uint32_t bits = 4u * w[0] + 12u * w[1] + 16u * (w[2] + w[3] + w[4]);
  const uint32_t nwords = (bits + 31u) >> 5;
  uint32_t agg;
  const uint32_t local = wg_exclusive_scan(nwords, s_scan, &agg);
  const uint32_t wave_base = __shfl(local, 0, 64);
  const uint32_t wave_total = __shfl(local + nwords, 63, 64) - wave_base;
  const uint32_t c0 = in[8 + chunk], c1 = in[8 + chunk + 1];
  if (threadIdx.x == 0 && (c1 < c0 || c1 - c0 != agg)) atomicOr(p.flags, kZcCorrupt);

  // the wave's payload -> LDS, 64 consecutive words per load, all loads in
  // flight together; words past the LDS area (nearly incompressible blocks
  // only) are read from the stream
  const int64_t src0 = p.pay_base + (int64_t)c0 + wave_base;
  if (lane == 0 && src0 + wave_total > p.cap_words) atomicOr(p.flags, kZcCorrupt);
  const uint32_t nstaged = min(wave_total, (uint32_t)STAGE);
  {
    constexpr int kPer = STAGE / 64;
    uint32_t t[kPer];
#pragma unroll
    for (int q = 0; q < kPer; ++q) {
      const uint32_t k = q * 64 + lane;
      t[q] = (k < nstaged && src0 + k < p.cap_words) ? ld(in + src0 + k) : 0u;
    }
#pragma unroll
    for (int q = 0; q < kPer; ++q) {
      const uint32_t k = q * 64 + lane;
      if (k < nstaged) row[k] = t[q];
    }
  }
  wave_sync();

  // unpack this lane's block
  int32_t v[64];
  const uint32_t my0 = local - wave_base, my1 = my0 + nwords;
  if (wave_total <= (uint32_t)STAGE) {
    // the whole payload is in LDS: every coefficient is extracted on its own
    // from its bit offset, so no read waits for another
#pragma unroll
    for (int c = 0; c < 64; ++c) {
      const int wc = w[band_of(c / kB, c % kB)];
      const uint32_t pos = count_before(c, 0) * w[0] + count_before(c, 1) * w[1] + count_before(c, 2) * w[2] +
                           count_before(c, 3) * w[3] + count_before(c, 4) * w[4];
      const uint32_t wi = my0 + (pos >> 5);
      const uint32_t lo = row[min(wi, (uint32_t)STAGE - 1)];
      const uint32_t hi = row[min(wi + 1, (uint32_t)STAGE - 1)];
      const uint64_t both = (uint64_t)(wi < my1 ? lo : 0u) | ((uint64_t)(wi + 1 < my1 ? hi : 0u) << 32);
      v[c] = unzigzag((uint32_t)((both >> (pos & 31)) & ((1ull << wc) - 1ull)));
      if ((c & 7) == 7) __builtin_amdgcn_sched_barrier(0);  // one row of reads in flight at a time
    }
  } else {
    // nearly incompressible: words past the LDS area come from the stream;
    // one word is read ahead
    uint32_t k = 0;
    uint32_t next = payload_word(row, in, my0, my1, nstaged, src0, p.cap_words);
    uint64_t acc = 0;
    int have = 0;
#pragma unroll
    for (int c = 0; c < 64; ++c) {
      const int wc = w[band_of(c / kB, c % kB)];
      if (have < wc) {
        acc |= (uint64_t)next << have;
        have += 32;
        next = payload_word(row, in, my0 + (++k), my1, nstaged, src0, p.cap_words);
      }
      const uint32_t uc = (uint32_t)(acc & ((1ull << wc) - 1ull));
      acc >>= wc;
      have -= wc;
      v[c] = unzigzag(uc);
    }
  }
  unlift_level<2>(v);
  unlift_level<4>(v);
  unlift_level<8>(v);
  wave_sync();  // every lane has read its payload out of the LDS area

  // this lane's block rows -> the row buffer -> the array, one row at a time
  // (no bounds tests when all 64 blocks of the wave lie inside the array)
  WaveBlocks wb;
  wave_blocks(p, b0, lane, wb);
  const int j = lane & 7;
  bool inside = true;
#pragma unroll
  for (int k = 0; k < 8; ++k) inside &= wb.live[k] && wb.z0[k] + kB <= p.rows && wb.x0[k] + kB <= p.cols;
  const bool all_inside = __all(inside);
#pragma unroll
  for (int i = 0; i < kB; ++i) {
    uint32_t e[8];
#pragma unroll
    for (int jj = 0; jj < kB; ++jj)
      e[jj] = __float_as_uint(MODE == 0 ? (float)((double)v[i * kB + jj] * p.step) : key_float(v[i * kB + jj]));
    reinterpret_cast<uint4*>(row)[2 * lane] = make_uint4(e[0], e[1], e[2], e[3]);
    reinterpret_cast<uint4*>(row)[2 * lane + 1] = make_uint4(e[4], e[5], e[6], e[7]);
    wave_sync();
    if (all_inside) {
#pragma unroll
      for (int k = 0; k < 8; ++k)
        st(__uint_as_float(row[64 * k + lane]), p.y + wb.img[k] + (int64_t)(wb.z0[k] + i) * p.cols + wb.x0[k] + j);
    } else {
#pragma unroll
      for (int k = 0; k < 8; ++k) {
        const int32_t z = wb.z0[k] + i, x = wb.x0[k] + j;
        if (wb.live[k] && z < p.rows && x < p.cols)
          st(__uint_as_float(row[64 * k + lane]), p.y + wb.img[k] + (int64_t)z * p.cols + x);
      }
    }
    wave_sync();
  }
}

// ---------------------------------------------------------------------------
// Scratch of the allocation-free encoder.  Host code never passes the
// array's name to a kernel or a copy (on the host it is a stand-in, not a
// device address): it uses the address hipGetSymbolAddress returns on each
// device, kept per device below.
// ---------------------------------------------------------------------------
static __device__ __align__(256) uint8_t scratch[kZcNoAllocBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};
}  // namespace

hipError_t zc_noalloc_scratch_init(int device) {
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (g_scratch_ptr[device]) return hipSuccess;
  void* ptr = nullptr;
  const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (e != hipSuccess) return e;
  if (!ptr) return hipErrorInvalidSymbol;
  g_scratch_ptr[device] = ptr;
  return hipSuccess;
}

void* zc_noalloc_scratch(int device) {
  if (device < 0 || device >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  return g_scratch_ptr[device];
}

hipError_t launch_zc_encode(const ZcParams& p, hipStream_t s) {
  if (p.nchunks < 1) return hipErrorInvalidValue;
  if (p.mode == 0)
    k_zc_encode<0><<<p.nchunks, kZcChunk, 0, s>>>(p);
  else
    k_zc_encode<1><<<p.nchunks, kZcChunk, 0, s>>>(p);
  return hipGetLastError();
}

hipError_t launch_zc_decode(const ZcParams& p, hipStream_t s) {
  if (p.nchunks < 1) return hipErrorInvalidValue;
  // mean payload words per wave decide the LDS area (the last chunk may be
  // partial; the estimate only picks a variant)
  constexpr int kSmall = 2496;
  const int64_t words = p.cap_words - p.pay_base;
  const bool small = words <= (int64_t)p.nchunks * 4 * (kSmall * 9 / 10);
  if (small) {
    if (p.mode == 0)
      k_zc_decode<0, kSmall, 4><<<p.nchunks, kZcChunk, 0, s>>>(p);
    else
      k_zc_decode<1, kSmall, 4><<<p.nchunks, kZcChunk, 0, s>>>(p);
  } else {
    if (p.mode == 0)
      k_zc_decode<0, kStageWords, 3><<<p.nchunks, kZcChunk, 0, s>>>(p);
    else
      k_zc_decode<1, kStageWords, 3><<<p.nchunks, kZcChunk, 0, s>>>(p);
  }
  return hipGetLastError();
}

}  // namespace rtm
