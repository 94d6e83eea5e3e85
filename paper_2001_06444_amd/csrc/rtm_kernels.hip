// rtm_kernels.hip -- gfx950 kernels of the RTM hot path.
//
// The time-step kernel is the whole per-step work of every job in a launch
// (arXiv:2001.06444, Sec. 2.2 and Sec. 3, Stage 2):
//   forward step n:   u^{n+1} = G (2u^n + c (L u^n + w^n e_s/(dx dz))) - G^2 u^{n-1}
//                     + boundary-ring save (reconstruct mode), snapshot write with
//                       per-snapshot power-of-two scale (store mode), or trace
//                       sampling (modelling);
//   backward step m:  R^m = G (2R^{m+1} + c (L R^{m+1} + d^m at receivers)) - G^2 R^{m+2}
//                     + source-wavefield S^m (time reversal of the forward recursion
//                       on the physical interior with the ring restored, or the
//                       decoded snapshot) + imaging I += k S^m R^{m+1} (Eq. 5 numerator).
// The stencil is HBM-bound (~2 flop/byte), so it runs on the vector ALUs: a
// workgroup owns a 64-column x TZ-row tile, stages the stencil operand with
// its 4-cell halo in LDS using 16-byte loads, and each thread marches down a
// column with the z-neighbours in registers.
#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "rtm_device.h"
#include "rtm_internal.h"

namespace rtm {

// Streaming hints: outputs of a step are not read again within the step, and
// pointwise operands are read exactly once per step.
#ifndef RTM_NT_STORE
#define RTM_NT_STORE 1
#endif
#ifndef RTM_NT_LOAD
#define RTM_NT_LOAD 1
#endif

// Pointers read from a job descriptor are generic; tagging them with the
// global address space lets the compiler issue global_load/global_store
// (vector-memory counter only) instead of flat accesses, whose waits also
// drain the LDS counter and serialise the loads issued up front.
#define RTM_GLOBAL __attribute__((address_space(1)))
template <class T>
__device__ __forceinline__ RTM_GLOBAL T* gp(T* p) {
  return (RTM_GLOBAL T*)p;
}
template <class T>
__device__ __forceinline__ const RTM_GLOBAL T* gp(const T* p) {
  return (const RTM_GLOBAL T*)p;
}

// p + i for an element index 0 <= i < 2^30: the byte offset fits 32 bits, so
// the access can add a per-lane 32-bit offset to the wavefront-uniform base
// in scalar registers instead of forming a 64-bit address in each lane.
template <class T>
__device__ __forceinline__ RTM_GLOBAL T* at(RTM_GLOBAL T* p, uint32_t i) {
  return (RTM_GLOBAL T*)((RTM_GLOBAL char*)p + i * (uint32_t)sizeof(T));
}
template <class T>
__device__ __forceinline__ const RTM_GLOBAL T* at(const RTM_GLOBAL T* p, uint32_t i) {
  return (const RTM_GLOBAL T*)((const RTM_GLOBAL char*)p + i * (uint32_t)sizeof(T));
}

template <class T>
__device__ __forceinline__ void st_stream(RTM_GLOBAL T* p, T v) {
#if RTM_NT_STORE
  __builtin_nontemporal_store(v, p);
#else
  *p = v;
#endif
}

template <class T>
__device__ __forceinline__ T ld_stream(const RTM_GLOBAL T* p) {
#if RTM_NT_LOAD
  return __builtin_nontemporal_load(p);
#else
  return *p;
#endif
}

// c = v^2 dt^2 is read with ordinary loads: the shots of a batch on one
// window share one c array, and its lines are then served from the caches
// to the jobs that follow.
template <class T>
__device__ __forceinline__ T ld_medium(const RTM_GLOBAL T* p) {
  return *p;
}

// ---------------------------------------------------------------------------
// 16-bit snapshot codec: q = RNE(x * s), x = q / s with s = 2^(15 - e) where
// max|S^n| = f 2^e, f in [1/2, 1).  The scale is a power of two, so encoding
// and decoding add no rounding beyond the 16-bit cast itself.
// ---------------------------------------------------------------------------
__device__ __forceinline__ float snap_scale_from_max(float m) {
  if (!(m > 0.0f)) return 1.0f;
  int e = ilogbf(m) + 1;  // m = f 2^e, f in [1/2, 1)
  return ldexpf(1.0f, 15 - e);
}

__device__ __forceinline__ uint16_t bf16_rne(float x) {
  uint32_t u = __float_as_uint(x);
  u += 0x7FFFu + ((u >> 16) & 1u);  // round half to even on the dropped 16 bits
  return (uint16_t)(u >> 16);
}

__device__ __forceinline__ float bf16_to_f32(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }

__device__ __forceinline__ uint16_t fp16_rne(float x) { return __half_as_ushort(__float2half_rn(x)); }

__device__ __forceinline__ float fp16_to_f32(uint16_t h) { return __half2float(__ushort_as_half(h)); }

// ---------------------------------------------------------------------------
// LDS staging of a (TZ + 8) x 72 tile with its halo, as 16-byte loads.  The
// loads land in registers first (load()) and go to LDS later (store()), so
// the caller can issue every global load of the step before waiting on any.
// ---------------------------------------------------------------------------
typedef float f32x4 __attribute__((ext_vector_type(4)));

template <int TZ>
struct TileStage {
  static constexpr int kRows = TZ + 2 * kHalo;
  static constexpr int kVec = kLdsW / 4;  // 18 float4 per row
  static constexpr int kN = kRows * kVec;
  static constexpr int kIt = (kN + kThreads - 1) / kThreads;
  f32x4 v[kIt];

  __device__ __forceinline__ void load(const RTM_GLOBAL float* __restrict__ fld, int pitch, int z0, int x0) {
    const RTM_GLOBAL float* base = fld + (int64_t)(z0 - kHalo) * pitch + (x0 - kHalo);
#pragma unroll
    for (int it = 0; it < kIt; ++it) {
      // surplus threads of the last round re-load the last vector (no branch
      // around the load, so no wait at a join); store() skips them
      const int i = min((int)threadIdx.x + it * kThreads, kN - 1);
      const int r = i / kVec, q = i - r * kVec;
      v[it] = *(const RTM_GLOBAL f32x4*)at(base, (uint32_t)(r * pitch + q * 4));
    }
  }
  __device__ __forceinline__ void store(float* __restrict__ lds) const {
#pragma unroll
    for (int it = 0; it < kIt; ++it) {
      const int i = threadIdx.x + it * kThreads;
      if (i < kN) {
        const int r = i / kVec, q = i - r * kVec;
        *reinterpret_cast<f32x4*>(lds + r * kLdsW + q * 4) = v[it];
      }
    }
  }
};

// a + b rounded on its own.  The source term is a product (wavelet sample x
// 1/(dx dz)); left to itself the compiler may fuse that product into the
// addition at some call sites and not at others, and kernels that must agree
// bit for bit would then round the source node differently.
__device__ __forceinline__ float add_unfused(float a, float b) {
#pragma clang fp contract(off)
  return a + b;
}

// One leapfrog update with the sponge, u_new = G (2u + c lap) - G^2 u_old,
// written as explicit fused operations so that every kernel that applies it
// (one step or two per launch) rounds identically.
__device__ __forceinline__ float leapfrog(float G, float c, float lap, float u, float u_old) {
  return fmaf(-(G * G), u_old, G * fmaf(c, lap, 2.0f * u));
}

// 8th-order Laplacian at LDS row `row` (centre) of column `col` (LDS coords),
// z-neighbours from the register window zw[k .. k+8] (zw[k+4] is the centre).
template <int RZ, int W = kLdsW>
__device__ __forceinline__ float lap8(const float* __restrict__ lds, int row, int col,
                                      const float (&zw)[RZ + 8], int k, float c0,
                                      const float (&cz)[4], const float (&cx)[4]) {
  // One address register per call, opaque to the compiler: left to itself
  // it pairs the neighbour reads into ds_read2 instructions, whose 8-bit
  // offsets cannot hold the arrays' LDS offsets, and adds a base per pair.
  typedef __attribute__((address_space(3))) const float lds_f;
  lds_f* rp = (lds_f*)(lds + row * W + col - kHalo);  // rp[kHalo] is the centre
  asm("" : "+v"(rp));
  float s = c0 * zw[k + 4];
  s = fmaf(cz[0], zw[k + 3] + zw[k + 5], s);
  s = fmaf(cx[0], rp[3] + rp[5], s);
  s = fmaf(cz[1], zw[k + 2] + zw[k + 6], s);
  s = fmaf(cx[1], rp[2] + rp[6], s);
  s = fmaf(cz[2], zw[k + 1] + zw[k + 7], s);
  s = fmaf(cx[2], rp[1] + rp[7], s);
  s = fmaf(cz[3], zw[k + 0] + zw[k + 8], s);
  s = fmaf(cx[3], rp[0] + rp[8], s);
  return s;
}

// Index of a physical node (pz, px) in the boundary ring: the 4-cell band
// inside the physical perimeter, ordered top band, bottom band, then the
// left/right bands row by row.  Returns -1 for interior nodes.
// Written with selects only, so callers can use it between loads without
// creating divergent branches.
__device__ __forceinline__ int ring_slot(int pz, int px, int nz, int nx) {
  const int band = pz < 4 ? pz : pz - (nz - 8);              // row within the top/bottom bands
  const int s_tb = band * nx + px;                            // top: rows 0-3, bottom: rows 4-7
  const int s_lr = 8 * nx + (pz - 4) * 8 + (px < 4 ? px : px - (nx - 8));
  const bool tb = pz < 4 || pz >= nz - 4;
  const bool lr = px < 4 || px >= nx - 4;
  return tb ? s_tb : (lr ? s_lr : -1);
}

// ---------------------------------------------------------------------------
// The time-step kernel
// ---------------------------------------------------------------------------
template <int TZ, bool kHasB>
struct StepSmem {
  float a[(TZ + 2 * kHalo) * kLdsW];             // stencil operand (u^n or R^{m+1})
  float b[kHasB ? (TZ + 2 * kHalo) * kLdsW : 4];  // S^{m+1} for reconstruction
  float inj[TZ * kTileX];                        // receiver injection / trace staging
  float red[4];
};

// Snapshot of level lev (a multiple of the stride) at physical row pz, padded
// column x: FP32, or 16-bit after scaling by sc.
__device__ __forceinline__ void store_snap(const DevJob& J, int lev, int pz, int x, float u, float sc) {
  const int64_t off = ((int64_t)(lev / J.snap_stride) * J.nz + pz) * J.pitch + x;
  if (J.snap_dtype == 0)
    st_stream(gp(reinterpret_cast<float*>(J.snap)) + off, u);
  else if (J.snap_dtype == 1)
    st_stream(gp(reinterpret_cast<uint16_t*>(J.snap)) + off, bf16_rne(u * sc));
  else
    st_stream(gp(reinterpret_cast<uint16_t*>(J.snap)) + off, fp16_rne(u * sc));
}

// Snapshot of level lev at physical row pz, padded column x, as a float
// (16-bit codes multiplied by dsc).
__device__ __forceinline__ float load_snap(const DevJob& J, int lev, int pz, int x, float dsc) {
  const int64_t off = ((int64_t)(lev / J.snap_stride) * J.nz + pz) * J.pitch + x;
  if (J.snap_dtype == 0) return ld_stream(gp(reinterpret_cast<const float*>(J.snap)) + off) * dsc;
  const uint16_t q = ld_stream(gp(reinterpret_cast<const uint16_t*>(J.snap)) + off);
  return (J.snap_dtype == 1 ? bf16_to_f32(q) : fp16_to_f32(q)) * dsc;
}

template <int TZ, class Smem>
__device__ __forceinline__ void forward_tile(const DevJob& J, const Tile& tl, int n, Smem& sm) {
  constexpr int RZ = TZ / 4;
  const int lane = threadIdx.x & 63;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // wavefront-uniform
  const int pitch = J.pitch;
  const RTM_GLOBAL float* __restrict__ cur = gp(J.f[n & 3]);
  const RTM_GLOBAL float* __restrict__ old = gp(J.f[(n + 3) & 3]);  // u^{n-1}
  RTM_GLOBAL float* __restrict__ nxt = gp(J.f[(n + 1) & 3]);        // u^{n+1}
  const RTM_GLOBAL float* __restrict__ cc = gp(J.c);
  const RTM_GLOBAL float* __restrict__ gz = gp(J.gz);
  const RTM_GLOBAL float* __restrict__ gx = gp(J.gx);
  const int x = tl.x0 + lane;
  const int z0 = tl.z0 + w * RZ;
  const bool colok = x < J.nxp;

  // ---- issue every global load of the step first ----
  TileStage<TZ> st;
  st.load(cur, pitch, tl.z0, tl.x0);
  // Pointwise operands: every lane loads (addresses clamped into the grid, so
  // there is no branch around a load); lanes outside the grid never use them.
  float cv[RZ], pv[RZ], gzv[RZ];
  const int xcl = min(x, J.nxp - 1);
#pragma unroll
  for (int k = 0; k < RZ; ++k) {
    const int zc = min(z0 + k, J.nzp - 1);
    const int64_t idx = (int64_t)zc * pitch + xcl;
    cv[k] = ld_medium(cc + idx);
    pv[k] = ld_stream(old + idx);
    gzv[k] = gz[zc];
  }
  const float gxv = colok ? gx[xcl] : 0.0f;
  const float wsrc = gp(J.wavelet)[n] * J.inv_cell;
  const int mode = J.mode;
  const bool snap_now = mode == kModeStore && (n % J.snap_stride) == 0;
  // u^{n-1}, when a two-step launch computed it as its first step: that
  // launch could not scale it (its maximum was not complete), so the launch
  // after it stores it
  const bool snap_prev = mode == kModeStore && J.two_step && (n & 1) == 0 && n >= 2 &&
                         ((n - 1) % J.snap_stride) == 0 && two_step_pair(n - 2, J.nt, J.nsteps, mode);
  const bool want_max = mode == kModeStore && J.snap_dtype != 0 && ((n + 1) % J.snap_stride) == 0 &&
                        (n + 1) <= J.nt - 2;
  // per-snapshot scale from the max-abs of u^n, kept as kMaxSlots partial maxima
  float sc = 1.0f, scp = 1.0f;
  if (snap_now && J.snap_dtype != 0)
    sc = snap_scale_from_max(wave_max(__uint_as_float(gp(J.maxbits)[(int64_t)n * kMaxSlots + lane])));
  if (snap_prev && J.snap_dtype != 0)
    scp = snap_scale_from_max(wave_max(__uint_as_float(gp(J.maxbits)[(int64_t)(n - 1) * kMaxSlots + lane])));
  st.store(sm.a);
  __syncthreads();

  const float c0 = J.c0;
  const float cz[4] = {J.cz[0], J.cz[1], J.cz[2], J.cz[3]};
  const float cx[4] = {J.cx[0], J.cx[1], J.cx[2], J.cx[3]};
  const int px = x - J.nb;
  const bool colphys = px >= 0 && px < J.nx;

  float zw[RZ + 8];
#pragma unroll
  for (int j = 0; j < RZ + 8; ++j) zw[j] = sm.a[(w * RZ + j) * kLdsW + lane + kHalo];

  float vmax = 0.0f;
#pragma clang loop unroll(full)
  for (int k = 0; k < RZ; ++k) {
    const int lz = w * RZ + k;
    const int z = z0 + k;
    if (colok && z < J.nzp) {
      const int64_t idx = (int64_t)z * pitch + x;
      float lap = lap8<RZ>(sm.a, lz + kHalo, lane + kHalo, zw, k, c0, cz, cx);
      if (z == J.src_z && x == J.src_x) lap = add_unfused(lap, wsrc);
      const float G = gzv[k] * gxv;
      const float u = zw[k + 4];
      const float un = leapfrog(G, cv[k], lap, u, pv[k]);
      st_stream(nxt + idx, un);
      const int pz = z - J.nb;
      const bool phys = colphys && pz >= 0 && pz < J.nz;
      if (mode == kModeModel) {
        sm.inj[lz * kTileX + lane] = un;
      } else if (phys) {
        if (mode == kModeRecon) {
          int slot = ring_slot(pz, px, J.nz, J.nx);
          if (slot >= 0) st_stream(gp(J.ring) + (int64_t)(n + 1) * J.ring_len + slot, un);
        } else {
          if (snap_now) store_snap(J, n, pz, x, u, sc);
          if (snap_prev) store_snap(J, n - 1, pz, x, pv[k], scp);
          vmax = fmaxf(vmax, fabsf(un));
        }
      }
    }
  }
  if (want_max) {
    const int tile_id = (tl.z0 / TZ) * J.tiles_x + tl.x0 / kTileX;
    wg_atomic_max(vmax, &J.maxbits[(int64_t)(n + 1) * kMaxSlots + (tile_id & (kMaxSlots - 1))], sm.red);
  }
  if (mode == kModeModel && tl.rec_count > 0 && J.traces != nullptr) {
    __syncthreads();
    for (int i = threadIdx.x; i < tl.rec_count; i += kThreads) {
      int2 r = J.recs[tl.rec_begin + i];
      gp(J.traces)[(int64_t)(n + 1) * J.nrec + r.y] = sm.inj[r.x];
    }
  }
}

template <int TZ, class Smem>
__device__ __forceinline__ void backward_tile(const DevJob& J, const Tile& tl, int m, Smem& sm) {
  constexpr int RZ = TZ / 4;
  const int lane = threadIdx.x & 63;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // wavefront-uniform
  const int pitch = J.pitch;
  const int nt = J.nt;
  const RTM_GLOBAL float* __restrict__ rcur = gp(J.r[(m + 1) & 3]);  // R^{m+1}
  const RTM_GLOBAL float* __restrict__ rold = gp(J.r[(m + 2) & 3]);  // R^{m+2}
  RTM_GLOBAL float* __restrict__ rout = gp(J.r[m & 3]);              // R^m
  const RTM_GLOBAL float* __restrict__ scur = gp(J.f[(m + 1) & 3]);  // S^{m+1}
  const RTM_GLOBAL float* __restrict__ sold = gp(J.f[(m + 2) & 3]);  // S^{m+2}
  RTM_GLOBAL float* __restrict__ sout = gp(J.f[m & 3]);  // S^m (left by the forward pass when m >= nt-2)
  RTM_GLOBAL float* __restrict__ image = gp(J.image);
  RTM_GLOBAL float* __restrict__ illum = gp(J.illum);
  const RTM_GLOBAL float* __restrict__ cc = gp(J.c);
  const RTM_GLOBAL float* __restrict__ gz = gp(J.gz);
  const RTM_GLOBAL float* __restrict__ gx = gp(J.gx);
  const int mode = J.mode;
  const int x = tl.x0 + lane;
  const int z0 = tl.z0 + w * RZ;
  const bool colok = x < J.nxp;
  const int px = x - J.nb;
  const bool colphys = px >= 0 && px < J.nx;

  // Does this tile touch the physical window?  Which source-side work runs?
  const int pz0 = tl.z0 - J.nb, px0 = tl.x0 - J.nb;
  const bool tile_phys = pz0 < J.nz && pz0 + TZ > 0 && px0 < J.nx && px0 + kTileX > 0;
  const bool imaging = tile_phys && m <= nt - 2 &&
                       (mode == kModeRecon || (m % J.snap_stride) == 0);
  const bool recon = imaging && mode == kModeRecon && m <= nt - 3;

  // ---- issue every global load of the step first ----
  TileStage<TZ> sa;
  sa.load(rcur, pitch, tl.z0, tl.x0);
  TileStage<TZ> sb;
  if (recon) sb.load(scur, pitch, tl.z0, tl.x0);
  // Pointwise operands, loaded by every lane from addresses clamped into the
  // grid / the physical window (no branch around a load; only wavefront-
  // uniform branches on the mode); lanes outside never use their values.
  float cv[RZ], pv[RZ], iv[RZ], sv[RZ], gzv[RZ];
  bool ring_pt[RZ];
  const int xcl = min(x, J.nxp - 1);
  const int xph = min(max(x, J.nb), J.nb + J.nx - 1);  // padded column clamped to the window
#pragma unroll
  for (int k = 0; k < RZ; ++k) {
    const int zc = min(z0 + k, J.nzp - 1);
    const int64_t idx = (int64_t)zc * pitch + xcl;
    cv[k] = ld_medium(cc + idx);
    pv[k] = ld_stream(rold + idx);
    gzv[k] = gz[zc];
    iv[k] = 0.0f;
    sv[k] = 0.0f;
    ring_pt[k] = false;
  }
  if (imaging) {
#pragma unroll
    for (int k = 0; k < RZ; ++k) {
      const int pzc = min(max(z0 + k - J.nb, 0), J.nz - 1);
      iv[k] = ld_stream((const RTM_GLOBAL float*)image + (int64_t)pzc * pitch + xph);
    }
    if (recon) {
#pragma unroll
      for (int k = 0; k < RZ; ++k) {
        const int pzc = min(max(z0 + k - J.nb, 0), J.nz - 1);
        const int slot = ring_slot(pzc, xph - J.nb, J.nz, J.nx);
        ring_pt[k] = slot >= 0;
        // ring nodes are restored from storage; interior nodes need S^{m+2}
        const RTM_GLOBAL float* sp =
            slot >= 0 ? gp(J.ring) + (int64_t)m * J.ring_len + slot
                      : sold + (int64_t)(pzc + J.nb) * pitch + xph;
        sv[k] = ld_stream(sp);
      }
    } else if (mode == kModeRecon) {
#pragma unroll
      for (int k = 0; k < RZ; ++k) {  // S^{nt-2}, left by the forward pass
        const int pzc = min(max(z0 + k - J.nb, 0), J.nz - 1);
        sv[k] = ld_stream((const RTM_GLOBAL float*)sout + (int64_t)(pzc + J.nb) * pitch + xph);
      }
    } else {
      const int64_t base = (int64_t)(m / J.snap_stride) * J.nz;
      if (J.snap_dtype == 0) {
        const RTM_GLOBAL float* sp = gp(reinterpret_cast<const float*>(J.snap));
#pragma unroll
        for (int k = 0; k < RZ; ++k)
          sv[k] = ld_stream(sp + (base + min(max(z0 + k - J.nb, 0), J.nz - 1)) * pitch + xph);
      } else {
        const RTM_GLOBAL uint16_t* sp = gp(reinterpret_cast<const uint16_t*>(J.snap));
        const bool bf = J.snap_dtype == 1;
#pragma unroll
        for (int k = 0; k < RZ; ++k) {
          const uint16_t q = ld_stream(sp + (base + min(max(z0 + k - J.nb, 0), J.nz - 1)) * pitch + xph);
          sv[k] = bf ? bf16_to_f32(q) : fp16_to_f32(q);
        }
      }
    }
  }
  const float gxv = colok ? gx[xcl] : 0.0f;
  const float wsrc = (recon ? gp(J.wavelet)[m + 1] : 0.0f) * J.inv_cell;
  float dsc = 1.0f;
  if (imaging && mode == kModeStore && J.snap_dtype != 0)  // exact: power of two
    dsc = 1.0f / snap_scale_from_max(wave_max(__uint_as_float(gp(J.maxbits)[(int64_t)m * kMaxSlots + lane])));
  sa.store(sm.a);
  if (recon) sb.store(sm.b);
  if (tl.rec_count > 0) {
    for (int i = threadIdx.x; i < TZ * kTileX; i += kThreads) sm.inj[i] = 0.0f;
    __syncthreads();
    const RTM_GLOBAL float* dm = gp(J.data) + (int64_t)m * J.nrec;
    for (int i = threadIdx.x; i < tl.rec_count; i += kThreads) {
      int2 r = J.recs[tl.rec_begin + i];
      atomicAdd(&sm.inj[r.x], dm[r.y]);
    }
  }
  __syncthreads();

  const float c0 = J.c0;
  const float cz[4] = {J.cz[0], J.cz[1], J.cz[2], J.cz[3]};
  const float cx[4] = {J.cx[0], J.cx[1], J.cx[2], J.cx[3]};
  const bool has_inj = tl.rec_count > 0;
  const float kfac = J.kfac;

  float zr[RZ + 8];
#pragma unroll
  for (int j = 0; j < RZ + 8; ++j) zr[j] = sm.a[(w * RZ + j) * kLdsW + lane + kHalo];
  float zs[RZ + 8];
  if (recon) {
#pragma unroll
    for (int j = 0; j < RZ + 8; ++j) zs[j] = sm.b[(w * RZ + j) * kLdsW + lane + kHalo];
  }

#pragma clang loop unroll(full)
  for (int k = 0; k < RZ; ++k) {
    const int lz = w * RZ + k;
    const int z = z0 + k;
    if (colok && z < J.nzp) {
      const int64_t idx = (int64_t)z * pitch + x;
      float lap = lap8<RZ>(sm.a, lz + kHalo, lane + kHalo, zr, k, c0, cz, cx);
      if (has_inj) lap += sm.inj[lz * kTileX + lane];
      const float G = gzv[k] * gxv;
      const float r1 = zr[k + 4];  // R^{m+1}
      st_stream(rout + idx, leapfrog(G, cv[k], lap, r1, pv[k]));
      const int pz = z - J.nb;
      if (imaging && colphys && pz >= 0 && pz < J.nz) {
        float s;
        if (mode == kModeRecon) {
          if (recon) {
            if (ring_pt[k]) {
              s = sv[k];
            } else {
              float ls = lap8<RZ>(sm.b, lz + kHalo, lane + kHalo, zs, k, c0, cz, cx);
              if (z == J.src_z && x == J.src_x) ls = add_unfused(ls, wsrc);
              s = fmaf(cv[k], ls, 2.0f * zs[k + 4]) - sv[k];
            }
            st_stream(sout + idx, s);
          } else {
            s = sv[k];
          }
        } else {
          s = sv[k] * dsc;
        }
        const int64_t io = (int64_t)pz * pitch + x;
        st_stream(image + io, fmaf(kfac * s, r1, iv[k]));
        if (illum) illum[io] = fmaf(kfac * s, s, illum[io]);
      }
    }
  }
}

template <int TZ, class Smem>
__device__ __forceinline__ void born_tile(const DevJob& J, const Tile& tl, int n, Smem& sm) {
  // Born (single-scattering) modelling, step n, background and scattered
  // field in lockstep:
  //   u0^{n+1} = G(2u0^n + c(L u0^n + w^n e_s/(dx dz))) - G^2 u0^{n-1}
  //   du^{n+1} = G(2du^n + c(L du^n + m u0^n)) - G^2 du^{n-1},  dd[n+1][r] = du^{n+1}(r)
  // m is the velocity-model perturbation on the physical window (zero in the
  // sponge); u0^n is the centre value the background stencil already holds.
  constexpr int RZ = TZ / 4;
  const int lane = threadIdx.x & 63;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // wavefront-uniform
  const int pitch = J.pitch;
  const RTM_GLOBAL float* __restrict__ ucur = gp(J.f[n & 3]);
  const RTM_GLOBAL float* __restrict__ uold = gp(J.f[(n + 3) & 3]);
  RTM_GLOBAL float* __restrict__ unxt = gp(J.f[(n + 1) & 3]);
  const RTM_GLOBAL float* __restrict__ dcur = gp(J.r[n & 3]);
  const RTM_GLOBAL float* __restrict__ dold = gp(J.r[(n + 3) & 3]);
  RTM_GLOBAL float* __restrict__ dnxt = gp(J.r[(n + 1) & 3]);
  const RTM_GLOBAL float* __restrict__ mp = gp(J.image);
  const RTM_GLOBAL float* __restrict__ cc = gp(J.c);
  const RTM_GLOBAL float* __restrict__ gz = gp(J.gz);
  const RTM_GLOBAL float* __restrict__ gx = gp(J.gx);
  const int x = tl.x0 + lane;
  const int z0 = tl.z0 + w * RZ;
  const bool colok = x < J.nxp;
  const int px = x - J.nb;
  const bool colphys = px >= 0 && px < J.nx;

  TileStage<TZ> sa, sb;
  sa.load(ucur, pitch, tl.z0, tl.x0);
  sb.load(dcur, pitch, tl.z0, tl.x0);
  float cv[RZ], pv[RZ], qv[RZ], mv[RZ], gzv[RZ];
  const int xcl = min(x, J.nxp - 1);
  const int xph = min(max(x, J.nb), J.nb + J.nx - 1);
#pragma unroll
  for (int k = 0; k < RZ; ++k) {
    const int zc = min(z0 + k, J.nzp - 1);
    const int64_t idx = (int64_t)zc * pitch + xcl;
    cv[k] = ld_medium(cc + idx);
    pv[k] = ld_stream(uold + idx);
    qv[k] = ld_stream(dold + idx);
    gzv[k] = gz[zc];
    const int pzc = min(max(z0 + k - J.nb, 0), J.nz - 1);
    mv[k] = ld_stream(mp + (int64_t)pzc * pitch + xph);
  }
  const float gxv = colok ? gx[xcl] : 0.0f;
  const float wsrc = gp(J.wavelet)[n] * J.inv_cell;
  sa.store(sm.a);
  sb.store(sm.b);
  __syncthreads();

  const float c0 = J.c0;
  const float cz[4] = {J.cz[0], J.cz[1], J.cz[2], J.cz[3]};
  const float cx[4] = {J.cx[0], J.cx[1], J.cx[2], J.cx[3]};
  float zu[RZ + 8], zd[RZ + 8];
#pragma unroll
  for (int j = 0; j < RZ + 8; ++j) {
    zu[j] = sm.a[(w * RZ + j) * kLdsW + lane + kHalo];
    zd[j] = sm.b[(w * RZ + j) * kLdsW + lane + kHalo];
  }
#pragma clang loop unroll(full)
  for (int k = 0; k < RZ; ++k) {
    const int lz = w * RZ + k;
    const int z = z0 + k;
    if (colok && z < J.nzp) {
      const int64_t idx = (int64_t)z * pitch + x;
      const int pz = z - J.nb;
      const bool phys = colphys && pz >= 0 && pz < J.nz;
      const float G = gzv[k] * gxv;
      const float u = zu[k + 4];
      float lu = lap8<RZ>(sm.a, lz + kHalo, lane + kHalo, zu, k, c0, cz, cx);
      if (z == J.src_z && x == J.src_x) lu = add_unfused(lu, wsrc);
      st_stream(unxt + idx, leapfrog(G, cv[k], lu, u, pv[k]));
      float ld = lap8<RZ>(sm.b, lz + kHalo, lane + kHalo, zd, k, c0, cz, cx);
      if (phys) ld = fmaf(mv[k], u, ld);
      const float dn = leapfrog(G, cv[k], ld, zd[k + 4], qv[k]);
      st_stream(dnxt + idx, dn);
      sm.inj[lz * kTileX + lane] = dn;
    }
  }
  if (tl.rec_count > 0 && J.traces != nullptr) {
    __syncthreads();
    for (int i = threadIdx.x; i < tl.rec_count; i += kThreads) {
      int2 r = J.recs[tl.rec_begin + i];
      gp(J.traces)[(int64_t)(n + 1) * J.nrec + r.y] = sm.inj[r.x];
    }
  }
}

// ---------------------------------------------------------------------------
// Two time steps per launch (reconstruct and store mode).  A two-step tile owns output
// rows [z0, z0 + TZ) and columns [x0, x0 + 56).  Its first step covers the
// middle region, the tile grown by the stencil radius (rows z0 - 4 ..
// z0 + TZ + 4, columns x0 - 4 .. x0 + 60: one column per lane), from inputs
// staged with an 8-cell halo; the second step reads the middle region from
// LDS.  Middle-region values outside the grid are set to zero, the value the
// ghost cells hold for a one-step launch, so every node goes through the same
// operations on the same operands as in two one-step launches and the
// results agree bit for bit.  Each job then moves its two stepped fields
// once per two steps instead of once per step.
// ---------------------------------------------------------------------------
// Two-step kernels read and write through the caches: the levels a launch
// writes are the ones the next launch reads, and ordinary accesses let the
// caches keep part of them (measured on the 100-shot survey: backward pair
// 878 -> 818 us, forward pair 418 -> 398 us).  The one-step kernels keep the
// streaming hints, which measured better for the serving engine's mixed
// launches (1024-RTM ensemble 3.14e11 against 3.01e11 updates/s).
template <class T>
__device__ __forceinline__ T ld_cached(const RTM_GLOBAL T* p) {
  return *p;
}
template <class T>
__device__ __forceinline__ void st_cached(RTM_GLOBAL T* p, T v) {
  *p = v;
}

template <int ROWS>
struct TileStageW {  // ROWS x 72 floats from (zs, xs), as 16-byte loads
  static constexpr int kVec = kLdsW / 4;
  static constexpr int kN = ROWS * kVec;
  static constexpr int kIt = (kN + kThreads - 1) / kThreads;
  f32x4 v[kIt];

  __device__ __forceinline__ void load(const RTM_GLOBAL float* __restrict__ fld, int pitch, int zs, int xs) {
    const RTM_GLOBAL float* base = fld + (int64_t)zs * pitch + xs;
#pragma unroll
    for (int it = 0; it < kIt; ++it) {
      const int i = min((int)threadIdx.x + it * kThreads, kN - 1);
      const int r = i / kVec, q = i - r * kVec;
      v[it] = *(const RTM_GLOBAL f32x4*)at(base, (uint32_t)(r * pitch + q * 4));
    }
  }
  __device__ __forceinline__ void store(float* __restrict__ lds) const {
#pragma unroll
    for (int it = 0; it < kIt; ++it) {
      const int i = threadIdx.x + it * kThreads;
      if (i < kN) {
        const int r = i / kVec, q = i - r * kVec;
        *reinterpret_cast<f32x4*>(lds + r * kLdsW + q * 4) = v[it];
      }
    }
  }
};

// kRecon: the backward pass reconstructs S (reconstruct mode), which needs
// the staged S^{m+1}; a store-mode backward pair stages R only.
template <int TZ, bool kBwd, bool kRecon = true>
struct Step2Smem {
  float a[(TZ + 4 * kHalo) * kLdsW];                         // u^n or R^{m+1}, 8-cell halo
  float b[kBwd && kRecon ? (TZ + 4 * kHalo) * kLdsW : 4];    // S^{m+1}
  float ma[(TZ + 2 * kHalo) * kTileX];                       // middle region: u^{n+1} or R^m
  float mb[kBwd ? (TZ + 2 * kHalo) * kTileX : 4];            // middle region: S^m (store mode: receiver data)
  float red[4];                                              // workgroup max (store mode)
};

// Boundary-ring save of a forward value at level `lev` (reconstruct mode).
__device__ __forceinline__ void ring_save(const DevJob& J, int z, int x, int lev, float v) {
  const int pz = z - J.nb, px = x - J.nb;
  if (pz >= 0 && pz < J.nz && px >= 0 && px < J.nx) {
    const int slot = ring_slot(pz, px, J.nz, J.nx);
    if (slot >= 0) st_cached(gp(J.ring) + (int64_t)lev * J.ring_len + slot, v);
  }
}

// One two-step forward tile.  kFast: the middle region lies inside the grid
// and holds neither the source nor a boundary-ring node, so no node needs a
// zero, a source term or a ring save and the per-node tests drop out; the
// other tiles take the general path.  Offsets are 32-bit (a field holds
// fewer than 2^30 floats).
template <int TZ, bool kFast, bool kStore, class Smem>
__device__ __forceinline__ void forward2_body(const DevJob& J, const Tile& tl, int n, Smem& sm) {
  constexpr int RA = (TZ + 2 * kHalo) / 4;  // middle rows per wavefront (first step)
  constexpr int RB = TZ / 4;                // output rows per wavefront (second step)
  const int lane = threadIdx.x & 63;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // wavefront-uniform
  const int pitch = J.pitch;
  const RTM_GLOBAL float* __restrict__ u0 = gp(J.f[n & 3]);        // u^n
  const RTM_GLOBAL float* __restrict__ um = gp(J.f[(n + 3) & 3]);  // u^{n-1}
  RTM_GLOBAL float* __restrict__ u1 = gp(J.f[(n + 1) & 3]);        // u^{n+1}
  RTM_GLOBAL float* __restrict__ u2 = gp(J.f[(n + 2) & 3]);        // u^{n+2}
  const RTM_GLOBAL float* __restrict__ cc = gp(J.c);
  const RTM_GLOBAL float* __restrict__ gz = gp(J.gz);
  const RTM_GLOBAL float* __restrict__ gx = gp(J.gx);
  const int x = tl.x0 - kHalo + lane;      // this lane's column
  const int za0 = tl.z0 - kHalo + w * RA;  // first middle row of this wavefront
  const int zb0 = tl.z0 + w * RB;          // first output row of this wavefront
  const bool xin = x >= 0 && x < J.nxp;
  const bool xout = lane >= kHalo && lane < kHalo + kTileX2 && (kFast || x < J.nxp);
  const uint32_t xcl = (uint32_t)min(max(x, 0), J.nxp - 1);

  // ---- every global load first ----
  TileStageW<TZ + 4 * kHalo> st;
  st.load(u0, pitch, tl.z0 - 2 * kHalo, tl.x0 - 2 * kHalo);
  float cva[RA], pva[RA], gza[RA], cvb[RB], gzb[RB];
#pragma unroll
  for (int k = 0; k < RA; ++k) {
    const int zc = kFast ? za0 + k : min(max(za0 + k, 0), J.nzp - 1);
    const uint32_t off = (uint32_t)zc * (uint32_t)pitch + xcl;
    cva[k] = ld_medium(at(cc, off));
    pva[k] = ld_cached(at(um, off));
    gza[k] = gz[zc];
  }
#pragma unroll
  for (int k = 0; k < RB; ++k) {
    const int zc = kFast ? zb0 + k : min(zb0 + k, J.nzp - 1);
    cvb[k] = ld_medium(at(cc, (uint32_t)zc * (uint32_t)pitch + xcl));
    gzb[k] = gz[zc];
  }
  const float gxv = (kFast || xin) ? gx[xcl] : 0.0f;
  const float w0 = kFast ? 0.0f : gp(J.wavelet)[n] * J.inv_cell;
  const float w1 = kFast ? 0.0f : gp(J.wavelet)[n + 1] * J.inv_cell;
  // store mode: snapshots of the levels this launch reads (u^n; u^{n-1} when
  // the previous two-step launch computed it), each with the scale of its
  // complete maximum, and the partial maxima of the levels it computes
  constexpr bool store = kStore && !kFast;
  const int stride = J.snap_stride;
  const bool snap0 = store && (n % stride) == 0;
  const bool snapp = store && n >= 2 && ((n - 1) % stride) == 0 && two_step_pair(n - 2, J.nt, J.nsteps, J.mode);
  const bool want1 = store && J.snap_dtype != 0 && ((n + 1) % stride) == 0 && n + 1 <= J.nt - 2;
  const bool want2 = store && J.snap_dtype != 0 && ((n + 2) % stride) == 0 && n + 2 <= J.nt - 2;
  float sc0 = 1.0f, scp = 1.0f;
  if (snap0 && J.snap_dtype != 0)
    sc0 = snap_scale_from_max(wave_max(__uint_as_float(gp(J.maxbits)[(int64_t)n * kMaxSlots + lane])));
  if (snapp && J.snap_dtype != 0)
    scp = snap_scale_from_max(wave_max(__uint_as_float(gp(J.maxbits)[(int64_t)(n - 1) * kMaxSlots + lane])));
  const int px = x - J.nb;
  const bool colphys = px >= 0 && px < J.nx;
  float vmax1 = 0.0f, vmax2 = 0.0f;
  st.store(sm.a);
  __syncthreads();

  const float c0 = J.c0;
  const float cz[4] = {J.cz[0], J.cz[1], J.cz[2], J.cz[3]};
  const float cx[4] = {J.cx[0], J.cx[1], J.cx[2], J.cx[3]};

  // ---- first step: u^{n+1} on the middle region ----
  float zw[RA + 8];
#pragma unroll
  for (int j = 0; j < RA + 8; ++j) zw[j] = sm.a[(w * RA + j) * kLdsW + lane + kHalo];
#pragma clang loop unroll(full)
  for (int k = 0; k < RA; ++k) {
    const int r = w * RA + k;  // middle row (wavefront-uniform)
    const int z = za0 + k;
    float lap = lap8<RA>(sm.a, r + kHalo, lane + kHalo, zw, k, c0, cz, cx);
    if (!kFast && z == J.src_z && x == J.src_x) lap = add_unfused(lap, w0);
    const float G = gza[k] * gxv;
    float un = leapfrog(G, cva[k], lap, zw[k + 4], pva[k]);
    if (!kFast) un = (xin && z >= 0 && z < J.nzp) ? un : 0.0f;
    sm.ma[r * kTileX + lane] = un;
    if (r >= kHalo && r < TZ + kHalo && (kFast || z < J.nzp) && xout) {  // a node of the output tile
      st_cached(at(u1, (uint32_t)z * (uint32_t)pitch + (uint32_t)x), un);
      if (store) {
        const int pz = z - J.nb;
        if (colphys && pz >= 0 && pz < J.nz) {
          if (snap0) store_snap(J, n, pz, x, zw[k + 4], sc0);
          if (snapp) store_snap(J, n - 1, pz, x, pva[k], scp);
          vmax1 = fmaxf(vmax1, fabsf(un));
        }
      } else if (!kFast) {
        ring_save(J, z, x, n + 1, un);
      }
    }
  }
  __syncthreads();

  // ---- second step: u^{n+2} on the output tile ----
  float zm[RB + 8];
#pragma unroll
  for (int j = 0; j < RB + 8; ++j) zm[j] = sm.ma[(w * RB + j) * kTileX + lane];
#pragma clang loop unroll(full)
  for (int k = 0; k < RB; ++k) {
    const int z = zb0 + k;
    float lap = lap8<RB, kTileX>(sm.ma, w * RB + k + kHalo, lane, zm, k, c0, cz, cx);
    if (!kFast && z == J.src_z && x == J.src_x) lap = add_unfused(lap, w1);
    const float G = gzb[k] * gxv;
    const float uold = sm.a[(w * RB + k + 2 * kHalo) * kLdsW + lane + kHalo];  // u^n
    if (xout && (kFast || z < J.nzp)) {
      const float un = leapfrog(G, cvb[k], lap, zm[k + 4], uold);
      st_cached(at(u2, (uint32_t)z * (uint32_t)pitch + (uint32_t)x), un);
      if (store) {
        const int pz = z - J.nb;
        if (colphys && pz >= 0 && pz < J.nz) vmax2 = fmaxf(vmax2, fabsf(un));
      } else if (!kFast) {
        ring_save(J, z, x, n + 2, un);
      }
    }
  }
  if (want1 || want2) {  // wavefront-uniform: the whole workgroup takes this branch
    const int slot = ((tl.z0 / TZ) * J.tiles_x2 + tl.x0 / kTileX2) & (kMaxSlots - 1);
    if (want1) wg_atomic_max(vmax1, &J.maxbits[(int64_t)(n + 1) * kMaxSlots + slot], sm.red);
    if (want2) {
      __syncthreads();  // sm.red is reused
      wg_atomic_max(vmax2, &J.maxbits[(int64_t)(n + 2) * kMaxSlots + slot], sm.red);
    }
  }
}

// kStore: store-mode jobs (general path, snapshots); else reconstruct mode.
template <int TZ, bool kStore, class Smem>
__device__ __forceinline__ void forward2_tile(const DevJob& J, const Tile& tl, int n, Smem& sm) {
  if (kStore) {
    forward2_body<TZ, false, true>(J, tl, n, sm);
    return;
  }
  const int z0 = tl.z0, x0 = tl.x0;
  const bool inside = z0 >= kHalo && z0 + TZ + kHalo <= J.nzp && x0 >= kHalo && x0 + kTileX2 + kHalo <= J.nxp;
  const bool src = J.src_z >= z0 - kHalo && J.src_z < z0 + TZ + kHalo && J.src_x >= x0 - kHalo &&
                   J.src_x < x0 + kTileX2 + kHalo;
  // output nodes in the physical window but outside its interior hold ring nodes
  const int pz0 = z0 - J.nb, pz1 = z0 + TZ - J.nb, px0 = x0 - J.nb, px1 = x0 + kTileX2 - J.nb;
  const bool phys = pz0 < J.nz && pz1 > 0 && px0 < J.nx && px1 > 0;
  const bool interior = pz0 >= 4 && pz1 <= J.nz - 4 && px0 >= 4 && px1 <= J.nx - 4;
  if (inside && !src && !(phys && !interior))
    forward2_body<TZ, true, false>(J, tl, n, sm);
  else
    forward2_body<TZ, false, false>(J, tl, n, sm);
}

// One two-step backward tile, levels m and m - 1 (reconstruct mode, both
// levels imaged and reconstructed: 1 <= m <= nt - 3).  The first step gives
// R^m and S^m on the middle region, the second R^{m-1} and S^{m-1} on the
// output tile, and the second also applies both imaging terms in level order
// (image + k S^m R^{m+1}, then + k S^{m-1} R^m), as two one-step launches do.
// S is defined on the physical window only: its interior nodes are
// reconstructed, its boundary-ring nodes restored from storage, and
// elsewhere the middle region holds zeros that no interior node reads.
// KIND 1: the middle region lies in the interior of the physical window;
// KIND 2: it lies in the grid outside the physical window (sponge only, no
// S); neither holds the source or a receiver.  KIND 0 is the general path.
template <int TZ, int KIND, class Smem>
__device__ __forceinline__ void backward2_body(const DevJob& J, const Tile& tl, const int2* __restrict__ recs2,
                                               int m, Smem& sm) {
  constexpr bool kGen = KIND == 0, kSrc = KIND != 2;  // kSrc: S and imaging may be present
  constexpr int RA = (TZ + 2 * kHalo) / 4;
  constexpr int RB = TZ / 4;
  const int lane = threadIdx.x & 63;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // wavefront-uniform
  const int pitch = J.pitch;
  const RTM_GLOBAL float* __restrict__ r1 = gp(J.r[(m + 1) & 3]);  // R^{m+1}
  const RTM_GLOBAL float* __restrict__ r2 = gp(J.r[(m + 2) & 3]);  // R^{m+2}
  RTM_GLOBAL float* __restrict__ r0 = gp(J.r[m & 3]);              // R^m
  RTM_GLOBAL float* __restrict__ rn = gp(J.r[(m + 3) & 3]);        // R^{m-1}
  const RTM_GLOBAL float* __restrict__ s1 = gp(J.f[(m + 1) & 3]);  // S^{m+1}
  const RTM_GLOBAL float* __restrict__ s2 = gp(J.f[(m + 2) & 3]);  // S^{m+2}
  RTM_GLOBAL float* __restrict__ s0 = gp(J.f[m & 3]);              // S^m
  RTM_GLOBAL float* __restrict__ sn = gp(J.f[(m + 3) & 3]);        // S^{m-1}
  RTM_GLOBAL float* __restrict__ image = gp(J.image);
  const RTM_GLOBAL float* __restrict__ cc = gp(J.c);
  const RTM_GLOBAL float* __restrict__ gz = gp(J.gz);
  const RTM_GLOBAL float* __restrict__ gx = gp(J.gx);
  const int x = tl.x0 - kHalo + lane;
  const int za0 = tl.z0 - kHalo + w * RA;
  const int zb0 = tl.z0 + w * RB;
  const bool xin = x >= 0 && x < J.nxp;
  const bool xout = lane >= kHalo && lane < kHalo + kTileX2 && (!kGen || x < J.nxp);
  const uint32_t xcl = (uint32_t)min(max(x, 0), J.nxp - 1);
  const int px = x - J.nb;
  const bool colphys = px >= 0 && px < J.nx;
  const uint32_t xph = (uint32_t)min(max(x, J.nb), J.nb + J.nx - 1);  // column clamped into the window
  // general path: does the middle region reach the physical window?
  const bool tphys = kGen ? (tl.z0 - kHalo - J.nb < J.nz && tl.z0 + TZ + kHalo - J.nb > 0 &&
                             tl.x0 - kHalo - J.nb < J.nx && tl.x0 + kTileX2 + kHalo - J.nb > 0)
                          : KIND == 1;

  // ---- every global load first ----
  TileStageW<TZ + 4 * kHalo> sa, sb;
  sa.load(r1, pitch, tl.z0 - 2 * kHalo, tl.x0 - 2 * kHalo);
  if (kSrc && tphys) sb.load(s1, pitch, tl.z0 - 2 * kHalo, tl.x0 - 2 * kHalo);
  float cva[RA], pva[RA], gza[RA], sva[RA];
  bool ringa[RA];
#pragma unroll
  for (int k = 0; k < RA; ++k) {
    const int zc = kGen ? min(max(za0 + k, 0), J.nzp - 1) : za0 + k;
    const uint32_t off = (uint32_t)zc * (uint32_t)pitch + xcl;
    cva[k] = ld_medium(at(cc, off));
    pva[k] = ld_cached(at(r2, off));
    gza[k] = gz[zc];
    sva[k] = 0.0f;
    ringa[k] = false;
    if (KIND == 1) sva[k] = ld_cached(at(s2, off));
  }
  if (kGen && tphys) {
#pragma unroll
    for (int k = 0; k < RA; ++k) {  // S^{m+2}, or the stored ring value of level m
      const int pzc = min(max(za0 + k - J.nb, 0), J.nz - 1);
      const int slot = ring_slot(pzc, (int)xph - J.nb, J.nz, J.nx);
      ringa[k] = slot >= 0;
      const RTM_GLOBAL float* sp = slot >= 0 ? gp(J.ring) + (int64_t)m * J.ring_len + slot
                                             : s2 + ((uint32_t)(pzc + J.nb) * (uint32_t)pitch + xph);
      sva[k] = ld_cached(sp);
    }
  }
  float cvb[RB], gzb[RB], ivb[RB], svb[RB];
  bool ringb[RB];
#pragma unroll
  for (int k = 0; k < RB; ++k) {
    const int zc = kGen ? min(zb0 + k, J.nzp - 1) : zb0 + k;
    cvb[k] = ld_medium(at(cc, (uint32_t)zc * (uint32_t)pitch + xcl));
    gzb[k] = gz[zc];
    ivb[k] = 0.0f;
    svb[k] = 0.0f;
    ringb[k] = false;
    if (KIND == 1) ivb[k] = ld_cached(at(image, (uint32_t)(zb0 + k - J.nb) * (uint32_t)pitch + (uint32_t)x));
  }
  if (kGen && tphys) {
#pragma unroll
    for (int k = 0; k < RB; ++k) {  // image, and the stored ring value of level m - 1
      const int pzc = min(max(zb0 + k - J.nb, 0), J.nz - 1);
      ivb[k] = ld_cached(at(image, (uint32_t)pzc * (uint32_t)pitch + xph));
      const int slot = ring_slot(pzc, (int)xph - J.nb, J.nz, J.nx);
      ringb[k] = slot >= 0;
      svb[k] = ld_cached(gp(J.ring) + (int64_t)(m - 1) * J.ring_len + max(slot, 0));
    }
  }
  const float gxv = (!kGen || xin) ? gx[xcl] : 0.0f;
  const float wa = kGen ? gp(J.wavelet)[m + 1] * J.inv_cell : 0.0f;  // source term of S^m
  const float wb = kGen ? gp(J.wavelet)[m] * J.inv_cell : 0.0f;      // source term of S^{m-1}
  const float kfac = J.kfac;
  sa.store(sm.a);
  if (kSrc && tphys) sb.store(sm.b);

  // receiver data of levels m and m - 1, summed into zeroed middle-region
  // arrays as a one-step launch sums them
  const bool has_inj = kGen && tl.rec_count > 0;
  float inja[RA], injb[RB];
#pragma unroll
  for (int k = 0; k < RA; ++k) inja[k] = 0.0f;
#pragma unroll
  for (int k = 0; k < RB; ++k) injb[k] = 0.0f;
  if (has_inj) {
    for (int i = threadIdx.x; i < (TZ + 2 * kHalo) * kTileX; i += kThreads) {
      sm.ma[i] = 0.0f;
      sm.mb[i] = 0.0f;
    }
    __syncthreads();
    const RTM_GLOBAL float* da = gp(J.data) + (int64_t)m * J.nrec;
    const RTM_GLOBAL float* db = gp(J.data) + (int64_t)(m - 1) * J.nrec;
    for (int i = threadIdx.x; i < tl.rec_count; i += kThreads) {
      const int2 e = recs2[tl.rec_begin + i];
      atomicAdd(&sm.ma[e.x], da[e.y]);
      atomicAdd(&sm.mb[e.x], db[e.y]);
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < RA; ++k) inja[k] = sm.ma[(w * RA + k) * kTileX + lane];
#pragma unroll
    for (int k = 0; k < RB; ++k) injb[k] = sm.mb[(w * RB + k + kHalo) * kTileX + lane];
  }
  __syncthreads();

  const float c0 = J.c0;
  const float cz[4] = {J.cz[0], J.cz[1], J.cz[2], J.cz[3]};
  const float cx[4] = {J.cx[0], J.cx[1], J.cx[2], J.cx[3]};

  // ---- first step: R^m and S^m on the middle region ----
  {
    float zr[RA + 8], zs[RA + 8];
#pragma unroll
    for (int j = 0; j < RA + 8; ++j) zr[j] = sm.a[(w * RA + j) * kLdsW + lane + kHalo];
    if (kSrc && tphys) {
#pragma unroll
      for (int j = 0; j < RA + 8; ++j) zs[j] = sm.b[(w * RA + j) * kLdsW + lane + kHalo];
    }
#pragma clang loop unroll(full)
    for (int k = 0; k < RA; ++k) {
      const int r = w * RA + k;
      const int z = za0 + k;
      float lap = lap8<RA>(sm.a, r + kHalo, lane + kHalo, zr, k, c0, cz, cx);
      if (has_inj) lap += inja[k];
      const float G = gza[k] * gxv;
      float rv = leapfrog(G, cva[k], lap, zr[k + 4], pva[k]);
      if (kGen) rv = (xin && z >= 0 && z < J.nzp) ? rv : 0.0f;
      sm.ma[r * kTileX + lane] = rv;
      float sv = 0.0f;
      const int pz = z - J.nb;
      const bool phys = KIND == 1 || (kGen && tphys && colphys && pz >= 0 && pz < J.nz);
      if (kSrc && tphys) {
        if (ringa[k]) {
          sv = sva[k];
        } else {
          float ls = lap8<RA>(sm.b, r + kHalo, lane + kHalo, zs, k, c0, cz, cx);
          if (kGen && z == J.src_z && x == J.src_x) ls = add_unfused(ls, wa);
          sv = fmaf(cva[k], ls, 2.0f * zs[k + 4]) - sva[k];
        }
        if (kGen) sv = phys ? sv : 0.0f;
        sm.mb[r * kTileX + lane] = sv;
      }
      if (r >= kHalo && r < TZ + kHalo && (!kGen || z < J.nzp) && xout) {  // a node of the output tile
        const uint32_t off = (uint32_t)z * (uint32_t)pitch + (uint32_t)x;
        st_cached(at(r0, off), rv);
        if (kSrc && phys) st_cached(at(s0, off), sv);
      }
    }
  }
  __syncthreads();

  // ---- second step: R^{m-1} and S^{m-1} on the output tile, imaging ----
  {
    float zr[RB + 8], zs[RB + 8];
#pragma unroll
    for (int j = 0; j < RB + 8; ++j) zr[j] = sm.ma[(w * RB + j) * kTileX + lane];
    if (kSrc && tphys) {
#pragma unroll
      for (int j = 0; j < RB + 8; ++j) zs[j] = sm.mb[(w * RB + j) * kTileX + lane];
    }
#pragma clang loop unroll(full)
    for (int k = 0; k < RB; ++k) {
      const int z = zb0 + k;
      float lap = lap8<RB, kTileX>(sm.ma, w * RB + k + kHalo, lane, zr, k, c0, cz, cx);
      if (has_inj) lap += injb[k];
      const float G = gzb[k] * gxv;
      const int lrow = (w * RB + k + 2 * kHalo) * kLdsW + lane + kHalo;  // centre in the staged tiles
      const float rc = sm.a[lrow];  // R^{m+1}
      if (xout && (!kGen || z < J.nzp)) {
        const uint32_t off = (uint32_t)z * (uint32_t)pitch + (uint32_t)x;
        st_cached(at(rn, off), leapfrog(G, cvb[k], lap, zr[k + 4], rc));
        const int pz = z - J.nb;
        const bool phys = KIND == 1 || (kGen && tphys && colphys && pz >= 0 && pz < J.nz);
        if (kSrc && phys) {
          float sv;
          if (ringb[k]) {
            sv = svb[k];
          } else {
            float ls = lap8<RB, kTileX>(sm.mb, w * RB + k + kHalo, lane, zs, k, c0, cz, cx);
            if (kGen && z == J.src_z && x == J.src_x) ls = add_unfused(ls, wb);
            sv = fmaf(cvb[k], ls, 2.0f * zs[k + 4]) - sm.b[lrow];
          }
          st_cached(at(sn, off), sv);
          const float im = fmaf(kfac * zs[k + 4], rc, ivb[k]);  // level m
          st_cached(at(image, (uint32_t)pz * (uint32_t)pitch + (uint32_t)x), fmaf(kfac * sv, zr[k + 4], im));
        }
      }
    }
  }
}

// One two-step backward tile of a store-mode job: R^m on the middle region,
// R^{m-1} on the output tile, and the imaging terms of levels m and m - 1
// (those on the snapshot stride) with the stored source wavefield, in level
// order, as two one-step launches apply them.
template <int TZ, class Smem>
__device__ __forceinline__ void backward2_store_body(const DevJob& J, const Tile& tl, const int2* __restrict__ recs2,
                                                     int m, Smem& sm) {
  constexpr int RA = (TZ + 2 * kHalo) / 4;
  constexpr int RB = TZ / 4;
  const int lane = threadIdx.x & 63;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // wavefront-uniform
  const int pitch = J.pitch;
  const RTM_GLOBAL float* __restrict__ r1 = gp(J.r[(m + 1) & 3]);  // R^{m+1}
  const RTM_GLOBAL float* __restrict__ r2 = gp(J.r[(m + 2) & 3]);  // R^{m+2}
  RTM_GLOBAL float* __restrict__ r0 = gp(J.r[m & 3]);              // R^m
  RTM_GLOBAL float* __restrict__ rn = gp(J.r[(m + 3) & 3]);        // R^{m-1}
  RTM_GLOBAL float* __restrict__ image = gp(J.image);
  const RTM_GLOBAL float* __restrict__ cc = gp(J.c);
  const RTM_GLOBAL float* __restrict__ gz = gp(J.gz);
  const RTM_GLOBAL float* __restrict__ gx = gp(J.gx);
  const int x = tl.x0 - kHalo + lane;
  const int za0 = tl.z0 - kHalo + w * RA;
  const int zb0 = tl.z0 + w * RB;
  const bool xin = x >= 0 && x < J.nxp;
  const bool xout = lane >= kHalo && lane < kHalo + kTileX2 && x < J.nxp;
  const uint32_t xcl = (uint32_t)min(max(x, 0), J.nxp - 1);
  const int px = x - J.nb;
  const bool colphys = px >= 0 && px < J.nx;
  const int xph = min(max(x, J.nb), J.nb + J.nx - 1);  // column clamped into the window
  const int stride = J.snap_stride;
  const bool tphys = tl.z0 - J.nb < J.nz && tl.z0 + TZ - J.nb > 0 && tl.x0 - J.nb < J.nx &&
                     tl.x0 + kTileX2 - J.nb > 0;  // the output tile reaches the window
  const bool img0 = tphys && (m % stride) == 0 && m <= J.nt - 2;              // level m imaged
  const bool img1 = tphys && ((m - 1) % stride) == 0 && m - 1 <= J.nt - 2;    // level m - 1 imaged

  // ---- every global load first ----
  TileStageW<TZ + 4 * kHalo> sa;
  sa.load(r1, pitch, tl.z0 - 2 * kHalo, tl.x0 - 2 * kHalo);
  float cva[RA], pva[RA], gza[RA];
#pragma unroll
  for (int k = 0; k < RA; ++k) {
    const int zc = min(max(za0 + k, 0), J.nzp - 1);
    const uint32_t off = (uint32_t)zc * (uint32_t)pitch + xcl;
    cva[k] = ld_medium(at(cc, off));
    pva[k] = ld_cached(at(r2, off));
    gza[k] = gz[zc];
  }
  float dsc0 = 1.0f, dsc1 = 1.0f;
  if (img0 && J.snap_dtype != 0)  // exact: powers of two
    dsc0 = 1.0f / snap_scale_from_max(wave_max(__uint_as_float(gp(J.maxbits)[(int64_t)m * kMaxSlots + lane])));
  if (img1 && J.snap_dtype != 0)
    dsc1 = 1.0f / snap_scale_from_max(wave_max(__uint_as_float(gp(J.maxbits)[(int64_t)(m - 1) * kMaxSlots + lane])));
  float cvb[RB], gzb[RB], ivb[RB], s0b[RB], s1b[RB];
#pragma unroll
  for (int k = 0; k < RB; ++k) {
    const int zc = min(zb0 + k, J.nzp - 1);
    cvb[k] = ld_medium(at(cc, (uint32_t)zc * (uint32_t)pitch + xcl));
    gzb[k] = gz[zc];
    ivb[k] = 0.0f;
    s0b[k] = 0.0f;
    s1b[k] = 0.0f;
  }
  if (img0 || img1) {
#pragma unroll
    for (int k = 0; k < RB; ++k) {  // image and snapshots, at addresses clamped into the window
      const int pzc = min(max(zb0 + k - J.nb, 0), J.nz - 1);
      ivb[k] = ld_cached(at(image, (uint32_t)pzc * (uint32_t)pitch + (uint32_t)xph));
      if (img0) s0b[k] = load_snap(J, m, pzc, xph, dsc0);
      if (img1) s1b[k] = load_snap(J, m - 1, pzc, xph, dsc1);
    }
  }
  const float gxv = xin ? gx[xcl] : 0.0f;
  const float kfac = J.kfac;
  sa.store(sm.a);

  // receiver data of levels m and m - 1, summed into zeroed middle-region
  // arrays as a one-step launch sums them
  const bool has_inj = tl.rec_count > 0;
  float inja[RA], injb[RB];
#pragma unroll
  for (int k = 0; k < RA; ++k) inja[k] = 0.0f;
#pragma unroll
  for (int k = 0; k < RB; ++k) injb[k] = 0.0f;
  if (has_inj) {
    for (int i = threadIdx.x; i < (TZ + 2 * kHalo) * kTileX; i += kThreads) {
      sm.ma[i] = 0.0f;
      sm.mb[i] = 0.0f;
    }
    __syncthreads();
    const RTM_GLOBAL float* da = gp(J.data) + (int64_t)m * J.nrec;
    const RTM_GLOBAL float* db = gp(J.data) + (int64_t)(m - 1) * J.nrec;
    for (int i = threadIdx.x; i < tl.rec_count; i += kThreads) {
      const int2 e = recs2[tl.rec_begin + i];
      atomicAdd(&sm.ma[e.x], da[e.y]);
      atomicAdd(&sm.mb[e.x], db[e.y]);
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < RA; ++k) inja[k] = sm.ma[(w * RA + k) * kTileX + lane];
#pragma unroll
    for (int k = 0; k < RB; ++k) injb[k] = sm.mb[(w * RB + k + kHalo) * kTileX + lane];
  }
  __syncthreads();

  const float c0 = J.c0;
  const float cz[4] = {J.cz[0], J.cz[1], J.cz[2], J.cz[3]};
  const float cx[4] = {J.cx[0], J.cx[1], J.cx[2], J.cx[3]};

  // ---- first step: R^m on the middle region ----
  {
    float zr[RA + 8];
#pragma unroll
    for (int j = 0; j < RA + 8; ++j) zr[j] = sm.a[(w * RA + j) * kLdsW + lane + kHalo];
#pragma clang loop unroll(full)
    for (int k = 0; k < RA; ++k) {
      const int r = w * RA + k;
      const int z = za0 + k;
      float lap = lap8<RA>(sm.a, r + kHalo, lane + kHalo, zr, k, c0, cz, cx);
      if (has_inj) lap += inja[k];
      float rv = leapfrog(gza[k] * gxv, cva[k], lap, zr[k + 4], pva[k]);
      rv = (xin && z >= 0 && z < J.nzp) ? rv : 0.0f;
      sm.ma[r * kTileX + lane] = rv;
      if (r >= kHalo && r < TZ + kHalo && z < J.nzp && xout)  // a node of the output tile
        st_cached(at(r0, (uint32_t)z * (uint32_t)pitch + (uint32_t)x), rv);
    }
  }
  __syncthreads();

  // ---- second step: R^{m-1} on the output tile, imaging ----
  {
    float zr[RB + 8];
#pragma unroll
    for (int j = 0; j < RB + 8; ++j) zr[j] = sm.ma[(w * RB + j) * kTileX + lane];
#pragma clang loop unroll(full)
    for (int k = 0; k < RB; ++k) {
      const int z = zb0 + k;
      float lap = lap8<RB, kTileX>(sm.ma, w * RB + k + kHalo, lane, zr, k, c0, cz, cx);
      if (has_inj) lap += injb[k];
      const float rc = sm.a[(w * RB + k + 2 * kHalo) * kLdsW + lane + kHalo];  // R^{m+1}
      if (xout && z < J.nzp) {
        const uint32_t off = (uint32_t)z * (uint32_t)pitch + (uint32_t)x;
        st_cached(at(rn, off), leapfrog(gzb[k] * gxv, cvb[k], lap, zr[k + 4], rc));
        const int pz = z - J.nb;
        if ((img0 || img1) && colphys && pz >= 0 && pz < J.nz) {
          float im = ivb[k];
          if (img0) im = fmaf(kfac * s0b[k], rc, im);         // level m:     S^m R^{m+1}
          if (img1) im = fmaf(kfac * s1b[k], zr[k + 4], im);  // level m - 1: S^{m-1} R^m
          st_cached(at(image, (uint32_t)pz * (uint32_t)pitch + (uint32_t)x), im);
        }
      }
    }
  }
}

// One two-step Born tile: the background u0 and the scattered field du
// from level n to n + 2, each step the Born step of born_tile (same
// operations on the same operands), and the receiver samples of du^{n+1}
// and du^{n+2} for the receivers on the output tile (a receiver in the
// middle region only is sampled by the tile whose output tile holds it).
template <int TZ, class Smem>
__device__ __forceinline__ void born2_body(const DevJob& J, const Tile& tl, const int2* __restrict__ recs2, int n,
                                           Smem& sm) {
  constexpr int RA = (TZ + 2 * kHalo) / 4;
  constexpr int RB = TZ / 4;
  const int lane = threadIdx.x & 63;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // wavefront-uniform
  const int pitch = J.pitch;
  const RTM_GLOBAL float* __restrict__ u0 = gp(J.f[n & 3]);        // u0^n
  const RTM_GLOBAL float* __restrict__ um = gp(J.f[(n + 3) & 3]);  // u0^{n-1}
  RTM_GLOBAL float* __restrict__ u1 = gp(J.f[(n + 1) & 3]);        // u0^{n+1}
  RTM_GLOBAL float* __restrict__ u2 = gp(J.f[(n + 2) & 3]);        // u0^{n+2}
  const RTM_GLOBAL float* __restrict__ d0 = gp(J.r[n & 3]);        // du^n
  const RTM_GLOBAL float* __restrict__ dm = gp(J.r[(n + 3) & 3]);  // du^{n-1}
  RTM_GLOBAL float* __restrict__ d1 = gp(J.r[(n + 1) & 3]);        // du^{n+1}
  RTM_GLOBAL float* __restrict__ d2 = gp(J.r[(n + 2) & 3]);        // du^{n+2}
  const RTM_GLOBAL float* __restrict__ mp = gp(J.image);           // m, physical window
  const RTM_GLOBAL float* __restrict__ cc = gp(J.c);
  const RTM_GLOBAL float* __restrict__ gz = gp(J.gz);
  const RTM_GLOBAL float* __restrict__ gx = gp(J.gx);
  const int x = tl.x0 - kHalo + lane;
  const int za0 = tl.z0 - kHalo + w * RA;
  const int zb0 = tl.z0 + w * RB;
  const bool xin = x >= 0 && x < J.nxp;
  const bool xout = lane >= kHalo && lane < kHalo + kTileX2 && x < J.nxp;
  const uint32_t xcl = (uint32_t)min(max(x, 0), J.nxp - 1);
  const int px = x - J.nb;
  const bool colphys = px >= 0 && px < J.nx;
  const uint32_t xph = (uint32_t)min(max(x, J.nb), J.nb + J.nx - 1);  // column clamped into the window

  // ---- every global load first ----
  TileStageW<TZ + 4 * kHalo> sa, sb;
  sa.load(u0, pitch, tl.z0 - 2 * kHalo, tl.x0 - 2 * kHalo);
  sb.load(d0, pitch, tl.z0 - 2 * kHalo, tl.x0 - 2 * kHalo);
  float cva[RA], pva[RA], qva[RA], gza[RA], mva[RA];
#pragma unroll
  for (int k = 0; k < RA; ++k) {
    const int zc = min(max(za0 + k, 0), J.nzp - 1);
    const uint32_t off = (uint32_t)zc * (uint32_t)pitch + xcl;
    cva[k] = ld_medium(at(cc, off));
    pva[k] = ld_cached(at(um, off));
    qva[k] = ld_cached(at(dm, off));
    gza[k] = gz[zc];
    const int pzc = min(max(za0 + k - J.nb, 0), J.nz - 1);
    mva[k] = ld_medium(at(mp, (uint32_t)pzc * (uint32_t)pitch + xph));
  }
  float cvb[RB], gzb[RB], mvb[RB];
#pragma unroll
  for (int k = 0; k < RB; ++k) {
    const int zc = min(zb0 + k, J.nzp - 1);
    cvb[k] = ld_medium(at(cc, (uint32_t)zc * (uint32_t)pitch + xcl));
    gzb[k] = gz[zc];
    const int pzc = min(max(zb0 + k - J.nb, 0), J.nz - 1);
    mvb[k] = ld_medium(at(mp, (uint32_t)pzc * (uint32_t)pitch + xph));
  }
  const float gxv = xin ? gx[xcl] : 0.0f;
  const float w0 = gp(J.wavelet)[n] * J.inv_cell;
  const float w1 = gp(J.wavelet)[n + 1] * J.inv_cell;
  sa.store(sm.a);
  sb.store(sm.b);
  __syncthreads();

  const float c0 = J.c0;
  const float cz[4] = {J.cz[0], J.cz[1], J.cz[2], J.cz[3]};
  const float cx[4] = {J.cx[0], J.cx[1], J.cx[2], J.cx[3]};

  // ---- first step: u0^{n+1} and du^{n+1} on the middle region ----
  {
    float zu[RA + 8], zd[RA + 8];
#pragma unroll
    for (int j = 0; j < RA + 8; ++j) {
      zu[j] = sm.a[(w * RA + j) * kLdsW + lane + kHalo];
      zd[j] = sm.b[(w * RA + j) * kLdsW + lane + kHalo];
    }
#pragma clang loop unroll(full)
    for (int k = 0; k < RA; ++k) {
      const int r = w * RA + k;  // middle row (wavefront-uniform)
      const int z = za0 + k;
      const float G = gza[k] * gxv;
      const float u = zu[k + 4];
      float lu = lap8<RA>(sm.a, r + kHalo, lane + kHalo, zu, k, c0, cz, cx);
      if (z == J.src_z && x == J.src_x) lu = add_unfused(lu, w0);
      float un = leapfrog(G, cva[k], lu, u, pva[k]);
      float ld = lap8<RA>(sm.b, r + kHalo, lane + kHalo, zd, k, c0, cz, cx);
      const int pz = z - J.nb;
      if (colphys && pz >= 0 && pz < J.nz) ld = fmaf(mva[k], u, ld);
      float dn = leapfrog(G, cva[k], ld, zd[k + 4], qva[k]);
      const bool inside = xin && z >= 0 && z < J.nzp;
      un = inside ? un : 0.0f;
      dn = inside ? dn : 0.0f;
      sm.ma[r * kTileX + lane] = un;
      sm.mb[r * kTileX + lane] = dn;
      if (r >= kHalo && r < TZ + kHalo && z < J.nzp && xout) {  // a node of the output tile
        const uint32_t off = (uint32_t)z * (uint32_t)pitch + (uint32_t)x;
        st_cached(at(u1, off), un);
        st_cached(at(d1, off), dn);
      }
    }
  }
  __syncthreads();

  // ---- second step: u0^{n+2} and du^{n+2} on the output tile ----
  float dout[RB];
  {
    float zu[RB + 8], zd[RB + 8];
#pragma unroll
    for (int j = 0; j < RB + 8; ++j) {
      zu[j] = sm.ma[(w * RB + j) * kTileX + lane];
      zd[j] = sm.mb[(w * RB + j) * kTileX + lane];
    }
#pragma clang loop unroll(full)
    for (int k = 0; k < RB; ++k) {
      const int z = zb0 + k;
      dout[k] = 0.0f;
      if (xout && z < J.nzp) {
        const float G = gzb[k] * gxv;
        const int lrow = (w * RB + k + 2 * kHalo) * kLdsW + lane + kHalo;  // centre in the staged tiles
        const float u = zu[k + 4];
        float lu = lap8<RB, kTileX>(sm.ma, w * RB + k + kHalo, lane, zu, k, c0, cz, cx);
        if (z == J.src_z && x == J.src_x) lu = add_unfused(lu, w1);
        const uint32_t off = (uint32_t)z * (uint32_t)pitch + (uint32_t)x;
        st_cached(at(u2, off), leapfrog(G, cvb[k], lu, u, sm.a[lrow]));
        float ld = lap8<RB, kTileX>(sm.mb, w * RB + k + kHalo, lane, zd, k, c0, cz, cx);
        const int pz = z - J.nb;
        if (colphys && pz >= 0 && pz < J.nz) ld = fmaf(mvb[k], u, ld);
        const float dn = leapfrog(G, cvb[k], ld, zd[k + 4], sm.b[lrow]);
        st_cached(at(d2, off), dn);
        dout[k] = dn;
      }
    }
  }

  // ---- receiver samples of du^{n+1} (middle region array) and du^{n+2} ----
  if (tl.rec_count > 0 && J.traces != nullptr) {  // workgroup-uniform
    __syncthreads();  // every wavefront is done with sm.ma
#pragma unroll
    for (int k = 0; k < RB; ++k) sm.ma[(w * RB + k + kHalo) * kTileX + lane] = dout[k];
    __syncthreads();
    for (int i = threadIdx.x; i < tl.rec_count; i += kThreads) {
      const int2 e = recs2[tl.rec_begin + i];
      const int r = e.x / kTileX, c = e.x - r * kTileX;
      if (r >= kHalo && r < TZ + kHalo && c >= kHalo && c < kHalo + kTileX2) {
        gp(J.traces)[(int64_t)(n + 1) * J.nrec + e.y] = sm.mb[e.x];
        gp(J.traces)[(int64_t)(n + 2) * J.nrec + e.y] = sm.ma[e.x];
      }
    }
  }
}

template <int TZ, class Smem>
__device__ __forceinline__ void backward2_tile(const DevJob& J, const Tile& tl, const int2* recs2, int m,
                                               Smem& sm) {
  const int z0 = tl.z0, x0 = tl.x0;
  // middle region [mz0, mz1) x [mx0, mx1), padded coordinates
  const int mz0 = z0 - kHalo, mz1 = z0 + TZ + kHalo, mx0 = x0 - kHalo, mx1 = x0 + kTileX2 + kHalo;
  const bool src = J.src_z >= mz0 && J.src_z < mz1 && J.src_x >= mx0 && J.src_x < mx1;
  const bool quiet = !src && tl.rec_count == 0;
  const int nb = J.nb;
  const bool interior = mz0 >= nb + 4 && mz1 <= nb + J.nz - 4 && mx0 >= nb + 4 && mx1 <= nb + J.nx - 4;
  const bool inside = mz0 >= 0 && mz1 <= J.nzp && mx0 >= 0 && mx1 <= J.nxp;
  const bool sponge = inside && (mz1 <= nb || mz0 >= nb + J.nz || mx1 <= nb || mx0 >= nb + J.nx);
  if (quiet && interior)
    backward2_body<TZ, 1>(J, tl, recs2, m, sm);
  else if (quiet && sponge)
    backward2_body<TZ, 2>(J, tl, recs2, m, sm);
  else
    backward2_body<TZ, 0>(J, tl, recs2, m, sm);
}

// kStore: a launch over store-mode jobs; else over reconstruct-mode jobs
// (the two take separate instances, so neither carries the other's code).
template <int TZ, int PH, bool kStore>
__global__ __launch_bounds__(kThreads) void k_step2(const DevJob* __restrict__ jobs,
                                                     const Tile* __restrict__ tiles,
                                                     const int2* __restrict__ recs2,
                                                     const StepCtl* __restrict__ ctl, int ntiles_arg,
                                                     int use_ctl_tick, int tick_off) {
  __shared__ Step2Smem<TZ, (PH & (kPhBwd | kPhBorn)) != 0, !kStore> sm;
  // Steps tick and tick + 1 of every job; same XCD-aware mapping as k_step,
  // except that every other launch walks each XCD's run of tiles backwards:
  // it then starts on the tiles the previous launch wrote last, whose data
  // are still in the caches (measured: 2 % shorter launches).  The grid may
  // be sized for more tiles than the table holds (graph replays read the
  // count from the control block).
  int ntiles = ntiles_arg;
  if (ntiles_arg < 0) {
    ntiles = (PH & kPhFwd) ? ctl->ntiles_fw : ctl->ntiles_bw;
    tiles += (PH & kPhFwd) ? ctl->base_fw : ctl->base_bw;
  }
  const int tick = (use_ctl_tick ? ctl->tick : 0) + tick_off;
  const int per = (ntiles + 7) >> 3;
  const int local0 = (int)(blockIdx.x >> 3);
  if (local0 >= per) return;  // before the reversal, which would turn it negative
  const int local = ((tick >> 1) & 1) ? per - 1 - local0 : local0;
  const int t = (blockIdx.x & 7) * per + local;
  if (t >= ntiles) return;
  const Tile tl = tiles[t];
  const DevJob& J = jobs[tl.job];
  const int s = tick - J.start_tick;
  if constexpr (PH == kPhBorn) {  // Born pairs: steps s, s + 1 (s even) of the job's nsteps
    if (J.mode == kModeBorn && s >= 0 && (s & 1) == 0 && s + 1 < J.nsteps) born2_body<TZ>(J, tl, recs2, s, sm);
    return;
  }
  if (J.mode != (kStore ? kModeStore : kModeRecon) || J.illum != nullptr ||
      !two_step_pair(s, J.nt, J.nsteps, J.mode))
    return;
  const int nf = J.nt - 1;  // forward steps
  if (s + 1 < nf) {
    if (PH & kPhFwd) forward2_tile<TZ, kStore>(J, tl, s, sm);
  } else if (PH & kPhBwd) {
    const int m = J.nt - 1 - (s - nf);  // levels m and m - 1
    if (kStore)
      backward2_store_body<TZ>(J, tl, recs2, m, sm);
    else
      backward2_tile<TZ>(J, tl, recs2, m, sm);
  }
}

template <int TZ, int PH>
__global__ __launch_bounds__(kThreads) void k_step(const DevJob* __restrict__ jobs,
                                                    const Tile* __restrict__ tiles,
                                                    const StepCtl* __restrict__ ctl, int ntiles_arg,
                                                    int use_ctl_tick, int tick_off, int skip_pairs) {
  __shared__ StepSmem<TZ, (PH & (kPhBwd | kPhBorn)) != 0> sm;
  // Global step: a base read from the control block (advanced by k_advance
  // after every group of graph-replayed launches) plus this launch's offset.
  int ntiles = ntiles_arg;
  if (ntiles_arg < 0) {
    ntiles = ctl->ntiles;
    tiles += ctl->base;
  }
  const int tick = (use_ctl_tick ? ctl->tick : 0) + tick_off;
  // XCD-aware mapping: workgroups are dealt round-robin to the 8 XCDs, so
  // give XCD k (blockIdx % 8) a contiguous run of tiles; neighbouring tiles,
  // and the halo rows they share, then meet in the same L2.  The grid may be
  // sized for more tiles than are active (graph replays).
  const int per = (ntiles + 7) >> 3;
  const int local = (int)(blockIdx.x >> 3);
  const int t = (blockIdx.x & 7) * per + local;
  if (local >= per || t >= ntiles) return;
  const Tile tl = tiles[t];
  const DevJob& J = jobs[tl.job];
  const int s = tick - J.start_tick;
  if (s < 0 || s >= J.nsteps) return;
  // serving engine: a job marked two_step starts at an even tick, and the
  // steps s & ~1, (s & ~1) + 1 that a two-step launch takes are skipped here
  if (skip_pairs && J.two_step && two_step_pair(s & ~1, J.nt, J.nsteps, J.mode)) return;
  if (J.mode == kModeBorn) {
    if (PH & kPhBorn) born_tile<TZ>(J, tl, s, sm);
    return;
  }
  const int nf = (J.mode == kModeModel) ? J.nsteps : J.nt - 1;  // forward steps
  if (s < nf) {
    if (PH & kPhFwd) forward_tile<TZ>(J, tl, s, sm);
  } else {
    if (PH & kPhBwd) backward_tile<TZ>(J, tl, J.nt - 1 - (s - nf), sm);
  }
}

__global__ void k_advance(StepCtl* ctl, int k) { ctl->tick += k; }

hipError_t launch_advance(StepCtl* ctl, int k, hipStream_t s) {
  hipLaunchKernelGGL(k_advance, dim3(1), dim3(1), 0, s, ctl, k);
  return hipGetLastError();
}

__global__ void k_set_ctl(StepCtl* ctl, StepCtl v) { *ctl = v; }

hipError_t launch_set_ctl(StepCtl* ctl, StepCtl v, hipStream_t s) {
  hipLaunchKernelGGL(k_set_ctl, dim3(1), dim3(1), 0, s, ctl, v);
  return hipGetLastError();
}

template <int TZ>
static hipError_t launch_step_tz(int phases, const DevJob* jobs, const Tile* tiles, int ntiles,
                                 int grid_tiles, const StepCtl* ctl, int use_ctl_tick, int tick_off,
                                 int skip_pairs, hipStream_t s) {
  const int per = (grid_tiles + 7) / 8;
  dim3 grid(8 * per), block(kThreads);
  if (phases == kPhFwd)
    hipLaunchKernelGGL((k_step<TZ, kPhFwd>), grid, block, 0, s, jobs, tiles, ctl, ntiles, use_ctl_tick, tick_off,
                       skip_pairs);
  else if (phases == kPhBwd)
    hipLaunchKernelGGL((k_step<TZ, kPhBwd>), grid, block, 0, s, jobs, tiles, ctl, ntiles, use_ctl_tick, tick_off,
                       skip_pairs);
  else if (phases == kPhBorn)
    hipLaunchKernelGGL((k_step<TZ, kPhBorn>), grid, block, 0, s, jobs, tiles, ctl, ntiles, use_ctl_tick, tick_off,
                       skip_pairs);
  else
    hipLaunchKernelGGL((k_step<TZ, kPhAny>), grid, block, 0, s, jobs, tiles, ctl, ntiles, use_ctl_tick, tick_off,
                       skip_pairs);
  return hipGetLastError();
}

hipError_t launch_step2(int tz, int phases, int store, const DevJob* jobs, const Tile* tiles, const int2* recs2,
                        int ntiles, int grid_tiles, const StepCtl* ctl, int use_ctl_tick, int tick_off,
                        hipStream_t s) {
  if (grid_tiles <= 0) return hipSuccess;
  const int per = (grid_tiles + 7) / 8;
  dim3 grid(8 * per), block(kThreads);
#define RTM_STEP2(T, P, M) \
  hipLaunchKernelGGL((k_step2<T, P, M>), grid, block, 0, s, jobs, tiles, recs2, ctl, ntiles, use_ctl_tick, tick_off)
#define RTM_STEP2_TZ(T)                                       \
  if (tz == T) {                                              \
    if (phases == kPhFwd && !store) RTM_STEP2(T, kPhFwd, false); \
    else if (phases == kPhBwd && !store) RTM_STEP2(T, kPhBwd, false); \
    else if (phases == kPhFwd) RTM_STEP2(T, kPhFwd, true);    \
    else if (phases == kPhBwd) RTM_STEP2(T, kPhBwd, true);    \
    else if (phases == kPhBorn && !store) RTM_STEP2(T, kPhBorn, false); \
    else return hipErrorInvalidValue;                         \
    return hipGetLastError();                                 \
  }
  RTM_STEP2_TZ(24)
  RTM_STEP2_TZ(16)
  RTM_STEP2_TZ(32)
#undef RTM_STEP2_TZ
#undef RTM_STEP2
  return hipErrorInvalidValue;
}

hipError_t launch_step(int tz, int phases, const DevJob* jobs, const Tile* tiles, int ntiles,
                       int grid_tiles, const StepCtl* ctl, int use_ctl_tick, int tick_off,
                       hipStream_t s, int skip_pairs) {
  switch (tz) {
    case 16:
      return launch_step_tz<16>(phases, jobs, tiles, ntiles, grid_tiles, ctl, use_ctl_tick, tick_off, skip_pairs, s);
    case 32:
      return launch_step_tz<32>(phases, jobs, tiles, ntiles, grid_tiles, ctl, use_ctl_tick, tick_off, skip_pairs, s);
    case 64:
      return launch_step_tz<64>(phases, jobs, tiles, ntiles, grid_tiles, ctl, use_ctl_tick, tick_off, skip_pairs, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace rtm
