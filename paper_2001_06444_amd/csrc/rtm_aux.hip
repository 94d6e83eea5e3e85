// rtm_aux.hip -- per-job and per-query kernels around the time-step kernel:
// model preparation and the CFL maximum, stacking over shots, the non-finite
// check, FP64 running statistics (Sec. 2.3 / Stage 3), the Stage-3 maps
// (Eq. 6, Eq. 7) and the post-stack Laplacian filter (Sec. 3).
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include <algorithm>

#include "rtm_device.h"
#include "rtm_internal.h"

namespace rtm {

// ---------------------------------------------------------------------------
// Job set-up: c = v^2 dt^2 on the padded window (velocity edge-replicated into
// the sponge) and the sponge profiles g(d) = exp(-(a d)^2).
// ---------------------------------------------------------------------------
__global__ void k_prep(const float* __restrict__ vel, int model_nx, int ix0, int nz, int nx, int nb,
                       int nzp, int nxp, int pitch, float dt2, float a, float* __restrict__ c,
                       float* __restrict__ gz, float* __restrict__ gx) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  const int z = blockIdx.y;
  if (x >= nxp || z >= nzp) return;
  int vz = min(max(z - nb, 0), nz - 1);
  int vx = min(max(x - nb, 0), nx - 1);
  float v = vel[(int64_t)vz * model_nx + ix0 + vx];
  c[(int64_t)z * pitch + x] = v * v * dt2;
  if (z == 0) {
    int d = x < nb ? nb - x : (x >= nb + nx ? x - (nb + nx - 1) : 0);
    float ad = a * (float)d;
    gx[x] = expf(-ad * ad);
  }
  if (x == 0) {
    int d = z < nb ? nb - z : (z >= nb + nz ? z - (nb + nz - 1) : 0);
    float ad = a * (float)d;
    gz[z] = expf(-ad * ad);
  }
}

hipError_t launch_prep(const float* vel, int model_nx, int ix0, const DevJob* hj, float* c,
                       float* gz, float* gx, float dt, float sponge_a, hipStream_t s) {
  dim3 block(256), grid((hj->nxp + 255) / 256, hj->nzp);
  float a = sponge_a > 0.0f ? sponge_a : (hj->nb > 0 ? 0.3f / (float)hj->nb : 0.0f);
  hipLaunchKernelGGL(k_prep, grid, block, 0, s, vel, model_nx, ix0, hj->nz, hj->nx, hj->nb,
                     hj->nzp, hj->nxp, hj->pitch, dt * dt, a, c, gz, gx);
  return hipGetLastError();
}

// max |v| over a window (float bits; the output must be zeroed first)
__global__ void k_vmax(const float* __restrict__ vel, int nz, int model_nx, int ix0, int width,
                       uint32_t* out) {
  __shared__ float red[4];
  float m = 0.0f;
  bool nan_seen = false;  // fmaxf drops NaN, so it is tracked on the side
  const int64_t n = (int64_t)nz * width;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    int64_t z = i / width, x = i - z * width;
    float v = fabsf(vel[z * model_nx + ix0 + x]);
    nan_seen |= (v != v);
    m = fmaxf(m, v);
  }
  wg_atomic_max(m, out, red);
  // NaN bits (0x7fc00000) sort above +inf under the unsigned max
  if (__any(nan_seen) && (threadIdx.x & 63) == 0) atomicMax(out, 0x7fc00000u);
}

hipError_t launch_vmax(const float* vel, int nz, int model_nx, int ix0, int width, uint32_t* out,
                       hipStream_t s) {
  int64_t n = (int64_t)nz * width;
  int blocks = (int)std::min<int64_t>((n + 255) / 256, 1024);
  hipLaunchKernelGGL(k_vmax, dim3(blocks), dim3(256), 0, s, vel, nz, model_nx, ix0, width, out);
  return hipGetLastError();
}

// Stack: dst[z][ix0 + x] += img[z][x]
__global__ void k_stack(float* __restrict__ dst, int dst_nx, int ix0, const float* __restrict__ img,
                        int img_pitch, int nz, int width) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  const int z = blockIdx.y;
  if (x < width && z < nz) dst[(int64_t)z * dst_nx + ix0 + x] += img[(int64_t)z * img_pitch + x];
}

hipError_t launch_stack(float* dst, int dst_nx, int ix0, const float* img, int img_pitch, int nz,
                        int width, hipStream_t s) {
  hipLaunchKernelGGL(k_stack, dim3((width + 255) / 256, nz), dim3(256), 0, s, dst, dst_nx, ix0, img,
                     img_pitch, nz, width);
  return hipGetLastError();
}

// Any non-finite value in an [nz][width] image (row pitch `pitch`) sets bit 0 of *flag.
__global__ void k_nonfinite(const float* __restrict__ img, int pitch, int nz, int width, uint32_t* flag) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  const int z = blockIdx.y;
  const bool bad = x < width && z < nz && !isfinite(img[(int64_t)z * pitch + x]);
  if (__any(bad) && (threadIdx.x & 63) == 0) atomicOr(flag, 1u);
}

hipError_t launch_nonfinite(const float* img, int pitch, int nz, int width, uint32_t* flag, hipStream_t s) {
  hipLaunchKernelGGL(k_nonfinite, dim3((width + 255) / 256, nz), dim3(256), 0, s, img, pitch, nz, width, flag);
  return hipGetLastError();
}

// Physical region of a padded field -> dense [nz][nx]
__global__ void k_copy_phys(float* __restrict__ dst, const float* __restrict__ fld, int nz, int nx,
                            int nb, int pitch) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  const int z = blockIdx.y;
  if (x < nx && z < nz) dst[(int64_t)z * nx + x] = fld[(int64_t)(z + nb) * pitch + nb + x];
}

hipError_t launch_copy_phys(float* dst, const float* fld, int nz, int nx, int nb, int pitch,
                            hipStream_t s) {
  hipLaunchKernelGGL(k_copy_phys, dim3((nx + 255) / 256, nz), dim3(256), 0, s, dst, fld, nz, nx, nb,
                     pitch);
  return hipGetLastError();
}

__global__ void k_fill_u32(uint32_t* p, uint32_t v, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

hipError_t launch_fill_u32(uint32_t* p, uint32_t v, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  int blocks = (int)std::min<int64_t>((n + 255) / 256, 4096);
  hipLaunchKernelGGL(k_fill_u32, dim3(blocks), dim3(256), 0, s, p, v, n);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Ensemble statistics (Sec. 2.3 / Stage 3): per-pixel FP64 Welford update
//   n += 1; d = x - mean; mean += d / n; M2 += d (x - mean)
// over the window [ix0, ix0 + width) of an [nz][nx_model] state.
// ---------------------------------------------------------------------------
__global__ void k_welford(double* __restrict__ mean, double* __restrict__ m2,
                          int32_t* __restrict__ count, int nx_model, const float* __restrict__ img,
                          int img_pitch, int nz, int width, int ix0) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  const int z = blockIdx.y;
  if (x >= width || z >= nz) return;
  const int64_t o = (int64_t)z * nx_model + ix0 + x;
  const double v = (double)img[(int64_t)z * img_pitch + x];
  const int32_t n = count[o] + 1;
  const double d = v - mean[o];
  const double mu = mean[o] + d / (double)n;
  m2[o] += d * (v - mu);
  mean[o] = mu;
  count[o] = n;
}

hipError_t launch_welford(double* mean, double* m2, int32_t* count, int nx_model, const float* img,
                          int img_pitch, int nz, int width, int ix0, hipStream_t s) {
  hipLaunchKernelGGL(k_welford, dim3((width + 255) / 256, nz), dim3(256), 0, s, mean, m2, count,
                     nx_model, img, img_pitch, nz, width, ix0);
  return hipGetLastError();
}

__global__ void k_stats_out(const double* __restrict__ mean, const double* __restrict__ m2,
                            const int32_t* __restrict__ count, int64_t n, double* mean_out,
                            double* std_out, int32_t* count_out) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    int32_t c = count[i];
    if (mean_out) mean_out[i] = c > 0 ? mean[i] : 0.0;
    if (std_out) std_out[i] = c > 1 ? sqrt(m2[i] / (double)(c - 1)) : 0.0;
    if (count_out) count_out[i] = c;
  }
}

hipError_t launch_stats_out(const double* mean, const double* m2, const int32_t* count, int64_t n,
                            double* mean_out, double* std_out, int32_t* count_out, hipStream_t s) {
  int blocks = (int)std::min<int64_t>((n + 255) / 256, 4096);
  hipLaunchKernelGGL(k_stats_out, dim3(blocks), dim3(256), 0, s, mean, m2, count, n, mean_out,
                     std_out, count_out);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Stage-3 maps.  The reductions they need (extremes of std for the
// confidence index, the largest illumination for the normalised image) run
// in two stages: each workgroup of a grid-stride pass writes its partial
// result and one workgroup folds the partials, so no address is hit by
// more than one write (with one atomic per wavefront on a single address,
// the 597k-pixel confidence map spent 95 us in its reduction).
// The streaming passes take four pixels per thread and step, as 16-byte
// loads and stores with two steps' loads in flight, when every array the
// pass touches is 16-byte aligned (kVec); otherwise, and for the pixels
// past the last whole group of four, one pixel per step.  The second pass
// of a map walks the arrays from their end, so it starts on the data the
// first pass read last, which the memory-side cache still holds (measured
// on 256 images side by side: the normalised image's second pass 10 %
// shorter than walking forward; the confidence map's unchanged).  The
// normalised image is written with non-temporal stores (3 % shorter; the
// confidence map's double stores were 20 % longer that way).
// ---------------------------------------------------------------------------
__device__ __forceinline__ void block_minmax(double& lo, double& hi, double* red) {
  for (int o = 32; o > 0; o >>= 1) {
    lo = fmin(lo, __shfl_xor(lo, o, 64));
    hi = fmax(hi, __shfl_xor(hi, o, 64));
  }
  const int w = threadIdx.x >> 6, nw = blockDim.x >> 6;
  if ((threadIdx.x & 63) == 0) {
    red[w] = lo;
    red[nw + w] = hi;
  }
  __syncthreads();
  if (threadIdx.x == 0)
    for (int k = 1; k < nw; ++k) {
      lo = fmin(lo, red[k]);
      hi = fmax(hi, red[nw + k]);
    }
}

typedef float f4v __attribute__((ext_vector_type(4)));  // for the non-temporal 16-byte store

static inline bool aligned16(const void* p) { return ((uintptr_t)p & 15) == 0; }

// Workgroups of a streaming pass over `units` groups (or pixels), at most cap.
static inline int stream_blocks(int64_t units, int cap) {
  return (int)std::max<int64_t>(1, std::min<int64_t>((units + 255) / 256, cap));
}

// Extremes of std over the pixels with count >= min_count (all pixels
// without counts), one (min, max) pair per workgroup.  std >= 0, so a
// workgroup without such pixels leaves (inf, 0), which orders as empty.
// min and max are exact, so the grouping of the pixels leaves the result
// unchanged.
template <bool kVec>
__global__ __launch_bounds__(256) void k_minmax_part(const double* __restrict__ sd,
                                                     const int32_t* __restrict__ count, int n,
                                                     int min_count, double* __restrict__ part) {
  __shared__ double red[8];
  double lo = INFINITY, hi = 0.0;
  auto take = [&](double v, int32_t c) {
    if (c >= min_count) {
      lo = fmin(lo, v);
      hi = fmax(hi, v);
    }
  };
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const int64_t t0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t head = 0;  // pixels [0, head) go through the vector loop
  if (kVec) {
    const int64_t ng = n >> 2;
    const double2* __restrict__ s2 = reinterpret_cast<const double2*>(sd);
    const int4* __restrict__ c4 = reinterpret_cast<const int4*>(count);
    const int4 all = make_int4(min_count, min_count, min_count, min_count);
    auto take4 = [&](double2 a, double2 b, int4 c) {
      take(a.x, c.x);
      take(a.y, c.y);
      take(b.x, c.z);
      take(b.y, c.w);
    };
    int64_t g = t0;
    for (; g + stride < ng; g += 2 * stride) {
      const int64_t h = g + stride;
      const double2 a0 = s2[2 * g], a1 = s2[2 * g + 1], b0 = s2[2 * h], b1 = s2[2 * h + 1];
      const int4 ca = count ? c4[g] : all, cb = count ? c4[h] : all;
      take4(a0, a1, ca);
      take4(b0, b1, cb);
    }
    if (g < ng) take4(s2[2 * g], s2[2 * g + 1], count ? c4[g] : all);
    head = ng << 2;
  }
  for (int64_t i = head + t0; i < n; i += stride) take(sd[i], count ? count[i] : min_count);
  block_minmax(lo, hi, red);
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = lo;
    part[2 * blockIdx.x + 1] = hi;
  }
}

__global__ __launch_bounds__(256) void k_minmax_fold(const double* __restrict__ part, int nparts,
                                                     double* __restrict__ mm) {
  __shared__ double red[8];
  double lo = INFINITY, hi = 0.0;
  for (int b = threadIdx.x; b < nparts; b += blockDim.x) {
    lo = fmin(lo, part[2 * b]);
    hi = fmax(hi, part[2 * b + 1]);
  }
  block_minmax(lo, hi, red);
  if (threadIdx.x == 0) {
    mm[0] = lo;
    mm[1] = hi;
  }
}

// Confidence index (Eq. 6) from the folded extremes mm = (s_min, s_max),
// walking the arrays from their end.
template <bool kVec>
__global__ __launch_bounds__(256) void k_confidence(const double* __restrict__ sd,
                                                    const int32_t* __restrict__ count, int n, int min_count,
                                                    const double* __restrict__ mm, double* __restrict__ out) {
  const double lo = mm[0], hi = mm[1];
  const bool any = hi > lo;
  auto conf = [&](double v, int32_t c) { return (c >= min_count && any) ? (hi - v) / (hi - lo) : 0.0; };
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const int64_t t0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t ng = kVec ? (n >> 2) : 0;
  for (int64_t j = t0; j < n - (ng << 2); j += stride) {  // pixels past the last group (all, unaligned)
    const int64_t i = n - 1 - j;
    out[i] = conf(sd[i], count ? count[i] : min_count);
  }
  if (kVec) {
    const double2* __restrict__ s2 = reinterpret_cast<const double2*>(sd);
    const int4* __restrict__ c4 = reinterpret_cast<const int4*>(count);
    double2* __restrict__ o2 = reinterpret_cast<double2*>(out);
    const int4 all = make_int4(min_count, min_count, min_count, min_count);
    auto put4 = [&](int64_t g, double2 a, double2 b, int4 c) {
      o2[2 * g] = make_double2(conf(a.x, c.x), conf(a.y, c.y));
      o2[2 * g + 1] = make_double2(conf(b.x, c.z), conf(b.y, c.w));
    };
    int64_t j = t0;
    for (; j + stride < ng; j += 2 * stride) {
      const int64_t g = ng - 1 - j, h = g - stride;
      const double2 a0 = s2[2 * g], a1 = s2[2 * g + 1], b0 = s2[2 * h], b1 = s2[2 * h + 1];
      const int4 ca = count ? c4[g] : all, cb = count ? c4[h] : all;
      put4(g, a0, a1, ca);
      put4(h, b0, b1, cb);
    }
    if (j < ng) {
      const int64_t g = ng - 1 - j;
      put4(g, s2[2 * g], s2[2 * g + 1], count ? c4[g] : all);
    }
  }
}

hipError_t launch_confidence(const double* sd, const int32_t* count, int n, int min_count,
                             double* out, double* scratch, hipStream_t s) {
  const bool vec = aligned16(sd) && (!count || aligned16(count)) && aligned16(out);
  const int64_t units = vec ? (n >> 2) : n;
  const int parts = stream_blocks(units, kRedBlocks);
  double* mm = scratch + 2 * kRedBlocks;
  if (vec)
    hipLaunchKernelGGL(k_minmax_part<true>, dim3(parts), dim3(256), 0, s, sd, count, n, min_count, scratch);
  else
    hipLaunchKernelGGL(k_minmax_part<false>, dim3(parts), dim3(256), 0, s, sd, count, n, min_count, scratch);
  hipLaunchKernelGGL(k_minmax_fold, dim3(1), dim3(256), 0, s, scratch, parts, mm);
  const int blocks = stream_blocks(units, 4096);
  if (vec)
    hipLaunchKernelGGL(k_confidence<true>, dim3(blocks), dim3(256), 0, s, sd, count, n, min_count, mm, out);
  else
    hipLaunchKernelGGL(k_confidence<false>, dim3(blocks), dim3(256), 0, s, sd, count, n, min_count, mm, out);
  return hipGetLastError();
}

// Ratio map (Eq. 7): r = std / mean, 0 where |mean| <= eps
__global__ void k_ratio(const double* __restrict__ sd, const double* __restrict__ mean, int n,
                        double eps, double* out) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    double mu = mean[i];
    out[i] = fabs(mu) > eps ? sd[i] / mu : 0.0;
  }
}

hipError_t launch_ratio(const double* sd, const double* mean, int n, double eps, double* out,
                        hipStream_t s) {
  int blocks = std::max(1, std::min((n + 255) / 256, 4096));
  hipLaunchKernelGGL(k_ratio, dim3(blocks), dim3(256), 0, s, sd, mean, n, eps, out);
  return hipGetLastError();
}

// Post-stack Laplacian filter: out = -L img, zero outside the image.  A
// thread filters kLapRows rows of one column, with the column's values in
// registers, so a pixel costs one new load along z and eight along x.
constexpr int kLapRows = 16;

__global__ __launch_bounds__(256) void k_lapfilter(const float* __restrict__ img, int nz, int nx,
                                                   float c0, float4 czv, float4 cxv,
                                                   float* __restrict__ out) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  const int z0 = blockIdx.y * kLapRows;
  if (x >= nx) return;
  const float cz[4] = {czv.x, czv.y, czv.z, czv.w};
  const float cx[4] = {cxv.x, cxv.y, cxv.z, cxv.w};
  auto at = [&](int zz, int xx) -> float {
    return (zz >= 0 && zz < nz && xx >= 0 && xx < nx) ? img[(int64_t)zz * nx + xx] : 0.0f;
  };
  float col[kLapRows + 8];
#pragma unroll
  for (int j = 0; j < kLapRows + 8; ++j) col[j] = at(z0 - 4 + j, x);
#pragma unroll
  for (int k = 0; k < kLapRows; ++k) {
    const int z = z0 + k;
    if (z >= nz) break;
    float s = c0 * col[k + 4];
#pragma unroll
    for (int q = 1; q <= 4; ++q) {
      s = fmaf(cz[q - 1], col[k + 4 - q] + col[k + 4 + q], s);
      s = fmaf(cx[q - 1], at(z, x - q) + at(z, x + q), s);
    }
    out[(int64_t)z * nx + x] = -s;
  }
}

hipError_t launch_lapfilter(const float* img, int nz, int nx, float dz, float dx, float* out,
                            hipStream_t s) {
  const double a[5] = {-205.0 / 72.0, 8.0 / 5.0, -1.0 / 5.0, 8.0 / 315.0, -1.0 / 560.0};
  const double iz2 = 1.0 / ((double)dz * dz), ix2 = 1.0 / ((double)dx * dx);
  float c0 = (float)(a[0] * (iz2 + ix2));
  float4 czv = make_float4((float)(a[1] * iz2), (float)(a[2] * iz2), (float)(a[3] * iz2),
                           (float)(a[4] * iz2));
  float4 cxv = make_float4((float)(a[1] * ix2), (float)(a[2] * ix2), (float)(a[3] * ix2),
                           (float)(a[4] * ix2));
  hipLaunchKernelGGL(k_lapfilter, dim3((nx + 255) / 256, (nz + kLapRows - 1) / kLapRows), dim3(256), 0, s,
                     img, nz, nx, c0, czv, cxv, out);
  return hipGetLastError();
}


// ---------------------------------------------------------------------------
// Source-normalised image (Eq. 5): out = I / (illum + eps_rel * max illum)
// ---------------------------------------------------------------------------
template <bool kVec>
__global__ __launch_bounds__(256) void k_max_part(const float* __restrict__ a, int n, float* __restrict__ part) {
  __shared__ float red[4];
  float m = 0.0f;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const int64_t t0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t head = 0;
  if (kVec) {
    const int64_t ng = n >> 2;
    const float4* __restrict__ a4 = reinterpret_cast<const float4*>(a);
    auto take4 = [&](float4 v) { m = fmaxf(fmaxf(m, v.x), fmaxf(fmaxf(v.y, v.z), v.w)); };
    int64_t g = t0;
    for (; g + stride < ng; g += 2 * stride) {
      const float4 u = a4[g], v = a4[g + stride];
      take4(u);
      take4(v);
    }
    if (g < ng) take4(a4[g]);
    head = ng << 2;
  }
  for (int64_t i = head + t0; i < n; i += stride) m = fmaxf(m, a[i]);
  m = wave_max(m);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0) part[blockIdx.x] = fmaxf(fmaxf(red[0], red[1]), fmaxf(red[2], red[3]));
}

__global__ __launch_bounds__(256) void k_max_fold(const float* __restrict__ part, int nparts, float* __restrict__ mx) {
  __shared__ float red[4];
  float m = 0.0f;
  for (int b = threadIdx.x; b < nparts; b += blockDim.x) m = fmaxf(m, part[b]);
  m = wave_max(m);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0) *mx = fmaxf(fmaxf(red[0], red[1]), fmaxf(red[2], red[3]));
}

// walks the arrays from their end, after k_max_part walked them from the start
template <bool kVec>
__global__ __launch_bounds__(256) void k_normalize(const float* __restrict__ img, const float* __restrict__ illum,
                                                   int n, float eps_rel, const float* __restrict__ mx,
                                                   float* __restrict__ out) {
  const float eps = eps_rel * *mx;
  auto norm = [&](float im, float il) {
    const float d = il + eps;
    return d > 0.0f ? im / d : 0.0f;
  };
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const int64_t t0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t ng = kVec ? (n >> 2) : 0;
  for (int64_t j = t0; j < n - (ng << 2); j += stride) {
    const int64_t i = n - 1 - j;
    out[i] = norm(img[i], illum[i]);
  }
  if (kVec) {
    const float4* __restrict__ i4 = reinterpret_cast<const float4*>(img);
    const float4* __restrict__ l4 = reinterpret_cast<const float4*>(illum);
    f4v* __restrict__ o4 = reinterpret_cast<f4v*>(out);
    auto put4 = [&](int64_t g, float4 u, float4 l) {
      __builtin_nontemporal_store(f4v{norm(u.x, l.x), norm(u.y, l.y), norm(u.z, l.z), norm(u.w, l.w)}, o4 + g);
    };
    int64_t j = t0;
    for (; j + stride < ng; j += 2 * stride) {
      const int64_t g = ng - 1 - j, h = g - stride;
      const float4 ua = i4[g], la = l4[g], ub = i4[h], lb = l4[h];
      put4(g, ua, la);
      put4(h, ub, lb);
    }
    if (j < ng) {
      const int64_t g = ng - 1 - j;
      put4(g, i4[g], l4[g]);
    }
  }
}

hipError_t launch_normalize(const float* img, const float* illum, int n, float eps_rel, float* out,
                            float* scratch, hipStream_t s) {
  const bool vec = aligned16(img) && aligned16(illum) && aligned16(out);
  const int64_t units = vec ? (n >> 2) : n;
  const int parts = stream_blocks(units, kRedBlocks);
  if (vec)
    hipLaunchKernelGGL(k_max_part<true>, dim3(parts), dim3(256), 0, s, illum, n, scratch);
  else
    hipLaunchKernelGGL(k_max_part<false>, dim3(parts), dim3(256), 0, s, illum, n, scratch);
  hipLaunchKernelGGL(k_max_fold, dim3(1), dim3(256), 0, s, scratch, parts, scratch + kRedBlocks);
  const int blocks = stream_blocks(units, 4096);
  if (vec)
    hipLaunchKernelGGL(k_normalize<true>, dim3(blocks), dim3(256), 0, s, img, illum, n, eps_rel,
                       scratch + kRedBlocks, out);
  else
    hipLaunchKernelGGL(k_normalize<false>, dim3(blocks), dim3(256), 0, s, img, illum, n, eps_rel,
                       scratch + kRedBlocks, out);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Chan et al. merge of two running (count, mean, M2) states, per pixel:
//   n = na + nb, d = mb - ma, mean = ma + d nb / n, M2 = M2a + M2b + d^2 na nb / n
// (combines per-GPU or per-stream statistics into one).
// ---------------------------------------------------------------------------
__global__ void k_chan_merge(double* __restrict__ ma, double* __restrict__ m2a, int32_t* __restrict__ na,
                             const double* __restrict__ mb, const double* __restrict__ m2b,
                             const int32_t* __restrict__ nb, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const int32_t a = na[i], b = nb[i];
    if (b == 0) continue;
    if (a == 0) {
      ma[i] = mb[i];
      m2a[i] = m2b[i];
      na[i] = b;
      continue;
    }
    const double nn = (double)a + (double)b;
    const double d = mb[i] - ma[i];
    ma[i] = ma[i] + d * ((double)b / nn);
    m2a[i] = m2a[i] + m2b[i] + d * d * ((double)a * (double)b / nn);
    na[i] = a + b;
  }
}

hipError_t launch_chan_merge(double* mean_a, double* m2_a, int32_t* n_a, const double* mean_b,
                             const double* m2_b, const int32_t* n_b, int64_t n, hipStream_t s) {
  const int blocks = (int)std::max<int64_t>(1, std::min<int64_t>((n + 255) / 256, 4096));
  hipLaunchKernelGGL(k_chan_merge, dim3(blocks), dim3(256), 0, s, mean_a, m2_a, n_a, mean_b, m2_b, n_b, n);
  return hipGetLastError();
}

}  // namespace rtm
