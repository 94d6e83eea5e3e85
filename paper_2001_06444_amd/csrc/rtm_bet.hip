// rtm_bet.hip -- Stage 1 of the workflow, Bayesian Eikonal tomography
// (Sec. 2.1, Eq. 1-3), as many reversible-jump chains advancing together.
//
// Model: Voronoi cells with a constant velocity each (a grid node takes the
// velocity of its nearest nucleus, ties to the lowest index).  Forward
// operator: first-arrival travel times of the Eikonal equation, first-order
// Godunov upwind scheme on a square grid, point sources at grid nodes.
// Likelihood: exp(-Phi / 2), Phi = sum ((T - d) / sigma)^2.  Proposals:
// add a nucleus (position and velocity from the uniform prior), delete one,
// or move one by a uniform step; every acceptance ratio is the likelihood
// ratio.  Random numbers: the counter form of splitmix64.
//
// One iteration of every chain is five launches: propose (a thread per
// chain), raster (nearest nucleus per node), eikonal (a wavefront per chain
// and source: fast sweeping over anti-diagonals in LDS), accept (a workgroup
// per chain: FP64 misfit, Metropolis test) and, on sampling iterations,
// sample (FP64 Welford of the chains' velocity grids per node).
//
// Arithmetic that decides a discrete outcome (positions, nearest nuclei,
// travel times, accept tests) is written without contraction, in the order
// the definition states, so it matches a plain CPU evaluation.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "rtm_bet.h"

#pragma clang fp contract(off)

namespace rtm {
namespace {

constexpr uint64_t kGamma = 0x9E3779B97F4A7C15ull;

__device__ inline uint64_t sm64_mix(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}
// output n of the splitmix64 stream seeded with s
__device__ inline uint64_t sm64_at(uint64_t s, uint64_t n) { return sm64_mix(s + (n + 1) * kGamma); }
// draw k of iteration t (t = -1: the initial model) of chain c
__device__ inline uint64_t bet_draw(uint64_t seed, int c, int t, int k) {
  return sm64_at(sm64_at(seed, (uint64_t)c), (uint64_t)(t + 1) * 256u + (uint64_t)k);
}
__device__ inline double unit_open0(uint64_t x) { return (double)(x >> 11) * 0x1.0p-53; }
__device__ inline double unit_open1(uint64_t x) { return (double)((x >> 11) + 1) * 0x1.0p-53; }

__device__ inline void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Godunov upwind value from the smaller z-neighbour and x-neighbour times
// and sh = slowness * h: one-sided lo + sh when hi - lo >= sh, else
// ((lo + hi) + sqrt((q + q) - d d)) / 2 with q = sh sh, d = hi - lo.
// (plain operators: this file turns contraction off, and sqrtf is the
// correctly rounded square root)
__device__ inline float godunov(float a, float b, float sh) {
  const float lo = a > b ? b : a, hi = a > b ? a : b;
  const float d = hi - lo;
  if (!(d < sh)) return lo + sh;
  const float q = sh * sh;
  return ((lo + hi) + sqrtf((q + q) - d * d)) * 0.5f;
}

// Fast sweeping by one wavefront on T[nz*nx] in LDS: the four orderings of
// Gauss-Seidel sweeps, each over anti-diagonals (the nodes of one diagonal are
// not neighbours, so a wavefront updates them together), repeated until a
// whole pass changes nothing.  Returns the passes used (kBetMaxSweeps: gave up).
template <class Slow>
__device__ int fsm_solve(float* T, int nz, int nx, float h, int si, int sj, Slow slow) {
  const int lane = threadIdx.x & 63;
  const int n = nz * nx;
  for (int p = lane; p < n; p += 64) T[p] = INFINITY;
  wave_sync();
  if (lane == 0) T[si * nx + sj] = 0.0f;
  wave_sync();
  int pass = 0;
  for (; pass < kBetMaxSweeps; ++pass) {
    bool changed = false;
    for (int o = 0; o < 4; ++o) {
      const bool fi = (o == 0 || o == 3), fj = (o < 2);
      for (int dg = 0; dg <= nz + nx - 2; ++dg) {
        const int ilo = max(0, dg - (nx - 1)), ihi = min(dg, nz - 1);
        for (int ii = ilo + lane; ii <= ihi; ii += 64) {
          const int jj = dg - ii;
          const int i = fi ? ii : nz - 1 - ii, j = fj ? jj : nx - 1 - jj;
          const int p = i * nx + j;
          const float up = i > 0 ? T[p - nx] : INFINITY, dn = i + 1 < nz ? T[p + nx] : INFINITY;
          const float lf = j > 0 ? T[p - 1] : INFINITY, rt = j + 1 < nx ? T[p + 1] : INFINITY;
          const float t = godunov(up < dn ? up : dn, lf < rt ? lf : rt, slow(p) * h);
          if (t < T[p]) {
            T[p] = t;
            changed = true;
          }
        }
        wave_sync();
      }
    }
    if (!__any(changed)) break;
  }
  return pass;
}

// The same sweeps with one row per lane (nz <= 64): in ordering (fi, fj) lane
// l owns the l-th row in sweep order and handles its column jj at step l + jj,
// which is the anti-diagonal schedule above.  A node's upwind neighbours were
// updated one step earlier -- the one in its row by this lane (kept in a
// register), the one in the previous row by lane l - 1 (a lane shift) -- and
// its downwind neighbours still hold their values from before this sweep
// (LDS that no lane overwrites before it has been read).  A step has no
// branches: reads use clamped in-bounds nodes and selects drop what lies
// outside the grid.
// lane l receives lane l - 1's value (lane 0 receives `edge`): a DPP wave
// shift, no LDS round trip
__device__ inline float from_lane_below(float v, float edge) {
  return __int_as_float(__builtin_amdgcn_update_dpp(__float_as_int(edge), __float_as_int(v), 0x138 /* wave_shr:1 */,
                                                    0xF, 0xF, false));
}

// Godunov value without branches: both forms computed, one selected (the
// same value as godunov())
__device__ inline float godunov_sel(float a, float b, float sh) {
  const float lo = a > b ? b : a, hi = a > b ? a : b;
  const float d = hi - lo;
  const float q = sh * sh;
  const float two = ((lo + hi) + sqrtf((q + q) - d * d)) * 0.5f;
  return !(d < sh) ? lo + sh : two;
}

template <class Slow>
__device__ int fsm_solve_rows(float* T, int nz, int nx, float h, int si, int sj, Slow slow) {
  const int lane = threadIdx.x & 63;
  const int n = nz * nx;
  for (int p = lane; p < n; p += 64) T[p] = INFINITY;
  wave_sync();
  if (lane == 0) T[si * nx + sj] = 0.0f;
  wave_sync();
  const bool row_ok = lane < nz;
  const bool has_dn = lane + 1 < nz;
  int pass = 0;
  for (; pass < kBetMaxSweeps; ++pass) {
    bool changed = false;
    for (int o = 0; o < 4; ++o) {
      const bool fi = (o == 0 || o == 3), fj = (o < 2);
      // lanes past the last row read row 0 and never change it
      const int i = row_ok ? (fi ? lane : nz - 1 - lane) : 0;
      const int idn = has_dn ? (fi ? i + 1 : i - 1) : i;  // the next row in sweep order
      float cur = INFINITY;  // this lane's node of the previous step
      for (int step = 0; step <= nz + nx - 2; ++step) {
        const int jj = step - lane;
        const bool active = row_ok && jj >= 0 && jj < nx;
        const int jc = jj < 0 ? 0 : (jj >= nx ? nx - 1 : jj);
        const int j = fj ? jc : nx - 1 - jc;
        const int p = i * nx + j;
        const int pr = jc + 1 < nx ? (fj ? p + 1 : p - 1) : p;
        const float dn_v = T[idn * nx + j], rt_v = T[pr], old = T[p];
        const float sl = slow(p);
        const float above = from_lane_below(cur, INFINITY);
        // up/left are this sweep's upwind times, dn/rt the downwind ones
        const float up = lane > 0 ? above : INFINITY;
        const float dn = has_dn ? dn_v : INFINITY;
        const float rt = jc + 1 < nx ? rt_v : INFINITY;
        const float left = jj > 0 ? cur : INFINITY;
        const float a = fi ? (up < dn ? up : dn) : (dn < up ? dn : up);
        const float b = fj ? (left < rt ? left : rt) : (rt < left ? rt : left);
        const float t = godunov_sel(a, b, sl * h);
        const bool better = active && t < old;
        cur = better ? t : old;
        // a lane with a row stores its own node (unchanged when inactive); a
        // lane past the last row stores to the discard slot T[n]
        T[row_ok ? p : n] = cur;
        changed |= better;
      }
      wave_sync();
    }
    if (!__any(changed)) break;
  }
  return pass;
}

// T[n + 1]: the grid's times and a discard slot
__device__ inline size_t bet_lds_t_bytes(int n) { return ((size_t)(n + 1) * 4 + 15) & ~(size_t)15; }
__device__ inline size_t bet_lds_c_bytes(int n) { return ((size_t)n + 15) & ~(size_t)15; }

}  // namespace

__global__ __launch_bounds__(64) void k_bet_propose(BetDev d, int t, int init) {
  const int c = blockIdx.x * 64 + threadIdx.x;
  if (c >= d.chains) return;
  const int K = d.k_max;
  const double Z = (double)(d.nz - 1) * d.h, X = (double)(d.nx - 1) * d.h;
  double* pz = d.pz + (size_t)c * K;
  double* px = d.px + (size_t)c * K;
  double* pv = d.pv + (size_t)c * K;
  if (init) {
    for (int q = 0; q < d.k_init; ++q) {
      pz[q] = unit_open0(bet_draw(d.seed, c, -1, 3 * q)) * Z;
      px[q] = unit_open0(bet_draw(d.seed, c, -1, 3 * q + 1)) * X;
      pv[q] = d.v_min + unit_open0(bet_draw(d.seed, c, -1, 3 * q + 2)) * (d.v_max - d.v_min);
    }
    d.pk[c] = d.k_init;
    d.valid[c] = 1;
    d.ptype[c] = 0;
    d.ua[c] = 1.0;
    return;
  }
  const int k = d.k[c];
  for (int q = 0; q < k; ++q) {
    pz[q] = d.z[(size_t)c * K + q];
    px[q] = d.x[(size_t)c * K + q];
    pv[q] = d.v[(size_t)c * K + q];
  }
  const double u0 = unit_open0(bet_draw(d.seed, c, t, 0));
  const double u1 = unit_open0(bet_draw(d.seed, c, t, 1));
  const double u2 = unit_open0(bet_draw(d.seed, c, t, 2));
  const double u3 = unit_open0(bet_draw(d.seed, c, t, 3));
  const double ua = unit_open1(bet_draw(d.seed, c, t, 4));
  const int type = u0 < d.p_birth ? 0 : (u0 < d.p_birth + d.p_death ? 1 : 2);
  int kk = k, valid = 1;
  if (type == 0) {
    if (k >= K) {
      valid = 0;
    } else {
      pz[k] = u1 * Z;
      px[k] = u2 * X;
      pv[k] = d.v_min + u3 * (d.v_max - d.v_min);
      kk = k + 1;
    }
  } else if (type == 1) {
    if (k <= d.k_min) {
      valid = 0;
    } else {
      int i = (int)(u1 * (double)k);
      if (i > k - 1) i = k - 1;
      for (int q = i; q < k - 1; ++q) {
        pz[q] = pz[q + 1];
        px[q] = px[q + 1];
        pv[q] = pv[q + 1];
      }
      kk = k - 1;
    }
  } else {
    int i = (int)(u1 * (double)k);
    if (i > k - 1) i = k - 1;
    const double nzp = pz[i] + (2.0 * u2 - 1.0) * d.move_dz;
    const double nxp = px[i] + (2.0 * u3 - 1.0) * d.move_dx;
    if (nzp < 0.0 || nzp > Z || nxp < 0.0 || nxp > X) {
      valid = 0;
    } else {
      pz[i] = nzp;
      px[i] = nxp;
    }
  }
  d.pk[c] = kk;
  d.valid[c] = valid;
  d.ptype[c] = type;
  d.ua[c] = ua;
}

// nearest nucleus of the proposal at every node (ties: lowest index)
__global__ __launch_bounds__(256) void k_bet_raster(BetDev d) {
  const int c = blockIdx.y;
  if (!d.valid[c]) return;
  const int n = d.nz * d.nx;
  const int p = blockIdx.x * 256 + threadIdx.x;
  if (p >= n) return;
  const int i = p / d.nx, j = p - (p / d.nx) * d.nx;
  const double z = (double)i * d.h, x = (double)j * d.h;
  const double* pz = d.pz + (size_t)c * d.k_max;
  const double* px = d.px + (size_t)c * d.k_max;
  const int kk = d.pk[c];
  int best = 0;
  double bd = INFINITY;
  for (int q = 0; q < kk; ++q) {
    const double dz = z - pz[q], dx = x - px[q];
    const double d2 = dz * dz + dx * dx;
    if (d2 < bd) {
      bd = d2;
      best = q;
    }
  }
  d.cell[(size_t)c * n + p] = (uint8_t)best;
}

// travel times of the proposal from source blockIdx.x of chain blockIdx.y
__global__ __launch_bounds__(64) void k_bet_eikonal(BetDev d) {
  extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
  const int e = blockIdx.x, c = blockIdx.y;
  if (!d.valid[c]) return;
  const int lane = threadIdx.x;
  const int n = d.nz * d.nx;
  float* T = reinterpret_cast<float*>(smem);
  uint8_t* cid = smem + bet_lds_t_bytes(n);
  float* stab = reinterpret_cast<float*>(smem + bet_lds_t_bytes(n) + bet_lds_c_bytes(n));
  const uint8_t* cell = d.cell + (size_t)c * n;
  for (int p = lane; p < n; p += 64) cid[p] = cell[p];
  const int kk = d.pk[c];
  for (int q = lane; q < kk; q += 64) stab[q] = (float)(1.0 / d.pv[(size_t)c * d.k_max + q]);
  wave_sync();
  const int2 s = d.src[e];
  auto slow = [&](int p) { return stab[cid[p]]; };
  const int passes = d.nz <= 64 ? fsm_solve_rows(T, d.nz, d.nx, (float)d.h, s.x, s.y, slow)
                                : fsm_solve(T, d.nz, d.nx, (float)d.h, s.x, s.y, slow);
  if (lane == 0) {
    if (passes >= kBetMaxSweeps) atomicOr(d.flags, kBetNoConverge);
    atomicAdd(d.work + 2 * (size_t)c, 1ull);
    atomicAdd(d.work + 2 * (size_t)c + 1, (unsigned long long)min(passes + 1, kBetMaxSweeps));
  }
  float* out = d.tt + ((size_t)c * d.nsrc + e) * d.nrec;
  for (int r = lane; r < d.nrec; r += 64) {
    const int2 q = d.rec[r];
    out[r] = T[q.x * d.nx + q.y];
  }
}

// misfit of the proposal and the Metropolis test (a workgroup per chain)
__global__ __launch_bounds__(256) void k_bet_accept(BetDev d, int init, int8_t* log_row) {
  __shared__ double red[256];
  __shared__ int s_acc;
  const int c = blockIdx.x, tid = threadIdx.x;
  const int valid = d.valid[c];
  const int type = d.ptype[c];
  if (valid) {
    const int nd = d.nsrc * d.nrec;
    const float* tt = d.tt + (size_t)c * nd;
    double part = 0.0;
    for (int q = tid; q < nd; q += 256) {
      const double r = ((double)tt[q] - (double)d.tt_obs[q]) / d.sigma;
      part += r * r;
    }
    red[tid] = part;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
      if (tid < w) red[tid] += red[tid + w];
      __syncthreads();
    }
    if (tid == 0) {
      const double phi = red[0];
      const int acc = init || (phi - d.misfit[c] < -2.0 * log(d.ua[c]));
      if (acc) {
        d.misfit[c] = phi;
        d.k[c] = d.pk[c];
      }
      if (!init) {
        ++d.proposed[(size_t)c * 3 + type];
        if (acc) ++d.accepted[(size_t)c * 3 + type];
      }
      s_acc = acc;
    }
    __syncthreads();
    if (s_acc) {
      const int kk = d.pk[c], K = d.k_max;
      for (int q = tid; q < kk; q += 256) {
        d.z[(size_t)c * K + q] = d.pz[(size_t)c * K + q];
        d.x[(size_t)c * K + q] = d.px[(size_t)c * K + q];
        d.v[(size_t)c * K + q] = d.pv[(size_t)c * K + q];
      }
    }
  }
  if (tid == 0 && log_row && !init) log_row[c] = (int8_t)(valid ? (s_acc ? 1 + type : 0) : -1);
}

// pooled FP64 Welford of every chain's current velocity grid (chains in order)
__global__ __launch_bounds__(256) void k_bet_sample(BetDev d) {
  const int n = d.nz * d.nx;
  const int p = blockIdx.x * 256 + threadIdx.x;
  if (p >= n) return;
  const int i = p / d.nx, j = p - (p / d.nx) * d.nx;
  const double z = (double)i * d.h, x = (double)j * d.h;
  double mean = d.mean[p], m2 = d.m2[p];
  int32_t cnt = d.count[p];
  for (int c = 0; c < d.chains; ++c) {
    const double* zs = d.z + (size_t)c * d.k_max;
    const double* xs = d.x + (size_t)c * d.k_max;
    const int k = d.k[c];
    int best = 0;
    double bd = INFINITY;
    for (int q = 0; q < k; ++q) {
      const double dz = z - zs[q], dx = x - xs[q];
      const double d2 = dz * dz + dx * dx;
      if (d2 < bd) {
        bd = d2;
        best = q;
      }
    }
    const double v = d.v[(size_t)c * d.k_max + best];
    ++cnt;
    const double delta = v - mean;
    mean += delta / (double)cnt;
    m2 += delta * (v - mean);
  }
  d.mean[p] = mean;
  d.m2[p] = m2;
  d.count[p] = cnt;
}

// travel times of one velocity grid from source blockIdx.x
__global__ __launch_bounds__(64) void k_eikonal_grid(const float* vel, int nz, int nx, float h, const int2* src,
                                                     const int2* rec, int nrec, float* tt, uint32_t* flags) {
  extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
  const int e = blockIdx.x, lane = threadIdx.x, n = nz * nx;
  float* T = reinterpret_cast<float*>(smem);
  float* S = reinterpret_cast<float*>(smem + bet_lds_t_bytes(n));
  for (int p = lane; p < n; p += 64) S[p] = (float)(1.0 / (double)vel[p]);
  wave_sync();
  const int2 s = src[e];
  auto slow = [&](int p) { return S[p]; };
  const int passes = nz <= 64 ? fsm_solve_rows(T, nz, nx, h, s.x, s.y, slow) : fsm_solve(T, nz, nx, h, s.x, s.y, slow);
  if (passes >= kBetMaxSweeps && lane == 0) atomicOr(flags, kBetNoConverge);
  for (int r = lane; r < nrec; r += 64) {
    const int2 q = rec[r];
    tt[(size_t)e * nrec + r] = T[q.x * nx + q.y];
  }
}

static size_t lds_bet(int n) {
  return (((size_t)(n + 1) * 4 + 15) & ~(size_t)15) + (((size_t)n + 15) & ~(size_t)15) + 4 * kBetMaxCells;
}
static size_t lds_grid(int n) { return (((size_t)(n + 1) * 4 + 15) & ~(size_t)15) + (((size_t)n * 4 + 15) & ~(size_t)15); }

hipError_t launch_bet_propose(const BetDev& d, int t, int init, hipStream_t s) {
  k_bet_propose<<<(d.chains + 63) / 64, 64, 0, s>>>(d, t, init);
  return hipGetLastError();
}

hipError_t launch_bet_raster(const BetDev& d, hipStream_t s) {
  const int n = d.nz * d.nx;
  k_bet_raster<<<dim3((n + 255) / 256, d.chains), 256, 0, s>>>(d);
  return hipGetLastError();
}

hipError_t launch_bet_eikonal(const BetDev& d, hipStream_t s) {
  const int n = d.nz * d.nx;
  if (n > kBetMaxNodes || d.k_max > kBetMaxCells) return hipErrorInvalidValue;
  const size_t lds = lds_bet(n);
  if (lds > 65536) {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_bet_eikonal),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  k_bet_eikonal<<<dim3(d.nsrc, d.chains), 64, lds, s>>>(d);
  return hipGetLastError();
}

hipError_t launch_bet_accept(const BetDev& d, int init, int8_t* log_row, hipStream_t s) {
  k_bet_accept<<<d.chains, 256, 0, s>>>(d, init, log_row);
  return hipGetLastError();
}

hipError_t launch_bet_sample(const BetDev& d, hipStream_t s) {
  const int n = d.nz * d.nx;
  k_bet_sample<<<(n + 255) / 256, 256, 0, s>>>(d);
  return hipGetLastError();
}

hipError_t launch_eikonal_grid(const float* vel, int nz, int nx, float h, const int2* src, int nsrc,
                               const int2* rec, int nrec, float* tt, uint32_t* flags, hipStream_t s) {
  const int n = nz * nx;
  if (n > kBetMaxNodes) return hipErrorInvalidValue;
  const size_t lds = lds_grid(n);
  if (lds > 65536) {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_eikonal_grid),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  k_eikonal_grid<<<nsrc, 64, lds, s>>>(vel, nz, nx, h, src, rec, nrec, tt, flags);
  return hipGetLastError();
}

}  // namespace rtm
