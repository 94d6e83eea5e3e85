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
// chain), raster (nearest nucleus per node, stored as the node's slowness
// terms), eikonal (a wavefront per chain and source: fast sweeping over
// anti-diagonals, times in LDS), accept (a workgroup per chain: FP64 misfit,
// Metropolis test) and, on sampling iterations, sample (FP64 Welford of the
// chains' velocity grids per node).
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

// Correctly rounded single-precision square root of x in [2^-60, 2^126],
// by Tuckerman's rounding test (Markstein, IBM J. Res. Dev. 34(1), 1990): the
// hardware estimate y is within one ulp of sqrt(x), and y is the rounded
// root exactly when pred(y) y < x <= y succ(y).  The two residuals come from
// fused multiply-adds, exact in sign over this range, and select pred(y), y
// or succ(y).  (Without the scaling and special cases of the library
// routine, which this range does not need.)
__device__ inline float sqrt_rn(float x) {
  const float y = __builtin_amdgcn_sqrtf(x);
  const float yd = __int_as_float(__float_as_int(y) - 1), yu = __int_as_float(__float_as_int(y) + 1);
  const float rd = __builtin_fmaf(-yd, y, x), ru = __builtin_fmaf(-yu, y, x);
  const float r = rd <= 0.0f ? yd : y;
  return ru > 0.0f ? yu : r;
}

// Godunov upwind value from the smaller z-neighbour and x-neighbour times
// and the node's sh = slowness * h, q2 = sh sh + sh sh: one-sided lo + sh
// when hi - lo >= sh, else ((lo + hi) + sqrt(q2 - d d)) / 2 with d = hi - lo.
// Both forms are computed and one selected, without branches.  Plain
// operators (this file turns contraction off); with sh in [kBetShMin,
// kBetShMax] the square root's argument in the two-sided case lies in
// [sh^2, 2 sh^2], inside the range of sqrt_rn.
__device__ inline BetSlowness slowness_h(float slow, float h) {
  const float sh = slow * h;
  const float q = sh * sh;
  return {sh, q + q};
}
// min and max of two times by their bit patterns: for non-negative floats
// (+inf included) the patterns order as integers the way the values do, and
// the times compared here are never negative or NaN where the result is
// used -- one integer instruction, the same value as a float comparison
__device__ inline float min_t(float a, float b) { return __int_as_float(min(__float_as_int(a), __float_as_int(b))); }
__device__ inline float max_t(float a, float b) { return __int_as_float(max(__float_as_int(a), __float_as_int(b))); }

__device__ inline float godunov(float a, float b, BetSlowness s) {
  const float lo = min_t(a, b), hi = max_t(a, b);
  const float d = hi - lo;
  const float two = ((lo + hi) + sqrt_rn(s.q2 - d * d)) * 0.5f;
  return !(d < s.sh) ? lo + s.sh : two;
}

// The node terms a solve reads, precomputed per node in global memory (for
// a chain's proposal by k_bet_raster, for a velocity grid by k_grid_terms);
// `ptr`/`at_ptr` read them through a pointer a sweep steps along a row.
// (a global-address-space pointer, so the reads are global loads, which
// count on the vector-memory counter only, not flat ones that also hold the
// LDS counter)
typedef const __attribute__((address_space(1))) BetSlowness* GlobalTerms;
struct NodeSlowness {
  GlobalTerms S;
  __device__ NodeSlowness(const BetSlowness* p) : S((GlobalTerms)p) {}
  __device__ BetSlowness at(int p) const { return {S[p].sh, S[p].q2}; }
  __device__ GlobalTerms ptr(int p) const { return S + p; }
  __device__ BetSlowness at_ptr(GlobalTerms q, int k) const { return {q[k].sh, q[k].q2}; }
};


// Both solvers run Gauss-Seidel sweeps of the four orderings in turn until a
// sweep changes nothing.  Such a sweep has updated every node from neighbours
// that did not change, so the times are a fixed point of every ordering: the
// times of repeating whole passes of four until a pass changes nothing.
// They return the sweeps used, negated when kBetMaxSweeps came first.
__device__ inline bool ordering_fi(int o) { return o == 0 || o == 3; }

// Fast sweeping by one wavefront over anti-diagonals (the nodes of one
// diagonal are not neighbours, so a wavefront updates them together), for
// any number of rows; T has row stride ld.
template <class Slow>
__device__ __forceinline__ int fsm_solve(float* T, int nz, int nx, int ld, int si, int sj, Slow sl) {
  const int lane = threadIdx.x & 63;
  for (int p = lane; p < nz * ld; p += 64) T[p] = INFINITY;
  wave_sync();
  if (lane == 0) T[si * ld + sj] = 0.0f;
  wave_sync();
  for (int sweeps = 0, o = 0; sweeps < kBetMaxSweeps; o = (o + 1) & 3) {
    const bool fi = ordering_fi(o), fj = (o < 2);
    bool changed = false;
    for (int dg = 0; dg <= nz + nx - 2; ++dg) {
      const int ilo = max(0, dg - (nx - 1)), ihi = min(dg, nz - 1);
      for (int ii = ilo + lane; ii <= ihi; ii += 64) {
        const int jj = dg - ii;
        const int i = fi ? ii : nz - 1 - ii, j = fj ? jj : nx - 1 - jj;
        const int p = i * ld + j;
        const float up = i > 0 ? T[p - ld] : INFINITY, dn = i + 1 < nz ? T[p + ld] : INFINITY;
        const float lf = j > 0 ? T[p - 1] : INFINITY, rt = j + 1 < nx ? T[p + 1] : INFINITY;
        const float t = godunov(up < dn ? up : dn, lf < rt ? lf : rt, sl.at(p));
        if (t < T[p]) {
          T[p] = t;
          changed = true;
        }
      }
      wave_sync();
    }
    ++sweeps;
    if (!__any(changed)) return sweeps;
  }
  return -kBetMaxSweeps;
}

// lane l receives lane l - 1's value (lane 0 receives `edge`): a DPP wave
// shift, no LDS round trip
__device__ inline float from_lane_below(float v, float edge) {
  return __int_as_float(__builtin_amdgcn_update_dpp(__float_as_int(edge), __float_as_int(v), 0x138 /* wave_shr:1 */,
                                                    0xF, 0xF, false));
}
// lane l receives lane l - 1's value, lane 0 lane 63's: a DPP wave rotation
__device__ inline float from_lane_below_rot(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(__float_as_int(v), __float_as_int(v), 0x13C /* wave_ror:1 */,
                                                    0xF, 0xF, false));
}

// One sweep with R rows per lane (nz <= 64 R): lane l owns the rows l,
// l + 64, ... in sweep order (row[r]: its first entry; a lane without an r-th
// row reads row 0 and never stores; below[r]: the next row in sweep order,
// the +inf row after the grid for the last) and handles column jj of its
// r-th row at step l + 64 r + jj, which is the anti-diagonal schedule.  A
// node's upwind neighbours were updated one step earlier -- the one in its
// row by this lane (kept in a register), the one in the previous row by lane
// l - 1 (a lane shift; for lane 0's r-th row, lane 63's (r - 1)-th row, a
// rotation) -- and every time a step reads from LDS is from before this
// sweep: its own node, the next node of its row (written by this lane a step
// later) and the node below it in the next row (written two steps later).
// So the times of step s + 1 are read during step s, and the node terms of
// step s + 2 as well, leaving only the arithmetic on the chain from step to
// step.  Steps have no branches: outside its row a lane reads guard, pad or
// neighbouring-row entries, whose values are never used except the +inf of
// the pad (or guard) entry on either side of the row, and stores to its
// discard slot.  Returns whether a node changed.
template <bool FJ, int R, class Slow>
__device__ __forceinline__ bool sweep_rows(float* T, int nx, int last, const int (&row)[R], const int (&below)[R],
                           const unsigned (&nx_own)[R], float* discard, Slow sl) {
  const int lane = threadIdx.x & 63;
  constexpr int dir = FJ ? 1 : -1;
  // node of sweep index jj in the r-th row (column jj or nx - 1 - jj), at
  // step 0 (jj = -lane - 64 r), and the offset to the node below
  int p0[R], to_dn[R];
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int jj0 = -lane - 64 * r;
    p0[r] = FJ ? row[r] + jj0 : row[r] + (nx - 1) - jj0;
    to_dn[r] = below[r] - row[r];
  }
  struct Stage {
    float old[R], rt[R], dn[R];
    BetSlowness s[R];
  };
  bool changed = false;
  float cur[R];  // this lane's nodes of the previous step
#pragma unroll
  for (int r = 0; r < R; ++r) cur[r] = INFINITY;
  // Three sets rotate (this step's, the next step's, the one after), so no
  // value is copied between registers while its read is in flight.
  using SPtr = decltype(sl.ptr(0));
  // pc[r]: node of the r-th row at this step; sc[r]: the same node's terms
  auto body = [&](int jj, const int (&pc)[R], const SPtr (&sc)[R], const Stage& P, Stage& Q, Stage& Rs) {
    // the reads first, then the arithmetic: the scheduler may not move
    // either across (work of the next step moved up, or reads moved down,
    // would wait on reads just issued)
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int p = pc[r];
      Q.old[r] = T[p + dir];
      Q.rt[r] = T[p + 2 * dir];
      Q.dn[r] = T[p + to_dn[r] + dir];
      Rs.s[r] = sl.at_ptr(sc[r], 2 * dir);
    }
    __builtin_amdgcn_sched_barrier(0);
    // up (the previous row's node of the previous step) and left (this
    // row's) are this sweep's upwind times, dn and rt the downwind ones; the
    // ups are taken before any of this step's nodes replace `cur`
    float up[R];
    // (the first row has no upwind row: it takes dn in place of +inf, the same min)
    up[0] = from_lane_below(cur[0], P.dn[0]);
#pragma unroll
    for (int r = 1; r < R; ++r) up[r] = from_lane_below_rot(lane == 63 ? cur[r - 1] : cur[r]);
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const bool active = (unsigned)(jj - 64 * r) < nx_own[r];
      const float a = min_t(up[r], P.dn[r]);
      const float b = min_t(cur[r], P.rt[r]);
      const float t = godunov(a, b, P.s[r]);
      const bool better = active && t < P.old[r];
      cur[r] = better ? t : P.old[r];
      *(active ? T + pc[r] : discard + 64 * r) = cur[r];
      changed |= better;
    }
  };
  Stage A, B, C;
#pragma unroll
  for (int r = 0; r < R; ++r) {
    A.old[r] = T[p0[r]];
    A.rt[r] = T[p0[r] + dir];
    A.dn[r] = T[p0[r] + to_dn[r]];
    A.s[r] = sl.at(p0[r]);
    B.s[r] = sl.at(p0[r] + dir);
  }
  int step = 0, jj = -lane;
  int p[R], p1[R], p2[R];  // this step's node of each row, and the next two steps'
  SPtr q[R], q1[R], q2[R];
#pragma unroll
  for (int r = 0; r < R; ++r) {
    p[r] = p0[r];
    q[r] = sl.ptr(p0[r]);
  }
  for (; step + 2 <= last; step += 3, jj += 3) {
#pragma unroll
    for (int r = 0; r < R; ++r) {
      p1[r] = p[r] + dir;
      p2[r] = p[r] + 2 * dir;
      q1[r] = q[r] + dir;
      q2[r] = q[r] + 2 * dir;
    }
    body(jj, p, q, A, B, C);
    body(jj + 1, p1, q1, B, C, A);
    body(jj + 2, p2, q2, C, A, B);
#pragma unroll
    for (int r = 0; r < R; ++r) {
      p[r] += 3 * dir;
      q[r] += 3 * dir;
    }
  }
#pragma unroll
  for (int r = 0; r < R; ++r) {
    p1[r] = p[r] + dir;
    q1[r] = q[r] + dir;
  }
  if (step <= last) body(jj, p, q, A, B, C);
  if (step + 1 <= last) body(jj + 1, p1, q1, B, C, A);
  return changed;
}

template <int R, class Slow>
__device__ __forceinline__ int fsm_solve_rows(float* T, int nz, int nx, int ld, int si, int sj, Slow sl) {
  const int lane = threadIdx.x & 63;
  // rows, pads, the row below the grid and guards: +inf (the discard slots
  // are in the first guard)
  for (int p = lane - kBetGuard; p < (nz + 1) * ld + kBetTail; p += 64) T[p] = INFINITY;
  wave_sync();
  if (lane == 0) T[si * ld + sj] = 0.0f;
  wave_sync();
  // 64 discard slots per row block, entries -132 .. -5 of the first guard:
  // never read for a value that is used
  float* const discard = T - kBetGuard + lane;
  const int last = nz + nx - 2;
  for (int sweeps = 0, o = 0; sweeps < kBetMaxSweeps; o = (o + 1) & 3) {
    const bool fi = ordering_fi(o);
    int row[R], below[R];
    unsigned nx_own[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int k = lane + 64 * r;  // this lane's r-th row in sweep order
      const bool ok = k < nz, has_dn = k + 1 < nz;
      const int i = ok ? (fi ? k : nz - 1 - k) : 0;
      row[r] = i * ld;
      below[r] = (has_dn ? (fi ? i + 1 : i - 1) : nz) * ld;  // the next row in sweep order, or the +inf row
      nx_own[r] = ok ? (unsigned)nx : 0u;
    }
    const bool changed = o < 2 ? sweep_rows<true, R>(T, nx, last, row, below, nx_own, discard, sl)
                               : sweep_rows<false, R>(T, nx, last, row, below, nx_own, discard, sl);
    wave_sync();
    ++sweeps;
    if (!__any(changed)) return sweeps;
  }
  return -kBetMaxSweeps;
}

// the solver for a grid of nz rows: one or two rows per lane up to 128 rows,
// else the anti-diagonal sweep (inlined into each kernel, where T is known
// to be LDS)
template <class Slow>
__device__ __forceinline__ int fsm_solve_any(float* T, int nz, int nx, int ld, int si, int sj, Slow sl) {
  if (nz <= 64) return fsm_solve_rows<1>(T, nz, nx, ld, si, sj, sl);
  if (nz <= 128) return fsm_solve_rows<2>(T, nz, nx, ld, si, sj, sl);
  return fsm_solve(T, nz, nx, ld, si, sj, sl);
}

}  // namespace

__global__ __launch_bounds__(64) void k_bet_propose(BetDev d, int t, int init, int c0, int cn) {
  const int lc = blockIdx.x * 64 + threadIdx.x;
  if (lc >= cn) return;
  const int c = c0 + lc;
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
__global__ __launch_bounds__(256) void k_bet_raster(BetDev d, int c0) {
  const int c = c0 + blockIdx.y;
  if (!d.valid[c]) return;
  const int nz = d.nz, nx = d.nx, ld = bet_ld(nz, nx);
  const int q = blockIdx.x * 256 + threadIdx.x;
  if (q >= bet_grid_entries(nz, nx)) return;
  const int e = q - kBetGuard, i = e / ld, j = e - (e / ld) * ld;
  BetSlowness out{0.0f, 0.0f};  // guards and pads
  if (e >= 0 && i < nz && j < nx) {
    const double z = (double)i * d.h, x = (double)j * d.h;
    const double* pz = d.pz + (size_t)c * d.k_max;
    const double* px = d.px + (size_t)c * d.k_max;
    const int kk = d.pk[c];
    int best = 0;
    double bd = INFINITY;
    for (int k = 0; k < kk; ++k) {
      const double dz = z - pz[k], dx = x - px[k];
      const double d2 = dz * dz + dx * dx;
      if (d2 < bd) {
        bd = d2;
        best = k;
      }
    }
    out = slowness_h((float)(1.0 / d.pv[(size_t)c * d.k_max + best]), (float)d.h);
  }
  d.node[(size_t)c * bet_grid_entries(nz, nx) + q] = out;
}

// travel times of the proposal of chain c0 + lc from source e.  Blocks map
// to (lc, e) so that all of a chain's solves run on one XCD (blocks go to the
// XCDs in turn), whose L2 then holds that chain's node terms.
__global__ __launch_bounds__(64) void k_bet_eikonal(BetDev d, int c0, int cn) {
  extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
  const int xcd = blockIdx.x & 7, r = blockIdx.x >> 3;
  const int e = r % d.nsrc, lc = (r / d.nsrc) * 8 + xcd;
  if (lc >= cn) return;
  const int c = c0 + lc;
  if (!d.valid[c]) return;
  const int lane = threadIdx.x;
  const int nz = d.nz, nx = d.nx, ld = bet_ld(nz, nx);
  float* T = reinterpret_cast<float*>(smem) + kBetGuard;  // times, with guards
  const NodeSlowness sl{d.node + (size_t)c * bet_grid_entries(nz, nx) + kBetGuard};
  const int2 s = d.src[e];
  const int sweeps = fsm_solve_any(T, nz, nx, ld, s.x, s.y, sl);
  if (lane == 0) {
    if (sweeps < 0) atomicOr(d.flags, kBetNoConverge);
    atomicAdd(d.work + 2 * (size_t)c, 1ull);
    atomicAdd(d.work + 2 * (size_t)c + 1, (unsigned long long)(sweeps < 0 ? -sweeps : sweeps));
  }
  float* out = d.tt + ((size_t)c * d.nsrc + e) * d.nrec;
  for (int q = lane; q < d.nrec; q += 64) {
    const int2 m = d.rec[q];
    out[q] = T[m.x * ld + m.y];
  }
}

// misfit of the proposal and the Metropolis test (a workgroup per chain)
__global__ __launch_bounds__(256) void k_bet_accept(BetDev d, int init, int8_t* log_row, int c0, int slot) {
  __shared__ double red[256];
  __shared__ int s_acc;
  const int c = c0 + blockIdx.x, tid = threadIdx.x;
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
  if (slot >= 0) {  // a sampling iteration: the chain's state after this decision
    __syncthreads();
    const int k = d.k[c], K = d.k_max;
    const size_t o = ((size_t)slot * d.chains + c) * K;
    if (tid == 0) d.snap_k[(size_t)slot * d.chains + c] = k;
    for (int q = tid; q < k; q += 256) {
      d.snap_z[o + q] = d.z[(size_t)c * K + q];
      d.snap_x[o + q] = d.x[(size_t)c * K + q];
      d.snap_v[o + q] = d.v[(size_t)c * K + q];
    }
  }
}

// pooled FP64 Welford of every chain's current velocity grid (chains in order)
// velocity of every chain's recorded state at every node (a thread per node
// and chain): the nearest nucleus, ties to the lowest index
__global__ __launch_bounds__(256) void k_bet_sample_vel(BetDev d, int slot) {
  const int n = d.nz * d.nx, c = blockIdx.y;
  const int p = blockIdx.x * 256 + threadIdx.x;
  if (p >= n) return;
  const int i = p / d.nx, j = p - (p / d.nx) * d.nx;
  const double z = (double)i * d.h, x = (double)j * d.h;
  const size_t o = (size_t)slot * d.chains + c;
  const double* zs = d.snap_z + o * d.k_max;
  const double* xs = d.snap_x + o * d.k_max;
  const int k = d.snap_k[o];
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
  d.sample_v[(size_t)c * n + p] = d.snap_v[o * d.k_max + best];
}

// pooled FP64 Welford update of every node with the chains' velocities, in
// chain order (a thread per node)
__global__ __launch_bounds__(256) void k_bet_sample(BetDev d) {
  const int n = d.nz * d.nx;
  const int p = blockIdx.x * 256 + threadIdx.x;
  if (p >= n) return;
  double mean = d.mean[p], m2 = d.m2[p];
  int32_t cnt = d.count[p];
  for (int c = 0; c < d.chains; ++c) {
    const double v = d.sample_v[(size_t)c * n + p];
    ++cnt;
    const double delta = v - mean;
    mean += delta / (double)cnt;
    m2 += delta * (v - mean);
  }
  d.mean[p] = mean;
  d.m2[p] = m2;
  d.count[p] = cnt;
}

// node terms of a velocity grid (a thread per entry of the padded layout;
// guards and pads: 0), flagging any node whose h / v leaves the range the
// solves' square root is exact in (velocities not positive and finite
// included)
__global__ __launch_bounds__(256) void k_grid_terms(const float* vel, int nz, int nx, float h, BetSlowness* node,
                                                    uint32_t* flags) {
  const int ld = bet_ld(nz, nx);
  const int q = blockIdx.x * 256 + threadIdx.x;
  if (q >= bet_grid_entries(nz, nx)) return;
  const int e = q - kBetGuard, i = e / ld, j = e - (e / ld) * ld;
  BetSlowness out{0.0f, 0.0f};
  if (e >= 0 && i < nz && j < nx) {
    out = slowness_h((float)(1.0 / (double)vel[i * nx + j]), h);
    if (!(out.sh >= kBetShMin && out.sh <= kBetShMax)) atomicOr(flags, kBetBadSlowness);
  }
  node[q] = out;
}

// travel times of one velocity grid from source blockIdx.x (the node terms
// from k_grid_terms; nothing is solved if it flagged a node)
__global__ __launch_bounds__(64) void k_eikonal_grid(const BetSlowness* node, int nz, int nx, const int2* src,
                                                     const int2* rec, int nrec, float* tt, uint32_t* flags) {
  extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
  if (__hip_atomic_load(flags, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) & kBetBadSlowness) return;
  const int e = blockIdx.x, lane = threadIdx.x, ld = bet_ld(nz, nx);
  float* T = reinterpret_cast<float*>(smem) + kBetGuard;  // times, with guards
  const int2 s = src[e];
  const NodeSlowness sl{node + kBetGuard};
  const int sweeps = fsm_solve_any(T, nz, nx, ld, s.x, s.y, sl);
  if (sweeps < 0 && lane == 0) atomicOr(flags, kBetNoConverge);
  for (int r = lane; r < nrec; r += 64) {
    const int2 q = rec[r];
    tt[(size_t)e * nrec + r] = T[q.x * ld + q.y];
  }
}

// Velocity grid [nz][nx] of chain c's current model sampled at nodes
// (i h, j h): the nearest nucleus's velocity (FP64 distances, ties to the
// lowest index), as float.
__global__ __launch_bounds__(256) void k_bet_model(BetDev d, int c, int nz, int nx, double h, float* vel) {
  const int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (p >= (int64_t)nz * nx) return;
  const int i = (int)(p / nx), j = (int)(p - (p / nx) * nx);
  const double z = (double)i * h, x = (double)j * h;
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
  vel[p] = (float)d.v[(size_t)c * d.k_max + best];
}

hipError_t launch_bet_model(const BetDev& d, int c, int nz, int nx, double h, float* vel, hipStream_t s) {
  const int64_t n = (int64_t)nz * nx;
  k_bet_model<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(d, c, nz, nx, h, vel);
  return hipGetLastError();
}

// Counts the float bit patterns in [lo, hi) where sqrt_rn differs from the
// correctly rounded square root (a thread per 256 patterns).
__global__ __launch_bounds__(256) void k_sqrt_check(uint32_t lo, uint32_t hi, unsigned long long* bad) {
  const uint64_t b0 = (uint64_t)lo + ((uint64_t)blockIdx.x * 256 + threadIdx.x) * 256;
  unsigned long long nb = 0;
  for (uint32_t q = 0; q < 256; ++q) {
    const uint64_t b = b0 + q;
    if (b >= hi) break;
    const float x = __uint_as_float((uint32_t)b);
    nb += __float_as_uint(sqrt_rn(x)) != __float_as_uint(sqrtf(x));
  }
  if (nb) atomicAdd(bad, nb);
}

hipError_t launch_sqrt_check(uint32_t lo, uint32_t hi, unsigned long long* bad, hipStream_t s) {
  const uint64_t threads = ((uint64_t)(hi - lo) + 255) / 256;
  k_sqrt_check<<<(unsigned)((threads + 255) / 256), 256, 0, s>>>(lo, hi, bad);
  return hipGetLastError();
}

static size_t lds_bet(int nz, int nx) { return bet_lds_sampler(nz, nx); }
static size_t lds_grid(int nz, int nx) { return bet_lds_grid(nz, nx); }

hipError_t launch_bet_propose(const BetDev& d, int t, int init, int c0, int cn, hipStream_t s) {
  k_bet_propose<<<(cn + 63) / 64, 64, 0, s>>>(d, t, init, c0, cn);
  return hipGetLastError();
}

hipError_t launch_bet_raster(const BetDev& d, int c0, int cn, hipStream_t s) {
  const int m = bet_grid_entries(d.nz, d.nx);
  k_bet_raster<<<dim3((m + 255) / 256, cn), 256, 0, s>>>(d, c0);
  return hipGetLastError();
}

hipError_t launch_bet_eikonal(const BetDev& d, int c0, int cn, hipStream_t s) {
  const int n = d.nz * d.nx;
  const size_t lds = lds_bet(d.nz, d.nx);
  if (n > kBetMaxNodes || d.k_max > kBetMaxCells || lds > kBetMaxLds) return hipErrorInvalidValue;
  if (lds > 65536) {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_bet_eikonal),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  // 8 blocks (one per XCD) per source and group of 8 chains
  k_bet_eikonal<<<8 * d.nsrc * ((cn + 7) / 8), 64, lds, s>>>(d, c0, cn);
  return hipGetLastError();
}

hipError_t launch_bet_accept(const BetDev& d, int init, int8_t* log_row, int c0, int cn, int slot, hipStream_t s) {
  k_bet_accept<<<cn, 256, 0, s>>>(d, init, log_row, c0, slot);
  return hipGetLastError();
}

hipError_t launch_bet_sample(const BetDev& d, int slot, hipStream_t s) {
  const int n = d.nz * d.nx;
  k_bet_sample_vel<<<dim3((n + 255) / 256, d.chains), 256, 0, s>>>(d, slot);
  k_bet_sample<<<(n + 255) / 256, 256, 0, s>>>(d);
  return hipGetLastError();
}

hipError_t launch_eikonal_grid(const float* vel, int nz, int nx, float h, const int2* src, int nsrc,
                               const int2* rec, int nrec, float* tt, uint32_t* flags, BetSlowness* node,
                               hipStream_t s) {
  const int n = nz * nx;
  const size_t lds = lds_grid(nz, nx);
  if (n > kBetMaxNodes || lds > kBetMaxLds) return hipErrorInvalidValue;
  if (lds > 65536) {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_eikonal_grid),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  const int m = bet_grid_entries(nz, nx);
  k_grid_terms<<<(m + 255) / 256, 256, 0, s>>>(vel, nz, nx, h, node, flags);
  k_eikonal_grid<<<nsrc, 64, lds, s>>>(node, nz, nx, src, rec, nrec, tt, flags);
  return hipGetLastError();
}

}  // namespace rtm
