// rtm_bet.h -- device state and launchers of the Stage-1 sampler
// (rtm_bet.hip), shared with the host runtime (rtm_runtime.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace rtm {

constexpr int kBetMaxCells = 64;     // Voronoi nuclei per model
constexpr int kBetMaxChains = 65535; // chains per sampler (a launch dimension)
constexpr int kBetMaxNodes = 40000;  // Eikonal grid nodes (a solve's times in LDS: 4 B per node)
// Fast sweeps before giving up: the solvers stop at the first sweep that
// changes nothing, and a quiet sweep within 1021 sweeps is exactly a quiet
// whole pass (four orderings) within 256 passes.
constexpr int kBetMaxSweeps = 1021;
// chain states recorded per sampling iteration before they are pooled
constexpr int kBetSnapSlots = 16;

// Layout of the grids a travel-time solve reads (times in LDS, the node
// slowness in global memory).  Up to 128 rows (the row-per-lane sweeps, one
// or two rows per lane) the row stride ld leaves at least one pad column
// after each row, and is even: a step touches addresses l (ld - 1) + c or
// l (ld + 1) + c over the lanes l, and an odd multiplier sends the lanes to
// distinct LDS banks.  kBetGuard entries before row 0, one more row after
// the last (+inf in the times: the row below the grid) and kBetTail entries
// after that keep the reads of lanes outside the grid in bounds (a lane's
// second row starts 127 columns before the grid at most).
constexpr int kBetGuard = 132, kBetTail = 132;
__host__ __device__ inline int bet_ld(int nz, int nx) { return nz <= 128 ? (nx + 1) + ((nx + 1) & 1) : nx; }
__host__ __device__ inline int bet_grid_entries(int nz, int nx) {
  return kBetGuard + (nz + 1) * bet_ld(nz, nx) + kBetTail;
}
// LDS of one solve: its times; a grid must fit the CU's 160 KB
constexpr size_t kBetMaxLds = 163840;
__host__ __device__ inline size_t bet_lds_bytes(int nz, int nx) {
  return ((size_t)bet_grid_entries(nz, nx) * 4 + 15) & ~(size_t)15;
}
__host__ __device__ inline size_t bet_lds_sampler(int nz, int nx) { return bet_lds_bytes(nz, nx); }
__host__ __device__ inline size_t bet_lds_grid(int nz, int nx) { return bet_lds_bytes(nz, nx); }

// sh = slowness * h and q2 = sh sh + sh sh of a node, in single precision:
// the two terms of the Godunov update that depend on the node alone
struct BetSlowness {
  float sh, q2;
};

// error bits raised by the kernels in BetDev::flags
constexpr uint32_t kBetNoConverge = 1u;  // a travel-time solve hit the sweep limit
constexpr uint32_t kBetBadSlowness = 2u; // a node's slowness * h outside [kBetShMin, kBetShMax]

// Range of sh = slowness * h (s, single precision) in which the Godunov
// update is evaluated: its square root then only sees normal arguments.
constexpr float kBetShMin = 1e-9f, kBetShMax = 1e18f;

struct BetDev {
  // grid, data
  int32_t nz, nx, nsrc, nrec;
  double h;  // node spacing (m); the travel-time sweeps use it rounded to float
  int32_t chains, k_min, k_max, k_init;
  int32_t burn_in, thin, pad0, pad1;
  double v_min, v_max, p_birth, p_death, move_dz, move_dx, sigma;
  uint64_t seed;
  const int2* src;      // [nsrc] (iz, ix)
  const int2* rec;      // [nrec]
  const float* tt_obs;  // [nsrc][nrec]
  // chain state [chains][k_max] / [chains]
  int32_t* k;
  double *z, *x, *v, *misfit;
  // proposal
  int32_t *pk, *valid, *ptype;
  double *pz, *px, *pv, *ua;
  BetSlowness* node;  // [chains][bet_grid_entries]: the proposal's node slowness terms (guards and pads: 0)
  float* tt;       // [chains][nsrc][nrec] travel times of the proposal
  // counters [chains][3] (birth, death, move); work [chains][2]: travel-time
  // solves, fast sweeps (one ordering each)
  int64_t *proposed, *accepted;
  unsigned long long* work;
  // chain states at sampling iterations: snap_k [kBetSnapSlots][chains],
  // snap_z/x/v [kBetSnapSlots][chains][k_max]
  int32_t* snap_k;
  double *snap_z, *snap_x, *snap_v;
  double* sample_v;  // [chains][nz*nx] velocities of one snapshot slot
  // pooled post-burn-in statistics of the velocity grid
  double *mean, *m2;
  int32_t* count;
  uint32_t* flags;
};

// Each step of an iteration works on the chains c0 .. c0 + cn - 1.
hipError_t launch_bet_propose(const BetDev& d, int t, int init, int c0, int cn, hipStream_t s);
hipError_t launch_bet_raster(const BetDev& d, int c0, int cn, hipStream_t s);
hipError_t launch_bet_eikonal(const BetDev& d, int c0, int cn, hipStream_t s);
// log_row (nullable): [chains] outcome of this iteration (-1 invalid, 0 rejected, 1 + move type);
// slot >= 0: also record the chains' states in snapshot slot `slot`
hipError_t launch_bet_accept(const BetDev& d, int init, int8_t* log_row, int c0, int cn, int slot, hipStream_t s);
// adds the states of snapshot slot `slot` (every chain, in order) to the pooled statistics
hipError_t launch_bet_sample(const BetDev& d, int slot, hipStream_t s);
// velocity grid [nz][nx] (float) of chain c's current model at nodes (i h, j h)
hipError_t launch_bet_model(const BetDev& d, int c, int nz, int nx, double h, float* vel, hipStream_t s);
// mismatches (added to *bad) of the solver's square root against the
// correctly rounded one over the float bit patterns [lo, hi), lo < hi
hipError_t launch_sqrt_check(uint32_t lo, uint32_t hi, unsigned long long* bad, hipStream_t s);
// travel times of one velocity grid (m/s) for every source: tt [nsrc][nrec];
// node: scratch of bet_grid_entries(nz, nx) node terms
hipError_t launch_eikonal_grid(const float* vel, int nz, int nx, float h, const int2* src, int nsrc,
                               const int2* rec, int nrec, float* tt, uint32_t* flags, BetSlowness* node,
                               hipStream_t s);

}  // namespace rtm
