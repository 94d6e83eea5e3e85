// rtm_internal.h -- device-side job and tile descriptors shared by the HIP
// kernels (rtm_kernels.hip) and the host runtime (rtm_runtime.hip).
//
// Memory layout of a job (all in the context arena, HBM):
//   A job runs on its own padded grid: the physical aperture window
//   (nz rows x nx columns) plus nb sponge cells on each side, nzp = nz + 2nb
//   rows by nxp = nx + 2nb columns.  Each wavefield array is stored row-major
//   with a row pitch `pitch` = roundup(nxp + 4, 64) floats (256-byte rows), so
//   every row starts on a 256-byte boundary and ends with >= 4 zero columns
//   that double as the left/right ghost cells of the 8th-order stencil.
//   Nine zero rows precede row 0 and the allocation extends to
//   roundup(nzp, 64) + 9 rows, which covers the top/bottom ghost rows and the
//   8-cell halo a two-step tile reads.  Points outside [0,nzp) x [0,nxp) are
//   zero and are never written.
//   Time level n of a wavefield lives in buffer n & 3 of four, so a launch
//   that advances two steps never overwrites a level a neighbouring tile
//   still reads.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace rtm {

constexpr int kTileX = 64;       // tile width: one 64-lane wavefront per row
constexpr int kHalo = 4;         // stencil radius
constexpr int kLdsW = kTileX + 2 * kHalo;  // 72 floats per LDS row
constexpr int kTopRows = 9;      // zero rows before padded row 0 (two-step halo + 1)
constexpr int kRedBlocks = 1024;  // workgroup partials of the maps' two-stage reductions
constexpr int kRowAlign = 64;    // rows rounded up to the tallest tile
constexpr int kThreads = 256;    // 4 wavefronts per workgroup
constexpr int kMaxSlots = 64;    // partial max-abs slots per stored step (spreads the atomics)
constexpr int kTileX2 = 56;      // output width of a two-step tile: its first step covers
                                 // 56 + 2 * 4 = 64 columns, one wavefront

enum JobMode : int32_t { kModeModel = 0, kModeStore = 1, kModeRecon = 2, kModeBorn = 3 };
enum PhaseSet : int { kPhFwd = 1, kPhBwd = 2, kPhAny = 3, kPhBorn = 4 };

// Device descriptor of one job.  Read-only for the step kernel except the
// arrays it points to.
struct alignas(16) DevJob {
  int32_t nzp, nxp, pitch, nz;     // padded rows/cols, row pitch, physical rows
  int32_t nx, nb, nt, mode;        // physical cols, sponge width, time samples, JobMode
  int32_t snap_dtype, snap_stride, flags, nsteps;  // snapshots; RTM_IMG_*; steps of the job
  int32_t src_z, src_x, nrec, ring_len;            // padded source node; receivers; ring size
  int32_t start_tick, tiles_x, tiles_z, tiles_x2;  // first global tick; tile grid; two-step tile columns
  float inv_cell, c0, kfac;        // 1/(dx dz); a0 (1/dz^2 + 1/dx^2); imaging weight k
  int32_t two_step;                // job whose pairable steps run in two-step launches
  float cz[4], cx[4];              // a_k / dz^2, a_k / dx^2, k = 1..4
  const float* c;                  // v^2 dt^2, padded grid (field layout)
  const float* gz;                 // sponge profile per padded row [nzp]
  const float* gx;                 // sponge profile per padded column [nxp]
  float* f[4];                     // source wavefield: S^n / u^n in f[n & 3]
  float* r[4];                     // receiver wavefield R^m in r[m & 3] (Born: scattered field du^n)
  const float* wavelet;            // [nt]
  const float* data;               // [nt][nrec] injected at receivers (migration)
  float* traces;                   // [nt][nrec] sampled at receivers (modelling)
  void* snap;                      // [nsnap][nz][pitch] stored S^n at padded columns (store mode)
  float* ring;                     // [nt][ring_len] boundary ring of S^n (reconstruct)
  uint32_t* maxbits;               // [nt][kMaxSlots] partial max |u^n| over the physical window (float bits)
  float* image;                    // [nz][pitch]: physical (pz, px) at pz * pitch + px + nb
                                   // (Born modelling: the perturbation m, same layout)
  float* illum;                    // same layout, or null
  const int2* recs;                // receivers sorted by tile: {local index, receiver id}
  uint32_t* health;                // [1] bit 0: a non-finite value was seen
};

// One tile of one job: rows [z0, z0+TZ), columns [x0, x0+64) of its padded grid
// (columns [x0, x0+56) for a two-step tile).
struct alignas(16) Tile {
  int32_t job, z0, x0, rec_begin;
  int32_t rec_count, pad0, pad1, pad2;
};

// Launch control block for graph-replayed launches: a launch's global step
// is ctl->tick + its own offset; k_advance moves ctl->tick after each group.
// A launch that passes ntiles < 0 takes its tiles from the control block:
// ntiles_* tiles from index base_* of the table it is given (the batched
// path moves the range from one group of shots to the next; the serving
// engine keeps the bases at 0).
struct alignas(16) StepCtl {
  int32_t tick;       // global step base; job step = tick + offset - start_tick
  int32_t ntiles_fw;  // two-step tiles of the forward table
  int32_t ntiles;     // one-step tiles
  int32_t ntiles_bw;  // two-step tiles of the backward table
  int32_t base_fw, base, base_bw;  // first tile of each range
  int32_t pad_;
};

// Does a two-step launch advance a reconstruct- or store-mode job from its
// step s (s even for the jobs that take two-step launches) through s + 1?
// Forward steps s and s + 1 both before the backward phase, or backward
// levels m = nt - 1 - (s - nf) and m - 1 with 1 <= m <= nt - 3 (levels
// nt - 1 and nt - 2 are imaged without reconstruction, and a last single
// level runs alone).  A store-mode job also keeps its last forward level
// nt - 2 out of a pair's first step: the snapshot of that level is written
// by the launch after the one that computes it (its 16-bit scale needs the
// whole level's maximum), and no forward launch follows.  The one-step
// launches of the serving engine skip exactly these steps of a job marked
// two_step; the two-step kernel takes exactly these.
__host__ __device__ inline bool two_step_pair(int s, int nt, int nsteps, int mode) {
  const int nf = nt - 1;
  if (s < 0 || s + 1 >= nsteps) return false;
  if (s + 1 < nf) return mode != kModeStore || s + 2 < nf;
  if (s < nf) return false;
  const int m = nt - 1 - (s - nf);
  return m <= nt - 3 && m >= 1;
}

inline int64_t field_rows(int nzp) { return ((nzp + kRowAlign - 1) / kRowAlign) * kRowAlign + 2 * kTopRows; }
inline int32_t field_pitch(int nxp) { return ((nxp + kHalo + 63) / 64) * 64; }
inline int64_t field_floats(int nzp, int nxp) { return field_rows(nzp) * field_pitch(nxp); }
inline int64_t field_origin(int nxp) { return (int64_t)kTopRows * field_pitch(nxp); }
inline int32_t ring_len_of(int nz, int nx) { return 8 * (nz + nx - 8); }

// ---- kernel launchers (rtm_kernels.hip) ----
// ntiles < 0: the launch reads the tile count from the control block (its
// grid is sized for grid_tiles).  skip_pairs: leave the steps of jobs marked
// two_step that a two-step launch takes (serving engine).
hipError_t launch_step(int tz, int phases, const DevJob* jobs, const Tile* tiles, int ntiles,
                       int grid_tiles, const StepCtl* ctl, int use_ctl_tick, int tick_off,
                       hipStream_t s, int skip_pairs = 0);
// store: the launch covers store-mode jobs (else reconstruct-mode jobs)
hipError_t launch_step2(int tz, int phases, int store, const DevJob* jobs, const Tile* tiles, const int2* recs2,
                        int ntiles, int grid_tiles, const StepCtl* ctl, int use_ctl_tick, int tick_off,
                        hipStream_t s);
hipError_t launch_advance(StepCtl* ctl, int k, hipStream_t s);
hipError_t launch_set_ctl(StepCtl* ctl, StepCtl v, hipStream_t s);  // *ctl = v, in stream order
hipError_t launch_prep(const float* vel, int model_nx, int ix0, const DevJob* host_job,
                       float* c, float* gz, float* gx, float dt, float sponge_a, hipStream_t s);
hipError_t launch_vmax(const float* vel, int nz, int model_nx, int ix0, int width,
                       uint32_t* out_bits, hipStream_t s);
hipError_t launch_stack(float* dst, int dst_nx, int ix0, const float* img, int img_pitch, int nz,
                        int width, hipStream_t s);
hipError_t launch_copy_phys(float* dst, const float* field, int nz, int nx, int nb, int pitch,
                            hipStream_t s);
hipError_t launch_nonfinite(const float* img, int pitch, int nz, int width, uint32_t* flag, hipStream_t s);
// scratch: at least kRedBlocks + 1 floats of device memory
hipError_t launch_normalize(const float* img, const float* illum, int n, float eps_rel, float* out,
                            float* scratch, hipStream_t s);
hipError_t launch_chan_merge(double* mean_a, double* m2_a, int32_t* n_a, const double* mean_b,
                             const double* m2_b, const int32_t* n_b, int64_t n, hipStream_t s);
hipError_t launch_fill_u32(uint32_t* p, uint32_t v, int64_t n, hipStream_t s);
hipError_t launch_welford(double* mean, double* m2, int32_t* count, int nx_model, const float* img,
                          int img_pitch, int nz, int width, int ix0, hipStream_t s);
hipError_t launch_stats_out(const double* mean, const double* m2, const int32_t* count, int64_t n,
                            double* mean_out, double* std_out, int32_t* count_out, hipStream_t s);
// scratch: at least 2 kRedBlocks + 2 doubles of device memory
hipError_t launch_confidence(const double* sd, const int32_t* count, int n, int min_count,
                             double* out, double* scratch, hipStream_t s);
hipError_t launch_ratio(const double* sd, const double* mean, int n, double eps, double* out,
                        hipStream_t s);
hipError_t launch_lapfilter(const float* img, int nz, int nx, float dz, float dx, float* out,
                            hipStream_t s);

}  // namespace rtm
