// rtm_runtime.hip -- host runtime and C ABI of the RTM library (include/rtm.h).
//
// Pieces:
//   Arena      first-fit sub-allocator over the caller's device buffer, with
//              frees deferred until the stream work that used the blocks is done
//   HostJob    one migration / modelling job: geometry, arena blocks, tiles,
//              device descriptor (rtm_internal.h)
//   plain      rtm_propagate / rtm_migrate_shot: one kernel launch per step
//   batched    rtm_migrate_batch: all shots of a model advance in each launch,
//              launches replayed from a captured hipGraph, device-side tick
//   ensemble   rtm_ensemble_*: a scheduler thread admits queued jobs by arena
//              footprint, runs every active job (any phase, any size) in the
//              same launches, finalises finished jobs (stack, FP64 Welford) and
//              admits new ones between graph replays (continuous batching)
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>
#include <stdarg.h>
#include <string.h>

#include <algorithm>
#include <array>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstdio>
#include <cstdlib>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "../../include/rtm.h"
#include "rtm_arena.h"
#include "rtm_bet.h"
#include "rtm_codec.h"
#include "rtm_internal.h"
#include "rtm_sched.h"
#include "rtm_zfp.h"

#include <rocprofiler-sdk-roctx/roctx.h>

using namespace rtm;

// Named ranges for profiler timelines (rocprofv3 --marker-trace): the
// scheduler's admission, launch and finalisation, and the batched phases.
struct RoctxRange {
  explicit RoctxRange(const char* name) { roctxRangePushA(name); }
  ~RoctxRange() { roctxRangePop(); }
  RoctxRange(const RoctxRange&) = delete;
  RoctxRange& operator=(const RoctxRange&) = delete;
};
using rtm::Arena;

// ===========================================================================
// errors
// ===========================================================================
static thread_local std::string g_last_error;

static int fail(int code, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
static int fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return code;
}

#define HIP_OK(expr)                                                                       \
  do {                                                                                     \
    hipError_t e_ = (expr);                                                                \
    if (e_ != hipSuccess)                                                                  \
      return fail(RTM_E_DEVICE, "%s failed: %s (%s:%d)", #expr, hipGetErrorString(e_),     \
                  __FILE__, __LINE__);                                                     \
  } while (0)

static double now_s() {
  using namespace std::chrono;
  return duration<double>(steady_clock::now().time_since_epoch()).count();
}

using rtm::align256;

// 8th-order central weights of the 2nd derivative; a0 + 2 sum a_k = 0.
static const double kA[5] = {-205.0 / 72.0, 8.0 / 5.0, -1.0 / 5.0, 8.0 / 315.0, -1.0 / 560.0};

// ===========================================================================
// Arena
// ===========================================================================
struct Block {
  void* p = nullptr;
  size_t n = 0;
};

// Blocks (and host staging, graphs) released once an event has completed.
struct Deferred {
  hipEvent_t ev = nullptr;
  std::vector<Block> blocks;
  std::vector<std::shared_ptr<void>> keep;  // host-side objects kept alive
  std::vector<hipGraphExec_t> graphs;
};

// ===========================================================================
// Jobs
// ===========================================================================
struct JobGeom {
  int nz = 0, model_nx = 0, ix0 = 0, width = 0, nb = 0, nt = 0;
  float dz = 0, dx = 0, dt = 0, sponge_a = 0;
  int mode = kModeModel;
  int snap_dtype = 0, snap_stride = 1;
  uint32_t flags = 0;
  int nrec = 0;
  int nbuf = 2;  // buffers per wavefield: 4 for jobs that take two-step launches
};

static int snap_bytes(int dtype) { return dtype == RTM_SNAP_FP32 ? 4 : 2; }
static int nsnap_of(int nt, int k) { return (nt - 2) / k + 1; }

struct Footprint {
  size_t field = 0, total = 0;
};

static Footprint footprint(const JobGeom& g) {
  Footprint f;
  const int nzp = g.nz + 2 * g.nb, nxp = g.width + 2 * g.nb;
  f.field = align256((size_t)field_floats(nzp, nxp) * 4);
  size_t t = 0;
  t += f.field;                                  // c
  t += g.nbuf * f.field;                             // f
  if (g.mode != kModeModel) t += g.nbuf * f.field;   // r
  t += align256((size_t)nzp * 4) + align256((size_t)nxp * 4);
  if (g.mode != kModeModel) {
    t += align256((size_t)g.nz * field_pitch(nxp) * 4);  // image (field-aligned rows)
    if (g.flags & RTM_IMG_ILLUM) t += align256((size_t)g.nz * field_pitch(nxp) * 4);
  }
  if (g.mode == kModeRecon) t += align256((size_t)g.nt * ring_len_of(g.nz, g.width) * 4);
  if (g.mode == kModeStore)
    t += align256((size_t)nsnap_of(g.nt, g.snap_stride) * g.nz * field_pitch(nxp) * snap_bytes(g.snap_dtype));
  t += align256((size_t)g.nt * kMaxSlots * 4);   // maxbits
  t += align256((size_t)std::max(g.nrec, 1) * 8);  // receivers
  t += 256;                                      // health
  f.total = t;
  return f;
}

// Arena bytes of a job's medium (c and the two sponge profiles).
static size_t medium_bytes(const JobGeom& g) {
  const int nzp = g.nz + 2 * g.nb, nxp = g.width + 2 * g.nb;
  return footprint(g).field + align256((size_t)nzp * 4) + align256((size_t)nxp * 4);
}

struct HostJob {
  JobGeom g;
  DevJob d{};
  std::vector<Tile> tiles;       // job-local (job field set when a table is built)
  std::vector<int2> recs;        // sorted by tile
  std::vector<Block> blocks;     // arena blocks of the job's working set
  Block image_blk;               // the per-job image (kept after the job for polling)
  uint64_t updates = 0, alg_bytes = 0;
  bool owns_medium = true;       // false: c and the sponge profiles are another job's
};

static void count_work(HostJob& j) {
  const JobGeom& g = j.g;
  const uint64_t Npad = (uint64_t)(g.nz + 2 * g.nb) * (g.width + 2 * g.nb);
  const uint64_t Nph = (uint64_t)g.nz * g.width;
  const uint64_t ring = (uint64_t)ring_len_of(g.nz, g.width);
  const uint64_t nt = g.nt;
  // 16 B per update: read u^n, u^{n-1}, c, write u^{n+1}; c is counted only
  // for the job that owns it when several jobs read one medium.
  const uint64_t u = j.owns_medium ? 16 : 12;
  if (g.mode == kModeModel) {
    j.updates = (nt - 1) * Npad;
    j.alg_bytes = (nt - 1) * (Npad * u + (uint64_t)g.nrec * 4);
    return;
  }
  if (g.mode == kModeBorn) {  // background and scattered field: 2 x 16 B, c shared, + m
    j.updates = 2 * (nt - 1) * Npad;
    j.alg_bytes = (nt - 1) * (Npad * (u + 12) + Nph * 4 + (uint64_t)g.nrec * 4);
    return;
  }
  j.updates = (nt - 1) * Npad + nt * Npad;
  uint64_t b = (nt - 1) * Npad * u + nt * Npad * u + nt * (uint64_t)g.nrec * 4;
  if (g.mode == kModeRecon) {
    j.updates += (nt >= 2 ? nt - 2 : 0) * Nph;
    b += (nt - 1) * ring * 4;                 // ring save
    b += (nt - 2) * (Nph * 12 - ring * 4);    // reconstruct S (interior 12 B, ring 8 B)
    b += (nt - 1) * Nph * 8;                  // image read-modify-write
  } else {
    const uint64_t ns = nsnap_of(g.nt, g.snap_stride), sb = snap_bytes(g.snap_dtype);
    b += ns * Nph * (2 * sb + 8);             // snapshot write + read, image RMW
  }
  if (g.flags & RTM_IMG_ILLUM) b += (g.mode == kModeRecon ? (nt - 1) : nsnap_of(g.nt, g.snap_stride)) * Nph * 8;
  j.alg_bytes = b;
}

// ===========================================================================
// Context
// ===========================================================================
struct Model {
  int nz = 0, nx = 0;
  rtm_grid grid{};
  Block vel;
  float vmax = 0;
  // statistics (allocated on first use)
  Block mean, m2, count, stack;
};

// What the runtime keeps of a served job beside its JobBook entry (state,
// timestamps): the request and, once admitted, its working set.
struct EnsJob {
  uint64_t ticket = 0;
  rtm_job spec{};
  std::unique_ptr<HostJob> job;
  double gpu_ms = 0;  // share of the launch time of the cycles it ran in (by algorithmic bytes)
};

struct StatsAcc {
  int nz = 0, nx = 0;
  Block mean, m2, count;
};

// most streams the batched path alternates its shot groups over
constexpr int kMaxGroupStreams = 4;

struct rtm_ctx {
  int device = 0;
  hipStream_t stream = nullptr;        // caller's stream (plain / batched / copies)
  hipStream_t sched_stream = nullptr;  // scheduler thread's stream
  hipStream_t work_stream = nullptr;   // batched path (graph capture needs a non-null stream)
  // batched path: further streams that shot groups alternate over, with
  // the events that fork them from work_stream and join them back
  hipStream_t group_stream[kMaxGroupStreams - 1] = {};
  hipEvent_t ev_fork = nullptr, ev_join[kMaxGroupStreams - 1] = {};
  hipEvent_t ev_in = nullptr, ev_out = nullptr;
  // phase timing of the last batched call (events on work_stream)
  hipEvent_t ph_ev[3] = {nullptr, nullptr, nullptr};
  int ph_launches[2] = {0, 0};  // time steps of each phase
  int ph_steps_per_launch = 1;
  int ph_tz2[2] = {0, 0};  // two-step tile height of each phase (0: one step per launch)
  int ph_groups[2] = {1, 1};  // shot groups of each phase (a launch covers one group)
  int born_groups = 0;        // shot groups of the last Born batch
  uint64_t ph_bytes[2] = {0, 0};
  bool ph_valid = false;
  Arena arena;
  void* own_arena = nullptr;
  std::mutex defer_mu;
  std::deque<Deferred> deferred;
  int tile_z = 0;                      // tile height of the last tuned launch set
  std::mutex tune_mu;
  std::map<std::string, int> tune_cache;  // geometry key -> tile height
  bool tune_file_loaded = false;
  // counters
  std::atomic<uint64_t> steps_launched{0}, graph_replays{0}, grid_updates{0}, alg_bytes{0};

  // ensemble
  std::mutex mu;
  std::condition_variable cv, cv_done;
  std::map<int, Model> models;
  std::unordered_map<uint64_t, std::unique_ptr<EnsJob>> jobs;  // payloads, by ticket
  std::unique_ptr<JobBook> book;  // queue, admission order, states, timestamps
  bool stop = false;
  std::thread sched;
  bool sched_started = false;
  FILE* job_log = nullptr;  // RTM_LOG: one JSON line per job reaching a final state
  uint32_t* scratch_u32 = nullptr;     // small device scratch (vmax etc.)
  double* scratch_f64 = nullptr;      // partials of the maps' reductions (2 kRedBlocks + 2 doubles)
  // last codec call: HIP events around its kernel, algorithmic bytes, 1 encode / 2 decode
  hipEvent_t zc_ev[2] = {nullptr, nullptr};
  int zc_op = 0;
  uint64_t zc_bytes = 0;
  // last rtm_bet_run call: events around its last iteration (start, before and
  // after the travel-time launch, end)
  hipEvent_t bet_ev[4] = {nullptr, nullptr, nullptr, nullptr};
  bool bet_valid = false;
};

// ---- deferred frees ----
static void reap(rtm_ctx* ctx, bool wait_one) {
  std::vector<Deferred> done;
  {
    std::lock_guard<std::mutex> lk(ctx->defer_mu);
    while (!ctx->deferred.empty()) {
      Deferred& d = ctx->deferred.front();
      hipError_t q = hipEventQuery(d.ev);
      if (q == hipErrorNotReady) {
        if (!wait_one) break;
        (void)hipEventSynchronize(d.ev);
        wait_one = false;
      }
      done.push_back(std::move(d));
      ctx->deferred.pop_front();
    }
  }
  for (auto& d : done) {
    for (auto& b : d.blocks) ctx->arena.release(b.p, b.n);
    for (auto g : d.graphs) (void)hipGraphExecDestroy(g);
    (void)hipEventDestroy(d.ev);
  }
}

static int defer(rtm_ctx* ctx, hipStream_t s, Deferred&& d) {
  HIP_OK(hipEventCreateWithFlags(&d.ev, hipEventDisableTiming));
  HIP_OK(hipEventRecord(d.ev, s));
  std::lock_guard<std::mutex> lk(ctx->defer_mu);
  ctx->deferred.push_back(std::move(d));
  return RTM_OK;
}

static void* arena_alloc(rtm_ctx* ctx, size_t n) {
  reap(ctx, false);
  for (;;) {
    void* p = ctx->arena.alloc(n);
    if (p) return p;
    bool pending;
    {
      std::lock_guard<std::mutex> lk(ctx->defer_mu);
      pending = !ctx->deferred.empty();
    }
    if (!pending) return nullptr;
    reap(ctx, true);
  }
}

static bool alloc_block(rtm_ctx* ctx, std::vector<Block>& list, size_t n, void** out) {
  void* p = arena_alloc(ctx, n);
  if (!p) return false;
  list.push_back({p, align256(n)});
  *out = p;
  return true;
}

static void release_blocks(rtm_ctx* ctx, std::vector<Block>& list) {
  for (auto& b : list) ctx->arena.release(b.p, b.n);
  list.clear();
}

// ===========================================================================
// Validation
// ===========================================================================
extern "C" double rtm_cfl_limit(void) {
  // |symbol| of the 1-D stencil at the Nyquist wavenumber: -(a0 + 2 sum (-1)^k a_k)
  double s = kA[0];
  for (int k = 1; k <= 4; ++k) s += 2.0 * ((k & 1) ? -kA[k] : kA[k]);
  return 2.0 / sqrt(-s);
}

extern "C" double rtm_cfl_number(float v_max, float dt, float dz, float dx) {
  return (double)v_max * dt * sqrt(1.0 / ((double)dx * dx) + 1.0 / ((double)dz * dz));
}

static int check_grid(const rtm_grid* g) {
  if (!g) return fail(RTM_E_INVAL, "grid is NULL");
  if (g->nz < 1 || g->nx < 1) return fail(RTM_E_INVAL, "nz, nx must be >= 1 (got %d, %d)", g->nz, g->nx);
  if (g->nb < 0 || g->nb > 4096) return fail(RTM_E_INVAL, "nb out of range (%d)", g->nb);
  if (g->nt < 2) return fail(RTM_E_INVAL, "nt must be >= 2 (got %d)", g->nt);
  if (!(g->dz > 0) || !(g->dx > 0) || !(g->dt > 0))
    return fail(RTM_E_INVAL, "dz, dx, dt must be > 0");
  return RTM_OK;
}

static int check_cfl(float vmax, float dt, float dz, float dx) {
  if (!std::isfinite(vmax) || !(vmax > 0)) return fail(RTM_E_NONFINITE, "velocity max is %g", (double)vmax);
  double cn = rtm_cfl_number(vmax, dt, dz, dx), lim = rtm_cfl_limit();
  if (cn > lim)
    return fail(RTM_E_CFL, "Courant number %.5f exceeds the stability limit %.5f (v_max %.1f)", cn, lim,
                (double)vmax);
  return RTM_OK;
}

static int device_vmax(rtm_ctx* ctx, hipStream_t s, const float* vel, int nz, int model_nx, int ix0,
                       int width, float* out) {
  HIP_OK(hipMemsetAsync(ctx->scratch_u32, 0, 4, s));
  HIP_OK(launch_vmax(vel, nz, model_nx, ix0, width, ctx->scratch_u32, s));
  uint32_t bits = 0;
  HIP_OK(hipMemcpyAsync(&bits, ctx->scratch_u32, 4, hipMemcpyDeviceToHost, s));
  HIP_OK(hipStreamSynchronize(s));
  memcpy(out, &bits, 4);
  return RTM_OK;
}

// ===========================================================================
// Job construction
// ===========================================================================
static int env_tz() {
  const char* e = getenv("RTM_TILE_Z");
  if (!e) return 0;
  int tz = atoi(e);
  return (tz == 16 || tz == 32 || tz == 64) ? tz : 0;
}

// Tile height of the last launch set (forced or tuned).
static int choose_tz(rtm_ctx* ctx) { return ctx->tile_z ? ctx->tile_z : 16; }

// Every pointer a job's kernels dereference, for the job's mode, must be set
// before the job reaches a launch.
static int check_devjob(const DevJob& d) {
  const char* miss = nullptr;
  if (!d.c || !d.gz || !d.gx || !d.f[0] || !d.f[3] || !d.wavelet || !d.maxbits || !d.health) miss = "core arrays";
  else if (d.nrec > 0 && !d.recs) miss = "receiver table";
  else if ((d.mode == kModeModel || d.mode == kModeBorn) && d.nrec > 0 && !d.traces) miss = "traces";
  else if (d.mode != kModeModel && (!d.r[0] || !d.r[3] || !d.image)) miss = "second wavefield or image";
  else if ((d.mode == kModeStore || d.mode == kModeRecon) && d.nrec > 0 && !d.data) miss = "receiver data";
  else if (d.mode == kModeRecon && !d.ring) miss = "ring storage";
  else if (d.mode == kModeStore && !d.snap) miss = "snapshot storage";
  else if ((d.flags & RTM_IMG_ILLUM) && d.mode != kModeModel && !d.illum) miss = "illumination";
  if (miss) return fail(RTM_E_INVAL, "job descriptor is missing its %s", miss);
  if (d.src_z < 0 || d.src_z >= d.nzp || d.src_x < 0 || d.src_x >= d.nxp)
    return fail(RTM_E_INVAL, "job source outside its grid");
  return RTM_OK;
}

// The medium of a job: c = v^2 dt^2 on its padded window and the sponge
// profiles.  Two jobs over the same velocity array with equal window,
// depth, sponge and time step have identical media.
static bool same_medium(const JobGeom& a, const JobGeom& b) {
  return a.nz == b.nz && a.model_nx == b.model_nx && a.ix0 == b.ix0 && a.width == b.width && a.nb == b.nb &&
         a.dt == b.dt && a.sponge_a == b.sponge_a;
}

// Allocates the job's working set and enqueues its set-up on stream s.
// src/recs are in model coordinates.  On failure nothing stays allocated.
// `medium`, if given, is a job of the same velocity array whose medium is
// the same (same_medium): the new job reads that job's c and sponge
// profiles instead of building its own, so a batch of shots on one window
// streams one c through the caches.  The caller keeps `medium` alive as
// long as the new job.
static int build_job(rtm_ctx* ctx, hipStream_t s, const JobGeom& g, int tz, const float* vel,
                     const float* wavelet, rtm_point src, const rtm_point* recs, const float* data,
                     float* traces, HostJob& j, const HostJob* medium) {
  j.g = g;
  const int nzp = g.nz + 2 * g.nb, nxp = g.width + 2 * g.nb;
  DevJob& d = j.d;
  memset(&d, 0, sizeof d);
  d.nzp = nzp;
  d.nxp = nxp;
  d.pitch = field_pitch(nxp);
  d.nz = g.nz;
  d.nx = g.width;
  d.nb = g.nb;
  d.nt = g.nt;
  d.mode = g.mode;
  d.snap_dtype = g.snap_dtype;
  d.snap_stride = g.mode == kModeStore ? g.snap_stride : 1;
  d.flags = g.flags;
  d.nsteps = (g.mode == kModeModel || g.mode == kModeBorn) ? g.nt - 1 : 2 * g.nt - 1;
  d.src_z = src.iz + g.nb;
  d.src_x = src.ix - g.ix0 + g.nb;
  d.nrec = g.nrec;
  d.ring_len = ring_len_of(g.nz, g.width);
  d.start_tick = 0;
  d.tiles_x = (nxp + kTileX - 1) / kTileX;
  d.tiles_z = (nzp + tz - 1) / tz;
  d.tiles_x2 = (nxp + kTileX2 - 1) / kTileX2;
  d.inv_cell = (float)(1.0 / ((double)g.dx * g.dz));
  const double iz2 = 1.0 / ((double)g.dz * g.dz), ix2 = 1.0 / ((double)g.dx * g.dx);
  d.c0 = (float)(kA[0] * (iz2 + ix2));
  for (int k = 0; k < 4; ++k) {
    d.cz[k] = (float)(kA[k + 1] * iz2);
    d.cx[k] = (float)(kA[k + 1] * ix2);
  }
  d.kfac = (float)d.snap_stride;

  // ---- arena blocks ----
  Footprint fp = footprint(g);
  const size_t F = fp.field;
  void* p = nullptr;
  bool ok = true;
  auto A = [&](size_t n) -> void* {
    if (!ok) return nullptr;
    void* q = nullptr;
    if (!alloc_block(ctx, j.blocks, n, &q)) ok = false;
    return q;
  };
  const int64_t org = field_origin(nxp);
  float* cbuf = medium ? nullptr : static_cast<float*>(A(F));
  float* fb[4] = {nullptr, nullptr, nullptr, nullptr};
  float* rb[4] = {nullptr, nullptr, nullptr, nullptr};
  // Level n lives in buffer n & 3.  A job that only takes one-step launches
  // needs two buffers: slots 2 and 3 then alias slots 0 and 1.
  const int nbuf = g.nbuf == 4 ? 4 : 2;
  for (int k = 0; k < nbuf; ++k) fb[k] = static_cast<float*>(A(F));
  if (g.mode != kModeModel)
    for (int k = 0; k < nbuf; ++k) rb[k] = static_cast<float*>(A(F));
  float* gz = medium ? nullptr : static_cast<float*>(A((size_t)nzp * 4));
  float* gx = medium ? nullptr : static_cast<float*>(A((size_t)nxp * 4));
  float* illum = nullptr;
  const size_t img_bytes = (size_t)g.nz * field_pitch(nxp) * 4;
  if (g.mode != kModeModel && (g.flags & RTM_IMG_ILLUM)) illum = static_cast<float*>(A(img_bytes));
  float* ring = nullptr;
  void* snap = nullptr;
  if (g.mode == kModeRecon) ring = static_cast<float*>(A((size_t)g.nt * d.ring_len * 4));
  if (g.mode == kModeStore)
    snap = A((size_t)nsnap_of(g.nt, g.snap_stride) * g.nz * field_pitch(nxp) * snap_bytes(g.snap_dtype));
  uint32_t* maxbits = static_cast<uint32_t*>(A((size_t)g.nt * kMaxSlots * 4));
  int2* recd = static_cast<int2*>(A((size_t)std::max(g.nrec, 1) * 8));
  uint32_t* health = static_cast<uint32_t*>(A(256));
  float* image = nullptr;
  if (ok && g.mode != kModeModel) {
    image = static_cast<float*>(arena_alloc(ctx, img_bytes));
    if (!image) ok = false;
    else j.image_blk = {image, align256(img_bytes)};
  }
  (void)p;
  if (!ok) {
    release_blocks(ctx, j.blocks);
    return fail(RTM_E_NOMEM, "arena exhausted: job needs %zu bytes, arena %zu used of %zu", fp.total,
                ctx->arena.used(), ctx->arena.size());
  }
  d.c = medium ? medium->d.c : cbuf + org;
  d.gz = medium ? medium->d.gz : gz;
  d.gx = medium ? medium->d.gx : gx;
  for (int k = 0; k < 4; ++k) {
    const int b = k % nbuf;
    d.f[k] = fb[b] + org;
    if (rb[b]) d.r[k] = rb[b] + org;
  }
  d.wavelet = wavelet;
  d.data = data;
  d.traces = traces;
  d.snap = snap;
  d.ring = ring;
  d.maxbits = maxbits;
  d.image = image;
  d.illum = illum;
  d.recs = recd;
  d.health = health;
  if (int rc = check_devjob(d)) {
    release_blocks(ctx, j.blocks);
    if (j.image_blk.p) ctx->arena.release(j.image_blk.p, j.image_blk.n);
    j.image_blk = {};
    return rc;
  }

  // ---- tiles and receivers ----
  std::vector<std::pair<int, int2>> keyed;
  keyed.reserve(g.nrec);
  for (int r = 0; r < g.nrec; ++r) {
    int z = recs[r].iz + g.nb, x = recs[r].ix - g.ix0 + g.nb;
    int t = (z / tz) * d.tiles_x + x / kTileX;
    int local = (z % tz) * kTileX + (x % kTileX);
    keyed.push_back({t, make_int2(local, r)});
  }
  std::stable_sort(keyed.begin(), keyed.end(),
                   [](const std::pair<int, int2>& a, const std::pair<int, int2>& b) { return a.first < b.first; });
  j.recs.resize(g.nrec);
  for (int r = 0; r < g.nrec; ++r) j.recs[r] = keyed[r].second;
  j.tiles.clear();
  size_t kk = 0;
  for (int tzi = 0; tzi < d.tiles_z; ++tzi)
    for (int txi = 0; txi < d.tiles_x; ++txi) {
      int t = tzi * d.tiles_x + txi;
      Tile tl{};
      tl.job = 0;
      tl.z0 = tzi * tz;
      tl.x0 = txi * kTileX;
      tl.rec_begin = (int)kk;
      while (kk < keyed.size() && keyed[kk].first == t) ++kk;
      tl.rec_count = (int)kk - tl.rec_begin;
      j.tiles.push_back(tl);
    }

  // ---- device set-up ----
  const size_t fbytes = (size_t)field_floats(nzp, nxp) * 4;
  for (int k = 0; k < nbuf; ++k) {
    HIP_OK(hipMemsetAsync(fb[k], 0, fbytes, s));
    if (rb[k]) HIP_OK(hipMemsetAsync(rb[k], 0, fbytes, s));
  }
  if (cbuf) HIP_OK(hipMemsetAsync(cbuf, 0, fbytes, s));
  if (image) HIP_OK(hipMemsetAsync(image, 0, img_bytes, s));
  if (illum) HIP_OK(hipMemsetAsync(illum, 0, img_bytes, s));
  if (ring) HIP_OK(hipMemsetAsync(ring, 0, (size_t)d.ring_len * 4, s));  // ring of u^0 = 0
  HIP_OK(hipMemsetAsync(maxbits, 0, (size_t)g.nt * kMaxSlots * 4, s));
  HIP_OK(hipMemsetAsync(health, 0, 4, s));
  if (traces) HIP_OK(hipMemsetAsync(traces, 0, (size_t)g.nrec * 4, s));  // d[0] = u^0 = 0
  if (g.nrec) HIP_OK(hipMemcpyAsync(recd, j.recs.data(), (size_t)g.nrec * 8, hipMemcpyHostToDevice, s));
  if (cbuf) HIP_OK(launch_prep(vel, g.model_nx, g.ix0, &d, cbuf + org, gz, gx, g.dt, g.sponge_a, s));
  j.owns_medium = cbuf != nullptr;
  count_work(j);
  return RTM_OK;
}

// Validation of a job's geometry (model coordinates).
static int check_job(const JobGeom& g, rtm_point src, const rtm_point* recs) {
  if (g.width < 1 || g.ix0 < 0 || g.ix0 + g.width > g.model_nx)
    return fail(RTM_E_INVAL, "window [%d, %d) outside the model's %d columns", g.ix0, g.ix0 + g.width,
                g.model_nx);
  if (g.nt < 2) return fail(RTM_E_INVAL, "nt must be >= 2");
  // the step kernels address a field with 32-bit byte offsets
  const int64_t nzp = (int64_t)g.nz + 2 * g.nb, nxp = (int64_t)g.width + 2 * g.nb;
  if (nzp > (1 << 30) || nxp > (1 << 30) || field_floats((int)nzp, (int)nxp) >= ((int64_t)1 << 30))
    return fail(RTM_E_INVAL, "padded window %lld x %lld too large: a wavefield must hold fewer than 2^30 floats",
                (long long)nzp, (long long)nxp);
  if (g.mode == kModeRecon && (g.nz < 9 || g.width < 9))
    return fail(RTM_E_INVAL, "reconstruct mode needs a window of at least 9 x 9 (got %d x %d)", g.nz, g.width);
  if (g.mode == kModeStore) {
    if (g.snap_stride < 1) return fail(RTM_E_INVAL, "snap_stride must be >= 1");
    if (g.snap_dtype < 0 || g.snap_dtype > 2) return fail(RTM_E_INVAL, "unknown snap_dtype %d", g.snap_dtype);
  }
  auto inside = [&](rtm_point p) {
    return p.iz >= 0 && p.iz < g.nz && p.ix >= g.ix0 && p.ix < g.ix0 + g.width;
  };
  if (!inside(src)) return fail(RTM_E_INVAL, "source (%d, %d) outside the window", src.iz, src.ix);
  if (g.nrec < 0 || (g.nrec > 0 && !recs)) return fail(RTM_E_INVAL, "bad receiver list");
  for (int r = 0; r < g.nrec; ++r)
    if (!inside(recs[r]))
      return fail(RTM_E_INVAL, "receiver %d (%d, %d) outside the window", r, recs[r].iz, recs[r].ix);
  // Receivers must be distinct nodes: the step kernels add each receiver's
  // sample into its node with one atomic add per receiver, which is exact
  // (order-free) only while every node receives at most one sample.
  if (g.nrec > 1) {
    std::vector<std::pair<int64_t, int>> key(g.nrec);
    for (int r = 0; r < g.nrec; ++r) key[r] = {(int64_t)recs[r].iz * g.model_nx + recs[r].ix, r};
    std::sort(key.begin(), key.end());
    for (int r = 1; r < g.nrec; ++r)
      if (key[r].first == key[r - 1].first)
        return fail(RTM_E_INVAL, "receivers %d and %d are the same node (%d, %d)", key[r - 1].second, key[r].second,
                    recs[key[r].second].iz, recs[key[r].second].ix);
  }
  return RTM_OK;
}

// ===========================================================================
// Tile-height autotuner
// ===========================================================================
// The step kernel is compiled for tile heights 16, 32 and 64 rows.  For a
// launch set, the tuner builds scratch jobs of the same window, mode and
// snapshot type (nt = 16, zero data, so nothing real is touched), times a
// few forward and backward launches of each height with HIP events and keeps
// the fastest.  Results are cached per geometry key in the context and, if
// RTM_AUTOTUNE_CACHE names a file, in that JSON file across processes.
// RTM_TILE_Z forces a height.
static std::string tune_key(const JobGeom& g, int batch) {
  int b = batch <= 1 ? 1 : batch <= 4 ? 4 : batch <= 16 ? 16 : 64;
  char buf[128];
  snprintf(buf, sizeof buf, "gfx950/nzp%d/nxp%d/mode%d/snap%d/b%d", g.nz + 2 * g.nb, g.width + 2 * g.nb,
           g.mode, g.mode == kModeStore ? g.snap_dtype : -1, b);
  return buf;
}

static void tune_file_load(rtm_ctx* ctx) {
  ctx->tune_file_loaded = true;
  const char* path = getenv("RTM_AUTOTUNE_CACHE");
  if (!path) return;
  FILE* f = fopen(path, "r");
  if (!f) return;
  char line[512];
  while (fgets(line, sizeof line, f)) {
    char key[400];
    int tz;
    if (sscanf(line, " \"%399[^\"]\" : %d", key, &tz) != 2) continue;
    const bool two = strstr(key, "/step2/") != nullptr;
    if (two ? (tz == 16 || tz == 24 || tz == 32) : (tz == 16 || tz == 32 || tz == 64)) ctx->tune_cache[key] = tz;
  }
  fclose(f);
}

static void tune_file_save(rtm_ctx* ctx) {
  const char* path = getenv("RTM_AUTOTUNE_CACHE");
  if (!path) return;
  std::string tmp = std::string(path) + ".tmp";
  FILE* f = fopen(tmp.c_str(), "w");
  if (!f) return;
  fprintf(f, "{\n");
  size_t i = 0;
  for (auto& kv : ctx->tune_cache)
    fprintf(f, "  \"%s\": %d%s\n", kv.first.c_str(), kv.second, ++i < ctx->tune_cache.size() ? "," : "");
  fprintf(f, "}\n");
  fclose(f);
  (void)rename(tmp.c_str(), path);
}

static int build_job(rtm_ctx* ctx, hipStream_t s, const JobGeom& g, int tz, const float* vel,
                     const float* wavelet, rtm_point src, const rtm_point* recs, const float* data,
                     float* traces, HostJob& j, const HostJob* medium);
static int upload_table(rtm_ctx* ctx, hipStream_t s, const std::vector<HostJob*>& js, struct Table& t, int tz2f,
                        int tz2b);

static int time_tz(rtm_ctx* ctx, hipStream_t s, const JobGeom& g0, const float* vel, int batch, int tz,
                   float* ms_out);

static int autotune_tz(rtm_ctx* ctx, hipStream_t s, const JobGeom& g0, const float* vel, int batch) {
  if (int tz = env_tz()) return ctx->tile_z = tz;
  std::lock_guard<std::mutex> lk(ctx->tune_mu);
  if (!ctx->tune_file_loaded) tune_file_load(ctx);
  const std::string key = tune_key(g0, batch);
  auto it = ctx->tune_cache.find(key);
  if (it != ctx->tune_cache.end()) return ctx->tile_z = it->second;
  // Three rounds over the candidates, keeping each height's fastest trial,
  // so one noisy trial does not decide the choice.
  const int cand[3] = {16, 32, 64};
  float best_of[3] = {1e30f, 1e30f, 1e30f};
  for (int round = 0; round < 3; ++round)
    for (int c = 0; c < 3; ++c) {
      float ms = 0;
      if (time_tz(ctx, s, g0, vel, batch, cand[c], &ms) == RTM_OK)  // no room: skip the height
        best_of[c] = std::min(best_of[c], ms);
    }
  int best = 16;
  float best_ms = 1e30f;
  for (int c = 0; c < 3; ++c)
    if (best_of[c] < best_ms) {
      best_ms = best_of[c];
      best = cand[c];
    }
  if (best_ms < 1e30f) {  // keep only measured choices
    ctx->tune_cache[key] = best;
    tune_file_save(ctx);
  }
  return ctx->tile_z = best;
}

// ===========================================================================
// Job tables on the device
// ===========================================================================
struct Table {
  DevJob* jobs = nullptr;
  Tile* tiles = nullptr;
  StepCtl* ctl = nullptr;
  StepCtl* side_ctl[kMaxGroupStreams - 1] = {};  // the batched path's further streams of shot groups
  int ntiles = 0;
  // two-step tiles (tz rows x 56 columns) of the forward and the backward
  // phase, with the receivers of each tile's middle region:
  // {index in the middle region, receiver}
  struct TwoStep {
    Tile* tiles = nullptr;
    int2* recs = nullptr;
    int ntiles = 0, tz = 0;
    std::shared_ptr<std::vector<Tile>> htiles = std::make_shared<std::vector<Tile>>();
    std::shared_ptr<std::vector<int2>> hrecs = std::make_shared<std::vector<int2>>();
    std::vector<int> first;  // first tile of each job (njobs + 1 entries)
  } fw, bw;
  std::vector<int> first;  // first one-step tile of each job (njobs + 1 entries)
  std::vector<Block> blocks;
  std::shared_ptr<std::vector<DevJob>> hjobs;
  std::shared_ptr<std::vector<Tile>> htiles;
};

// The host arrays a table's uploads read, kept alive until the work that
// follows them has run.
static void keep_table(Deferred& d, const Table& t) {
  d.keep.push_back(t.hjobs);
  d.keep.push_back(t.htiles);
  d.keep.push_back(t.fw.htiles);
  d.keep.push_back(t.fw.hrecs);
  d.keep.push_back(t.bw.htiles);
  d.keep.push_back(t.bw.hrecs);
}

// Two-step tile height.  RTM_TILE_Z2 unset: the tuner picks the height of
// each phase (autotune_tz2); 16, 24 or 32 forces that height for both
// phases; 0, or any other value, turns two-step launches off.
static int env_tz2() {
  const char* e = getenv("RTM_TILE_Z2");
  if (!e) return -1;
  const int v = atoi(e);
  return v == 16 || v == 24 || v == 32 ? v : 0;
}
static bool two_step_on() { return env_tz2() != 0; }

// Reconstruct- and store-mode jobs without illumination advance two steps per
// launch where the scheme allows (four buffers per wavefield); the others,
// and all jobs when RTM_TILE_Z2 = 0, one step per launch.
static bool pairs_mode(const JobGeom& g) {
  return (g.mode == kModeRecon || g.mode == kModeStore) && !(g.flags & RTM_IMG_ILLUM);
}
// The serving engine pairs reconstruct-mode jobs, and store-mode jobs only
// when RTM_SERVE_STORE_PAIRS=1.  Its jobs sit in different phases, so a cycle
// with pairs launches forward pairs, backward pairs (one launch per job mode
// present) and one-step launches for the steps no pair covers.  That paid
// off for the reconstruct-mode ensemble (3.17e11 -> 3.82e11 updates/s).  On
// the store-mode stream (Poisson, 20 jobs/s, 300 timed jobs) pairs cut the
// median latency of the mostly lone jobs (42 -> 36 ms) but lengthen the tail
// and the saturation run, where many jobs in different phases split every
// step into more launches (p99 89 -> 133 ms; saturation 101 -> 77 images/s),
// so store-mode jobs run one step per launch by default.  Pairs only for the
// store-mode jobs admitted into an empty running set were no better (1200
// timed jobs: p50 40 against 37 ms, p99 102 against 80 ms; saturation
// unchanged): the later jobs admitted beside a paired one add launches.
// At saturation the pair kernels took as long as the one-step kernel for
// the same work, and the GPU was busy 74 % of the wall time against 97 %,
// most likely waiting on table rebuilds, which the jobs' changing launch
// kinds trigger in most cycles.
static bool served_two_step(const JobGeom& g) {
  const char* e = getenv("RTM_SERVE_STORE_PAIRS");
  const bool store_pairs = e && atoi(e) == 1;
  return (g.mode == kModeRecon || (store_pairs && g.mode == kModeStore)) && !(g.flags & RTM_IMG_ILLUM) &&
         two_step_on();
}


// A two-step tile reads 8 rows past its last row, and the staged rows of the
// last tile column run past the row end into the next row: the last tile
// must end within the 64-row rounding of the field allocation, whose 9 zero
// rows after it take the halo and that overrun.  Heights that divide 64
// always do; a 24-row tile may not, and then the phase takes 16-row tiles.
static bool tz2_fits(const std::vector<HostJob*>& js, int tz2) {
  for (auto* j : js) {
    const int nzp = j->d.nzp, z0last = ((nzp - 1) / tz2) * tz2;
    if (z0last + tz2 > field_rows(nzp) - 2 * kTopRows) return false;
  }
  return true;
}

// Appends the two-step tiles of a job (tz2 rows x 56 columns) with the
// receivers of each tile's middle region, {index in the middle region,
// receiver}, to tiles / recs; the tiles name job `job_index`.
static void append_two_step_tiles(const HostJob& hj, int job_index, int tz2, std::vector<Tile>& tiles,
                                  std::vector<int2>& recs) {
  const DevJob& d = hj.d;
  // receiver nodes (padded coordinates) from the one-step tiles' lists,
  // whose local index is (row in tile) * 64 + (column in tile)
  std::vector<std::pair<int, int>> rz(hj.recs.size());  // (row, receiver), sorted by row
  std::vector<int> rx(hj.recs.size());
  for (const Tile& one : hj.tiles)
    for (int q = one.rec_begin; q < one.rec_begin + one.rec_count; ++q) {
      const int local = hj.recs[q].x, r = hj.recs[q].y;
      rz[r] = {one.z0 + local / kTileX, r};
      rx[r] = one.x0 + local % kTileX;
    }
  std::sort(rz.begin(), rz.end());
  for (int z0 = 0; z0 < d.nzp; z0 += tz2)
    for (int x0 = 0; x0 < d.nxp; x0 += kTileX2) {
      Tile tl{};
      tl.job = job_index;
      tl.z0 = z0;
      tl.x0 = x0;
      tl.rec_begin = (int)recs.size();
      // receivers in the middle region rows [z0 - 4, z0 + tz2 + 4), columns [x0 - 4, x0 + 60)
      auto lo = std::lower_bound(rz.begin(), rz.end(), std::make_pair(z0 - kHalo, -1));
      for (auto it = lo; it != rz.end() && it->first < z0 + tz2 + kHalo; ++it) {
        const int xr = rx[it->second];
        if (xr >= x0 - kHalo && xr < x0 + kTileX2 + kHalo)
          recs.push_back(make_int2((it->first - (z0 - kHalo)) * kTileX + (xr - (x0 - kHalo)), it->second));
      }
      tl.rec_count = (int)recs.size() - tl.rec_begin;
      tiles.push_back(tl);
    }
}

// tz2f / tz2b > 0 also build the two-step tile tables of the forward and the
// backward phase (reconstruct- and store-mode jobs without illumination).
static int upload_table(rtm_ctx* ctx, hipStream_t s, const std::vector<HostJob*>& js, Table& t, int tz2f,
                        int tz2b) {
  t.hjobs = std::make_shared<std::vector<DevJob>>();
  t.htiles = std::make_shared<std::vector<Tile>>();
  for (size_t i = 0; i < js.size(); ++i) {
    t.hjobs->push_back(js[i]->d);
    t.first.push_back((int)t.htiles->size());
    for (Tile tl : js[i]->tiles) {
      tl.job = (int)i;
      t.htiles->push_back(tl);
    }
  }
  t.ntiles = (int)t.htiles->size();
  t.first.push_back(t.ntiles);
  bool pairs = true;
  for (auto* j : js) pairs = pairs && (pairs_mode(j->g) || j->g.mode == kModeBorn) && j->g.nbuf == 4;
  for (auto [tw, tz2] : {std::make_pair(&t.fw, tz2f), std::make_pair(&t.bw, tz2b)}) {
    if (!pairs || (tz2 != 16 && tz2 != 24 && tz2 != 32)) continue;
    if (!tz2_fits(js, tz2)) tz2 = 16;
    for (size_t i = 0; i < js.size(); ++i) {
      tw->first.push_back((int)tw->htiles->size());
      append_two_step_tiles(*js[i], (int)i, tz2, *tw->htiles, *tw->hrecs);
    }
    tw->ntiles = (int)tw->htiles->size();
    tw->first.push_back(tw->ntiles);
    tw->tz = tz2;
  }
  // jobs whose forward steps run in pairs (store mode: the launch after a
  // pair writes the snapshot of the pair's first level)
  if (t.fw.ntiles > 0)
    for (DevJob& dj : *t.hjobs) dj.two_step = 1;
  void* p;
  if (!alloc_block(ctx, t.blocks, t.hjobs->size() * sizeof(DevJob), &p)) return fail(RTM_E_NOMEM, "arena exhausted (job table)");
  t.jobs = static_cast<DevJob*>(p);
  if (!alloc_block(ctx, t.blocks, std::max<size_t>(t.htiles->size(), 1) * sizeof(Tile), &p)) {
    release_blocks(ctx, t.blocks);
    return fail(RTM_E_NOMEM, "arena exhausted (tile table)");
  }
  t.tiles = static_cast<Tile*>(p);
  if (!alloc_block(ctx, t.blocks, sizeof(StepCtl), &p)) {
    release_blocks(ctx, t.blocks);
    return fail(RTM_E_NOMEM, "arena exhausted (control block)");
  }
  t.ctl = static_cast<StepCtl*>(p);
  for (auto& sc : t.side_ctl) {
    if (!alloc_block(ctx, t.blocks, sizeof(StepCtl), &p)) {
      release_blocks(ctx, t.blocks);
      return fail(RTM_E_NOMEM, "arena exhausted (control block)");
    }
    sc = static_cast<StepCtl*>(p);
  }
  for (auto* tw : {&t.fw, &t.bw}) {
    if (tw->ntiles == 0) continue;
    if (!alloc_block(ctx, t.blocks, tw->htiles->size() * sizeof(Tile), &p)) {
      release_blocks(ctx, t.blocks);
      return fail(RTM_E_NOMEM, "arena exhausted (two-step tile table)");
    }
    tw->tiles = static_cast<Tile*>(p);
    HIP_OK(hipMemcpyAsync(tw->tiles, tw->htiles->data(), tw->htiles->size() * sizeof(Tile), hipMemcpyHostToDevice, s));
    if (!alloc_block(ctx, t.blocks, std::max<size_t>(tw->hrecs->size(), 1) * sizeof(int2), &p)) {
      release_blocks(ctx, t.blocks);
      return fail(RTM_E_NOMEM, "arena exhausted (two-step receiver table)");
    }
    tw->recs = static_cast<int2*>(p);
    if (!tw->hrecs->empty())
      HIP_OK(hipMemcpyAsync(tw->recs, tw->hrecs->data(), tw->hrecs->size() * sizeof(int2), hipMemcpyHostToDevice, s));
  }
  HIP_OK(hipMemcpyAsync(t.jobs, t.hjobs->data(), t.hjobs->size() * sizeof(DevJob), hipMemcpyHostToDevice, s));
  HIP_OK(hipMemcpyAsync(t.tiles, t.htiles->data(), t.htiles->size() * sizeof(Tile), hipMemcpyHostToDevice, s));
  StepCtl c{};
  c.ntiles = t.ntiles;
  HIP_OK(hipMemcpyAsync(t.ctl, &c, sizeof c, hipMemcpyHostToDevice, s));
  for (StepCtl* sc : t.side_ctl) HIP_OK(hipMemcpyAsync(sc, &c, sizeof c, hipMemcpyHostToDevice, s));
  HIP_OK(hipStreamSynchronize(s));  // host-side staging copies are complete
  return RTM_OK;
}

// One timing trial of the tuner: B scratch jobs (B = min(batch, 8)), nt = 16.
static int time_tz(rtm_ctx* ctx, hipStream_t s, const JobGeom& g0, const float* vel, int batch, int tz,
                   float* ms_out) {
  const int B = std::max(1, std::min(batch, 8));
  JobGeom g = g0;
  g.nt = 16;
  g.nrec = g.width;
  g.flags = 0;
  const bool model = g.mode == kModeModel || g.mode == kModeBorn;  // forward-only job kinds
  const int nsteps = model ? g.nt - 1 : 2 * g.nt - 1;
  std::vector<Block> scratch;
  void *zero = nullptr, *traces = nullptr;
  if (!alloc_block(ctx, scratch, (size_t)g.nt * g.width * 4 + 256, &zero)) return RTM_E_NOMEM;
  HIP_OK(hipMemsetAsync(zero, 0, (size_t)g.nt * g.width * 4 + 256, s));
  if (model) {  // modelling trials sample traces: give them somewhere to go
    if (!alloc_block(ctx, scratch, (size_t)B * g.nt * g.width * 4, &traces)) {
      release_blocks(ctx, scratch);
      return RTM_E_NOMEM;
    }
  }
  std::vector<rtm_point> recs(g.width);
  for (int r = 0; r < g.width; ++r) recs[r] = {0, g.ix0 + r};
  rtm_point src{g.nz / 2, g.ix0 + g.width / 2};
  std::vector<std::unique_ptr<HostJob>> jobs;
  std::vector<HostJob*> ptrs;
  int rc = RTM_OK;
  for (int b = 0; b < B && rc == RTM_OK; ++b) {
    auto j = std::make_unique<HostJob>();
    float* tr = traces ? static_cast<float*>(traces) + (size_t)b * g.nt * g.width : nullptr;
    rc = build_job(ctx, s, g, tz, vel, static_cast<const float*>(zero), src, recs.data(),
                   static_cast<const float*>(zero), tr, *j, jobs.empty() ? nullptr : jobs[0].get());
    if (rc == RTM_OK) {
      ptrs.push_back(j.get());
      jobs.push_back(std::move(j));
    }
  }
  Table t;
  if (rc == RTM_OK) rc = upload_table(ctx, s, ptrs, t, 0, 0);
  hipEvent_t e[3] = {nullptr, nullptr, nullptr};
  if (rc == RTM_OK) {
    for (auto& ev : e) (void)hipEventCreate(&ev);
    const int nf = g.nt - 1;
    for (int st = 0; st < nsteps && rc == RTM_OK; ++st) {
      if (st == 2) (void)hipEventRecord(e[0], s);
      if (st == nf - 1 && model) (void)hipEventRecord(e[1], s);
      if (st == nf && !model) (void)hipEventRecord(e[1], s);
      const int ph = g.mode == kModeBorn ? kPhBorn : (st < nf ? kPhFwd : kPhBwd);
      if (launch_step(tz, ph, t.jobs, t.tiles, t.ntiles, t.ntiles, t.ctl, 0, st, s) != hipSuccess)
        rc = fail(RTM_E_DEVICE, "tuning launch failed");
    }
    (void)hipEventRecord(e[2], s);
    (void)hipStreamSynchronize(s);
    float a = 0, b = 0;
    if (rc == RTM_OK && hipEventElapsedTime(&a, e[0], e[1]) == hipSuccess &&
        hipEventElapsedTime(&b, e[1], e[2]) == hipSuccess)
      *ms_out = model ? a / (nf - 3) : a / (nf - 2) + b / g.nt;  // one forward (+ one backward) launch
    for (auto ev : e)
      if (ev) (void)hipEventDestroy(ev);
  }
  (void)hipStreamSynchronize(s);
  for (auto& j : jobs) {
    release_blocks(ctx, j->blocks);
    if (j->image_blk.p) ctx->arena.release(j->image_blk.p, j->image_blk.n);
  }
  release_blocks(ctx, t.blocks);
  release_blocks(ctx, scratch);
  return rc;
}

// Two-step tile heights (forward phase, backward phase) of a batch of
// reconstruct-mode jobs.  For each height that fits the geometry (16, 24,
// 32 rows; tz2_fits), scratch jobs of the batch's widest window (B =
// min(batch, 16) sharing one medium, nt = 24, zero data) run their two-step
// launches of each phase, timed with HIP events; three rounds, best trial
// per height, fastest height per phase.  Cached per geometry key in the
// context and the RTM_AUTOTUNE_CACHE file like the one-step heights.
static int time_tz2(rtm_ctx* ctx, hipStream_t s, const JobGeom& g0, const float* vel, int batch, int tz2,
                    float* ms_fwd, float* ms_bwd) {
  const int B = std::max(1, std::min(batch, 16));
  JobGeom g = g0;
  g.nt = 24;
  g.nrec = g.width;
  g.flags = 0;
  g.mode = kModeRecon;
  g.nbuf = 4;
  std::vector<Block> scratch;
  void* zero = nullptr;
  if (!alloc_block(ctx, scratch, (size_t)g.nt * g.width * 4 + 256, &zero)) return RTM_E_NOMEM;
  HIP_OK(hipMemsetAsync(zero, 0, (size_t)g.nt * g.width * 4 + 256, s));
  std::vector<rtm_point> recs(g.width);
  for (int r = 0; r < g.width; ++r) recs[r] = {0, g.ix0 + r};
  rtm_point src{g.nz / 2, g.ix0 + g.width / 2};
  std::vector<std::unique_ptr<HostJob>> jobs;
  std::vector<HostJob*> ptrs;
  int rc = RTM_OK;
  for (int b = 0; b < B && rc == RTM_OK; ++b) {
    auto j = std::make_unique<HostJob>();
    rc = build_job(ctx, s, g, 16, vel, static_cast<const float*>(zero), src, recs.data(),
                   static_cast<const float*>(zero), nullptr, *j, jobs.empty() ? nullptr : jobs[0].get());
    if (rc == RTM_OK) {
      ptrs.push_back(j.get());
      jobs.push_back(std::move(j));
    }
  }
  Table t;
  if (rc == RTM_OK && !tz2_fits(ptrs, tz2)) rc = RTM_E_INVAL;  // this height does not fit: skip it
  if (rc == RTM_OK) rc = upload_table(ctx, s, ptrs, t, tz2, tz2);
  hipEvent_t e[4] = {nullptr, nullptr, nullptr, nullptr};
  if (rc == RTM_OK) {
    for (auto& ev : e) (void)hipEventCreate(&ev);
    const int nf = g.nt - 1, nsteps = 2 * g.nt - 1;
    hipError_t er = hipSuccess;
    // forward pairs at steps 0, 2, ..; the first two are not timed
    int nfw = 0, nbw = 0;
    for (int st = 0; st + 1 < nf && er == hipSuccess; st += 2) {
      if (st == 4) er = hipEventRecord(e[0], s);
      if (er == hipSuccess) er = launch_step2(tz2, kPhFwd, 0, t.jobs, t.fw.tiles, t.fw.recs, t.fw.ntiles, t.fw.ntiles, t.ctl, 0, st, s);
      nfw += st >= 4;
    }
    if (er == hipSuccess) er = hipEventRecord(e[1], s);
    // backward pairs from level nt - 3 down (steps nf + 2, nf + 4, ..)
    for (int st = nf + 2, k = 0; st + 1 < nsteps && er == hipSuccess; st += 2, ++k) {
      if (k == 2) er = hipEventRecord(e[2], s);
      if (er == hipSuccess) er = launch_step2(tz2, kPhBwd, 0, t.jobs, t.bw.tiles, t.bw.recs, t.bw.ntiles, t.bw.ntiles, t.ctl, 0, st, s);
      nbw += k >= 2;
    }
    if (er == hipSuccess) er = hipEventRecord(e[3], s);
    if (er != hipSuccess) rc = fail(RTM_E_DEVICE, "tuning launch failed: %s", hipGetErrorString(er));
    (void)hipStreamSynchronize(s);
    float a = 0, b = 0;
    if (rc == RTM_OK && nfw > 0 && nbw > 0 && hipEventElapsedTime(&a, e[0], e[1]) == hipSuccess &&
        hipEventElapsedTime(&b, e[2], e[3]) == hipSuccess) {
      *ms_fwd = a / nfw;
      *ms_bwd = b / nbw;
    } else if (rc == RTM_OK) {
      rc = RTM_E_INVAL;
    }
    for (auto ev : e)
      if (ev) (void)hipEventDestroy(ev);
  }
  (void)hipStreamSynchronize(s);
  for (auto& j : jobs) {
    release_blocks(ctx, j->blocks);
    if (j->image_blk.p) ctx->arena.release(j->image_blk.p, j->image_blk.n);
  }
  release_blocks(ctx, t.blocks);
  release_blocks(ctx, scratch);
  return rc;
}

static std::string tune_key2(const JobGeom& g, int batch) {
  int b = batch <= 1 ? 1 : batch <= 4 ? 4 : batch <= 16 ? 16 : 64;
  char buf[128];
  snprintf(buf, sizeof buf, "gfx950/step2/nzp%d/nxp%d/b%d", g.nz + 2 * g.nb, g.width + 2 * g.nb, b);
  return buf;
}

static void autotune_tz2(rtm_ctx* ctx, hipStream_t s, const JobGeom& g0, const float* vel, int batch, int* tzf,
                         int* tzb) {
  const int forced = env_tz2();
  if (forced >= 0) {
    *tzf = *tzb = forced;
    return;
  }
  std::lock_guard<std::mutex> lk(ctx->tune_mu);
  if (!ctx->tune_file_loaded) tune_file_load(ctx);
  const std::string key = tune_key2(g0, batch);
  auto f = ctx->tune_cache.find(key + "/fwd"), b = ctx->tune_cache.find(key + "/bwd");
  if (f != ctx->tune_cache.end() && b != ctx->tune_cache.end()) {
    *tzf = f->second;
    *tzb = b->second;
    return;
  }
  const int cand[3] = {16, 24, 32};
  float bf[3] = {1e30f, 1e30f, 1e30f}, bb[3] = {1e30f, 1e30f, 1e30f};
  for (int round = 0; round < 3; ++round)
    for (int c = 0; c < 3; ++c) {
      float mf = 0, mb = 0;
      if (time_tz2(ctx, s, g0, vel, batch, cand[c], &mf, &mb) == RTM_OK) {  // no fit / no room: skip
        bf[c] = std::min(bf[c], mf);
        bb[c] = std::min(bb[c], mb);
      }
    }
  // 24 rows (the best on the survey) unless another height measured at
  // least 5 % faster, or 24 rows could not be measured: heights within the
  // trials' noise (a few per cent on the survey's shot groups, where 16 and
  // 24 rows run equally fast) do not flip from one tuning to the next
  int kf = 1, kb = 1;
  for (int c : {0, 2}) {
    if (bf[c] < (bf[kf] < 1e30f ? 0.95f : 1.0f) * bf[kf]) kf = c;
    if (bb[c] < (bb[kb] < 1e30f ? 0.95f : 1.0f) * bb[kb]) kb = c;
  }
  *tzf = cand[kf];
  *tzb = cand[kb];
  if (bf[kf] < 1e30f && bb[kb] < 1e30f) {  // keep only measured choices
    ctx->tune_cache[key + "/fwd"] = *tzf;
    ctx->tune_cache[key + "/bwd"] = *tzb;
    tune_file_save(ctx);
  }
}

// ===========================================================================
// C ABI: helpers and context
// ===========================================================================
extern "C" const char* rtm_status_str(int st) {
  switch (st) {
    case RTM_OK: return "ok";
    case RTM_E_INVAL: return "invalid argument";
    case RTM_E_CFL: return "CFL stability limit exceeded";
    case RTM_E_NOMEM: return "arena exhausted";
    case RTM_E_AGAIN: return "queue full, retry";
    case RTM_E_NOTFOUND: return "not found";
    case RTM_E_NONFINITE: return "non-finite value";
    case RTM_E_DEVICE: return "HIP runtime error";
    case RTM_E_CANCELLED: return "cancelled";
    default: return "unknown status";
  }
}

extern "C" const char* rtm_last_error(void) { return g_last_error.c_str(); }

extern "C" int rtm_version(void) { return 10000; }

static void sched_main(rtm_ctx* ctx);

extern "C" int rtm_ctx_create(rtm_ctx** out, int device, void* arena_dev, size_t arena_bytes,
                              void* hip_stream, uint32_t flags) {
  (void)flags;
  if (!out) return fail(RTM_E_INVAL, "out is NULL");
  *out = nullptr;
  if (arena_bytes < (1u << 20)) return fail(RTM_E_INVAL, "arena must be at least 1 MiB");
  int ndev = 0;
  HIP_OK(hipGetDeviceCount(&ndev));
  if (device < 0 || device >= ndev) return fail(RTM_E_INVAL, "device %d not present (%d devices)", device, ndev);
  HIP_OK(hipSetDevice(device));
  // address of the allocation-free encoder's scratch on this device (looked
  // up once per device, with the device current)
  HIP_OK(zc_noalloc_scratch_init(device));
  auto ctx = std::make_unique<rtm_ctx>();
  ctx->device = device;
  ctx->stream = static_cast<hipStream_t>(hip_stream);
  if (!arena_dev) {
    HIP_OK(hipMalloc(&ctx->own_arena, arena_bytes));
    arena_dev = ctx->own_arena;
  }
  if ((reinterpret_cast<uintptr_t>(arena_dev) & 255) != 0)
    return fail(RTM_E_INVAL, "arena must be 256-byte aligned");
  ctx->arena.init(arena_dev, arena_bytes);
  HIP_OK(hipStreamCreateWithFlags(&ctx->sched_stream, hipStreamNonBlocking));
  HIP_OK(hipStreamCreateWithFlags(&ctx->work_stream, hipStreamNonBlocking));
  for (auto& gs : ctx->group_stream) HIP_OK(hipStreamCreateWithFlags(&gs, hipStreamNonBlocking));
  HIP_OK(hipEventCreateWithFlags(&ctx->ev_fork, hipEventDisableTiming));
  for (auto& e : ctx->ev_join) HIP_OK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
  HIP_OK(hipEventCreateWithFlags(&ctx->ev_in, hipEventDisableTiming));
  HIP_OK(hipEventCreateWithFlags(&ctx->ev_out, hipEventDisableTiming));
  for (auto& e : ctx->ph_ev) HIP_OK(hipEventCreate(&e));
  for (auto& e : ctx->zc_ev) HIP_OK(hipEventCreate(&e));
  for (auto& e : ctx->bet_ev) HIP_OK(hipEventCreate(&e));
  // A served job must fit the arena beside a few KB of tables; larger ones are
  // refused at submit.
  ctx->book = std::make_unique<JobBook>(now_s, arena_bytes > 4096 ? arena_bytes - 4096 : 0);
  if (const char* path = getenv("RTM_LOG")) ctx->job_log = fopen(path, "a");
  ctx->scratch_u32 = static_cast<uint32_t*>(ctx->arena.alloc(256));
  ctx->scratch_f64 = static_cast<double*>(ctx->arena.alloc((2 * kRedBlocks + 2) * sizeof(double)));
  if (!ctx->scratch_u32 || !ctx->scratch_f64) return fail(RTM_E_NOMEM, "arena too small for the context's scratch");
  HIP_OK(hipMemset(ctx->scratch_u32, 0, 256));
  *out = ctx.release();
  return RTM_OK;
}

extern "C" int rtm_ctx_synchronize(rtm_ctx* ctx) {
  if (!ctx) return fail(RTM_E_INVAL, "ctx is NULL");
  HIP_OK(hipSetDevice(ctx->device));
  HIP_OK(hipStreamSynchronize(ctx->stream));
  reap(ctx, false);
  // images of plain / batched calls are checked for non-finite values as they
  // finish; report (and clear) the flag here
  uint32_t flag = 0;
  HIP_OK(hipMemcpy(&flag, ctx->scratch_u32 + 1, 4, hipMemcpyDeviceToHost));
  if (flag) {
    HIP_OK(hipMemset(ctx->scratch_u32 + 1, 0, 4));
    return fail(RTM_E_NONFINITE, "a migrated image contained non-finite values since the last synchronize");
  }
  return RTM_OK;
}

extern "C" int rtm_ctx_destroy(rtm_ctx* ctx) {
  if (!ctx) return RTM_OK;
  (void)hipSetDevice(ctx->device);
  {
    std::lock_guard<std::mutex> lk(ctx->mu);
    ctx->stop = true;
  }
  ctx->cv.notify_all();
  if (ctx->sched.joinable()) ctx->sched.join();
  (void)hipStreamSynchronize(ctx->stream);
  (void)hipStreamSynchronize(ctx->sched_stream);
  reap(ctx, false);
  while (true) {
    bool empty;
    {
      std::lock_guard<std::mutex> lk(ctx->defer_mu);
      empty = ctx->deferred.empty();
    }
    if (empty) break;
    reap(ctx, true);
  }
  (void)hipStreamSynchronize(ctx->work_stream);
  for (auto gs : ctx->group_stream) (void)hipStreamSynchronize(gs);
  reap(ctx, false);
  (void)hipStreamDestroy(ctx->sched_stream);
  (void)hipStreamDestroy(ctx->work_stream);
  for (auto gs : ctx->group_stream) (void)hipStreamDestroy(gs);
  (void)hipEventDestroy(ctx->ev_fork);
  for (auto e : ctx->ev_join) (void)hipEventDestroy(e);
  (void)hipEventDestroy(ctx->ev_in);
  (void)hipEventDestroy(ctx->ev_out);
  for (auto e : ctx->ph_ev) (void)hipEventDestroy(e);
  for (auto e : ctx->zc_ev) (void)hipEventDestroy(e);
  for (auto e : ctx->bet_ev) (void)hipEventDestroy(e);
  if (ctx->own_arena) (void)hipFree(ctx->own_arena);
  if (ctx->job_log) fclose(ctx->job_log);
  delete ctx;
  return RTM_OK;
}

// ===========================================================================
// Plain path
// ===========================================================================
// Two-step tile height of Born jobs (RTM_TILE_Z2 forces 16, 24 or 32; 0
// keeps one step per launch).  A launch with few tiles needs the smaller
// tiles' extra workgroups more than the larger tiles' smaller halo share:
// measured on 351 x 1701 (nb 50, nt 4000), one shot per launch (627
// 24-row tiles) 2.95e11 updates/s at 16 rows, 2.75e11 at 24, 2.72e11 one
// step per launch; 16 shots per launch (10032 tiles) 3.77e11 at 16 rows,
// 3.86e11 at 24, 3.62e11 one step per launch.  So 16 rows below 2048
// 24-row tiles per launch, 24 from there (upload_table falls back to 16
// where a grid's last 24-row tile would not fit).
static int born_tz2(const JobGeom& g, int nshots) {
  const int e = env_tz2();
  if (e >= 0) return e;
  const int64_t tiles24 = (int64_t)nshots * ((g.nz + 2 * g.nb + 23) / 24) * ((g.width + 2 * g.nb + kTileX2 - 1) / kTileX2);
  return tiles24 < 2048 ? 16 : 24;
}

// The time steps of every job in js (jobs of one mode and step count: a
// single job, or the shots of a Born batch) over all their tiles: one launch
// per step, except that Born jobs built with four buffers per field
// (tz2 > 0) advance two steps per launch, the last step alone when the
// count is odd.
static int run_plain_jobs(rtm_ctx* ctx, hipStream_t s, const std::vector<HostJob*>& js, int tz, Table& t,
                          int tz2 = 0) {
  int rc = upload_table(ctx, s, js, t, tz2, 0);
  if (rc) return rc;
  const HostJob& j = *js[0];
  const int nsteps = j.d.nsteps;
  const int nf = j.g.mode == kModeModel ? nsteps : j.g.nt - 1;
  int st = 0;
  if (j.g.mode == kModeBorn && t.fw.ntiles > 0)
    for (; st + 1 < nsteps; st += 2)
      HIP_OK(launch_step2(t.fw.tz, kPhBorn, 0, t.jobs, t.fw.tiles, t.fw.recs, t.fw.ntiles, t.fw.ntiles, t.ctl, 0,
                          st, s));
  for (; st < nsteps; ++st) {
    const int ph = j.g.mode == kModeBorn ? kPhBorn : (st < nf ? kPhFwd : kPhBwd);
    HIP_OK(launch_step(tz, ph, t.jobs, t.tiles, t.ntiles, t.ntiles, t.ctl, 0, st, s));
  }
  ctx->steps_launched += nsteps;
  return RTM_OK;
}

static int run_plain(rtm_ctx* ctx, hipStream_t s, HostJob& j, int tz, Table& t) {
  return run_plain_jobs(ctx, s, std::vector<HostJob*>{&j}, tz, t);
}

static void finish_job_deferred(rtm_ctx* ctx, hipStream_t s, HostJob& j, Table& t, bool keep_image) {
  Deferred d;
  d.blocks = std::move(j.blocks);
  for (auto& b : t.blocks) d.blocks.push_back(b);
  t.blocks.clear();
  if (!keep_image && j.image_blk.p) d.blocks.push_back(j.image_blk);
  keep_table(d, t);
  defer(ctx, s, std::move(d));
}

extern "C" int rtm_propagate(rtm_ctx* ctx, const rtm_grid* grid, const float* vel_dev,
                             const float* wavelet_dev, rtm_point src, int32_t nrec,
                             const rtm_point* rec_host, float* traces_dev, float* final_field_dev) {
  if (!ctx) return fail(RTM_E_INVAL, "ctx is NULL");
  int rc = check_grid(grid);
  if (rc) return rc;
  if (!vel_dev || !wavelet_dev) return fail(RTM_E_INVAL, "vel_dev and wavelet_dev are required");
  if (nrec > 0 && !traces_dev) return fail(RTM_E_INVAL, "traces_dev is required when nrec > 0");
  JobGeom g;
  g.nz = grid->nz;
  g.model_nx = grid->nx;
  g.ix0 = 0;
  g.width = grid->nx;
  g.nb = grid->nb;
  g.nt = grid->nt;
  g.dz = grid->dz;
  g.dx = grid->dx;
  g.dt = grid->dt;
  g.sponge_a = grid->sponge_a;
  g.mode = kModeModel;
  g.nrec = nrec;
  if ((rc = check_job(g, src, rec_host))) return rc;
  HIP_OK(hipSetDevice(ctx->device));
  hipStream_t s = ctx->stream;
  float vmax = 0;
  if ((rc = device_vmax(ctx, s, vel_dev, g.nz, g.model_nx, 0, g.width, &vmax))) return rc;
  if ((rc = check_cfl(vmax, g.dt, g.dz, g.dx))) return rc;
  const int tz = autotune_tz(ctx, s, g, vel_dev, 1);
  HostJob j;
  if ((rc = build_job(ctx, s, g, tz, vel_dev, wavelet_dev, src, rec_host, nullptr, traces_dev, j, nullptr)))
    return rc;
  Table t;
  if ((rc = run_plain(ctx, s, j, tz, t))) {
    finish_job_deferred(ctx, s, j, t, false);
    return rc;
  }
  if (final_field_dev)
    HIP_OK(launch_copy_phys(final_field_dev, j.d.f[(g.nt - 1) & 3], g.nz, g.width, g.nb, j.d.pitch, s));
  ctx->grid_updates += j.updates;
  ctx->alg_bytes += j.alg_bytes;
  finish_job_deferred(ctx, s, j, t, false);
  return RTM_OK;
}

// A Born job runs over the whole model.
static void born_geom(const rtm_grid* grid, int32_t nrec, JobGeom& g) {
  g.nz = grid->nz;
  g.model_nx = grid->nx;
  g.ix0 = 0;
  g.width = grid->nx;
  g.nb = grid->nb;
  g.nt = grid->nt;
  g.dz = grid->dz;
  g.dx = grid->dx;
  g.dt = grid->dt;
  g.sponge_a = grid->sponge_a;
  g.mode = kModeBorn;
  g.nrec = nrec;
  if (env_tz2() != 0) g.nbuf = 4;  // two steps per launch
}

extern "C" int rtm_born(rtm_ctx* ctx, const rtm_grid* grid, const float* vel_dev, const float* wavelet_dev,
                        rtm_point src, const float* mpert_dev, int32_t nrec, const rtm_point* rec_host,
                        float* dtraces_dev) {
  if (!ctx) return fail(RTM_E_INVAL, "ctx is NULL");
  int rc = check_grid(grid);
  if (rc) return rc;
  if (!vel_dev || !wavelet_dev || !mpert_dev) return fail(RTM_E_INVAL, "vel_dev, wavelet_dev, mpert_dev are required");
  if (nrec > 0 && !dtraces_dev) return fail(RTM_E_INVAL, "dtraces_dev is required when nrec > 0");
  JobGeom g;
  born_geom(grid, nrec, g);
  if ((rc = check_job(g, src, rec_host))) return rc;
  HIP_OK(hipSetDevice(ctx->device));
  hipStream_t s = ctx->stream;
  float vmax = 0;
  if ((rc = device_vmax(ctx, s, vel_dev, g.nz, g.model_nx, 0, g.width, &vmax))) return rc;
  if ((rc = check_cfl(vmax, g.dt, g.dz, g.dx))) return rc;
  const int tz = autotune_tz(ctx, s, g, vel_dev, 1);
  HostJob j;
  if ((rc = build_job(ctx, s, g, tz, vel_dev, wavelet_dev, src, rec_host, nullptr, dtraces_dev, j, nullptr)))
    return rc;
  // the perturbation goes into the job's image buffer (field-aligned rows, padded columns)
  HIP_OK(hipMemcpy2DAsync(j.d.image + g.nb, (size_t)j.d.pitch * 4, mpert_dev, (size_t)g.width * 4,
                          (size_t)g.width * 4, g.nz, hipMemcpyDeviceToDevice, s));
  Table t;
  if ((rc = run_plain_jobs(ctx, s, std::vector<HostJob*>{&j}, tz, t, born_tz2(g, 1)))) {
    finish_job_deferred(ctx, s, j, t, false);
    return rc;
  }
  ctx->grid_updates += j.updates;
  ctx->alg_bytes += j.alg_bytes;
  finish_job_deferred(ctx, s, j, t, false);
  return RTM_OK;
}

static size_t group_budget();
static int group_streams();

// Shot groups of a Born batch: consecutive runs of near-equal size whose
// launches' working set (per shot two fields, two levels read and two
// written per launch; c and the perturbation once) fits the cache budget
// (RTM_GROUP_KB, as for the migration batch), shared by the streams whose
// groups run side by side.
static std::vector<std::pair<int, int>> born_groups(const JobGeom& g, int nshots, int streams) {
  const size_t pad = (size_t)(g.nz + 2 * g.nb) * field_pitch(g.width + 2 * g.nb) * 4;
  const size_t per = 8 * pad, shared = 2 * pad;
  const size_t budget = group_budget() == SIZE_MAX ? SIZE_MAX : group_budget() / streams;
  int ngroups = 1;
  if (budget != SIZE_MAX && shared + per * (size_t)nshots > budget) {
    const size_t fit = budget > shared + per ? (budget - shared) / per : 1;
    ngroups = (int)std::min<size_t>(nshots, ((size_t)nshots + fit - 1) / fit);
  }
  std::vector<std::pair<int, int>> out;
  for (int i = 0; i < ngroups; ++i) out.push_back({nshots * i / ngroups, nshots * (i + 1) / ngroups});
  return out;
}

// Born modelling of several shots in shared launches: every shot's job reads
// the first job's c, sponge profiles and perturbation (the Born step only
// reads them), and each launch advances the Born step of every shot.
extern "C" int rtm_born_batch(rtm_ctx* ctx, const rtm_grid* grid, const float* vel_dev, const float* wavelet_dev,
                              const float* mpert_dev, int32_t nshots, const rtm_born_shot* shots) {
  if (!ctx) return fail(RTM_E_INVAL, "ctx is NULL");
  int rc = check_grid(grid);
  if (rc) return rc;
  if (!vel_dev || !wavelet_dev || !mpert_dev) return fail(RTM_E_INVAL, "vel_dev, wavelet_dev, mpert_dev are required");
  if (nshots < 1 || !shots) return fail(RTM_E_INVAL, "need at least one shot");
  std::vector<JobGeom> geoms(nshots);
  size_t need = 0;
  for (int i = 0; i < nshots; ++i) {
    born_geom(grid, shots[i].nrec, geoms[i]);
    if (shots[i].nrec > 0 && !shots[i].dtraces_dev) return fail(RTM_E_INVAL, "shot %d has no dtraces_dev", i);
    if ((rc = check_job(geoms[i], shots[i].src, shots[i].rec_host))) return rc;
    need += footprint(geoms[i]).total - (i ? medium_bytes(geoms[i]) : 0);
  }
  if (need > ctx->arena.size())
    return fail(RTM_E_NOMEM, "batch needs %zu bytes, arena holds %zu", need, ctx->arena.size());
  HIP_OK(hipSetDevice(ctx->device));
  hipStream_t s = ctx->stream;
  float vmax = 0;
  if ((rc = device_vmax(ctx, s, vel_dev, grid->nz, grid->nx, 0, grid->nx, &vmax))) return rc;
  if ((rc = check_cfl(vmax, grid->dt, grid->dz, grid->dx))) return rc;
  const int tz = autotune_tz(ctx, s, geoms[0], vel_dev, nshots);
  std::vector<std::unique_ptr<HostJob>> jobs;
  std::vector<HostJob*> ptrs;
  for (int i = 0; i < nshots; ++i) {
    auto j = std::make_unique<HostJob>();
    rc = build_job(ctx, s, geoms[i], tz, vel_dev, wavelet_dev, shots[i].src, shots[i].rec_host, nullptr,
                   shots[i].dtraces_dev, *j, i ? jobs[0].get() : nullptr);
    if (rc) {
      (void)hipStreamSynchronize(s);
      for (auto& o : jobs) {
        release_blocks(ctx, o->blocks);
        if (o->image_blk.p) ctx->arena.release(o->image_blk.p, o->image_blk.n);
      }
      return rc;
    }
    ptrs.push_back(j.get());
    jobs.push_back(std::move(j));
  }
  // the perturbation, once, in the first job's image buffer (field-aligned
  // rows, padded columns); the other jobs read it there
  HostJob& j0 = *jobs[0];
  rc = hipMemcpy2DAsync(j0.d.image + j0.g.nb, (size_t)j0.d.pitch * 4, mpert_dev, (size_t)j0.g.width * 4,
                        (size_t)j0.g.width * 4, j0.g.nz, hipMemcpyDeviceToDevice, s) == hipSuccess
           ? RTM_OK
           : fail(RTM_E_DEVICE, "perturbation copy failed");
  for (auto& j : jobs) j->d.image = j0.d.image;
  // Shot groups sized for the memory-side cache, as the migration batch
  // runs them: each group advances all its steps before the next starts, so
  // the levels a launch writes are still cached when the group's next launch
  // reads them; the groups alternate between the context stream and the
  // further group streams (RTM_GROUP_STREAMS), forked from it and joined
  // back into it, so one group's launches fill what another's leave idle.
  // Every group has its own tables and control block.
  const int nreq = group_streams();
  const std::vector<std::pair<int, int>> groups = born_groups(geoms[0], nshots, nreq);
  const int ns = std::max(1, std::min<int>(nreq, (int)groups.size()));
  std::vector<Table> tables(groups.size());
  if (!rc && ns > 1) {
    rc = hipEventRecord(ctx->ev_fork, s) == hipSuccess ? RTM_OK : fail(RTM_E_DEVICE, "event record");
    for (int k = 1; k < ns && !rc; ++k)
      if (hipStreamWaitEvent(ctx->group_stream[k - 1], ctx->ev_fork, 0) != hipSuccess)
        rc = fail(RTM_E_DEVICE, "stream wait");
  }
  for (size_t gi = 0; gi < groups.size() && !rc; ++gi) {
    const auto [a, b] = groups[gi];
    const int side = (int)(gi % ns);
    std::vector<HostJob*> grp(ptrs.begin() + a, ptrs.begin() + b);
    rc = run_plain_jobs(ctx, side ? ctx->group_stream[side - 1] : s, grp, tz, tables[gi], born_tz2(geoms[0], b - a));
  }
  for (int k = 1; k < ns; ++k) {  // also after an error: deferred work on s waits for the group streams
    hipStream_t gs = ctx->group_stream[k - 1];
    if (hipEventRecord(ctx->ev_join[k - 1], gs) != hipSuccess || hipStreamWaitEvent(s, ctx->ev_join[k - 1], 0) != hipSuccess) {
      (void)hipStreamSynchronize(gs);
      if (!rc) rc = fail(RTM_E_DEVICE, "joining a group stream failed");
    }
  }
  if (!rc) ctx->born_groups = (int)groups.size();
  Deferred d;
  for (auto& j : jobs) {
    for (auto& b : j->blocks) d.blocks.push_back(b);
    j->blocks.clear();
    if (j->image_blk.p) d.blocks.push_back(j->image_blk);
    ctx->grid_updates += rc ? 0 : j->updates;
    ctx->alg_bytes += rc ? 0 : j->alg_bytes;
  }
  for (auto& t : tables) {
    for (auto& b : t.blocks) d.blocks.push_back(b);
    keep_table(d, t);
  }
  int rc2 = defer(ctx, s, std::move(d));
  return rc ? rc : rc2;
}

static int fill_geom_rtm(const rtm_grid* grid, int32_t ix0, int32_t width, const rtm_img_opts* opts, int nrec,
                         JobGeom& g) {
  g.nz = grid->nz;
  g.model_nx = grid->nx;
  g.ix0 = ix0;
  g.width = width;
  g.nb = grid->nb;
  g.nt = grid->nt;
  g.dz = grid->dz;
  g.dx = grid->dx;
  g.dt = grid->dt;
  g.sponge_a = grid->sponge_a;
  rtm_img_opts o{};
  o.src_mode = RTM_SRC_RECONSTRUCT;
  o.snap_stride = 1;
  if (opts) o = *opts;
  if (o.src_mode == RTM_SRC_RECONSTRUCT) {
    g.mode = kModeRecon;
    g.snap_stride = 1;
  } else if (o.src_mode == RTM_SRC_STORE) {
    g.mode = kModeStore;
    g.snap_stride = o.snap_stride;
    g.snap_dtype = o.snap_dtype;
  } else {
    return fail(RTM_E_INVAL, "unknown src_mode %d", o.src_mode);
  }
  g.flags = o.flags;
  g.nrec = nrec;
  return RTM_OK;
}

extern "C" int rtm_migrate_shot(rtm_ctx* ctx, const rtm_grid* grid, const float* vel_dev,
                                const float* wavelet_dev, rtm_point src, int32_t nrec,
                                const rtm_point* rec_host, const float* data_dev, int32_t ix0,
                                int32_t width, const rtm_img_opts* opts, float* image_dev,
                                float* illum_dev) {
  if (!ctx) return fail(RTM_E_INVAL, "ctx is NULL");
  int rc = check_grid(grid);
  if (rc) return rc;
  if (!vel_dev || !wavelet_dev || !image_dev) return fail(RTM_E_INVAL, "vel_dev, wavelet_dev, image_dev are required");
  if (nrec > 0 && !data_dev) return fail(RTM_E_INVAL, "data_dev is required when nrec > 0");
  JobGeom g;
  if ((rc = fill_geom_rtm(grid, ix0, width, opts, nrec, g))) return rc;
  if (illum_dev && !(g.flags & RTM_IMG_ILLUM)) g.flags |= RTM_IMG_ILLUM;
  if ((rc = check_job(g, src, rec_host))) return rc;
  HIP_OK(hipSetDevice(ctx->device));
  hipStream_t s = ctx->stream;
  float vmax = 0;
  if ((rc = device_vmax(ctx, s, vel_dev, g.nz, g.model_nx, ix0, width, &vmax))) return rc;
  if ((rc = check_cfl(vmax, g.dt, g.dz, g.dx))) return rc;
  const int tz = autotune_tz(ctx, s, g, vel_dev, 1);
  HostJob j;
  if ((rc = build_job(ctx, s, g, tz, vel_dev, wavelet_dev, src, rec_host, data_dev, nullptr, j, nullptr)))
    return rc;
  Table t;
  rc = run_plain(ctx, s, j, tz, t);
  if (!rc) {
    HIP_OK(launch_stack(image_dev, g.model_nx, ix0, j.d.image + g.nb, j.d.pitch, g.nz, width, s));
    HIP_OK(launch_nonfinite(j.d.image + g.nb, j.d.pitch, g.nz, width, ctx->scratch_u32 + 1, s));
    if (illum_dev && j.d.illum)
      HIP_OK(launch_stack(illum_dev, g.model_nx, ix0, j.d.illum + g.nb, j.d.pitch, g.nz, width, s));
    ctx->grid_updates += j.updates;
    ctx->alg_bytes += j.alg_bytes;
  }
  finish_job_deferred(ctx, s, j, t, false);
  return rc;
}

// ===========================================================================
// Batched path: all shots in every launch, hipGraph replays of K steps
// ===========================================================================
// Runs nsteps launches of the step kernel: whole groups of K as replays of a
// captured graph (K step launches with offsets 0..K-1, then one k_advance
// node), the remainder as direct launches followed by one k_advance.  The
// launches take their tiles from the control block (a range of the table,
// sized for up to grid[kind] tiles: one-step, forward and backward two-step),
// so one captured graph serves every group of shots; `*graph` keeps it.
// With `two_step` and a two-step table for the phase the launches go two
// steps each; an odd last step runs as a one-step launch.  The caller starts
// the backward phase with two one-step launches (levels nt - 1 and nt - 2 are
// not reconstructed) before it asks for pairs.
static int graph_steps(rtm_ctx* ctx, hipStream_t s, StepCtl* ctl, int tz, int ph, Table& t, const int (&grid)[3],
                       int nsteps, int K, hipGraphExec_t* graph, bool two_step) {
  const Table::TwoStep& tw = ph == kPhFwd ? t.fw : t.bw;
  const bool pairs = two_step && tw.ntiles > 0 && (ph == kPhFwd || ph == kPhBwd);
  const int store = !t.hjobs->empty() && (*t.hjobs)[0].mode == kModeStore;  // one mode per batch
  if (pairs) K = std::max(2, K & ~1);
  auto one = [&](int off, int left) -> hipError_t {  // the launch at offset `off`
    if (pairs && left >= 2)
      return launch_step2(tw.tz, ph, store, t.jobs, tw.tiles, tw.recs, -1, grid[ph == kPhFwd ? 1 : 2], ctl, 1, off, s);
    return launch_step(tz, ph, t.jobs, t.tiles, -1, grid[0], ctl, 1, off, s);
  };
  int done = 0;
  if (nsteps >= K && K > 1) {
    if (!*graph) {
      hipGraph_t g = nullptr;
      HIP_OK(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
      hipError_t e = hipSuccess;
      for (int i = 0; i < K && e == hipSuccess; i += pairs ? 2 : 1) e = one(i, K - i);
      if (e == hipSuccess) e = launch_advance(ctl, K, s);
      hipError_t e2 = hipStreamEndCapture(s, &g);
      if (e != hipSuccess || e2 != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        return fail(RTM_E_DEVICE, "graph capture failed: %s", hipGetErrorString(e != hipSuccess ? e : e2));
      }
      e = hipGraphInstantiate(graph, g, nullptr, nullptr, 0);
      (void)hipGraphDestroy(g);
      if (e != hipSuccess) {
        *graph = nullptr;
        return fail(RTM_E_DEVICE, "hipGraphInstantiate: %s", hipGetErrorString(e));
      }
    }
    for (; done + K <= nsteps; done += K) {
      HIP_OK(hipGraphLaunch(*graph, s));
      ctx->graph_replays++;
    }
  }
  if (done < nsteps) {
    for (int i = 0; done + i < nsteps;) {
      const int left = nsteps - done - i;
      HIP_OK(one(i, left));
      i += pairs && left >= 2 ? 2 : 1;
    }
    HIP_OK(launch_advance(ctl, nsteps - done, s));
  }
  ctx->steps_launched += nsteps;
  return RTM_OK;
}

// Shot groups of the batched path.  Every launch of a phase reads the levels
// the previous launch wrote; when the levels of all the shots in a launch fit
// in the memory-side cache (256 MB on MI355X) with room to spare, the next
// launch reads them from there instead of HBM.  So the shots run in groups,
// one group after another through a phase, each group's per-launch working
// set (the field bytes a launch reads or writes, the image, c once) at most
// the budget RTM_GROUP_KB (KiB, default 200 MiB; 0: one group).  Measured on
// the 351 x 1701 survey (nt 1000): 7.7 shots per backward launch and 14.3 per
// forward launch, 6.5 us and 2.8 us of launch time per shot, against 7.6 and
// 3.7 us with all 100 shots in every launch; larger groups spill out of the
// cache (11 shots per backward launch: 7.8 us per shot).  Groups are
// consecutive runs of jobs of near-equal working set.  When two streams run
// groups side by side, each group takes half the budget.
static size_t group_budget() {
  const char* e = getenv("RTM_GROUP_KB");
  const long v = e ? atol(e) : 200 << 10;
  return v <= 0 ? SIZE_MAX : (size_t)v << 10;
}

// Running-set budget of the serving engine (RTM_SERVE_KB, KiB; unset or 0:
// none, admission is limited by the arena only).  Unlike the batch path's
// shot groups it did not pay off on the served workloads: the 1024-RTM
// ensemble ran at 3.94e11 updates/s without it and 3.42e11, 3.72e11 and
// 3.82e11 at 128, 160 and 200 MiB (each job's own c counted), and the
// 400-job saturation run at 96.1 images/s without it and 86.0 / 98.6 at 200
// / 400 MiB (c not counted); served jobs own their c and the running set
// then splits into smaller launches.
static size_t serve_budget() {
  const char* e = getenv("RTM_SERVE_KB");
  const long v = e ? atol(e) : 0;
  return v <= 0 ? SIZE_MAX : (size_t)v << 10;
}

static size_t launch_working_set(const JobGeom& g, int ph) {
  const size_t row = (size_t)field_pitch(g.width + 2 * g.nb) * 4;
  const size_t pad = (size_t)(g.nz + 2 * g.nb) * row, phys = (size_t)g.nz * row;
  if (ph == kPhFwd) return 4 * pad;  // two levels read, two written
  // R: two levels read, two written; S likewise on the window, and the image
  // (reconstruct mode); a stored snapshot and the image (store mode)
  return 4 * pad + (g.mode == kModeRecon ? 5 * phys : 2 * phys);
}

// A served job's share: its backward launch's field bytes and its own c.
static size_t served_working_set(const JobGeom& g) {
  return launch_working_set(g, kPhBwd) + (size_t)(g.nz + 2 * g.nb) * field_pitch(g.width + 2 * g.nb) * 4;
}

static std::vector<std::pair<int, int>> shot_groups(const std::vector<JobGeom>& gs, int ph, int streams) {
  std::vector<std::pair<int, int>> out;
  const int n = (int)gs.size();
  if (n == 0) return out;
  size_t total = 0, medium = 0;
  for (const JobGeom& g : gs) {
    total += launch_working_set(g, ph);
    medium = std::max(medium, (size_t)(g.nz + 2 * g.nb) * field_pitch(g.width + 2 * g.nb) * 4);  // c
  }
  const size_t budget = group_budget() == SIZE_MAX ? SIZE_MAX : group_budget() / streams;
  if (budget == SIZE_MAX || total + medium <= budget) return {{0, n}};
  const size_t room = budget > medium ? budget - medium : 1;
  const int ngroups = (int)std::min<size_t>(n, (total + room - 1) / room);
  if (ngroups == n) {  // one job per group
    for (int i = 0; i < n; ++i) out.push_back({i, i + 1});
    return out;
  }
  // job i joins group floor(ngroups x (middle of its share) / total), a
  // non-decreasing index: runs of near-equal working set
  size_t before = 0;
  int last = -1;
  for (int i = 0; i < n; ++i) {
    const size_t w = launch_working_set(gs[i], ph);
    const int gi = (int)std::min<size_t>(ngroups - 1, (2 * before + w) * ngroups / (2 * total));
    if (gi != last) {
      out.push_back({i, i + 1});
      last = gi;
    } else {
      out.back().second = i + 1;
    }
    before += w;
  }
  return out;
}

// Streams the batched path runs its shot groups on (RTM_GROUP_STREAMS, 1 to
// 4; default 2).  With several, the groups go to the work stream and the
// context's further group streams in turn, each stream with its own control
// block and captured graphs, so one group's launches fill the workgroup
// slots another group's launch leaves idle as it drains; each group then
// gets its share of the cache budget.  Measured on the 351 x 1701 survey
// (nt 1000, 200 MiB): 484 ms per migration of 100 shots on two streams
// against 512 ms on one; one stream with groups of the two-stream size took
// 572 ms, so the gain is the overlap, not the smaller groups.  Three and
// four streams (smaller groups again) took 550 and 522 ms.
static int group_streams() {
  const char* e = getenv("RTM_GROUP_STREAMS");
  const int v = e ? atoi(e) : 2;
  return std::max(1, std::min(v, kMaxGroupStreams));
}

// One phase of the batch, group by group: the group's control block is
// pointed at its tile ranges with the tick at `tick0`, then the group's
// steps run (a backward phase with two-step tiles opens with two one-step
// launches).  Group i runs on stream i mod nstreams (stream 0: s), the
// further streams forked from s and joined back into it before the call
// returns (also on an error, so that work deferred on s waits for them).
// graph[k] keeps stream k's captured graph.
static int run_phase_groups(rtm_ctx* ctx, hipStream_t s, int nstreams, int tz, int ph, Table& t,
                            const std::vector<std::pair<int, int>>& groups, int tick0, int nsteps, int K,
                            hipGraphExec_t (&graph)[kMaxGroupStreams], bool two_step) {
  const Table::TwoStep& tw = ph == kPhFwd ? t.fw : t.bw;
  const bool pairs = two_step && tw.ntiles > 0;
  const bool store = !t.hjobs->empty() && (*t.hjobs)[0].mode == kModeStore;  // one mode per batch
  const int ns = std::max(1, std::min<int>(nstreams, (int)groups.size()));
  int grid[3] = {0, 0, 0};
  for (auto [a, b] : groups) {
    grid[0] = std::max(grid[0], t.first[b] - t.first[a]);
    if (pairs) grid[ph == kPhFwd ? 1 : 2] = std::max(grid[ph == kPhFwd ? 1 : 2], tw.first[b] - tw.first[a]);
  }
  if (ns > 1) {
    HIP_OK(hipEventRecord(ctx->ev_fork, s));
    for (int k = 1; k < ns; ++k) HIP_OK(hipStreamWaitEvent(ctx->group_stream[k - 1], ctx->ev_fork, 0));
  }
  auto run = [&](int gi, int a, int b) -> int {
    const int side = gi % ns;
    hipStream_t gs = side ? ctx->group_stream[side - 1] : s;
    StepCtl* ctl = side ? t.side_ctl[side - 1] : t.ctl;
    StepCtl c{};
    c.tick = tick0;
    c.ntiles = t.first[b] - t.first[a];
    c.base = t.first[a];
    if (pairs && ph == kPhFwd) {
      c.ntiles_fw = tw.first[b] - tw.first[a];
      c.base_fw = tw.first[a];
    } else if (pairs) {
      c.ntiles_bw = tw.first[b] - tw.first[a];
      c.base_bw = tw.first[a];
    }
    HIP_OK(launch_set_ctl(ctl, c, gs));
    if (ph == kPhBwd && pairs && nsteps >= 4) {
      // levels nt - 1 and nt - 2 are imaged without reconstruction: one step each
      for (int i = 0; i < 2; ++i) HIP_OK(launch_step(tz, kPhBwd, t.jobs, t.tiles, -1, grid[0], ctl, 1, i, gs));
      HIP_OK(launch_advance(ctl, 2, gs));
      ctx->steps_launched += 2;
      return graph_steps(ctx, gs, ctl, tz, ph, t, grid, nsteps - 2, K, &graph[side], true);
    }
    if (ph == kPhFwd && pairs && store) {
      // store mode: pairs as long as a forward step follows them (two_step_pair),
      // then one step per launch
      const int np = (nsteps - 1) & ~1;
      const int rc = graph_steps(ctx, gs, ctl, tz, ph, t, grid, np, K, &graph[side], true);
      if (rc) return rc;
      for (int i = 0; i < nsteps - np; ++i)
        HIP_OK(launch_step(tz, kPhFwd, t.jobs, t.tiles, -1, grid[0], ctl, 1, i, gs));
      if (nsteps > np) {
        HIP_OK(launch_advance(ctl, nsteps - np, gs));
        ctx->steps_launched += nsteps - np;
      }
      return RTM_OK;
    }
    return graph_steps(ctx, gs, ctl, tz, ph, t, grid, nsteps, K, &graph[side], pairs && ph == kPhFwd);
  };
  int rc = RTM_OK;
  for (int gi = 0; gi < (int)groups.size() && !rc; ++gi) rc = run(gi, groups[gi].first, groups[gi].second);
  for (int k = 1; k < ns; ++k) {
    hipStream_t gs = ctx->group_stream[k - 1];
    const bool joined = hipEventRecord(ctx->ev_join[k - 1], gs) == hipSuccess &&
                        hipStreamWaitEvent(s, ctx->ev_join[k - 1], 0) == hipSuccess;
    if (!joined) {
      (void)hipStreamSynchronize(gs);
      if (!rc) rc = fail(RTM_E_DEVICE, "joining a group stream failed");
    }
  }
  return rc;
}

static int graph_k() {
  const char* e = getenv("RTM_GRAPH_STEPS");
  int k = e ? atoi(e) : 64;
  return k < 1 ? 1 : k;
}

extern "C" int rtm_migrate_batch(rtm_ctx* ctx, const rtm_grid* grid, const float* vel_dev,
                                 const float* wavelet_dev, int32_t nshots, const rtm_shot_desc* shots,
                                 const rtm_img_opts* opts, float* image_dev, float* illum_dev) {
  if (!ctx) return fail(RTM_E_INVAL, "ctx is NULL");
  int rc = check_grid(grid);
  if (rc) return rc;
  if (nshots < 1 || !shots) return fail(RTM_E_INVAL, "need at least one shot");
  if (!vel_dev || !wavelet_dev || !image_dev) return fail(RTM_E_INVAL, "vel_dev, wavelet_dev, image_dev are required");
  std::vector<JobGeom> geoms(nshots);
  for (int i = 0; i < nshots; ++i) {
    if ((rc = fill_geom_rtm(grid, shots[i].ix0, shots[i].width, opts, shots[i].nrec, geoms[i]))) return rc;
    if (illum_dev) geoms[i].flags |= RTM_IMG_ILLUM;
    if (pairs_mode(geoms[i]) && !illum_dev && two_step_on())
      geoms[i].nbuf = 4;  // two-step launches
    if ((rc = check_job(geoms[i], shots[i].src, shots[i].rec_host))) return rc;
    if (shots[i].nrec > 0 && !shots[i].data_dev) return fail(RTM_E_INVAL, "shot %d has no data", i);
  }
  size_t need = 0;
  for (int i = 0; i < nshots; ++i) {
    need += footprint(geoms[i]).total;
    for (int k = 0; k < i; ++k)
      if (same_medium(geoms[k], geoms[i])) {  // reads shot k's medium
        need -= medium_bytes(geoms[i]);
        break;
      }
  }
  if (need > ctx->arena.size())
    return fail(RTM_E_NOMEM, "batch needs %zu bytes, arena holds %zu", need, ctx->arena.size());
  HIP_OK(hipSetDevice(ctx->device));
  // All batch work runs on the library's work stream, ordered after and
  // before the caller's stream by events (capture is not allowed on the
  // legacy null stream).
  hipStream_t s = ctx->work_stream;
  HIP_OK(hipEventRecord(ctx->ev_in, ctx->stream));
  HIP_OK(hipStreamWaitEvent(s, ctx->ev_in, 0));
  float vmax = 0;
  if ((rc = device_vmax(ctx, s, vel_dev, grid->nz, grid->nx, 0, grid->nx, &vmax))) return rc;
  if ((rc = check_cfl(vmax, grid->dt, grid->dz, grid->dx))) return rc;
  // tile height for the widest window of the batch
  int widest = 0;
  for (int i = 1; i < nshots; ++i)
    if (geoms[i].width > geoms[widest].width) widest = i;
  const int tz = autotune_tz(ctx, s, geoms[widest], vel_dev, nshots);
  // shot groups of each phase; two-step heights, tuned at the size of the
  // backward groups (the dominant launches) before the batch takes its
  // arena blocks
  const int nstreams = group_streams();
  const auto gf = shot_groups(geoms, kPhFwd, nstreams), gb = shot_groups(geoms, kPhBwd, nstreams);
  int gmax = 1;
  for (auto [a, b] : gb) gmax = std::max(gmax, b - a);
  int tz2f = 0, tz2b = 0;
  if (geoms[widest].nbuf == 4) autotune_tz2(ctx, s, geoms[widest], vel_dev, gmax, &tz2f, &tz2b);
  std::vector<std::unique_ptr<HostJob>> jobs;
  std::vector<HostJob*> ptrs;
  auto cleanup = [&]() {
    for (auto& j : jobs) {
      release_blocks(ctx, j->blocks);
      if (j->image_blk.p) ctx->arena.release(j->image_blk.p, j->image_blk.n);
    }
  };
  for (int i = 0; i < nshots; ++i) {
    auto j = std::make_unique<HostJob>();
    const HostJob* medium = nullptr;
    for (auto& o : jobs)
      if (o->owns_medium && same_medium(o->g, geoms[i])) {
        medium = o.get();
        break;
      }
    rc = build_job(ctx, s, geoms[i], tz, vel_dev, wavelet_dev, shots[i].src, shots[i].rec_host,
                   shots[i].data_dev, nullptr, *j, medium);
    if (rc) {
      (void)hipStreamSynchronize(s);
      cleanup();
      return rc;
    }
    ptrs.push_back(j.get());
    jobs.push_back(std::move(j));
  }
  Table t;
  if ((rc = upload_table(ctx, s, ptrs, t, tz2f, tz2b))) {
    cleanup();
    return rc;
  }
  const int nt = grid->nt, K = graph_k();
  hipGraphExec_t graphs[2][kMaxGroupStreams] = {};  // [phase][stream]
  HIP_OK(hipEventRecord(ctx->ph_ev[0], s));
  roctxRangePushA("rtm.batch.forward");  // host-side enqueue of the phase
  rc = run_phase_groups(ctx, s, nstreams, tz, kPhFwd, t, gf, 0, nt - 1, K, graphs[0], true);
  roctxRangePop();
  roctxRangePushA("rtm.batch.backward");
  if (!rc) rc = hipEventRecord(ctx->ph_ev[1], s) == hipSuccess ? RTM_OK : fail(RTM_E_DEVICE, "event record");
  if (!rc) rc = run_phase_groups(ctx, s, nstreams, tz, kPhBwd, t, gb, nt - 1, nt, K, graphs[1], t.bw.ntiles > 0 && nt >= 4);
  roctxRangePop();
  if (!rc) rc = hipEventRecord(ctx->ph_ev[2], s) == hipSuccess ? RTM_OK : fail(RTM_E_DEVICE, "event record");
  if (!rc) {
    // algorithmic bytes of one forward / one backward launch over all shots
    uint64_t bf = 0, bb = 0;
    for (auto& j : jobs) {
      const JobGeom& g = j->g;
      const uint64_t Npad = (uint64_t)(g.nz + 2 * g.nb) * (g.width + 2 * g.nb), Nph = (uint64_t)g.nz * g.width;
      const uint64_t ring = ring_len_of(g.nz, g.width);
      const uint64_t u = j->owns_medium ? 16 : 12;  // c counted once per medium
      bf += Npad * u + (g.mode == kModeRecon ? ring * 4 : 0);
      bb += Npad * u + (uint64_t)g.nrec * 4;
      // interior: S^{m+1}, S^{m+2} read + S^m written (12 B) + image (8 B); ring: stored value read + S^m written
      if (g.mode == kModeRecon) bb += Nph * 20 - ring * 4;
    }
    ctx->ph_launches[0] = nt - 1;
    ctx->ph_launches[1] = nt;
    ctx->ph_groups[0] = (int)gf.size();
    ctx->ph_groups[1] = (int)gb.size();
    ctx->ph_steps_per_launch = t.fw.ntiles > 0 && t.bw.ntiles > 0 && nt >= 4 ? 2 : 1;  // both phases ran pairs
    ctx->ph_tz2[0] = t.fw.ntiles > 0 && nt >= 3 ? t.fw.tz : 0;
    ctx->ph_tz2[1] = t.bw.ntiles > 0 && nt >= 4 ? t.bw.tz : 0;
    ctx->ph_bytes[0] = bf;
    ctx->ph_bytes[1] = bb;
    ctx->ph_valid = true;
  }
  if (!rc) {
    for (int i = 0; i < nshots && !rc; ++i) {
      const DevJob& d = jobs[i]->d;
      hipError_t e = launch_stack(image_dev, grid->nx, geoms[i].ix0, d.image + d.nb, d.pitch, grid->nz,
                                  geoms[i].width, s);
      if (e == hipSuccess)
        e = launch_nonfinite(d.image + d.nb, d.pitch, grid->nz, geoms[i].width, ctx->scratch_u32 + 1, s);
      if (e == hipSuccess && illum_dev)
        e = launch_stack(illum_dev, grid->nx, geoms[i].ix0, d.illum + d.nb, d.pitch, grid->nz, geoms[i].width, s);
      if (e != hipSuccess) rc = fail(RTM_E_DEVICE, "stack launch failed: %s", hipGetErrorString(e));
    }
  }
  Deferred d;
  for (auto& j : jobs) {
    for (auto& b : j->blocks) d.blocks.push_back(b);
    j->blocks.clear();
    if (j->image_blk.p) d.blocks.push_back(j->image_blk);
    ctx->grid_updates += rc ? 0 : j->updates;
    ctx->alg_bytes += rc ? 0 : j->alg_bytes;
  }
  for (auto& b : t.blocks) d.blocks.push_back(b);
  keep_table(d, t);
  for (auto& gp : graphs)
    for (auto g : gp)
      if (g) d.graphs.push_back(g);
  int rc2 = defer(ctx, s, std::move(d));
  HIP_OK(hipEventRecord(ctx->ev_out, s));
  HIP_OK(hipStreamWaitEvent(ctx->stream, ctx->ev_out, 0));
  return rc ? rc : rc2;
}

// ===========================================================================
// Ensemble path: model bank, job queue, scheduler thread
// ===========================================================================
extern "C" int rtm_model_register(rtm_ctx* ctx, int32_t realization, const float* vel_dev, int32_t nz,
                                  int32_t nx, const rtm_grid* grid) {
  if (!ctx) return fail(RTM_E_INVAL, "ctx is NULL");
  int rc = check_grid(grid);
  if (rc) return rc;
  if (!vel_dev || nz != grid->nz || nx != grid->nx)
    return fail(RTM_E_INVAL, "velocity [%d][%d] does not match the grid [%d][%d]", nz, nx, grid->nz, grid->nx);
  HIP_OK(hipSetDevice(ctx->device));
  std::unique_lock<std::mutex> lk(ctx->mu);
  if (!ctx->models.empty()) {
    const Model& m0 = ctx->models.begin()->second;
    if (m0.nz != nz || m0.nx != nx)
      return fail(RTM_E_INVAL, "all registered models must share one size (%d x %d)", m0.nz, m0.nx);
  }
  if (ctx->book->in_flight(realization) > 0)
    return fail(RTM_E_AGAIN, "realization %d has jobs in flight", realization);
  lk.unlock();
  Block vb;
  vb.n = align256((size_t)nz * nx * 4);
  vb.p = arena_alloc(ctx, vb.n);
  if (!vb.p) return fail(RTM_E_NOMEM, "arena exhausted (velocity bank)");
  hipStream_t s = ctx->stream;
  hipError_t e = hipMemcpyAsync(vb.p, vel_dev, (size_t)nz * nx * 4, hipMemcpyDeviceToDevice, s);
  float vmax = 0;
  if (e != hipSuccess || (rc = device_vmax(ctx, s, static_cast<float*>(vb.p), nz, nx, 0, nx, &vmax))) {
    ctx->arena.release(vb.p, vb.n);
    return e != hipSuccess ? fail(RTM_E_DEVICE, "copy failed: %s", hipGetErrorString(e)) : rc;
  }
  lk.lock();
  // Re-check under the lock: a job of this realization may have been queued,
  // or a model of another size registered, while the copy ran unlocked.
  const bool busy = ctx->book->in_flight(realization) > 0;
  bool other_size = false;
  for (auto& kv : ctx->models)
    if (kv.first != realization && (kv.second.nz != nz || kv.second.nx != nx)) other_size = true;
  if (busy || other_size) {
    ctx->arena.release(vb.p, vb.n);  // the copy and the v_max pass have finished (synchronised)
    return busy ? fail(RTM_E_AGAIN, "realization %d has jobs in flight", realization)
                : fail(RTM_E_INVAL, "all registered models must share one size");
  }
  Model& m = ctx->models[realization];
  if (m.vel.p) {
    // jobs that read the old velocity have finished, but release it behind
    // whatever the scheduler stream still holds
    Deferred d;
    d.blocks.push_back(m.vel);
    if (int drc = defer(ctx, ctx->sched_stream, std::move(d))) return drc;
  }
  m.nz = nz;
  m.nx = nx;
  m.grid = *grid;
  m.vel = vb;
  m.vmax = vmax;
  return RTM_OK;
}

extern "C" int rtm_ensemble_submit(rtm_ctx* ctx, const rtm_job* job, uint64_t* ticket) {
  if (!ctx || !job || !ticket) return fail(RTM_E_INVAL, "ctx, job and ticket are required");
  std::unique_lock<std::mutex> lk(ctx->mu);
  auto it = ctx->models.find(job->realization);
  if (it == ctx->models.end()) return fail(RTM_E_NOTFOUND, "realization %d is not registered", job->realization);
  Model& m = it->second;
  rtm_grid gr = m.grid;
  gr.nt = job->nt;
  int rc = check_grid(&gr);
  if (rc) return rc;
  if (!job->wavelet_dev || !job->data_dev) return fail(RTM_E_INVAL, "wavelet_dev and data_dev are required");
  JobGeom g;
  if ((rc = fill_geom_rtm(&gr, job->ix0, job->width, &job->img, job->width, g))) return rc;
  // receivers: every window column at row rec_iz
  if (job->rec_iz < 0 || job->rec_iz >= gr.nz) return fail(RTM_E_INVAL, "rec_iz %d outside the model", job->rec_iz);
  rtm_point probe{job->rec_iz, job->ix0};
  g.nrec = 0;
  if ((rc = check_job(g, job->src, &probe))) return rc;
  g.nrec = job->width;
  if (served_two_step(g)) g.nbuf = 4;  // as the scheduler builds it
  if ((rc = check_cfl(m.vmax, gr.dt, gr.dz, gr.dx))) return rc;
  uint64_t t = 0;
  rc = ctx->book->submit(job->realization, footprint(g).total, &t);
  if (rc == kSchedNomem)
    return fail(RTM_E_NOMEM, "job needs %zu bytes, larger than the whole arena (%zu)", footprint(g).total,
                ctx->arena.size());
  if (rc == kSchedAgain) return fail(RTM_E_AGAIN, "queue full (%zu jobs)", ctx->book->queued());
  auto ej = std::make_unique<EnsJob>();
  ej->ticket = t;
  ej->spec = *job;
  *ticket = t;
  ctx->jobs.emplace(t, std::move(ej));
  if (!ctx->sched_started) {
    ctx->sched_started = true;
    ctx->sched = std::thread(sched_main, ctx);
  }
  lk.unlock();
  ctx->cv.notify_all();
  return RTM_OK;
}

// Allocates a realization's statistics (mean, M2, count) and stack on first
// use.  All-or-nothing: the three statistics blocks are taken together or
// not at all, so a Model never holds a partial set (a later job would
// otherwise be admitted and its Welford update write through a null M2).
static int ensure_stats(rtm_ctx* ctx, hipStream_t s, Model& m, bool stats, bool stack) {
  const size_t n = (size_t)m.nz * m.nx;
  if (stats && !m.mean.p) {
    Block mean{arena_alloc(ctx, n * 8), align256(n * 8)};
    Block m2{mean.p ? arena_alloc(ctx, n * 8) : nullptr, align256(n * 8)};
    Block count{m2.p ? arena_alloc(ctx, n * 4) : nullptr, align256(n * 4)};
    if (!mean.p || !m2.p || !count.p) {
      ctx->arena.release(mean.p, mean.n);
      ctx->arena.release(m2.p, m2.n);
      ctx->arena.release(count.p, count.n);
      return fail(RTM_E_NOMEM, "arena exhausted (statistics)");
    }
    HIP_OK(launch_fill_u32(static_cast<uint32_t*>(mean.p), 0, (int64_t)(n * 2), s));
    HIP_OK(launch_fill_u32(static_cast<uint32_t*>(m2.p), 0, (int64_t)(n * 2), s));
    HIP_OK(launch_fill_u32(static_cast<uint32_t*>(count.p), 0, (int64_t)n, s));
    m.mean = mean;
    m.m2 = m2;
    m.count = count;
  }
  if (stack && !m.stack.p) {
    Block st{arena_alloc(ctx, n * 4), align256(n * 4)};
    if (!st.p) return fail(RTM_E_NOMEM, "arena exhausted (stack)");
    HIP_OK(launch_fill_u32(static_cast<uint32_t*>(st.p), 0, (int64_t)n, s));
    m.stack = st;
  }
  return RTM_OK;
}

static bool has_stats(const Model& m) { return m.mean.p && m.m2.p && m.count.p; }

// Device tables of the serving engine's launches.  A job that takes two-step
// launches (reconstruct or store mode without illumination, marked two_step) is in
// the forward or backward two-step table for the cycles in which it has a
// step pair of that phase, and in the one-step table for the cycles in
// which it has a step that no pair covers (the first backward levels, an odd
// phase boundary, a last single level); every other job is in the one-step
// table.  The tables are rebuilt when the active jobs or these memberships
// change.
struct SchedTables {
  std::vector<Block> blocks;
  DevJob* jobs = nullptr;
  Tile* tiles = nullptr;                              // one-step tiles
  Tile* tiles_f = nullptr;                            // two-step tiles, forward phase
  Tile* tiles_b = nullptr;                            // two-step tiles, backward phase
  int2* recs_f = nullptr;                             // their receivers
  int2* recs_b = nullptr;
  StepCtl* ctl = nullptr;
  size_t cap_jobs = 0, cap_tiles = 0, cap_f = 0, cap_b = 0, cap_rf = 0, cap_rb = 0;
  // launch buckets (one-step, forward, backward; modes present) -> graph
  std::map<std::array<int, 4>, hipGraphExec_t> graphs;
  std::vector<DevJob> hjobs;
  std::vector<Tile> htiles, htf, htb;
  std::vector<int2> hrf, hrb;
  std::vector<uint8_t> kinds;  // per active job: 1 one-step, 2 forward pairs, 4 backward pairs
  std::array<int32_t, 3> counts{};  // ntiles_fw, ntiles, ntiles_bw as the control block holds them
  int modes = 0;  // two-step tables: bit 0 forward reconstruct, 1 forward store, 2 backward reconstruct, 3 backward store
  hipEvent_t ev[2] = {nullptr, nullptr};  // around each cycle's launches
};

static int tile_bucket(int n) {
  int b = 256;
  while (b < n) b <<= 1;
  return b;
}

// Launch kinds a job needs in the cycle of ticks [tick, tick + K) (K even,
// jobs start at even ticks): 1 one-step launches, 2 forward pairs, 4
// backward pairs.
static uint8_t cycle_kinds(const DevJob& d, int tick, int K) {
  if (!d.two_step) return 1;
  uint8_t k = 0;
  for (int t = tick; t < tick + K; t += 2) {
    const int s = t - d.start_tick;
    if (s < 0 || s >= d.nsteps) continue;
    if (two_step_pair(s, d.nt, d.nsteps, d.mode)) k |= (s + 1 < d.nt - 1) ? 2 : 4;
    else k |= 1;
  }
  return k;
}

template <class T>
static int grow(rtm_ctx* ctx, SchedTables& Tb, T*& p, size_t& cap, size_t need) {
  if (need <= cap && p) return RTM_OK;
  cap = (size_t)tile_bucket((int)std::max<size_t>(need, 1));
  void* q = nullptr;
  if (!alloc_block(ctx, Tb.blocks, cap * sizeof(T), &q)) return fail(RTM_E_NOMEM, "arena exhausted (scheduler tables)");
  p = static_cast<T*>(q);
  return RTM_OK;
}

// K steps of every active job: one graph replay of K one-step launches, or,
// when jobs take two-step launches, K/2 rounds of (forward pairs, backward
// pairs, one-step launch of the even tick, one-step launch of the odd tick).
static int sched_cycle(rtm_ctx* ctx, SchedTables& T, std::vector<EnsJob*>& active, bool& changed, int& tick,
                       int tz, int tzf, int tzb, int K, float* cycle_ms) {
  hipStream_t s = ctx->sched_stream;
  RoctxRange range("rtm.sched.cycle");
  *cycle_ms = 0;
  if (!T.ev[0]) {
    HIP_OK(hipEventCreate(&T.ev[0]));
    HIP_OK(hipEventCreate(&T.ev[1]));
  }
  std::vector<uint8_t> kinds(active.size());
  for (size_t i = 0; i < active.size(); ++i) kinds[i] = cycle_kinds(active[i]->job->d, tick, K);
  if (changed || kinds != T.kinds) {
    T.hjobs.clear();
    T.htiles.clear();
    T.htf.clear();
    T.htb.clear();
    T.hrf.clear();
    T.hrb.clear();
    for (size_t i = 0; i < active.size(); ++i) {
      const HostJob& j = *active[i]->job;
      T.hjobs.push_back(j.d);
      if (kinds[i] & 1)
        for (Tile tl : j.tiles) {
          tl.job = (int)i;
          T.htiles.push_back(tl);
        }
      if (kinds[i] & 2) append_two_step_tiles(j, (int)i, tzf, T.htf, T.hrf);
      if (kinds[i] & 4) append_two_step_tiles(j, (int)i, tzb, T.htb, T.hrb);
    }
    T.modes = 0;
    for (size_t i = 0; i < active.size(); ++i) {
      const int st = active[i]->job->d.mode == kModeStore ? 1 : 0;
      if (kinds[i] & 2) T.modes |= 1 << st;
      if (kinds[i] & 4) T.modes |= 4 << st;
    }
    const bool fits = T.hjobs.size() <= T.cap_jobs && T.htiles.size() <= T.cap_tiles && T.htf.size() <= T.cap_f &&
                      T.htb.size() <= T.cap_b && T.hrf.size() <= T.cap_rf && T.hrb.size() <= T.cap_rb && T.ctl;
    if (!fits) {  // new device tables (graphs hold the old pointers: drop them)
      HIP_OK(hipStreamSynchronize(s));
      for (auto& kv : T.graphs) (void)hipGraphExecDestroy(kv.second);
      T.graphs.clear();
      release_blocks(ctx, T.blocks);
      T.jobs = nullptr;
      T.tiles = T.tiles_f = T.tiles_b = nullptr;
      T.recs_f = T.recs_b = nullptr;
      T.ctl = nullptr;
      T.cap_jobs = T.cap_tiles = T.cap_f = T.cap_b = T.cap_rf = T.cap_rb = 0;
      size_t one = 1;
      if (int rc = grow(ctx, T, T.jobs, T.cap_jobs, std::max<size_t>(T.hjobs.size(), 64))) return rc;
      if (int rc = grow(ctx, T, T.tiles, T.cap_tiles, T.htiles.size())) return rc;
      if (int rc = grow(ctx, T, T.tiles_f, T.cap_f, T.htf.size())) return rc;
      if (int rc = grow(ctx, T, T.tiles_b, T.cap_b, T.htb.size())) return rc;
      if (int rc = grow(ctx, T, T.recs_f, T.cap_rf, T.hrf.size())) return rc;
      if (int rc = grow(ctx, T, T.recs_b, T.cap_rb, T.hrb.size())) return rc;
      if (int rc = grow(ctx, T, T.ctl, one, 1)) return rc;
      StepCtl c{};
      c.tick = tick;
      HIP_OK(hipMemcpyAsync(T.ctl, &c, sizeof c, hipMemcpyHostToDevice, s));
    }
    auto up = [&](void* dst, const void* src, size_t bytes) -> hipError_t {
      return bytes ? hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, s) : hipSuccess;
    };
    HIP_OK(up(T.jobs, T.hjobs.data(), T.hjobs.size() * sizeof(DevJob)));
    HIP_OK(up(T.tiles, T.htiles.data(), T.htiles.size() * sizeof(Tile)));
    HIP_OK(up(T.tiles_f, T.htf.data(), T.htf.size() * sizeof(Tile)));
    HIP_OK(up(T.tiles_b, T.htb.data(), T.htb.size() * sizeof(Tile)));
    HIP_OK(up(T.recs_f, T.hrf.data(), T.hrf.size() * sizeof(int2)));
    HIP_OK(up(T.recs_b, T.hrb.data(), T.hrb.size() * sizeof(int2)));
    T.counts = {(int32_t)T.htf.size(), (int32_t)T.htiles.size(), (int32_t)T.htb.size()};
    HIP_OK(up(&T.ctl->ntiles_fw, T.counts.data(), sizeof(int32_t) * 3));
    HIP_OK(hipStreamSynchronize(s));  // the host staging is reused next time
    T.kinds = kinds;
    changed = false;
  }
  const int n1 = T.counts[1], nf = T.counts[0], nb = T.counts[2];
  const std::array<int, 4> key = {n1 ? tile_bucket(n1) : 0, nf ? tile_bucket(nf) : 0, nb ? tile_bucket(nb) : 0,
                                  T.modes};
  auto git = T.graphs.find(key);
  if (git == T.graphs.end()) {
    hipGraph_t g = nullptr;
    HIP_OK(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
    hipError_t e0 = hipSuccess;
    if (!key[1] && !key[2]) {
      for (int i = 0; i < K && e0 == hipSuccess; ++i)
        e0 = launch_step(tz, kPhAny, T.jobs, T.tiles, -1, key[0], T.ctl, 1, i, s, 1);
    } else {
      for (int i = 0; i < K && e0 == hipSuccess; i += 2) {
        // one launch per phase and job mode present (each kernel instance
        // takes the tiles of its mode's jobs and passes over the others)
        for (int st = 0; st < 2 && e0 == hipSuccess; ++st) {
          if (key[1] && (key[3] & (1 << st)))
            e0 = launch_step2(tzf, kPhFwd, st, T.jobs, T.tiles_f, T.recs_f, -1, key[1], T.ctl, 1, i, s);
          if (e0 == hipSuccess && key[2] && (key[3] & (4 << st)))
            e0 = launch_step2(tzb, kPhBwd, st, T.jobs, T.tiles_b, T.recs_b, -1, key[2], T.ctl, 1, i, s);
        }
        for (int k = 0; k < 2 && key[0] && e0 == hipSuccess; ++k)
          e0 = launch_step(tz, kPhAny, T.jobs, T.tiles, -1, key[0], T.ctl, 1, i + k, s, 1);
      }
    }
    if (e0 == hipSuccess) e0 = launch_advance(T.ctl, K, s);
    hipError_t e1 = hipStreamEndCapture(s, &g);
    if (e0 != hipSuccess || e1 != hipSuccess) {
      if (g) (void)hipGraphDestroy(g);
      return fail(RTM_E_DEVICE, "graph capture failed: %s", hipGetErrorString(e0 != hipSuccess ? e0 : e1));
    }
    hipGraphExec_t ex = nullptr;
    hipError_t e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) return fail(RTM_E_DEVICE, "hipGraphInstantiate: %s", hipGetErrorString(e));
    git = T.graphs.emplace(key, ex).first;
  }
  HIP_OK(hipEventRecord(T.ev[0], s));
  HIP_OK(hipGraphLaunch(git->second, s));
  HIP_OK(hipEventRecord(T.ev[1], s));
  ctx->graph_replays++;
  ctx->steps_launched += K;
  tick += K;
  HIP_OK(hipStreamSynchronize(s));
  (void)hipEventElapsedTime(cycle_ms, T.ev[0], T.ev[1]);
  return RTM_OK;
}

// One JSON line per job reaching a final state, appended to the file named
// by RTM_LOG (opened at context creation): the job's request, state and
// status, host timestamps (s), queueing / running / total times (ms), its
// grid updates and algorithmic HBM bytes, and gpu_ms, its share of the
// launch time of the scheduler cycles it ran in (each cycle's HIP-event time
// split over the jobs in it in proportion to their algorithmic bytes per
// step).  Called with ctx->mu held.
static void log_job(rtm_ctx* ctx, const SchedEntry& e, const EnsJob& ej) {
  if (!ctx->job_log) return;
  static const char* kState[] = {"queued", "running", "done", "failed", "cancelled", "queued"};
  static const char* kMode[] = {"store", "reconstruct"};
  static const char* kDtype[] = {"fp32", "bf16", "fp16"};
  const rtm_job& j = ej.spec;
  const bool admitted = e.t_admit > 0;
  const int mode = j.img.src_mode == RTM_SRC_RECONSTRUCT ? 1 : 0;
  const int dt = j.img.snap_dtype >= 0 && j.img.snap_dtype <= 2 ? j.img.snap_dtype : 0;
  fprintf(ctx->job_log,
          "{\"ticket\": %llu, \"user_tag\": %llu, \"realization\": %d, \"state\": \"%s\", \"status\": %d, "
          "\"src\": [%d, %d], \"ix0\": %d, \"width\": %d, \"nt\": %d, \"mode\": \"%s\", \"snap_dtype\": \"%s\", "
          "\"snap_stride\": %d, \"t_submit\": %.6f, \"t_admit\": %.6f, \"t_done\": %.6f, \"queue_ms\": %.3f, "
          "\"run_ms\": %.3f, \"latency_ms\": %.3f, \"gpu_ms\": %.3f, \"grid_updates\": %llu, \"alg_bytes\": %llu}\n",
          (unsigned long long)e.ticket, (unsigned long long)j.user_tag, j.realization, kState[e.state], e.status,
          j.src.iz, j.src.ix, j.ix0, j.width, j.nt, kMode[mode], kDtype[dt], mode ? 1 : j.img.snap_stride, e.t_submit,
          e.t_admit, e.t_done, 1e3 * ((admitted ? e.t_admit : e.t_done) - e.t_submit),
          admitted ? 1e3 * (e.t_done - e.t_admit) : 0.0, 1e3 * (e.t_done - e.t_submit), ej.gpu_ms,
          (unsigned long long)(ej.job ? ej.job->updates : 0), (unsigned long long)(ej.job ? ej.job->alg_bytes : 0));
  fflush(ctx->job_log);
}

// The scheduler thread.  Each round: an admission pass over the queue (a
// candidate's working set is built without the context mutex; the JobBook
// marks it ADMITTING meanwhile), K steps of every admitted job in one graph
// replay, then the finished jobs' images go through the non-finite check
// into the statistics and stack, and their memory is released behind the
// stream.
static void sched_main(rtm_ctx* ctx) {
  (void)hipSetDevice(ctx->device);
  hipStream_t s = ctx->sched_stream;
  SchedTables T;
  std::vector<EnsJob*> active;
  bool changed = false;
  int tick = 0;  // advances by K, so every job starts at an even tick
  int tz = 0;    // tuned on the first admitted job; every job of the scheduler shares it
  int tzf = 0, tzb = 0;  // two-step heights, tuned on the first job that takes pairs (0: off)
  bool tz2_tuned = false;
  const int K = std::max(2, std::min(graph_k(), 64) & ~1);
  for (;;) {
    {
      std::unique_lock<std::mutex> lk(ctx->mu);
      if (ctx->stop) break;
      if (active.empty() && ctx->book->queued() == 0) {
        ctx->cv_done.notify_all();
        ctx->cv.wait(lk, [&] { return ctx->stop || ctx->book->queued() > 0; });
        continue;
      }
    }
    // ---- admission pass (first come, first served, bounded bypass) ----
    {
      RoctxRange range("rtm.sched.admit");
      AdmitPass pass;
      // field bytes the running jobs' launches touch: admission stops at
      // the budget (a job runs alone if it alone exceeds it)
      size_t running_ws = 0;
      for (EnsJob* a : active) running_ws += served_working_set(a->job->g);
      const size_t budget = serve_budget();
      for (;;) {
        uint64_t t = 0;
        EnsJob* ej = nullptr;
        JobGeom g;
        const float* vel = nullptr;
        int rc = RTM_OK;
        {
          std::lock_guard<std::mutex> lk(ctx->mu);
          if (ctx->stop) break;
          t = ctx->book->next_candidate(pass);
          if (!t) break;
          ej = ctx->jobs.at(t).get();
          Model& m = ctx->models[ej->spec.realization];
          rtm_grid gr = m.grid;
          gr.nt = ej->spec.nt;
          fill_geom_rtm(&gr, ej->spec.ix0, ej->spec.width, &ej->spec.img, ej->spec.width, g);
          if (served_two_step(g)) g.nbuf = 4;
          vel = static_cast<const float*>(m.vel.p);  // stable while the job is in flight
          const size_t ws = served_working_set(g);
          if (running_ws > 0 && budget != SIZE_MAX && running_ws + ws > budget) {
            ctx->book->admit_result(pass, t, kSchedAgain);  // the running set is full
            break;
          }
          running_ws += ws;
          rc = ensure_stats(ctx, s, m, ej->spec.flags & RTM_JOB_ACC_STATS, ej->spec.flags & RTM_JOB_ACC_STACK);
        }
        // the working set, built without the mutex (polls and submits go on)
        auto hj = std::make_unique<HostJob>();
        // The one-step tile height is tuned for a lone job (batch 1): at low
        // load a served job mostly runs alone, one small launch per step, and
        // its latency is those launches' duration, which the height sets;
        // under load the launches are large enough for any height.  On the
        // store-mode stream (300 timed jobs) the batch-16 tuner's 64 rows gave
        // p50 44 ms, p99 84 ms, 96.3 images/s at saturation; 16 rows 39 ms,
        // 79 ms, 96.9 images/s.
        if (!rc && tz == 0) tz = autotune_tz(ctx, s, g, vel, 1);
        const bool pairs = served_two_step(g);
        if (!rc && pairs && !tz2_tuned) {
          autotune_tz2(ctx, s, g, vel, 16, &tzf, &tzb);
          tz2_tuned = true;
        }
        if (!rc) {
          std::vector<rtm_point> recs(ej->spec.width);
          for (int r = 0; r < ej->spec.width; ++r) recs[r] = {ej->spec.rec_iz, ej->spec.ix0 + r};
          rc = build_job(ctx, s, g, tz, vel, ej->spec.wavelet_dev, ej->spec.src, recs.data(), ej->spec.data_dev,
                         nullptr, *hj, nullptr);
        }
        // steps that two-step launches take: only with heights whose last tile
        // stays inside this job's field allocation
        if (!rc && pairs && tzf > 0 && tzb > 0) {
          std::vector<HostJob*> one{hj.get()};
          hj->d.two_step = tz2_fits(one, tzf) && tz2_fits(one, tzb);
        }
        std::lock_guard<std::mutex> lk(ctx->mu);
        ctx->book->admit_result(pass, t, rc == RTM_E_NOMEM ? kSchedNomem : rc);
        if (rc == RTM_OK) {
          hj->d.start_tick = tick;
          ej->job = std::move(hj);
          active.push_back(ej);
          changed = true;
        } else {
          running_ws -= served_working_set(g);  // not admitted
          if (rc != RTM_E_NOMEM) log_job(ctx, *ctx->book->find(t), *ej);
        }
      }
    }
    if (active.empty()) {
      bool pending;
      {
        std::lock_guard<std::mutex> lk(ctx->defer_mu);
        pending = !ctx->deferred.empty();
      }
      if (pending) {  // memory is on its way back: wait for it, then retry
        reap(ctx, true);
        continue;
      }
      // Nothing runs and nothing is being freed, yet the head job does not
      // fit (the arena is held by results not yet released): fail it rather
      // than wait forever.
      std::lock_guard<std::mutex> lk(ctx->mu);
      if (uint64_t t = ctx->book->fail_head(RTM_E_NOMEM)) log_job(ctx, *ctx->book->find(t), *ctx->jobs.at(t));
      continue;
    }
    // ---- K steps of every active job ----
    float cycle_ms = 0;
    int rc = sched_cycle(ctx, T, active, changed, tick, tz, tzf, tzb, K, &cycle_ms);
    if (cycle_ms > 0) {
      double total = 0;
      for (EnsJob* ej : active) total += (double)ej->job->alg_bytes / ej->job->d.nsteps;
      for (EnsJob* ej : active)
        ej->gpu_ms += total > 0 ? cycle_ms * ((double)ej->job->alg_bytes / ej->job->d.nsteps) / total : 0.0;
    }
    // ---- finalise finished jobs ----
    std::vector<EnsJob*> still;
    std::vector<EnsJob*> finished;
    for (EnsJob* ej : active) {
      if (rc || ej->job->d.start_tick + ej->job->d.nsteps <= tick)
        finished.push_back(ej);
      else
        still.push_back(ej);
    }
    if (!finished.empty()) {
      RoctxRange range("rtm.sched.finalize");
      // non-finite check of every finished image before it reaches the statistics
      std::vector<uint32_t> health(finished.size(), 0);
      if (!rc) {
        for (size_t i = 0; i < finished.size(); ++i) {
          const HostJob& j = *finished[i]->job;
          (void)launch_nonfinite(j.d.image + j.g.nb, j.d.pitch, j.g.nz, j.g.width, j.d.health, s);
          (void)hipMemcpyAsync(&health[i], j.d.health, 4, hipMemcpyDeviceToHost, s);
        }
        (void)hipStreamSynchronize(s);
      }
      std::lock_guard<std::mutex> lk(ctx->mu);
      Deferred d;
      std::vector<int> status(finished.size());
      for (size_t fi = 0; fi < finished.size(); ++fi) {
        EnsJob* ej = finished[fi];
        HostJob& j = *ej->job;
        Model& m = ctx->models[ej->spec.realization];
        const int jrc = rc ? rc : (health[fi] ? RTM_E_NONFINITE : RTM_OK);
        status[fi] = jrc;
        if (!jrc) {
          if ((ej->spec.flags & RTM_JOB_ACC_STATS) && has_stats(m))
            (void)launch_welford(static_cast<double*>(m.mean.p), static_cast<double*>(m.m2.p),
                                 static_cast<int32_t*>(m.count.p), m.nx, j.d.image + j.g.nb, j.d.pitch,
                                 j.g.nz, j.g.width, j.g.ix0, s);
          if ((ej->spec.flags & RTM_JOB_ACC_STACK) && m.stack.p)
            (void)launch_stack(static_cast<float*>(m.stack.p), m.nx, j.g.ix0, j.d.image + j.g.nb, j.d.pitch,
                               j.g.nz, j.g.width, s);
          ctx->grid_updates += j.updates;
          ctx->alg_bytes += j.alg_bytes;
        }
        for (auto& b : j.blocks) d.blocks.push_back(b);
        j.blocks.clear();
      }
      (void)hipStreamSynchronize(s);  // the statistics include the job when it reads DONE
      for (size_t fi = 0; fi < finished.size(); ++fi) {
        ctx->book->finish(finished[fi]->ticket, status[fi]);
        log_job(ctx, *ctx->book->find(finished[fi]->ticket), *finished[fi]);
      }
      defer(ctx, s, std::move(d));
      active.swap(still);
      changed = true;
    }
    ctx->cv_done.notify_all();
  }
  (void)hipStreamSynchronize(s);
  for (auto& kv : T.graphs) (void)hipGraphExecDestroy(kv.second);
  for (auto e : T.ev)
    if (e) (void)hipEventDestroy(e);
  release_blocks(ctx, T.blocks);
  std::lock_guard<std::mutex> lk(ctx->mu);
  for (EnsJob* ej : active) {
    release_blocks(ctx, ej->job->blocks);
    ctx->book->cancel_running(ej->ticket);
  }
  ctx->cv_done.notify_all();
}

extern "C" int rtm_ensemble_poll(rtm_ctx* ctx, uint64_t ticket, rtm_job_info* info, float* image_dev,
                                 int32_t release) {
  if (!ctx) return fail(RTM_E_INVAL, "ctx is NULL");
  std::unique_lock<std::mutex> lk(ctx->mu);
  const SchedEntry* e = ctx->book->find(ticket);
  auto it = ctx->jobs.find(ticket);
  if (!e || it == ctx->jobs.end()) return fail(RTM_E_NOTFOUND, "unknown ticket %llu", (unsigned long long)ticket);
  EnsJob& ej = *it->second;
  const int state = JobBook::visible_state(*e);
  if (info) {
    info->state = state;
    info->status = e->status;
    info->t_submit = e->t_submit;
    info->t_admit = e->t_admit;
    info->t_done = e->t_done;
    info->grid_updates = ej.job ? ej.job->updates : 0;
    info->alg_bytes = ej.job ? ej.job->alg_bytes : 0;
    info->user_tag = ej.spec.user_tag;
  }
  const bool final = JobBook::final_state(state);
  if (state == RTM_JOB_DONE && image_dev && ej.job && ej.job->image_blk.p) {
    HIP_OK(hipSetDevice(ctx->device));
    const HostJob& hj = *ej.job;
    HIP_OK(hipMemcpy2DAsync(image_dev, (size_t)hj.g.width * 4, hj.d.image + hj.g.nb, (size_t)hj.d.pitch * 4,
                            (size_t)hj.g.width * 4, hj.g.nz, hipMemcpyDeviceToDevice, ctx->stream));
  }
  if (final && release) {
    Deferred d;
    if (ej.job && ej.job->image_blk.p) d.blocks.push_back(ej.job->image_blk);
    ctx->book->forget(ticket);
    ctx->jobs.erase(it);
    lk.unlock();
    return defer(ctx, ctx->stream, std::move(d));
  }
  return RTM_OK;
}

extern "C" int rtm_ensemble_cancel(rtm_ctx* ctx, uint64_t ticket) {
  if (!ctx) return fail(RTM_E_INVAL, "ctx is NULL");
  std::lock_guard<std::mutex> lk(ctx->mu);
  const int rc = ctx->book->cancel(ticket);
  if (rc == kSchedNotFound) return fail(RTM_E_NOTFOUND, "unknown ticket");
  if (rc != kSchedOk) return fail(RTM_E_INVAL, "job is no longer queued");
  log_job(ctx, *ctx->book->find(ticket), *ctx->jobs.at(ticket));
  ctx->cv_done.notify_all();
  return RTM_OK;
}

extern "C" int rtm_ensemble_drain(rtm_ctx* ctx) {
  if (!ctx) return fail(RTM_E_INVAL, "ctx is NULL");
  std::unique_lock<std::mutex> lk(ctx->mu);
  ctx->cv_done.wait(lk, [&] { return ctx->book->idle(); });
  lk.unlock();
  HIP_OK(hipSetDevice(ctx->device));
  HIP_OK(hipStreamSynchronize(ctx->sched_stream));
  return RTM_OK;
}

extern "C" int rtm_ensemble_stats(rtm_ctx* ctx, int32_t realization, double* mean_dev, double* std_dev,
                                  int32_t* count_dev) {
  if (!ctx) return fail(RTM_E_INVAL, "ctx is NULL");
  std::lock_guard<std::mutex> lk(ctx->mu);
  auto it = ctx->models.find(realization);
  if (it == ctx->models.end()) return fail(RTM_E_NOTFOUND, "realization %d is not registered", realization);
  Model& m = it->second;
  const int64_t n = (int64_t)m.nz * m.nx;
  HIP_OK(hipSetDevice(ctx->device));
  HIP_OK(hipStreamSynchronize(ctx->sched_stream));
  if (!has_stats(m)) {
    if (mean_dev) HIP_OK(hipMemsetAsync(mean_dev, 0, n * 8, ctx->stream));
    if (std_dev) HIP_OK(hipMemsetAsync(std_dev, 0, n * 8, ctx->stream));
    if (count_dev) HIP_OK(hipMemsetAsync(count_dev, 0, n * 4, ctx->stream));
    return RTM_OK;
  }
  HIP_OK(launch_stats_out(static_cast<double*>(m.mean.p), static_cast<double*>(m.m2.p),
                          static_cast<int32_t*>(m.count.p), n, mean_dev, std_dev, count_dev, ctx->stream));
  return RTM_OK;
}

extern "C" int rtm_ensemble_stack(rtm_ctx* ctx, int32_t realization, float* stack_dev) {
  if (!ctx || !stack_dev) return fail(RTM_E_INVAL, "ctx and stack_dev are required");
  std::lock_guard<std::mutex> lk(ctx->mu);
  auto it = ctx->models.find(realization);
  if (it == ctx->models.end()) return fail(RTM_E_NOTFOUND, "realization %d is not registered", realization);
  Model& m = it->second;
  const size_t n = (size_t)m.nz * m.nx;
  HIP_OK(hipSetDevice(ctx->device));
  HIP_OK(hipStreamSynchronize(ctx->sched_stream));
  if (!m.stack.p)
    HIP_OK(hipMemsetAsync(stack_dev, 0, n * 4, ctx->stream));
  else
    HIP_OK(hipMemcpyAsync(stack_dev, m.stack.p, n * 4, hipMemcpyDeviceToDevice, ctx->stream));
  return RTM_OK;
}

// ===========================================================================
// Explicit-image statistics, Stage-3 maps, post-stack filter
// ===========================================================================
struct rtm_stats {
  int nz = 0, nx = 0;
  Block mean, m2, count;
};

extern "C" int rtm_stats_create(rtm_ctx* ctx, rtm_stats** out, int32_t nz, int32_t nx) {
  if (!ctx || !out || nz < 1 || nx < 1) return fail(RTM_E_INVAL, "bad arguments");
  HIP_OK(hipSetDevice(ctx->device));
  auto st = std::make_unique<rtm_stats>();
  st->nz = nz;
  st->nx = nx;
  const size_t n = (size_t)nz * nx;
  st->mean = {arena_alloc(ctx, n * 8), align256(n * 8)};
  st->m2 = {arena_alloc(ctx, n * 8), align256(n * 8)};
  st->count = {arena_alloc(ctx, n * 4), align256(n * 4)};
  if (!st->mean.p || !st->m2.p || !st->count.p) {
    ctx->arena.release(st->mean.p, st->mean.n);
    ctx->arena.release(st->m2.p, st->m2.n);
    ctx->arena.release(st->count.p, st->count.n);
    return fail(RTM_E_NOMEM, "arena exhausted (statistics)");
  }
  HIP_OK(hipMemsetAsync(st->mean.p, 0, n * 8, ctx->stream));
  HIP_OK(hipMemsetAsync(st->m2.p, 0, n * 8, ctx->stream));
  HIP_OK(hipMemsetAsync(st->count.p, 0, n * 4, ctx->stream));
  *out = st.release();
  return RTM_OK;
}

extern "C" int rtm_stats_destroy(rtm_ctx* ctx, rtm_stats* st) {
  if (!ctx || !st) return fail(RTM_E_INVAL, "bad arguments");
  Deferred d;
  d.blocks = {st->mean, st->m2, st->count};
  delete st;
  return defer(ctx, ctx->stream, std::move(d));
}

extern "C" int rtm_stats_add(rtm_ctx* ctx, rtm_stats* st, const float* image_dev, int32_t ix0, int32_t width) {
  if (!ctx || !st || !image_dev) return fail(RTM_E_INVAL, "bad arguments");
  if (ix0 < 0 || width < 1 || ix0 + width > st->nx) return fail(RTM_E_INVAL, "window outside the image");
  HIP_OK(hipSetDevice(ctx->device));
  HIP_OK(launch_welford(static_cast<double*>(st->mean.p), static_cast<double*>(st->m2.p),
                        static_cast<int32_t*>(st->count.p), st->nx, image_dev, width, st->nz, width, ix0,
                        ctx->stream));
  return RTM_OK;
}

extern "C" int rtm_stats_get(rtm_ctx* ctx, rtm_stats* st, double* mean_dev, double* std_dev, int32_t* count_dev) {
  if (!ctx || !st) return fail(RTM_E_INVAL, "bad arguments");
  HIP_OK(hipSetDevice(ctx->device));
  HIP_OK(launch_stats_out(static_cast<double*>(st->mean.p), static_cast<double*>(st->m2.p),
                          static_cast<int32_t*>(st->count.p), (int64_t)st->nz * st->nx, mean_dev, std_dev,
                          count_dev, ctx->stream));
  return RTM_OK;
}

extern "C" int rtm_confidence_map(rtm_ctx* ctx, const double* std_dev, const int32_t* count_dev, int32_t n,
                                  int32_t min_count, double* conf_dev) {
  if (!ctx || !std_dev || !conf_dev || n < 1) return fail(RTM_E_INVAL, "bad arguments");
  HIP_OK(hipSetDevice(ctx->device));
  HIP_OK(launch_confidence(std_dev, count_dev, n, min_count, conf_dev, ctx->scratch_f64, ctx->stream));
  return RTM_OK;
}

extern "C" int rtm_ratio_map(rtm_ctx* ctx, const double* std_dev, const double* mean_dev, int32_t n, double eps,
                             double* ratio_dev) {
  if (!ctx || !std_dev || !mean_dev || !ratio_dev || n < 1 || !(eps >= 0))
    return fail(RTM_E_INVAL, "bad arguments");
  HIP_OK(hipSetDevice(ctx->device));
  HIP_OK(launch_ratio(std_dev, mean_dev, n, eps, ratio_dev, ctx->stream));
  return RTM_OK;
}

extern "C" int rtm_laplacian_filter(rtm_ctx* ctx, const float* img_dev, int32_t nz, int32_t nx, float dz, float dx,
                                    float* out_dev) {
  if (!ctx || !img_dev || !out_dev || nz < 1 || nx < 1 || !(dz > 0) || !(dx > 0))
    return fail(RTM_E_INVAL, "bad arguments");
  if (img_dev == out_dev) return fail(RTM_E_INVAL, "the filter cannot run in place");
  HIP_OK(hipSetDevice(ctx->device));
  HIP_OK(launch_lapfilter(img_dev, nz, nx, dz, dx, out_dev, ctx->stream));
  return RTM_OK;
}

extern "C" int rtm_normalize_image(rtm_ctx* ctx, const float* image_dev, const float* illum_dev, int32_t n,
                                   float eps_rel, float* out_dev) {
  if (!ctx || !image_dev || !illum_dev || !out_dev || n < 1 || !(eps_rel >= 0))
    return fail(RTM_E_INVAL, "bad arguments");
  HIP_OK(hipSetDevice(ctx->device));
  HIP_OK(launch_normalize(image_dev, illum_dev, n, eps_rel, out_dev, reinterpret_cast<float*>(ctx->scratch_f64),
                          ctx->stream));
  return RTM_OK;
}

extern "C" int rtm_stats_merge(rtm_ctx* ctx, rtm_stats* dst, const rtm_stats* src) {
  if (!ctx || !dst || !src || dst == src) return fail(RTM_E_INVAL, "bad arguments");
  if (dst->nz != src->nz || dst->nx != src->nx) return fail(RTM_E_INVAL, "statistics of different sizes");
  HIP_OK(hipSetDevice(ctx->device));
  HIP_OK(launch_chan_merge(static_cast<double*>(dst->mean.p), static_cast<double*>(dst->m2.p),
                           static_cast<int32_t*>(dst->count.p), static_cast<const double*>(src->mean.p),
                           static_cast<const double*>(src->m2.p), static_cast<const int32_t*>(src->count.p),
                           (int64_t)dst->nz * dst->nx, ctx->stream));
  return RTM_OK;
}

// ===========================================================================
// Codec (fixed-accuracy / lossless block-transform coder of float32 arrays)
// ===========================================================================
static int64_t zc_index_words(int64_t nblk) {
  return kZcHeaderWords + (nblk + kZcChunk - 1) / kZcChunk + 1 + nblk;
}

static int zc_geometry(int32_t count, int32_t rows, int32_t cols, ZcParams& p) {
  if (count < 1 || rows < 1 || cols < 1) return fail(RTM_E_INVAL, "count, rows and cols must be >= 1");
  const int64_t bz = (rows + 7) / 8, bx = (cols + 7) / 8, nblk = (int64_t)count * bz * bx;
  if (nblk > kZcMaxBlocks)
    return fail(RTM_E_INVAL, "%lld blocks exceed the limit of %lld per stream", (long long)nblk,
                (long long)kZcMaxBlocks);
  p.count = count;
  p.rows = rows;
  p.cols = cols;
  p.bz = (int32_t)bz;
  p.bx = (int32_t)bx;
  p.nblocks = (int32_t)nblk;
  p.nchunks = (int32_t)((nblk + kZcChunk - 1) / kZcChunk);
  p.hdr_base = kZcHeaderWords + p.nchunks + 1;
  p.pay_base = p.hdr_base + nblk;
  return RTM_OK;
}

// Geometry of a fixed-accuracy ZFP-method stream (4 x 4 blocks, chunks of 16).
static int zf_geometry(int32_t count, int32_t rows, int32_t cols, ZfParams& p) {
  if (count < 1 || rows < 1 || cols < 1) return fail(RTM_E_INVAL, "count, rows and cols must be >= 1");
  const int64_t bz = (rows + 3) / 4, bx = (cols + 3) / 4, nblk = (int64_t)count * bz * bx;
  if (nblk > kZfMaxBlocks)
    return fail(RTM_E_INVAL, "%lld blocks of 4 x 4 exceed the limit of %lld per stream", (long long)nblk,
                (long long)kZfMaxBlocks);
  p.count = count;
  p.rows = rows;
  p.cols = cols;
  p.bz = (int32_t)bz;
  p.bx = (int32_t)bx;
  p.nblocks = nblk;
  p.nchunks = (nblk + kZfChunk - 1) / kZfChunk;
  p.hdr_base = kZfHeaderWords;
  p.pay_base = kZfHeaderWords + p.nchunks + 1;
  return RTM_OK;
}

// Longest fixed-accuracy ZFP-method stream of a shape (-1: outside the limits).
static int64_t zf_max_bytes(int32_t count, int32_t rows, int32_t cols) {
  if (count < 1 || rows < 1 || cols < 1) return -1;
  const int64_t nblk = (int64_t)count * ((rows + 3) / 4) * ((cols + 3) / 4);
  if (nblk > kZfMaxBlocks) return -1;
  const int64_t nch = (nblk + kZfChunk - 1) / kZfChunk, last = nblk - (nch - 1) * kZfChunk;
  const int64_t full = ((int64_t)kZfChunk * kZfMaxBlockBits + 31) / 32, part = (last * kZfMaxBlockBits + 31) / 32;
  return 4 * (kZfHeaderWords + nch + 1 + (nch - 1) * full + part);
}

extern "C" int64_t rtm_codec_max_bytes(int32_t count, int32_t rows, int32_t cols) {
  if (count < 1 || rows < 1 || cols < 1) return -1;
  const int64_t nblk = (int64_t)count * ((rows + 7) / 8) * ((cols + 7) / 8);
  if (nblk > kZcMaxBlocks) return -1;
  const int64_t zf = zf_max_bytes(count, rows, cols);
  return std::max(4 * (zc_index_words(nblk) + 64 * nblk), zf);
}

// rtm_codec_encode with mode RTM_CODEC_ZFP.
static int zf_encode(rtm_ctx* ctx, const float* x_dev, int32_t count, int32_t rows, int32_t cols, double tol,
                     void* stream_dev, int64_t capacity_bytes, int64_t* stream_bytes) {
  if (!(tol >= 0x1p-60) || !std::isfinite(tol))
    return fail(RTM_E_INVAL, "the tolerance must be finite and at least 2^-60 for the ZFP-method coder");
  ZfParams p{};
  if (int st = zf_geometry(count, rows, cols, p)) return st;
  int e2 = 0;
  (void)frexp(tol, &e2);
  p.minexp = e2 - 1;  // floor(log2 tol)
  if (capacity_bytes < 4 * p.pay_base)
    return fail(RTM_E_NOMEM, "stream capacity %lld bytes is below the %lld-byte index",
                (long long)capacity_bytes, (long long)(4 * p.pay_base));
  p.cap_words = capacity_bytes / 4;
  p.x = x_dev;
  p.out = static_cast<uint32_t*>(stream_dev);
  uint32_t tw[2];
  memcpy(tw, &tol, 8);
  const uint32_t head[8] = {kZfMagic, (uint32_t)kZfMode, (uint32_t)count, (uint32_t)rows,
                            (uint32_t)cols, (uint32_t)kZfChunk, tw[0], tw[1]};
  memcpy(p.head, head, sizeof head);
  HIP_OK(hipSetDevice(ctx->device));
  // scratch: the look-back state (one word per encoder workgroup), the
  // workgroup ticket, flags and result words, all zeroed
  const int64_t nwg = (p.nblocks + kZfEncThreads - 1) / kZfEncThreads;
  const size_t status_bytes = align256(8 * (size_t)nwg);
  const size_t scratch_bytes = status_bytes + 256;
  char* scratch = static_cast<char*>(arena_alloc(ctx, scratch_bytes));
  if (!scratch) return fail(RTM_E_NOMEM, "arena exhausted (codec scratch)");
  uint32_t* tail = reinterpret_cast<uint32_t*>(scratch + status_bytes);
  p.status = reinterpret_cast<uint64_t*>(scratch);
  p.flags = tail;
  p.result = tail + 2;
  p.ticket = tail + 4;
  hipStream_t s = ctx->stream;
  uint32_t res[4] = {0, 0, 0, 0};
  hipError_t e = launch_fill_u32(reinterpret_cast<uint32_t*>(scratch), 0, (int64_t)(scratch_bytes / 4), s);
  if (e == hipSuccess) e = hipEventRecord(ctx->zc_ev[0], s);
  if (e == hipSuccess) e = launch_zf_encode(p, s);
  if (e == hipSuccess) e = hipEventRecord(ctx->zc_ev[1], s);
  if (e == hipSuccess) e = hipMemcpyAsync(res, tail, 16, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  ctx->arena.release(scratch, align256(scratch_bytes));
  if (e != hipSuccess) return fail(RTM_E_DEVICE, "codec encode: %s", hipGetErrorString(e));
  if (res[0] & kZfRange)
    return fail(RTM_E_INVAL, "a value is non-finite or |x| >= 2^100 (outside the ZFP-method coder's range)");
  if (res[0] & kZfSpin) return fail(RTM_E_DEVICE, "codec encode: a chunk offset did not arrive in time");
  const uint64_t payload = (uint64_t)res[2] | ((uint64_t)res[3] << 32);
  const int64_t bytes = 4 * (p.pay_base + (int64_t)payload);
  *stream_bytes = bytes;
  ctx->zc_op = 1;
  ctx->zc_bytes = 4 * (uint64_t)count * rows * cols + (uint64_t)bytes;
  if (bytes > capacity_bytes)
    return fail(RTM_E_NOMEM, "the stream needs %lld bytes, the buffer holds %lld", (long long)bytes,
                (long long)capacity_bytes);
  return RTM_OK;
}

// Validation of an encode and its launch parameters (no device work).
// max_chunks bounds the chunk count (the look-back state holds 8 bytes per
// chunk); larger arrays are rejected with RTM_E_INVAL.
static int zc_encode_params(rtm_ctx* ctx, const float* x_dev, int32_t count, int32_t rows, int32_t cols,
                            int32_t mode, double tol, void* stream_dev, int64_t capacity_bytes,
                            int64_t* stream_bytes, int64_t max_chunks, ZcParams& p) {
  if (!ctx || !x_dev || !stream_dev || !stream_bytes) return fail(RTM_E_INVAL, "bad arguments");
  *stream_bytes = 0;
  if (reinterpret_cast<uintptr_t>(stream_dev) & 3) return fail(RTM_E_INVAL, "stream must be 4-byte aligned");
  if (reinterpret_cast<uintptr_t>(x_dev) & 3) return fail(RTM_E_INVAL, "array must be 4-byte aligned");
  p = ZcParams{};
  if (mode == RTM_CODEC_TOL) {
    if (!(tol > 0) || !std::isfinite(tol)) return fail(RTM_E_INVAL, "the tolerance must be finite and > 0");
    p.r = 1.0 / (2.0 * tol);
    p.step = 2.0 * tol;
    if (!std::isfinite(p.r)) return fail(RTM_E_INVAL, "the tolerance is too small");
  } else if (mode == RTM_CODEC_LOSSLESS) {
    tol = 0.0;
  } else {
    return fail(RTM_E_INVAL, "unknown codec mode %d", mode);
  }
  p.mode = mode;
  if (int st = zc_geometry(count, rows, cols, p)) return st;
  if (p.nchunks > max_chunks)
    return fail(RTM_E_INVAL, "%d chunks of %d blocks exceed the %lld this call holds look-back state for",
                p.nchunks, kZcChunk, (long long)max_chunks);
  if (capacity_bytes < 4 * p.pay_base)
    return fail(RTM_E_NOMEM, "stream capacity %lld bytes is below the %lld-byte index",
                (long long)capacity_bytes, (long long)(4 * p.pay_base));
  p.cap_words = capacity_bytes / 4;
  p.x = x_dev;
  p.out = static_cast<uint32_t*>(stream_dev);
  uint32_t tw[2];
  memcpy(tw, &tol, 8);
  const uint32_t head[8] = {kZcMagic, (uint32_t)mode, (uint32_t)count, (uint32_t)rows,
                            (uint32_t)cols, (uint32_t)kZcChunk, tw[0], tw[1]};
  memcpy(p.head, head, sizeof head);
  return RTM_OK;
}

// Runs a validated encode with its look-back state in `scratch` (device
// memory of at least 8 nchunks + 64 bytes, cleared here by a fill kernel)
// and waits for it: the stream length comes back to the host.
static int zc_encode_run(rtm_ctx* ctx, ZcParams& p, void* scratch, int64_t capacity_bytes, int64_t* stream_bytes) {
  const size_t scratch_bytes = 8 * (size_t)p.nchunks + 64;
  uint32_t* tail = reinterpret_cast<uint32_t*>(static_cast<char*>(scratch) + 8 * (size_t)p.nchunks);
  p.status = static_cast<uint64_t*>(scratch);
  p.ticket = tail;
  p.flags = tail + 1;
  p.result = tail + 2;
  hipStream_t s = ctx->stream;
  uint32_t res[4] = {0, 0, 0, 0};
  hipError_t e = launch_fill_u32(static_cast<uint32_t*>(scratch), 0, (int64_t)scratch_bytes / 4, s);
  if (e == hipSuccess) e = hipEventRecord(ctx->zc_ev[0], s);
  if (e == hipSuccess) e = launch_zc_encode(p, s);
  if (e == hipSuccess) e = hipEventRecord(ctx->zc_ev[1], s);
  if (e == hipSuccess) e = hipMemcpyAsync(res, tail, 16, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return fail(RTM_E_DEVICE, "codec encode: %s", hipGetErrorString(e));
  const uint32_t flags = res[1];
  if (flags & kZcSpin) return fail(RTM_E_DEVICE, "codec encode: a chunk prefix did not arrive in time");
  if (flags & kZcRange)
    return fail(RTM_E_INVAL, "a value is non-finite or |x| / (2 tol) exceeds 2^31 - 1; use a larger "
                             "tolerance or the lossless mode");
  const int64_t bytes = 4 * (p.pay_base + (int64_t)res[2]);
  *stream_bytes = bytes;
  ctx->zc_op = 1;
  ctx->zc_bytes = 4 * (uint64_t)p.count * p.rows * p.cols + (uint64_t)bytes;
  if (flags & kZcCapacity)
    return fail(RTM_E_NOMEM, "the stream needs %lld bytes, the buffer holds %lld", (long long)bytes,
                (long long)capacity_bytes);
  return RTM_OK;
}

extern "C" int rtm_codec_encode(rtm_ctx* ctx, const float* x_dev, int32_t count, int32_t rows, int32_t cols,
                                int32_t mode, double tol, void* stream_dev, int64_t capacity_bytes,
                                int64_t* stream_bytes) {
  if (mode == RTM_CODEC_ZFP) {
    if (!ctx || !x_dev || !stream_dev || !stream_bytes) return fail(RTM_E_INVAL, "bad arguments");
    *stream_bytes = 0;
    if (reinterpret_cast<uintptr_t>(stream_dev) & 3) return fail(RTM_E_INVAL, "stream must be 4-byte aligned");
    if (reinterpret_cast<uintptr_t>(x_dev) & 3) return fail(RTM_E_INVAL, "array must be 4-byte aligned");
    return zf_encode(ctx, x_dev, count, rows, cols, tol, stream_dev, capacity_bytes, stream_bytes);
  }
  ZcParams p;
  if (int st = zc_encode_params(ctx, x_dev, count, rows, cols, mode, tol, stream_dev, capacity_bytes, stream_bytes,
                                INT64_MAX, p))
    return st;
  HIP_OK(hipSetDevice(ctx->device));
  const size_t scratch_bytes = 8 * (size_t)p.nchunks + 64;
  void* scratch = arena_alloc(ctx, scratch_bytes);
  if (!scratch) return fail(RTM_E_NOMEM, "arena exhausted (codec look-back state)");
  const int rc = zc_encode_run(ctx, p, scratch, capacity_bytes, stream_bytes);
  ctx->arena.release(scratch, align256(scratch_bytes));  // the run waited for the stream
  return rc;
}

// One lock per device: the allocation-free encoder's calls on a device share
// its scratch array, and each call returns only after its kernels finished,
// so holding the lock for the call keeps calls of this process from
// overlapping on one device.
static std::mutex g_zc_noalloc_mu[64];

extern "C" int rtm_codec_encode_noalloc(rtm_ctx* ctx, const float* x_dev, int32_t count, int32_t rows,
                                        int32_t cols, int32_t mode, double tol, void* stream_dev,
                                        int64_t capacity_bytes, int64_t* stream_bytes) {
  if (mode == RTM_CODEC_ZFP) return fail(RTM_E_INVAL, "the allocation-free encoder takes the TOL and LOSSLESS modes");
  ZcParams p;
  if (int st = zc_encode_params(ctx, x_dev, count, rows, cols, mode, tol, stream_dev, capacity_bytes, stream_bytes,
                                kZcNoAllocChunks, p))
    return st;
  void* scratch = zc_noalloc_scratch(ctx->device);
  if (!scratch || ctx->device < 0 || ctx->device >= 64)
    return fail(RTM_E_DEVICE, "the encoder's device scratch was not found on device %d", ctx->device);
  HIP_OK(hipSetDevice(ctx->device));
  std::lock_guard<std::mutex> lk(g_zc_noalloc_mu[ctx->device]);
  return zc_encode_run(ctx, p, scratch, capacity_bytes, stream_bytes);
}

extern "C" int rtm_codec_info(rtm_ctx* ctx, const void* stream_dev, int64_t stream_bytes, int32_t* mode,
                              int32_t* count, int32_t* rows, int32_t* cols, double* tol) {
  if (!ctx || !stream_dev) return fail(RTM_E_INVAL, "bad arguments");
  if (reinterpret_cast<uintptr_t>(stream_dev) & 3) return fail(RTM_E_INVAL, "stream must be 4-byte aligned");
  if (stream_bytes < 4 * kZcHeaderWords) return fail(RTM_E_INVAL, "stream shorter than its header");
  HIP_OK(hipSetDevice(ctx->device));
  uint32_t h[8];
  HIP_OK(hipMemcpyAsync(h, stream_dev, sizeof h, hipMemcpyDeviceToHost, ctx->stream));
  HIP_OK(hipStreamSynchronize(ctx->stream));
  if (h[0] == kZfMagic) {  // fixed-accuracy ZFP-method stream
    if (h[1] != (uint32_t)kZfMode) return fail(RTM_E_INVAL, "unknown codec mode %u", h[1]);
    if (h[5] != (uint32_t)kZfChunk) return fail(RTM_E_INVAL, "unsupported chunk size %u", h[5]);
    if (h[2] - 1 > 0x7ffffffeu || h[3] - 1 > 0x7ffffffeu || h[4] - 1 > 0x7ffffffeu)
      return fail(RTM_E_INVAL, "bad array shape in the stream header");
    double t;
    memcpy(&t, h + 6, 8);
    if (!(t >= 0x1p-60) || !std::isfinite(t)) return fail(RTM_E_INVAL, "bad tolerance in the stream header");
    ZfParams q{};
    if (int st = zf_geometry((int32_t)h[2], (int32_t)h[3], (int32_t)h[4], q)) return st;
    if (stream_bytes < 4 * q.pay_base) return fail(RTM_E_INVAL, "stream shorter than its index");
    if (mode) *mode = RTM_CODEC_ZFP;
    if (count) *count = q.count;
    if (rows) *rows = q.rows;
    if (cols) *cols = q.cols;
    if (tol) *tol = t;
    return RTM_OK;
  }
  if (h[0] != kZcMagic) return fail(RTM_E_INVAL, "not a codec stream (magic %08x)", h[0]);
  if (h[1] > 1) return fail(RTM_E_INVAL, "unknown codec mode %u", h[1]);
  if (h[5] != (uint32_t)kZcChunk) return fail(RTM_E_INVAL, "unsupported chunk size %u", h[5]);
  if (h[2] - 1 > 0x7ffffffeu || h[3] - 1 > 0x7ffffffeu || h[4] - 1 > 0x7ffffffeu)
    return fail(RTM_E_INVAL, "bad array shape in the stream header");
  double t;
  memcpy(&t, h + 6, 8);
  if (h[1] == RTM_CODEC_TOL && (!(t > 0) || !std::isfinite(t) || !std::isfinite(1.0 / (2.0 * t))))
    return fail(RTM_E_INVAL, "bad tolerance in the stream header");
  ZcParams p{};
  if (int st = zc_geometry((int32_t)h[2], (int32_t)h[3], (int32_t)h[4], p)) return st;
  if (stream_bytes < 4 * p.pay_base) return fail(RTM_E_INVAL, "stream shorter than its index");
  if (mode) *mode = (int32_t)h[1];
  if (count) *count = p.count;
  if (rows) *rows = p.rows;
  if (cols) *cols = p.cols;
  if (tol) *tol = t;
  return RTM_OK;
}

// rtm_codec_decode of a fixed-accuracy ZFP-method stream (header checked).
static int zf_decode(rtm_ctx* ctx, const void* stream_dev, int64_t stream_bytes, float* x_dev, int64_t capacity_floats,
                     int32_t count, int32_t rows, int32_t cols, double tol) {
  ZfParams p{};
  if (int st = zf_geometry(count, rows, cols, p)) return st;
  const int64_t n = (int64_t)count * rows * cols;
  if (capacity_floats < n)
    return fail(RTM_E_NOMEM, "the array holds %lld floats, the stream decodes to %lld",
                (long long)capacity_floats, (long long)n);
  int e2 = 0;
  (void)frexp(tol, &e2);
  p.minexp = e2 - 1;
  void* scratch = arena_alloc(ctx, 64);
  if (!scratch) return fail(RTM_E_NOMEM, "arena exhausted (codec flags)");
  p.in = static_cast<const uint32_t*>(stream_dev);
  p.y = x_dev;
  p.flags = static_cast<uint32_t*>(scratch);
  p.cap_words = stream_bytes / 4;
  hipStream_t s = ctx->stream;
  uint32_t flags = 0;
  hipError_t e = launch_fill_u32(p.flags, 0, 16, s);
  if (e == hipSuccess) e = hipEventRecord(ctx->zc_ev[0], s);
  // LDS budget of the decoder's staged payload (RTM_ZFP_STAGE_BYTES; unset: from
  // the stream's mean payload per workgroup; 0: no staging)
  const char* sb = getenv("RTM_ZFP_STAGE_BYTES");
  if (e == hipSuccess) e = launch_zf_decode(p, sb ? std::max(0ll, atoll(sb)) : -1ll, s);
  if (e == hipSuccess) e = hipEventRecord(ctx->zc_ev[1], s);
  if (e == hipSuccess) e = hipMemcpyAsync(&flags, p.flags, 4, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  ctx->arena.release(scratch, align256(64));
  if (e != hipSuccess) return fail(RTM_E_DEVICE, "codec decode: %s", hipGetErrorString(e));
  ctx->zc_op = 2;
  ctx->zc_bytes = (uint64_t)stream_bytes + 4 * (uint64_t)n;
  if (flags) return fail(RTM_E_INVAL, "corrupt codec stream (chunk table or block codes)");
  return RTM_OK;
}

extern "C" int rtm_codec_decode(rtm_ctx* ctx, const void* stream_dev, int64_t stream_bytes, float* x_dev,
                                int64_t capacity_floats) {
  if (!ctx || !stream_dev || !x_dev) return fail(RTM_E_INVAL, "bad arguments");
  if (reinterpret_cast<uintptr_t>(x_dev) & 3) return fail(RTM_E_INVAL, "array must be 4-byte aligned");
  int32_t mode = 0, count = 0, rows = 0, cols = 0;
  double tol = 0;
  if (int st = rtm_codec_info(ctx, stream_dev, stream_bytes, &mode, &count, &rows, &cols, &tol)) return st;
  if (mode == RTM_CODEC_ZFP) return zf_decode(ctx, stream_dev, stream_bytes, x_dev, capacity_floats, count, rows,
                                              cols, tol);
  ZcParams p{};
  if (int st = zc_geometry(count, rows, cols, p)) return st;
  const int64_t n = (int64_t)count * rows * cols;
  if (capacity_floats < n)
    return fail(RTM_E_NOMEM, "the array holds %lld floats, the stream decodes to %lld",
                (long long)capacity_floats, (long long)n);
  void* scratch = arena_alloc(ctx, 64);
  if (!scratch) return fail(RTM_E_NOMEM, "arena exhausted (codec flags)");
  p.mode = mode;
  p.step = 2.0 * tol;
  p.in = static_cast<const uint32_t*>(stream_dev);
  p.y = x_dev;
  p.flags = static_cast<uint32_t*>(scratch);
  p.cap_words = stream_bytes / 4;
  hipStream_t s = ctx->stream;
  uint32_t flags = 0;
  hipError_t e = launch_fill_u32(p.flags, 0, 16, s);
  if (e == hipSuccess) e = hipEventRecord(ctx->zc_ev[0], s);
  if (e == hipSuccess) e = launch_zc_decode(p, s);
  if (e == hipSuccess) e = hipEventRecord(ctx->zc_ev[1], s);
  if (e == hipSuccess) e = hipMemcpyAsync(&flags, p.flags, 4, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  ctx->arena.release(scratch, align256(64));
  if (e != hipSuccess) return fail(RTM_E_DEVICE, "codec decode: %s", hipGetErrorString(e));
  ctx->zc_op = 2;
  // payload words actually used: the chunk table's last entry is not read back,
  // so count the stream as handed in
  ctx->zc_bytes = (uint64_t)stream_bytes + 4 * (uint64_t)n;
  if (flags) return fail(RTM_E_INVAL, "corrupt codec stream (widths, chunk table or length)");
  return RTM_OK;
}

// ===========================================================================
// Stage 1: Bayesian Eikonal tomography
// ===========================================================================
// Chains are independent, so groups of them advance on streams of their own
// (the context stream and kBetGroups - 1 more): one group's last solves of
// an iteration overlap the other group's next iteration instead of idling
// the GPU at a per-iteration barrier.  Two groups: a process has few
// hardware queues (4 by default, shared with the context's other streams),
// and groups that share one run in turn (64 chains: 127.7k chain
// iterations/s with two groups, 125.2k with three, 129.1k with four).
constexpr int kBetGroups = 2;

struct rtm_bet {
  BetDev d{};
  std::vector<Block> blocks;
  int t = 0;  // iterations done
  int groups = 1;
  hipStream_t gs[kBetGroups] = {};     // gs[0] = the context stream (not owned)
  hipEvent_t fork = nullptr, join[kBetGroups] = {};
  ~rtm_bet() {
    for (int g = 1; g < kBetGroups; ++g)
      if (gs[g]) {
        (void)hipStreamSynchronize(gs[g]);
        (void)hipStreamDestroy(gs[g]);
      }
    if (fork) (void)hipEventDestroy(fork);
    for (auto e : join)
      if (e) (void)hipEventDestroy(e);
  }
  int c0(int g) const { return (int)((int64_t)d.chains * g / groups); }
  int cn(int g) const { return c0(g + 1) - c0(g); }
};

static int bet_points(const rtm_point* pts, int n, int nz, int nx, const char* what, std::vector<int2>& out) {
  if (n < 1 || !pts) return fail(RTM_E_INVAL, "no %s", what);
  out.resize(n);
  for (int i = 0; i < n; ++i) {
    if (pts[i].iz < 0 || pts[i].iz >= nz || pts[i].ix < 0 || pts[i].ix >= nx)
      return fail(RTM_E_INVAL, "%s %d at (%d, %d) is outside the %d x %d grid", what, i, pts[i].iz, pts[i].ix, nz,
                  nx);
    out[i] = make_int2(pts[i].iz, pts[i].ix);
  }
  return RTM_OK;
}

extern "C" int rtm_eikonal(rtm_ctx* ctx, const float* vel_dev, int32_t nz, int32_t nx, float h, int32_t nsrc,
                           const rtm_point* src_host, int32_t nrec, const rtm_point* rec_host, float* tt_dev) {
  if (!ctx || !vel_dev || !tt_dev) return fail(RTM_E_INVAL, "bad arguments");
  if (nz < 1 || nx < 1 || (int64_t)nz * nx > kBetMaxNodes || !(h > 0) || !std::isfinite(h))
    return fail(RTM_E_INVAL, "grid %d x %d, h %g: need 1..%d nodes and h > 0", nz, nx, (double)h, kBetMaxNodes);
  if (bet_lds_grid(nz, nx) > kBetMaxLds)
    return fail(RTM_E_INVAL, "grid %d x %d: a solve needs %zu bytes of LDS, at most %zu", nz, nx,
                bet_lds_grid(nz, nx), kBetMaxLds);
  std::vector<int2> src, rec;
  if (int st = bet_points(src_host, nsrc, nz, nx, "source", src)) return st;
  if (int st = bet_points(rec_host, nrec, nz, nx, "receiver", rec)) return st;
  HIP_OK(hipSetDevice(ctx->device));
  const size_t bs = align256(8 * (size_t)nsrc), br = align256(8 * (size_t)nrec);
  const size_t bn = align256(sizeof(BetSlowness) * (size_t)bet_grid_entries(nz, nx));
  char* buf = static_cast<char*>(arena_alloc(ctx, bs + br + 256 + bn));
  if (!buf) return fail(RTM_E_NOMEM, "arena exhausted (travel-time geometry and node terms)");
  hipStream_t s = ctx->stream;
  uint32_t* flags = reinterpret_cast<uint32_t*>(buf + bs + br);
  BetSlowness* node = reinterpret_cast<BetSlowness*>(buf + bs + br + 256);
  uint32_t flag = 0;
  hipError_t e = hipMemcpyAsync(buf, src.data(), 8 * (size_t)nsrc, hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipMemcpyAsync(buf + bs, rec.data(), 8 * (size_t)nrec, hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = launch_fill_u32(flags, 0, 1, s);
  if (e == hipSuccess)
    e = launch_eikonal_grid(vel_dev, nz, nx, h, reinterpret_cast<int2*>(buf), nsrc, reinterpret_cast<int2*>(buf + bs),
                            nrec, tt_dev, flags, node, s);
  if (e == hipSuccess) e = hipMemcpyAsync(&flag, flags, 4, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  ctx->arena.release(buf, align256(bs + br + 256 + bn));
  if (e != hipSuccess) return fail(RTM_E_DEVICE, "travel times: %s", hipGetErrorString(e));
  if (flag & kBetBadSlowness)
    return fail(RTM_E_INVAL, "velocity grid: h / v must lie in [%g, %g] s at every node", (double)kBetShMin,
                (double)kBetShMax);
  if (flag & kBetNoConverge) return fail(RTM_E_DEVICE, "a travel-time solve did not converge");
  return RTM_OK;
}

extern "C" int rtm_bet_create(rtm_ctx* ctx, const rtm_bet_config* cfg, int32_t nsrc, const rtm_point* src_host,
                              int32_t nrec, const rtm_point* rec_host, const float* tt_obs_dev, rtm_bet** out) {
  if (!ctx || !cfg || !tt_obs_dev || !out) return fail(RTM_E_INVAL, "bad arguments");
  *out = nullptr;
  const rtm_bet_config& c = *cfg;
  if (c.nz < 2 || c.nx < 2 || (int64_t)c.nz * c.nx > kBetMaxNodes || !(c.h > 0) || !std::isfinite(c.h) ||
      bet_lds_sampler(c.nz, c.nx) > kBetMaxLds)
    return fail(RTM_E_INVAL, "grid %d x %d, h %g: need 2..%d nodes per side product and h > 0", c.nz, c.nx, c.h,
                kBetMaxNodes);
  if (c.chains < 1 || c.chains > kBetMaxChains || c.k_min < 1 || c.k_init < c.k_min || c.k_max < c.k_init ||
      c.k_max > kBetMaxCells)
    return fail(RTM_E_INVAL, "need 1 <= chains <= %d and 1 <= k_min <= k_init <= k_max <= %d", kBetMaxChains,
                kBetMaxCells);
  if (!(c.v_min > 0) || !(c.v_max > c.v_min) || !std::isfinite(c.v_max))
    return fail(RTM_E_INVAL, "need 0 < v_min < v_max");
  {  // the node terms the solves will see, as the device computes them
    const float sh_lo = (float)(1.0 / c.v_max) * (float)c.h, sh_hi = (float)(1.0 / c.v_min) * (float)c.h;
    if (!(sh_lo >= kBetShMin && sh_hi <= kBetShMax))
      return fail(RTM_E_INVAL, "h / v must lie in [%g, %g] s over [v_min, v_max]", (double)kBetShMin,
                  (double)kBetShMax);
  }
  if (!(c.p_birth >= 0) || !(c.p_death >= 0) || !(c.p_birth + c.p_death <= 1.0))
    return fail(RTM_E_INVAL, "need p_birth, p_death >= 0 with p_birth + p_death <= 1");
  if (!(c.move_dz >= 0) || !(c.move_dx >= 0) || !(c.sigma > 0) || !std::isfinite(c.sigma) || c.burn_in < 0 ||
      c.thin < 1)
    return fail(RTM_E_INVAL, "need move half-widths >= 0, sigma > 0, burn_in >= 0, thin >= 1");
  std::vector<int2> src, rec;
  if (int st = bet_points(src_host, nsrc, c.nz, c.nx, "source", src)) return st;
  if (int st = bet_points(rec_host, nrec, c.nz, c.nx, "receiver", rec)) return st;
  HIP_OK(hipSetDevice(ctx->device));
  auto b = std::make_unique<rtm_bet>();
  BetDev& d = b->d;
  d.nz = c.nz;
  d.nx = c.nx;
  d.nsrc = nsrc;
  d.nrec = nrec;
  d.h = c.h;
  d.chains = c.chains;
  d.k_min = c.k_min;
  d.k_max = c.k_max;
  d.k_init = c.k_init;
  d.burn_in = c.burn_in;
  d.thin = c.thin;
  d.v_min = c.v_min;
  d.v_max = c.v_max;
  d.p_birth = c.p_birth;
  d.p_death = c.p_death;
  d.move_dz = c.move_dz;
  d.move_dx = c.move_dx;
  d.sigma = c.sigma;
  d.seed = c.seed;
  const size_t C = c.chains, K = c.k_max, n = (size_t)c.nz * c.nx, nd = (size_t)nsrc * nrec;
  bool ok = true;
  auto get = [&](size_t bytes) -> void* {
    void* q = nullptr;
    if (ok && !alloc_block(ctx, b->blocks, bytes, &q)) ok = false;
    return q;
  };
  d.src = static_cast<const int2*>(get(8 * (size_t)nsrc));
  d.rec = static_cast<const int2*>(get(8 * (size_t)nrec));
  d.tt_obs = static_cast<const float*>(get(4 * nd));
  d.k = static_cast<int32_t*>(get(4 * C));
  d.z = static_cast<double*>(get(8 * C * K));
  d.x = static_cast<double*>(get(8 * C * K));
  d.v = static_cast<double*>(get(8 * C * K));
  d.misfit = static_cast<double*>(get(8 * C));
  d.pk = static_cast<int32_t*>(get(4 * C));
  d.valid = static_cast<int32_t*>(get(4 * C));
  d.ptype = static_cast<int32_t*>(get(4 * C));
  d.pz = static_cast<double*>(get(8 * C * K));
  d.px = static_cast<double*>(get(8 * C * K));
  d.pv = static_cast<double*>(get(8 * C * K));
  d.ua = static_cast<double*>(get(8 * C));
  d.node = static_cast<BetSlowness*>(get(sizeof(BetSlowness) * C * (size_t)bet_grid_entries(c.nz, c.nx)));
  d.tt = static_cast<float*>(get(4 * C * nd));
  d.proposed = static_cast<int64_t*>(get(8 * 3 * C));
  d.accepted = static_cast<int64_t*>(get(8 * 3 * C));
  d.work = static_cast<unsigned long long*>(get(8 * 2 * C));
  d.snap_k = static_cast<int32_t*>(get(4 * (size_t)kBetSnapSlots * C));
  d.snap_z = static_cast<double*>(get(8 * (size_t)kBetSnapSlots * C * K));
  d.snap_x = static_cast<double*>(get(8 * (size_t)kBetSnapSlots * C * K));
  d.snap_v = static_cast<double*>(get(8 * (size_t)kBetSnapSlots * C * K));
  d.sample_v = static_cast<double*>(get(8 * C * n));
  d.mean = static_cast<double*>(get(8 * n));
  d.m2 = static_cast<double*>(get(8 * n));
  d.count = static_cast<int32_t*>(get(4 * n));
  d.flags = static_cast<uint32_t*>(get(256));
  if (!ok) {
    release_blocks(ctx, b->blocks);
    return fail(RTM_E_NOMEM, "arena exhausted (sampler state)");
  }
  hipStream_t s = ctx->stream;
  b->groups = std::min(kBetGroups, c.chains);
  b->gs[0] = s;
  {
    hipError_t e = hipEventCreateWithFlags(&b->fork, hipEventDisableTiming);
    for (int g = 0; g < b->groups && e == hipSuccess; ++g) {
      if (g > 0) e = hipStreamCreateWithFlags(&b->gs[g], hipStreamNonBlocking);
      if (e == hipSuccess) e = hipEventCreateWithFlags(&b->join[g], hipEventDisableTiming);
    }
    if (e != hipSuccess) {
      release_blocks(ctx, b->blocks);
      return fail(RTM_E_DEVICE, "sampler streams: %s", hipGetErrorString(e));
    }
  }
  HIP_OK(hipMemcpyAsync(const_cast<int2*>(d.src), src.data(), 8 * (size_t)nsrc, hipMemcpyHostToDevice, s));
  HIP_OK(hipMemcpyAsync(const_cast<int2*>(d.rec), rec.data(), 8 * (size_t)nrec, hipMemcpyHostToDevice, s));
  HIP_OK(hipMemcpyAsync(const_cast<float*>(d.tt_obs), tt_obs_dev, 4 * nd, hipMemcpyDeviceToDevice, s));
  HIP_OK(hipMemsetAsync(d.proposed, 0, 8 * 3 * C, s));
  HIP_OK(hipMemsetAsync(d.accepted, 0, 8 * 3 * C, s));
  HIP_OK(hipMemsetAsync(d.work, 0, 8 * 2 * C, s));
  HIP_OK(hipMemsetAsync(d.mean, 0, 8 * n, s));
  HIP_OK(hipMemsetAsync(d.m2, 0, 8 * n, s));
  HIP_OK(hipMemsetAsync(d.count, 0, 4 * n, s));
  HIP_OK(hipMemsetAsync(d.flags, 0, 256, s));
  // the initial model of every chain and its misfit
  HIP_OK(launch_bet_propose(d, -1, 1, 0, C, s));
  HIP_OK(launch_bet_raster(d, 0, C, s));
  HIP_OK(launch_bet_eikonal(d, 0, C, s));
  HIP_OK(launch_bet_accept(d, 1, nullptr, 0, C, -1, s));
  // the host vectors above are copied from before this call returns
  HIP_OK(hipStreamSynchronize(s));
  *out = b.release();
  return RTM_OK;
}

extern "C" int rtm_bet_run(rtm_ctx* ctx, rtm_bet* bet, int32_t iterations, int8_t* log_dev) {
  if (!ctx || !bet || iterations < 0) return fail(RTM_E_INVAL, "bad arguments");
  HIP_OK(hipSetDevice(ctx->device));
  hipStream_t s = ctx->stream;
  const BetDev& d = bet->d;
  const int G = bet->groups;
  auto sampling = [&](int t) { return t >= d.burn_in && (t - d.burn_in) % d.thin == 0; };
  // Segments of iterations holding at most kBetSnapSlots sampling iterations:
  // every group runs the segment on its stream, recording the chains' states
  // at sampling iterations; then the context stream pools them, chain by
  // chain in order, exactly as one stream would.
  for (int it = 0; it < iterations;) {
    int end = it, slots = 0;
    while (end < iterations && !(slots == kBetSnapSlots && sampling(bet->t + end))) slots += sampling(bet->t + end++);
    HIP_OK(hipEventRecord(bet->fork, s));  // the groups start after earlier work on the context stream
    for (int g = 1; g < G; ++g) HIP_OK(hipStreamWaitEvent(bet->gs[g], bet->fork, 0));
    // iteration by iteration, so that groups sharing a hardware queue alternate
    for (int q = it, slot = 0; q < end; ++q) {
      const int t = bet->t + q;
      for (int g = 0; g < G; ++g) {
        hipStream_t gs = bet->gs[g];
        const int c0 = bet->c0(g), cn = bet->cn(g);
        const bool timed = g == 0 && q == iterations - 1;  // the last iteration of the first group
        if (timed) HIP_OK(hipEventRecord(ctx->bet_ev[0], gs));
        HIP_OK(launch_bet_propose(d, t, 0, c0, cn, gs));
        HIP_OK(launch_bet_raster(d, c0, cn, gs));
        if (timed) HIP_OK(hipEventRecord(ctx->bet_ev[1], gs));
        HIP_OK(launch_bet_eikonal(d, c0, cn, gs));
        if (timed) HIP_OK(hipEventRecord(ctx->bet_ev[2], gs));
        HIP_OK(launch_bet_accept(d, 0, log_dev ? log_dev + (size_t)q * d.chains : nullptr, c0, cn,
                                 sampling(t) ? slot : -1, gs));
        if (timed) HIP_OK(hipEventRecord(ctx->bet_ev[3], gs));
      }
      slot += sampling(t);
    }
    for (int g = 1; g < G; ++g) {
      HIP_OK(hipEventRecord(bet->join[g], bet->gs[g]));
      HIP_OK(hipStreamWaitEvent(s, bet->join[g], 0));
    }
    for (int slot = 0; slot < slots; ++slot) HIP_OK(launch_bet_sample(d, slot, s));
    it = end;
  }
  if (iterations > 0) ctx->bet_valid = true;
  bet->t += iterations;
  return RTM_OK;
}

extern "C" int rtm_bet_chain(rtm_ctx* ctx, rtm_bet* bet, int32_t chain, rtm_bet_chain_info* info, double* z_host,
                             double* x_host, double* v_host) {
  if (!ctx || !bet || !info || chain < 0 || chain >= bet->d.chains) return fail(RTM_E_INVAL, "bad arguments");
  HIP_OK(hipSetDevice(ctx->device));
  const BetDev& d = bet->d;
  hipStream_t s = ctx->stream;
  const size_t K = d.k_max;
  uint32_t flag = 0;
  memset(info, 0, sizeof *info);
  HIP_OK(hipMemcpyAsync(&info->k, d.k + chain, 4, hipMemcpyDeviceToHost, s));
  HIP_OK(hipMemcpyAsync(&info->misfit, d.misfit + chain, 8, hipMemcpyDeviceToHost, s));
  HIP_OK(hipMemcpyAsync(info->proposed, d.proposed + 3 * (size_t)chain, 24, hipMemcpyDeviceToHost, s));
  HIP_OK(hipMemcpyAsync(info->accepted, d.accepted + 3 * (size_t)chain, 24, hipMemcpyDeviceToHost, s));
  HIP_OK(hipMemcpyAsync(&info->solves, d.work + 2 * (size_t)chain, 16, hipMemcpyDeviceToHost, s));
  if (z_host) HIP_OK(hipMemcpyAsync(z_host, d.z + chain * K, 8 * K, hipMemcpyDeviceToHost, s));
  if (x_host) HIP_OK(hipMemcpyAsync(x_host, d.x + chain * K, 8 * K, hipMemcpyDeviceToHost, s));
  if (v_host) HIP_OK(hipMemcpyAsync(v_host, d.v + chain * K, 8 * K, hipMemcpyDeviceToHost, s));
  HIP_OK(hipMemcpyAsync(&flag, d.flags, 4, hipMemcpyDeviceToHost, s));
  HIP_OK(hipStreamSynchronize(s));
  if (flag & kBetNoConverge) return fail(RTM_E_DEVICE, "a travel-time solve did not converge");
  return RTM_OK;
}

extern "C" int rtm_bet_stats(rtm_ctx* ctx, rtm_bet* bet, double* mean_dev, double* std_dev, int32_t* count_dev) {
  if (!ctx || !bet) return fail(RTM_E_INVAL, "bad arguments");
  HIP_OK(hipSetDevice(ctx->device));
  const BetDev& d = bet->d;
  HIP_OK(launch_stats_out(d.mean, d.m2, d.count, (int64_t)d.nz * d.nx, mean_dev, std_dev, count_dev, ctx->stream));
  return RTM_OK;
}

extern "C" int rtm_bet_model(rtm_ctx* ctx, rtm_bet* bet, int32_t chain, int32_t nz, int32_t nx, double h,
                             float* vel_dev) {
  if (!ctx || !bet || !vel_dev || chain < 0 || chain >= bet->d.chains) return fail(RTM_E_INVAL, "bad arguments");
  if (nz < 1 || nx < 1 || (int64_t)nz * nx > ((int64_t)1 << 31) || !(h > 0) || !std::isfinite(h))
    return fail(RTM_E_INVAL, "grid %d x %d, h %g: need positive sizes, at most 2^31 nodes, h > 0", nz, nx, h);
  HIP_OK(hipSetDevice(ctx->device));
  HIP_OK(launch_bet_model(bet->d, chain, nz, nx, h, vel_dev, ctx->stream));
  return RTM_OK;
}

extern "C" int rtm_bet_destroy(rtm_ctx* ctx, rtm_bet* bet) {
  if (!ctx || !bet) return fail(RTM_E_INVAL, "bad arguments");
  Deferred dd;
  dd.blocks = std::move(bet->blocks);
  delete bet;  // its streams have no work the context stream does not already wait for
  return defer(ctx, ctx->stream, std::move(dd));
}

extern "C" int rtm_sqrt_check(rtm_ctx* ctx, uint32_t lo_bits, uint32_t hi_bits, uint64_t* mismatches) {
  if (!ctx || !mismatches || !(lo_bits < hi_bits)) return fail(RTM_E_INVAL, "bad arguments");
  HIP_OK(hipSetDevice(ctx->device));
  unsigned long long* bad = static_cast<unsigned long long*>(arena_alloc(ctx, 256));
  if (!bad) return fail(RTM_E_NOMEM, "arena exhausted");
  hipStream_t s = ctx->stream;
  unsigned long long n = 0;
  hipError_t e = launch_fill_u32(reinterpret_cast<uint32_t*>(bad), 0, 2, s);
  if (e == hipSuccess) e = launch_sqrt_check(lo_bits, hi_bits, bad, s);
  if (e == hipSuccess) e = hipMemcpyAsync(&n, bad, 8, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  ctx->arena.release(bad, 256);
  if (e != hipSuccess) return fail(RTM_E_DEVICE, "square-root check: %s", hipGetErrorString(e));
  *mismatches = n;
  return RTM_OK;
}

extern "C" int rtm_ctx_stats(rtm_ctx* ctx, rtm_ctx_stats_t* out) {
  if (!ctx || !out) return fail(RTM_E_INVAL, "bad arguments");
  memset(out, 0, sizeof *out);
  {
    std::lock_guard<std::mutex> lk(ctx->mu);
    out->jobs_submitted = ctx->book->submitted();
    out->jobs_done = ctx->book->done();
    out->jobs_failed = ctx->book->failed();
    out->jobs_cancelled = ctx->book->cancelled();
    out->active_jobs = (int32_t)ctx->book->running();
    out->queued_jobs = (int32_t)ctx->book->queued();
  }
  out->steps_launched = ctx->steps_launched;
  out->graph_replays = ctx->graph_replays;
  out->grid_updates = ctx->grid_updates;
  out->alg_bytes = ctx->alg_bytes;
  out->arena_bytes = ctx->arena.size();
  out->arena_used = ctx->arena.used();
  out->arena_peak = ctx->arena.peak();
  out->tile_z = choose_tz(ctx);
  out->last_born_groups = ctx->born_groups;
  if (ctx->ph_valid) {
    float a = 0, b = 0;
    if (hipEventSynchronize(ctx->ph_ev[2]) == hipSuccess &&
        hipEventElapsedTime(&a, ctx->ph_ev[0], ctx->ph_ev[1]) == hipSuccess &&
        hipEventElapsedTime(&b, ctx->ph_ev[1], ctx->ph_ev[2]) == hipSuccess) {
      out->last_fwd_ms = a;
      out->last_bwd_ms = b;
      out->last_steps_per_launch = ctx->ph_steps_per_launch;
      out->last_tile_z2_fwd = ctx->ph_tz2[0];
      out->last_tile_z2_bwd = ctx->ph_tz2[1];
      out->last_groups_fwd = ctx->ph_groups[0];
      out->last_groups_bwd = ctx->ph_groups[1];
      out->last_fwd_launches = ctx->ph_launches[0];
      out->last_bwd_launches = ctx->ph_launches[1];
      out->last_fwd_launch_bytes = ctx->ph_bytes[0];
      out->last_bwd_launch_bytes = ctx->ph_bytes[1];
    }
  }
  if (ctx->bet_valid) {
    float a = 0, b = 0;
    if (hipEventSynchronize(ctx->bet_ev[3]) == hipSuccess &&
        hipEventElapsedTime(&a, ctx->bet_ev[1], ctx->bet_ev[2]) == hipSuccess &&
        hipEventElapsedTime(&b, ctx->bet_ev[0], ctx->bet_ev[3]) == hipSuccess) {
      out->last_bet_eikonal_ms = a;
      out->last_bet_iteration_ms = b;
    }
  }
  if (ctx->zc_op) {
    float ms = 0;
    if (hipEventSynchronize(ctx->zc_ev[1]) == hipSuccess &&
        hipEventElapsedTime(&ms, ctx->zc_ev[0], ctx->zc_ev[1]) == hipSuccess) {
      out->last_codec_ms = ms;
      out->last_codec_op = ctx->zc_op;
      out->last_codec_bytes = ctx->zc_bytes;
    }
  }
  std::lock_guard<std::mutex> lk(ctx->mu);

  return RTM_OK;
}
