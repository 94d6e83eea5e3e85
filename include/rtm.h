/*
 * rtm.h -- C ABI of the MI355X (gfx950) reverse-time-migration library.
 *
 * The library computes the data-parallel hot path of arXiv:2001.06444
 * ("A workflow for seismic imaging with quantified uncertainty"):
 *   - the acoustic isotropic two-way wave equation (Eq. 4), discretised
 *     2nd order in time and 8th order in space (Sec. 3, Stage 2), with a
 *     Cerjan absorbing sponge around each job's grid;
 *   - the forward source wavefield, driven by the wavelet (Sec. 2.2);
 *   - the source wavefield kept as snapshots (FP32, or BF16/FP16 with a
 *     per-snapshot power-of-two scale) or rebuilt backward from saved
 *     boundary rings (time reversal);
 *   - the backward receiver wavefield, driven by the seismogram (Sec. 2.2),
 *     computed as the exact discrete adjoint of the forward recursion
 *     (Sec. 3: the reverse problem is kept coercive, after Givoli 2014);
 *   - the zero-lag cross-correlation image (numerator of Eq. 5), optional
 *     source illumination (denominator of Eq. 5), stacking over shots
 *     (Fig. 2 caption), and running FP64 mean / standard deviation maps
 *     over velocity samples (Sec. 2.3, Stage 3);
 *   - the Stage-3 maps built from those statistics: the confidence index
 *     (Eq. 6) and the std/mean ratio (Eq. 7), and the post-stack Laplacian
 *     filter (Sec. 3, Stage 2).
 *
 * Discretisation (shared by every entry point):
 *   u^{n+1} = G (2u^n + c (L u^n + f^n)) - G^2 u^{n-1},   c = v^2 dt^2,
 * L the 17-point 8th-order Laplacian, G = g(d_z) g(d_x) with
 * g(d) = exp(-(a d)^2), d the number of cells outside the physical window.
 * Source term: f^n = w^n / (dx dz) at the source node.  Traces: d[n][r] =
 * u^n(r), n = 0..nt-1 (d[0] = 0).  Receiver wavefield: R^{nt} = R^{nt+1} = 0,
 * R^m = G(2R^{m+1} + c(L R^{m+1} + d[m] at receivers)) - G^2 R^{m+2}.
 * Image: I = k sum_{n in N} S^n R^{n+1}, N = {0, k, 2k, ...}, n <= nt-2,
 * over the physical window (k = snapshot stride; 1 in reconstruct mode).
 *
 * Conventions:
 *   - Arrays are row-major [z][x] with x contiguous; traces are [t][receiver].
 *   - Every pointer whose name ends in _dev is a caller-owned device pointer
 *     on the context's device; _host pointers are host memory.  The library
 *     never frees caller memory.
 *   - Calls that take a context enqueue work on the context stream and
 *     return before the work completes (stream-ordered), unless stated.
 *   - Every function returns RTM_OK (0) or a negative RTM_E_* code.  A call
 *     rejected by validation has done no device work.  rtm_last_error()
 *     gives a human-readable detail for the calling thread's last failure.
 */
#ifndef RTM_H
#define RTM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ---------------------------------------------------- */
enum {
    RTM_OK = 0,
    RTM_E_INVAL = -1,     /* invalid argument or geometry */
    RTM_E_CFL = -2,       /* v_max dt sqrt(1/dx^2 + 1/dz^2) above the stability limit */
    RTM_E_NOMEM = -3,     /* arena too small for the request */
    RTM_E_AGAIN = -4,     /* queue full; retry later */
    RTM_E_NOTFOUND = -5,  /* unknown ticket or realization */
    RTM_E_NONFINITE = -6, /* a wavefield became non-finite */
    RTM_E_DEVICE = -7,    /* a HIP runtime call failed */
    RTM_E_CANCELLED = -8  /* the job was cancelled */
};

/* ---- enumerations ---------------------------------------------------- */
enum { RTM_SNAP_FP32 = 0, RTM_SNAP_BF16 = 1, RTM_SNAP_FP16 = 2 };
enum { RTM_SRC_STORE = 0, RTM_SRC_RECONSTRUCT = 1 };
enum { RTM_IMG_ILLUM = 1u };
enum { RTM_JOB_QUEUED = 0, RTM_JOB_RUNNING = 1, RTM_JOB_DONE = 2, RTM_JOB_FAILED = 3,
       RTM_JOB_CANCELLED = 4 };

typedef struct rtm_ctx rtm_ctx;

/* Physical model grid and time axis.  A job's padded window, (nz + 2 nb)
 * rows by (window width + 2 nb) columns, must give wavefield arrays of
 * fewer than 2^30 floats (about 32000 x 32000 nodes; the step kernels
 * address a field with 32-bit byte offsets); larger windows are rejected
 * with RTM_E_INVAL before any device work. */
typedef struct {
    int32_t nz, nx;  /* model rows (depth) and columns */
    int32_t nb;      /* sponge width in cells, added on all four sides of a job window */
    int32_t nt;      /* time samples (>= 2) */
    float dz, dx;    /* grid spacing (m) */
    float dt;        /* time step (s) */
    float sponge_a;  /* Cerjan constant a; <= 0 selects 0.3 / nb */
} rtm_grid;

/* An on-grid node in model coordinates (row iz, column ix). */
typedef struct {
    int32_t iz, ix;
} rtm_point;

/* Source-wavefield handling and imaging options. */
typedef struct {
    int32_t src_mode;    /* RTM_SRC_STORE or RTM_SRC_RECONSTRUCT */
    int32_t snap_dtype;  /* RTM_SNAP_*; store mode only */
    int32_t snap_stride; /* k >= 1; store mode only (reconstruct images every step) */
    uint32_t flags;      /* RTM_IMG_ILLUM: also accumulate sum k (S^n)^2 */
} rtm_img_opts;

/* ---- library-level helpers ------------------------------------------- */

/* Static description of a status code. */
const char *rtm_status_str(int status);

/* Detail text of the calling thread's last failed call ("" if none). */
const char *rtm_last_error(void);

/* ABI version (major * 10000 + minor * 100 + patch). */
int rtm_version(void);

/* Courant number v_max dt sqrt(1/dx^2 + 1/dz^2) of a grid (host only). */
double rtm_cfl_number(float v_max, float dt, float dz, float dx);

/* Largest stable Courant number of the scheme (von Neumann limit,
 * 2 / sqrt(|sum of the 1-D stencil symbol at the Nyquist wavenumber|)),
 * about 0.78437; calls above it are rejected with RTM_E_CFL (Sec. 3: each
 * migration checks its own CFL condition).  Host only. */
double rtm_cfl_limit(void);

/* ---- context --------------------------------------------------------- */

/* Create a context on HIP device `device`: the device memory and streams
 * every migration of the Monte Carlo loop (Sec. 3, Stage 2) runs in.
 *   arena_dev, arena_bytes: caller-owned device buffer the library
 *     sub-allocates all its working memory from (wavefields, snapshot and
 *     boundary storage, per-job images, statistics).  It must stay alive
 *     until rtm_ctx_destroy.  arena_dev == NULL makes the library allocate
 *     arena_bytes itself (freed at destroy).
 *   hip_stream: hipStream_t the stream-ordered calls enqueue on (NULL =
 *     the device's null stream).
 *   flags: reserved, pass 0.
 * On success *out receives the context. */
int rtm_ctx_create(rtm_ctx **out, int device, void *arena_dev, size_t arena_bytes,
                   void *hip_stream, uint32_t flags);

/* Stop the scheduler, wait for all work, release the context. */
int rtm_ctx_destroy(rtm_ctx *ctx);

/* Wait until all work the context enqueued on its stream has finished. */
int rtm_ctx_synchronize(rtm_ctx *ctx);

/* ---- plain path (one launch per time step) --------------------------- */

/* Forward modelling of one shot over the whole model (Eq. 4 with the
 * wavelet as source term; Sec. 2.2).
 *   vel_dev [nz][nx] velocity (m/s); wavelet_dev [nt] source samples w^n;
 *   src: source node; rec_host [nrec]: receiver nodes (copied at call time),
 *     pairwise distinct (a repeated node is RTM_E_INVAL: every call adds one
 *     sample per node, so results do not depend on the order of additions);
 *   traces_dev [nt][nrec] out: d[n][r] = u^n(r);
 *   final_field_dev [nz][nx] out (nullable): u^{nt-1} on the model grid.
 * Errors: RTM_E_INVAL (bad sizes/nodes), RTM_E_CFL, RTM_E_NOMEM. */
int rtm_propagate(rtm_ctx *ctx, const rtm_grid *grid, const float *vel_dev,
                  const float *wavelet_dev, rtm_point src, int32_t nrec,
                  const rtm_point *rec_host, float *traces_dev, float *final_field_dev);

/* Born (single-scattering) modelling of one shot over the whole model: the
 * linearisation of Eq. 4 that migration is the exact adjoint of (Sec. 3,
 * reverse problem).  Background u0 as in rtm_propagate and
 *   du^{n+1} = G (2du^n + c (L du^n + m u0^n)) - G^2 du^{n-1},
 * dtraces[n][r] = du^n(r).  mpert_dev [nz][nx]: perturbation m (zero in the
 * sponge by construction); other arguments as in rtm_propagate.
 * Errors: RTM_E_INVAL, RTM_E_CFL, RTM_E_NOMEM. */
int rtm_born(rtm_ctx *ctx, const rtm_grid *grid, const float *vel_dev, const float *wavelet_dev,
             rtm_point src, const float *mpert_dev, int32_t nrec, const rtm_point *rec_host,
             float *dtraces_dev);

/* One shot of a Born batch: source, receivers and its output traces. */
typedef struct {
    rtm_point src;
    int32_t nrec;
    const rtm_point *rec_host; /* [nrec], model coordinates, pairwise distinct */
    float *dtraces_dev;        /* [nt][nrec] out: du^n at the receivers */
} rtm_born_shot;

/* Born modelling of nshots shots of one model and one perturbation (the
 * linearised operator of rtm_born, Sec. 3 reverse problem) in shared
 * kernel launches: each launch advances the background and scattered field
 * of every shot of a shot group by two time steps (one with RTM_TILE_Z2=0),
 * and the shots read one c array and one copy of mpert_dev.  Shot groups
 * are consecutive shots whose fields fit the memory-side cache budget
 * (RTM_GROUP_KB, KiB, default 200 MiB; 0 or less: one group), each running
 * all its steps before the next; groups alternate between ctx's stream and
 * the library's further group streams (RTM_GROUP_STREAMS, 1-4, default 2),
 * which are forked from ctx's stream and joined back into it, and the
 * budget is shared among them.  Each shot's dtraces equal rtm_born's for
 * that shot bit for bit, whatever the groups.  shots_host [nshots] is read
 * at call time; the other arguments as in rtm_born.  Stream-ordered on ctx's
 * stream; rtm_ctx_stats reports the group count.
 * Errors: RTM_E_INVAL (no shots, bad nodes, missing dtraces_dev),
 * RTM_E_CFL, RTM_E_NOMEM (the whole batch must fit the arena). */
int rtm_born_batch(rtm_ctx *ctx, const rtm_grid *grid, const float *vel_dev, const float *wavelet_dev,
                   const float *mpert_dev, int32_t nshots, const rtm_born_shot *shots_host);

/* Reverse time migration of one shot on the aperture window
 * [ix0, ix0 + width) of the model (Sec. 2.2, Eq. 5 numerator; the per-shot
 * forward + adjoint pair of the paper's migration code).
 *   vel_dev [nz][nx]: migration velocity; the window's sponge takes the
 *     window's edge velocities.
 *   data_dev [nt][nrec]: seismogram injected at the receivers.
 *   src, rec_host: nodes inside the window (model coordinates); receivers
 *     pairwise distinct, as in rtm_propagate.
 *   opts: source-wavefield mode, snapshot dtype and stride, flags.
 *   image_dev [nz][nx]: the shot image is ADDED into columns [ix0, ix0+width)
 *     (stack over shots).  illum_dev likewise (nullable; needs RTM_IMG_ILLUM).
 * Errors: RTM_E_INVAL, RTM_E_CFL, RTM_E_NOMEM. */
int rtm_migrate_shot(rtm_ctx *ctx, const rtm_grid *grid, const float *vel_dev,
                     const float *wavelet_dev, rtm_point src, int32_t nrec,
                     const rtm_point *rec_host, const float *data_dev, int32_t ix0,
                     int32_t width, const rtm_img_opts *opts, float *image_dev,
                     float *illum_dev);

/* ---- batched path ---------------------------------------------------- */

/* One shot of a batch: source, window, receivers and its seismogram. */
typedef struct {
    rtm_point src;
    int32_t ix0, width;        /* aperture window in model columns */
    int32_t nrec;
    const rtm_point *rec_host; /* [nrec], model coordinates */
    const float *data_dev;     /* [nt][nrec] */
} rtm_shot_desc;

/* Migrate nshots shots of one model together (Sec. 3, Stage 2: the shots of
 * one velocity model): the shots advance in shared kernel launches, two time
 * steps per launch in reconstruct and store mode without illumination (two-step tile
 * heights from the autotuner per phase; RTM_TILE_Z2 = 16, 24 or 32 forces a
 * height, 0 keeps one step per launch; results are the same bit for bit;
 * rtm_ctx_stats reports the heights used), launches are replayed from a
 * captured HIP graph, and the one-step tile shape comes from the autotuner.
 * All shots are resident at once; each phase runs them in groups of
 * consecutive shots whose levels fit the memory-side cache (RTM_GROUP_KB,
 * default 200 MiB of field bytes the launches in flight touch; 0 runs all
 * shots in every launch), the groups dealt in turn to RTM_GROUP_STREAMS
 * streams (1 to 4, default 2; each group then gets its share of the budget)
 * whose launches overlap, and groups on one stream one after another; none
 * of this changes a result.  The call is ordered after the work already on
 * ctx's stream, and work enqueued there afterwards waits for it.
 * Each shot's image is added into image_dev in shot order after all shots
 * finish (deterministic stack).  Shots with the same window (ix0, width)
 * share one c = v^2 dt^2 array and its sponge profiles, built once.  Same
 * argument meaning as rtm_migrate_shot; image_dev/illum_dev [nz][nx].
 * Errors: RTM_E_INVAL, RTM_E_CFL, RTM_E_NOMEM (the whole batch must fit). */
int rtm_migrate_batch(rtm_ctx *ctx, const rtm_grid *grid, const float *vel_dev,
                      const float *wavelet_dev, int32_t nshots, const rtm_shot_desc *shots_host,
                      const rtm_img_opts *opts, float *image_dev, float *illum_dev);

/* ---- ensemble / serving path ------------------------------------------
 *
 * Stage 2 migrates the seismograms for every velocity sample of Stage 1,
 * RTM wrapped in a Monte Carlo loop (Sec. 1; Sec. 2.2, last paragraph), and
 * the paper farms the migrations out as subgroups, each starting as soon as
 * the previous one finishes, with every migration checking its own CFL
 * condition (Sec. 3, Stage 2).  Here the subgroups become jobs of one
 * device: a scheduler thread admits queued jobs whenever arena memory frees
 * up and advances every admitted job in the same kernel launches
 * (continuous batching); finished images feed per-sample statistics on the
 * device (Sec. 2.3, Stage 3).  Reconstruct-mode jobs advance two steps per
 * launch where they can; RTM_SERVE_STORE_PAIRS=1 does the same for
 * store-mode jobs (shorter median latency of lone jobs, longer tail under
 * load).  RTM_SERVE_KB (KiB) optionally caps the field bytes the running
 * jobs' launches touch; admission then waits, in order, until running jobs
 * finish. */

/* Register velocity sample `realization` (Sec. 3, Stage 2: one migration
 * set per velocity sample).  The velocity is copied into the arena and v_max
 * cached for the per-job CFL check.  Model size must equal the context's
 * other registered models.  Re-registering a realization replaces it, only
 * when no job of it is queued or running (RTM_E_AGAIN otherwise, also when a
 * job of it was submitted while the call ran). */
int rtm_model_register(rtm_ctx *ctx, int32_t realization, const float *vel_dev, int32_t nz,
                       int32_t nx, const rtm_grid *grid);

/* One RTM job of a stream (velocity sample x shot x aperture x nt): one
 * member of a subgroup of Sec. 3, Stage 2. */
typedef struct {
    int32_t realization;
    rtm_point src;             /* model coordinates */
    int32_t ix0, width;        /* aperture window; receivers on every window
                                  column at row rec_iz */
    int32_t rec_iz;
    int32_t nt;                /* time samples of this job (>= 2) */
    const float *wavelet_dev;  /* [nt] */
    const float *data_dev;     /* [nt][width]; must stay alive until DONE */
    rtm_img_opts img;
    uint32_t flags;            /* RTM_JOB_* accumulation flags below */
    uint64_t user_tag;
} rtm_job;

enum {
    RTM_JOB_ACC_STATS = 1u, /* add the job image to its realization's running mean/std */
    RTM_JOB_ACC_STACK = 2u  /* add the job image to its realization's FP32 stack */
};

/* Queue a job (non-blocking; Sec. 3, Stage 2: a migration starts as soon as
 * room frees up).  Validation and the CFL check (cached v_max; each
 * migration checks its own CFL condition) happen here; a job larger than the
 * whole arena returns RTM_E_NOMEM, a full queue RTM_E_AGAIN.  Memory pressure
 * only delays admission: queued jobs are admitted first come, first served,
 * except that while the oldest waiting job does not fit, later jobs that do
 * fit may pass it, at most 8 times. */
int rtm_ensemble_submit(rtm_ctx *ctx, const rtm_job *job, uint64_t *ticket);

/* Job state and timing. */
typedef struct {
    int32_t state;   /* RTM_JOB_* state */
    int32_t status;  /* RTM_OK or the failure code */
    double t_submit, t_admit, t_done; /* host monotonic seconds */
    uint64_t grid_updates;            /* point updates the job performs */
    uint64_t alg_bytes;               /* algorithmic HBM bytes of the job */
    uint64_t user_tag;
} rtm_job_info;

/* Non-blocking status query of a submitted job (Sec. 3, Stage 2).  When
 * the job is DONE and image_dev is not
 * NULL, its [nz][width] image is copied there (stream-ordered on the
 * context stream).  A DONE/FAILED/CANCELLED job is forgotten after a poll
 * that passes release = 1. */
int rtm_ensemble_poll(rtm_ctx *ctx, uint64_t ticket, rtm_job_info *info, float *image_dev,
                      int32_t release);

/* Cancel a queued job (running jobs finish; RTM_E_INVAL once admitted).
 * RTM_E_NOTFOUND if unknown. */
int rtm_ensemble_cancel(rtm_ctx *ctx, uint64_t ticket);

/* Block until every submitted job has finished (DONE, FAILED or CANCELLED):
 * the end of the Monte Carlo loop over samples (Sec. 3, Stage 2). */
int rtm_ensemble_drain(rtm_ctx *ctx);

/* Running per-pixel statistics of a realization's job images (FP64
 * Welford; a pixel's samples are the images whose window covers it): the
 * mean and standard-deviation maps of Stage 3 (Sec. 2.3).
 *   mean_dev, std_dev [nz][nx] double (nullable), count_dev [nz][nx] int32
 *   (nullable).  std is the sample standard deviation (n - 1); 0 where
 *   count < 2.  Stream-ordered after every finished job's update. */
int rtm_ensemble_stats(rtm_ctx *ctx, int32_t realization, double *mean_dev, double *std_dev,
                       int32_t *count_dev);

/* FP32 shot stack of a realization (sum of its RTM_JOB_ACC_STACK job
 * images, window-placed; the stacked section of Fig. 2) copied to
 * stack_dev [nz][nx]. */
int rtm_ensemble_stack(rtm_ctx *ctx, int32_t realization, float *stack_dev);

/* ---- ensemble statistics over explicit images (Sec. 2.3) ------------- */

/* FP64 Welford accumulator over [nz][nx] images (one per velocity sample). */
typedef struct rtm_stats rtm_stats;

int rtm_stats_create(rtm_ctx *ctx, rtm_stats **out, int32_t nz, int32_t nx);
int rtm_stats_destroy(rtm_ctx *ctx, rtm_stats *st);
/* Add one FP32 image [nz][width] whose columns are [ix0, ix0 + width). */
int rtm_stats_add(rtm_ctx *ctx, rtm_stats *st, const float *image_dev, int32_t ix0,
                  int32_t width);
/* mean/std (double, nullable), count (int32, nullable) as in rtm_ensemble_stats. */
int rtm_stats_get(rtm_ctx *ctx, rtm_stats *st, double *mean_dev, double *std_dev,
                  int32_t *count_dev);

/* Chan merge of two accumulators of the same size: dst becomes the
 * statistics of the union of both sample sets (per pixel n = na + nb,
 * d = mb - ma, mean = ma + d nb/n, M2 = M2a + M2b + d^2 na nb/n).  This is
 * the combine step for statistics kept on several devices or streams. */
int rtm_stats_merge(rtm_ctx *ctx, rtm_stats *dst, const rtm_stats *src);

/* ---- Stage-3 maps and post-stack filter ------------------------------ */

/* Source-normalised image (Eq. 5): out = image / (illum + eps_rel *
 * max(illum)), with image and illum the numerator and denominator sums of a
 * migration run with RTM_IMG_ILLUM.  All arrays [n] float. */
int rtm_normalize_image(rtm_ctx *ctx, const float *image_dev, const float *illum_dev, int32_t n,
                        float eps_rel, float *out_dev);


/* Confidence index (Eq. 6): c = (s_max - s) / (s_max - s_min), s_min and
 * s_max the extremes of std over pixels with count >= min_count; pixels
 * below min_count get 0.  conf_dev [n] out (double). */
int rtm_confidence_map(rtm_ctx *ctx, const double *std_dev, const int32_t *count_dev,
                       int32_t n, int32_t min_count, double *conf_dev);

/* Ratio map (Eq. 7): r = std / mean where |mean| > eps, else 0.
 * ratio_dev [n] out (double). */
int rtm_ratio_map(rtm_ctx *ctx, const double *std_dev, const double *mean_dev, int32_t n,
                  double eps, double *ratio_dev);

/* Post-stack Laplacian filter (Sec. 3: attenuates the low-frequency
 * artefacts of the brute stack): out = -(8th-order Laplacian of img) with
 * zero values outside the image.  img_dev/out_dev [nz][nx] float. */
int rtm_laplacian_filter(rtm_ctx *ctx, const float *img_dev, int32_t nz, int32_t nx, float dz,
                         float dx, float *out_dev);

/* ---- codec: fixed-accuracy / lossless compression of float32 arrays ----
 *
 * The workflow compresses velocity models, migrated images and seismograms
 * between its stages with an error-bounded block-transform coder, in a lossy
 * fixed-accuracy setting and a lossless one (Sec. 3, data-compression
 * paragraph; Sec. 4.2, Tables 1 and 2).  This coder is the library's own
 * design for that job:
 *   - 8 x 8 blocks (edge rows / columns repeated), in the order
 *     (array, block row, block column);
 *   - fixed accuracy: q = rint(x / (2 tol)) (float64, ties to even), so every
 *     decoded value is within tol (1 + 2^-26) + 2^-24 |x'| of the input (the
 *     last term is the float32 rounding of the decoded value x');
 *     lossless: q = the float32 bit pattern as an order-preserving int32;
 *   - three levels of a 2-D integer Haar lifting (modulo 2^32, exactly
 *     invertible), zig-zag, five sub-bands each stored in its own bit width.
 * Stream (32-bit words): [0..7] magic 0x315A5452, mode, count, rows, cols,
 * blocks per chunk (256), tol (float64; 0 if lossless); chunk table
 * [nchunks + 1]; block headers [nblocks]; payload.  The stream is
 * self-describing and position independent.
 *
 * Arrays are dense [count][rows][cols] float32 (cols contiguous), caller
 * owned, on the context's device.  Both calls are stream-ordered on the
 * context stream and return after that stream has finished them (the encoder
 * must report the stream length, the decoder its validation result). */
enum { RTM_CODEC_TOL = 0, RTM_CODEC_LOSSLESS = 1, RTM_CODEC_ZFP = 2 };

/* RTM_CODEC_ZFP: the published ZFP method in fixed-accuracy mode (Lindstrom,
 * IEEE TVCG 20(12), 2014), the coder the paper uses (Sec. 4.2), for 2-D
 * float32 arrays:
 *   - 4 x 4 blocks (edges repeated) in the order (array, block row, block
 *     column); block floating point with the block's largest exponent e and
 *     30-bit integers q = trunc(x 2^(30 - e));
 *   - ZFP's decorrelating transform (integer lifting of
 *     T = 1/16 [[4,4,4,4],[5,1,-1,-5],[-4,4,4,-4],[-2,6,-6,2]]) on rows, then
 *     columns; coefficients by sequency; negabinary digits;
 *   - embedded bit-plane coding with group tests, planes from 31 down to
 *     32 - min(32, max(0, e - floor(log2 tol) + 6));
 *   - a zero block, or one below the tolerance, is one 0 bit; else a 1 bit,
 *     e + 127 in 8 bits and its planes.
 * Accepted: tol >= 2^-60, |x| < 2^100, finite.  Decoded values stay within
 * tol of the input (the method's guard planes; checked on the benchmark
 * banks and random data).  Stream: [0..7] magic 0x465A5452, mode 2, count,
 * rows, cols, 16 blocks per chunk, tol (float64); chunk table [nchunks + 1]
 * (payload word offset of each chunk of 16 blocks, then the total);
 * payload (each chunk's block codes, bits least-significant first, padded
 * to a word).  rtm_codec_decode reads either format. */

/* Largest stream the encoder can produce for this shape in any mode (64
 * words per 8 x 8 block plus the index, or 585 bits per 4 x 4 block plus the
 * chunk table for RTM_CODEC_ZFP, whichever is larger), or -1 for a shape that
 * is empty or exceeds 2^26 - 1 blocks of 8 x 8 per stream. */
int64_t rtm_codec_max_bytes(int32_t count, int32_t rows, int32_t cols);

/* Encode x_dev [count][rows][cols] into stream_dev (capacity_bytes, 4-byte
 * aligned).  mode RTM_CODEC_TOL needs a finite tol > 0, RTM_CODEC_ZFP a
 * finite tol >= 2^-60; RTM_CODEC_LOSSLESS ignores tol.  *stream_bytes receives the stream length, also when the
 * buffer is too small.
 * Errors: RTM_E_INVAL (bad shape or mode; a non-finite value or
 * |x| / (2 tol) > 2^31 - 1 in fixed-accuracy mode), RTM_E_NOMEM (capacity
 * below the length: nothing past capacity_bytes is written; arena
 * exhausted), RTM_E_DEVICE. */
int rtm_codec_encode(rtm_ctx *ctx, const float *x_dev, int32_t count, int32_t rows, int32_t cols,
                     int32_t mode, double tol, void *stream_dev, int64_t capacity_bytes,
                     int64_t *stream_bytes);

/* rtm_codec_encode for callers that cannot allocate memory (code that must
 * not call hipMalloc, e.g. under stream capture or in a serving loop with
 * fixed memory): same arguments, results and stream bytes as
 * rtm_codec_encode, but the look-back state lives in a 1 MiB device array
 * the library holds on every device it runs on until the process ends,
 * instead of the context arena, and the call allocates nothing.
 *   Limit: at most (2^20 - 256) / 8 = 131040 chunks of 256 8 x 8 blocks
 *   (about 2.1e9 values per call); larger arrays return RTM_E_INVAL before
 *   any device work.
 *   Calls on one device share the array and its last contents (cleared by
 *   each call before use): two calls overlapping on one device would race,
 *   so the library serialises these calls per device with a lock held
 *   until the call's kernels have finished.  Errors as rtm_codec_encode;
 *   RTM_E_DEVICE if the array's address was not found when the context was
 *   created. */
int rtm_codec_encode_noalloc(rtm_ctx *ctx, const float *x_dev, int32_t count, int32_t rows, int32_t cols,
                             int32_t mode, double tol, void *stream_dev, int64_t capacity_bytes,
                             int64_t *stream_bytes);

/* Read and validate a stream's header (copies its first 32 bytes to the
 * host).  Any output pointer may be NULL.  Errors: RTM_E_INVAL (not a codec
 * stream, bad header, stream shorter than its index). */
int rtm_codec_info(rtm_ctx *ctx, const void *stream_dev, int64_t stream_bytes, int32_t *mode,
                   int32_t *count, int32_t *rows, int32_t *cols, double *tol);

/* Decode stream_dev (stream_bytes long) into x_dev, which must hold
 * count * rows * cols floats (capacity_floats).  Reads never leave the
 * stream; a stream whose widths, chunk table or length disagree returns
 * RTM_E_INVAL (x_dev then holds partial output).  RTM_E_NOMEM: x_dev too
 * small.  For ZFP-method streams the environment variable
 * RTM_ZFP_STAGE_BYTES sets the LDS budget per decoder workgroup for its
 * staged payload (0: none; unset: chosen from the stream's mean payload);
 * the result does not depend on it. */
int rtm_codec_decode(rtm_ctx *ctx, const void *stream_dev, int64_t stream_bytes, float *x_dev,
                     int64_t capacity_floats);

/* ---- Stage 1: Bayesian Eikonal tomography ------------------------------
 *
 * Sec. 2.1 (Eq. 1-3): travel times are the Eikonal equation's first
 * arrivals; velocity samples come from reversible-jump Markov chains over
 * Voronoi tessellations with a constant velocity per cell; the likelihood is
 * exp(-Phi / 2), Phi = sum over sources and receivers of ((T - d) / sigma)^2.
 *   - Travel times: first-order Godunov upwind scheme on a square grid of
 *     spacing h (m), point sources and receivers at grid nodes, solved by
 *     fast sweeping in single precision: Gauss-Seidel sweeps in the four
 *     orderings in turn until four in a row change nothing (the times of
 *     repeating passes of four until a pass changes nothing), at most 1024
 *     sweeps.
 *   - Model: k nuclei (k_min <= k <= k_max <= 64) with positions in
 *     [0, (nz-1) h] x [0, (nx-1) h] and velocities; a node takes the velocity
 *     of the nearest nucleus (ties: lowest index).
 *   - Each iteration a chain proposes, with probabilities p_birth, p_death
 *     and 1 - p_birth - p_death, to add a nucleus (position and velocity
 *     drawn from the uniform prior), delete a uniformly chosen one, or move one
 *     by a uniform step of half-widths (move_dz, move_dx); proposals leaving
 *     the bounds are rejected; the rest are accepted with probability
 *     min(1, exp(-(Phi' - Phi) / 2)).
 *   - Random numbers: splitmix64 in counter form; chain c's stream is seeded
 *     by output c of the stream seeded with `seed`; iteration t (t = -1 for
 *     the initial model) uses its outputs (t + 1) * 256 + k.  Initial model:
 *     k_init nuclei from the prior.
 *   - After burn_in iterations, every thin-th iteration adds every chain's
 *     velocity grid (chains in order) to a pooled FP64 Welford mean / M2 per
 *     node: the velocity uncertainty maps of Stage 3.
 * Grids have at most 40000 nodes, and a solve's times must fit the 160 KB of
 * LDS of a compute unit: 4 (264 + (nz + 1) ld) bytes, with ld the even number
 * nx + 1 or nx + 2 up to 128 rows, else nx (e.g. 71 x 341 nodes: 100 KB). */
typedef struct {
    int32_t nz, nx;                 /* grid nodes */
    int32_t chains;                 /* chains advanced together */
    int32_t k_min, k_max, k_init;   /* Voronoi cells: bounds and initial count */
    int32_t burn_in, thin;          /* sampling of the velocity statistics */
    double h;                       /* node spacing (m) */
    double v_min, v_max;            /* uniform velocity prior (m/s) */
    double p_birth, p_death;        /* proposal probabilities; a move otherwise */
    double move_dz, move_dx;        /* half-widths of a nucleus move (m) */
    double sigma;                   /* travel-time noise standard deviation (s) */
    uint64_t seed;
} rtm_bet_config;

typedef struct {
    int32_t k;                      /* cells of the current model */
    int32_t pad_;
    double misfit;                  /* Phi of the current model */
    int64_t proposed[3], accepted[3];  /* birth, death, move (valid proposals) */
    int64_t solves;                 /* travel-time solves (one per source per valid proposal) */
    int64_t sweeps;                 /* fast sweeps (one ordering each) of those solves */
} rtm_bet_chain_info;

typedef struct rtm_bet rtm_bet;

/* Travel times tt_dev [nsrc][nrec] (s, float) of the velocity grid vel_dev
 * [nz][nx] (m/s, float) for sources src_host[nsrc] and receivers
 * rec_host[nrec] (grid nodes).  Synchronous.  Errors: RTM_E_INVAL (shape,
 * points outside the grid, a grid beyond the limits above, or a node where
 * h / v, in single precision, lies outside [1e-9, 1e18] s -- velocities must
 * be positive and finite), RTM_E_DEVICE (a solve did not converge). */
int rtm_eikonal(rtm_ctx *ctx, const float *vel_dev, int32_t nz, int32_t nx, float h, int32_t nsrc,
                const rtm_point *src_host, int32_t nrec, const rtm_point *rec_host, float *tt_dev);

/* Creates the sampler: copies the observed travel times tt_obs_dev
 * [nsrc][nrec] (s), draws every chain's initial model and computes its
 * misfit (stream-ordered).  Errors: RTM_E_INVAL (bad configuration:
 * chains outside 1..65535, k bounds outside 1..64, h / v outside
 * [1e-9, 1e18] s for v in [v_min, v_max], ...),
 * RTM_E_NOMEM (arena). */
int rtm_bet_create(rtm_ctx *ctx, const rtm_bet_config *cfg, int32_t nsrc, const rtm_point *src_host,
                   int32_t nrec, const rtm_point *rec_host, const float *tt_obs_dev, rtm_bet **out);

/* Advances every chain by `iterations` (stream-ordered, returns after
 * enqueue: the chains advance in two groups on streams the sampler owns,
 * which start after the context stream's earlier work and which the context
 * stream waits for).  log_dev (nullable) receives [iterations][chains]
 * outcomes: -1 invalid proposal, 0 rejected, 1 birth / 2 death / 3 move
 * accepted.  Calls on one sampler must not overlap. */
int rtm_bet_run(rtm_ctx *ctx, rtm_bet *bet, int32_t iterations, int8_t *log_dev);

/* Copies chain `chain`'s state to the host (synchronous): info, and the
 * nuclei z/x/v (k_max doubles each, nullable).  RTM_E_DEVICE if any solve
 * since creation hit the sweep limit. */
int rtm_bet_chain(rtm_ctx *ctx, rtm_bet *bet, int32_t chain, rtm_bet_chain_info *info, double *z_host,
                  double *x_host, double *v_host);

/* Pooled velocity statistics so far: mean_dev, std_dev (sample std) [nz][nx]
 * double and count_dev [nz][nx] int32, each nullable (stream-ordered). */
int rtm_bet_stats(rtm_ctx *ctx, rtm_bet *bet, double *mean_dev, double *std_dev, int32_t *count_dev);

/* The velocity grid vel_dev [nz][nx] (m/s, float) of chain `chain`'s current
 * model sampled at nodes (i h, j h): each node takes the velocity of its
 * nearest nucleus (ties: lowest index), the model definition of Sec. 2.1, at
 * any spacing -- how a sample of Stage 1 becomes a velocity model for the
 * migrations of Stage 2 (e.g. nz, nx, h of the RTM grid covering the same
 * extent).  Stream-ordered.  Errors: RTM_E_INVAL (chain out of range, sizes
 * not positive or above 2^31 nodes, h not positive). */
int rtm_bet_model(rtm_ctx *ctx, rtm_bet *bet, int32_t chain, int32_t nz, int32_t nx, double h, float *vel_dev);

int rtm_bet_destroy(rtm_ctx *ctx, rtm_bet *bet);

/* Self-check of the travel-time arithmetic: counts into *mismatches the
 * float bit patterns in [lo_bits, hi_bits) whose square root, as the
 * travel-time solves evaluate it (a hardware estimate corrected by
 * Tuckerman's rounding test), differs from the correctly rounded square
 * root.  Over [2^-60, 2^126] (bit patterns 0x21800000 to 0x7E800000), which
 * holds every argument the solves use within the accepted h / v range, the
 * count is 0.  Synchronous.  Errors: RTM_E_INVAL (lo_bits >= hi_bits). */
int rtm_sqrt_check(rtm_ctx *ctx, uint32_t lo_bits, uint32_t hi_bits, uint64_t *mismatches);

/* ---- observability --------------------------------------------------- */

typedef struct {
    uint64_t jobs_submitted, jobs_done, jobs_failed, jobs_cancelled;
    uint64_t steps_launched;     /* time-step kernel launches */
    uint64_t graph_replays;      /* hipGraph launches */
    uint64_t grid_updates;       /* point updates performed by finished jobs */
    uint64_t alg_bytes;          /* algorithmic HBM bytes of finished jobs */
    uint64_t arena_bytes, arena_used, arena_peak;
    int32_t tile_z;              /* tile height in use */
    int32_t active_jobs, queued_jobs;
    /* last rtm_migrate_batch call: time steps per launch of its step kernels
     * (2 when its reconstruct-mode shots advanced two steps per launch) */
    int32_t last_steps_per_launch;
    /* last rtm_migrate_batch call: HIP-event time of its forward and backward
     * phases (all launches of each, on the library's work stream), their time
     * steps, and the algorithmic HBM bytes of one time step of each phase
     * (the per-update figures summed over the shots; a two-step launch moves
     * less than twice this) */
    float last_fwd_ms, last_bwd_ms;
    int32_t last_fwd_launches, last_bwd_launches;  /* time steps, whatever the launches */
    uint64_t last_fwd_launch_bytes, last_bwd_launch_bytes;
    /* last codec call: HIP-event time of its kernel, 1 encode / 2 decode, and
     * its algorithmic HBM bytes (4 per value plus the stream length) */
    float last_codec_ms;
    int32_t last_codec_op;
    uint64_t last_codec_bytes;
    /* last rtm_bet_run call: HIP-event times, on the first chain group's
     * stream, of that group's travel-time launch and of all its launches in
     * the call's last iteration (the other group's work overlaps them) */
    float last_bet_eikonal_ms, last_bet_iteration_ms;
    /* last rtm_migrate_batch call: two-step tile height (rows) of its
     * forward and backward phases, 0 for a phase that ran one step per
     * launch */
    int32_t last_tile_z2_fwd, last_tile_z2_bwd;
    /* last rtm_migrate_batch call: shot groups of its forward and backward
     * phases (consecutive shots whose levels fit the memory-side cache run
     * through a phase together, one group after another; each launch covers
     * one group, so a phase made nsteps x groups launches) */
    int32_t last_groups_fwd, last_groups_bwd;
    /* last rtm_born_batch call: shot groups (consecutive shots whose fields
     * fit the memory-side cache advance through all their steps together,
     * one group after another) */
    int32_t last_born_groups;
} rtm_ctx_stats_t;

int rtm_ctx_stats(rtm_ctx *ctx, rtm_ctx_stats_t *out);

#ifdef __cplusplus
}
#endif

#endif /* RTM_H */
