/*
 * rtm_oracle.c -- plain FP64 CPU reference of the RTM hot path.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing on the product path links, loads or
 * calls this file; only the test-suite, the smoke check and the CPU-baseline
 * leg of the benchmark do.  It shares no source, header or table with the
 * HIP library.
 *
 * What it computes (arXiv:2001.06444, Sec. 2.2 "Reverse Time Migration"):
 *   - the acoustic isotropic wave equation (Eq. 4), discretised 2nd order in
 *     time and 8th order in space (Sec. 3, paragraph on Stage 2), with a
 *     point-source wavelet as the source term;
 *   - the receiver wavefield driven by the recorded seismogram (Sec. 2.2,
 *     text after Eq. 5), taken here as the exact discrete adjoint of the
 *     forward recursion (the paper's "reverse problem" with a coercive adjoint,
 *     Sec. 3, citing Givoli 2014);
 *   - the zero-lag cross-correlation imaging condition (numerator of Eq. 5),
 *     with the optional source illumination (denominator of Eq. 5).
 *
 * Readings of points the paper leaves open (each is a project definition):
 *   - absorbing boundary: Cerjan sponge of nb cells on all four sides of the
 *     physical grid, g(d) = exp(-(a d)^2), a = 0.3/nb by default, G = g(dz)g(dx),
 *     applied in the fused form  u+ = G(2u + c(Lu + f)) - G^2 u-;
 *   - four rigid (zero) ghost cells beyond the padded grid;
 *   - point source injected as c * w^n / (dx dz) at an on-grid node, i.e. the
 *     right-hand side w(t) delta(x - xs) of (1/v^2) p_tt - lap p;
 *   - traces d[n][r] = u^n(r), n = 0..nt-1, d[0] = 0;
 *   - receiver wavefield: R^{nt} = R^{nt+1} = 0 and
 *       R^m = G(2R^{m+1} + c(L R^{m+1} + sum_r d[m][r] e_r)) - G^2 R^{m+2};
 *   - image I = k * sum_{n in N} S^n (.) R^{n+1},  N = {0, k, 2k, ..} and n <= nt-2,
 *     over the physical region only (the S^n R^{n+1} pairing is the one that
 *     makes migration the exact adjoint of Born modelling);
 *   - 16-bit snapshot emulation: per-snapshot power-of-two scale s = 2^(15-e)
 *     where max|S^n| = f 2^e, f in [1/2, 1); stored value RNE(S s) in the
 *     16-bit format, decoded as q / s.
 *
 * Everything is double precision.  The loops are deliberately plain: bounds
 * checks on every stencil access, no blocking, no fusion beyond what the
 * recursion states.  OpenMP splits rows only.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* Central 8th-order second-derivative weights a_0..a_4 (standard finite
 * difference weights for the 2nd derivative; a_0 + 2 sum a_k = 0). */
static const double ORC_A[5] = {-205.0 / 72.0, 8.0 / 5.0, -1.0 / 5.0, 8.0 / 315.0,
                                -1.0 / 560.0};

typedef struct {
    int32_t nz, nx;    /* physical grid */
    int32_t nb;        /* sponge width in cells (0 allowed) */
    int32_t nt;        /* number of time samples */
    double dz, dx, dt; /* spacings (m, m, s) */
    double sponge_a;   /* Cerjan constant a; <= 0 selects 0.3/nb */
    int32_t periodic;  /* 1: periodic wrap, no sponge (test mode; nb must be 0) */
    int32_t pad_;
} orc_grid;

enum { ORC_OK = 0, ORC_EINVAL = -1, ORC_ENOMEM = -2 };

/* ---------------------------------------------------------------------- */
/* Model on the padded grid                                                */
/* ---------------------------------------------------------------------- */
typedef struct {
    int nz, nx, nb, nzp, nxp, periodic;
    double dz, dx, dt;
    double *c; /* v^2 dt^2, padded, velocity edge-replicated into the sponge */
    double *G; /* sponge factor g(dz) g(dx), 1 inside the physical region */
} orc_model;

static size_t npad(const orc_model *m) { return (size_t)m->nzp * (size_t)m->nxp; }

static int clampi(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }

static double sponge_g(int d, double a) { return exp(-(a * d) * (a * d)); }

static int model_init(orc_model *m, const orc_grid *g, const double *vel) {
    if (g->nz <= 0 || g->nx <= 0 || g->nb < 0 || g->nt < 1) return ORC_EINVAL;
    if (g->periodic && g->nb != 0) return ORC_EINVAL;
    m->nz = g->nz;
    m->nx = g->nx;
    m->nb = g->nb;
    m->nzp = g->nz + 2 * g->nb;
    m->nxp = g->nx + 2 * g->nb;
    m->periodic = g->periodic;
    m->dz = g->dz;
    m->dx = g->dx;
    m->dt = g->dt;
    m->c = (double *)malloc(npad(m) * sizeof(double));
    m->G = (double *)malloc(npad(m) * sizeof(double));
    if (!m->c || !m->G) {
        free(m->c);
        free(m->G);
        return ORC_ENOMEM;
    }
    double a = g->sponge_a > 0 ? g->sponge_a : (g->nb > 0 ? 0.3 / g->nb : 0.0);
    for (int iz = 0; iz < m->nzp; iz++) {
        /* cells outside the physical region along z (0 inside) */
        int dzc = iz < m->nb ? m->nb - iz : (iz >= m->nb + m->nz ? iz - (m->nb + m->nz - 1) : 0);
        for (int ix = 0; ix < m->nxp; ix++) {
            int dxc = ix < m->nb ? m->nb - ix : (ix >= m->nb + m->nx ? ix - (m->nb + m->nx - 1) : 0);
            int vz = clampi(iz - m->nb, 0, m->nz - 1);
            int vx = clampi(ix - m->nb, 0, m->nx - 1);
            double v = vel[(size_t)vz * m->nx + vx];
            size_t i = (size_t)iz * m->nxp + ix;
            m->c[i] = v * v * m->dt * m->dt;
            m->G[i] = sponge_g(dzc, a) * sponge_g(dxc, a);
        }
    }
    return ORC_OK;
}

static void model_free(orc_model *m) {
    free(m->c);
    free(m->G);
    m->c = m->G = NULL;
}

/* Field value with rigid zero ghosts (or periodic wrap in test mode). */
static double fval(const orc_model *m, const double *u, int iz, int ix) {
    if (m->periodic) {
        iz = ((iz % m->nzp) + m->nzp) % m->nzp;
        ix = ((ix % m->nxp) + m->nxp) % m->nxp;
    } else if (iz < 0 || iz >= m->nzp || ix < 0 || ix >= m->nxp) {
        return 0.0;
    }
    return u[(size_t)iz * m->nxp + ix];
}

/* 8th-order Laplacian at one node: sum_k a_|k| (u[z+k,x]/dz^2 + u[z,x+k]/dx^2). */
static double lap_at(const orc_model *m, const double *u, int iz, int ix) {
    double idz2 = 1.0 / (m->dz * m->dz), idx2 = 1.0 / (m->dx * m->dx);
    double s = ORC_A[0] * (idz2 + idx2) * fval(m, u, iz, ix);
    for (int k = 1; k <= 4; k++) {
        s += ORC_A[k] * (fval(m, u, iz - k, ix) + fval(m, u, iz + k, ix)) * idz2;
        s += ORC_A[k] * (fval(m, u, iz, ix - k) + fval(m, u, iz, ix + k)) * idx2;
    }
    return s;
}

/* One step of the damped leapfrog recursion
 *     next = G (2 cur + c (L cur + f)) - G^2 prev
 * where f is zero except at npt listed nodes (padded linear index pidx[j],
 * value pval[j]; repeated nodes add).  f is folded in after the sweep as
 * G c f, which is the same expression.  next may alias prev. */
static void leapfrog(const orc_model *m, const double *cur, const double *prev, double *next,
                     int npt, const long *pidx, const double *pval) {
#pragma omp parallel for schedule(static)
    for (int iz = 0; iz < m->nzp; iz++) {
        for (int ix = 0; ix < m->nxp; ix++) {
            size_t i = (size_t)iz * m->nxp + ix;
            double G = m->G[i];
            double L = lap_at(m, cur, iz, ix);
            next[i] = G * (2.0 * cur[i] + m->c[i] * L) - G * G * prev[i];
        }
    }
    for (int j = 0; j < npt; j++) {
        long i = pidx[j];
        next[i] += m->G[i] * m->c[i] * pval[j];
    }
}

static long pidx_of(const orc_model *m, int iz_phys, int ix_phys) {
    return (long)(iz_phys + m->nb) * m->nxp + (ix_phys + m->nb);
}

static int in_phys(const orc_model *m, int iz, int ix) {
    return iz >= 0 && iz < m->nz && ix >= 0 && ix < m->nx;
}

/* copy the physical region of a padded field into a dense nz x nx array */
static void phys_copy(const orc_model *m, const double *u, double *out) {
    for (int iz = 0; iz < m->nz; iz++)
        memcpy(out + (size_t)iz * m->nx, u + (size_t)(iz + m->nb) * m->nxp + m->nb,
               (size_t)m->nx * sizeof(double));
}

/* ---------------------------------------------------------------------- */
/* 16-bit snapshot emulation                                               */
/* ---------------------------------------------------------------------- */

/* Round x to the nearest value with p significant bits (ties to even), with
 * a fixed quantum 2^qmin below the normal range: the value set of IEEE
 * binary16 (p = 11, qmin = -24) or bfloat16 (p = 8, qmin = -133).  No
 * overflow handling: callers stay far inside the range. */
static double round_sig(double x, int p, int qmin) {
    if (x == 0.0 || !isfinite(x)) return x;
    int e;
    frexp(x, &e); /* |x| = f 2^e, f in [1/2, 1) */
    int q = e - p; /* quantum exponent of the p-bit significand */
    if (q < qmin) q = qmin;
    return ldexp(nearbyint(ldexp(x, -q)), q); /* nearbyint: ties to even */
}

double orc_round_fp16(double x) { return round_sig(x, 11, -24); }
double orc_round_bf16(double x) { return round_sig(x, 8, -133); }

/* Scale s = 2^(15-e) from the snapshot max-abs, max = f 2^e, f in [1/2,1). */
double orc_snapshot_scale(double maxabs) {
    if (!(maxabs > 0.0)) return 1.0;
    int e;
    frexp(maxabs, &e);
    return ldexp(1.0, 15 - e);
}

/* Replace a physical snapshot by dequant(quant(.)) with the per-snapshot
 * power-of-two scale.  kind: 1 = bf16, 2 = fp16. */
static void emulate_16bit(double *s, size_t n, int kind) {
    double mx = 0.0;
    for (size_t i = 0; i < n; i++) mx = fmax(mx, fabs(s[i]));
    double sc = orc_snapshot_scale(mx);
    for (size_t i = 0; i < n; i++) {
        double q = kind == 1 ? orc_round_bf16(s[i] * sc) : orc_round_fp16(s[i] * sc);
        s[i] = q / sc;
    }
}

/* ---------------------------------------------------------------------- */
/* Public entry points                                                     */
/* ---------------------------------------------------------------------- */

/* 8th-order Laplacian of a dense nz x nx field (zero ghosts, or periodic). */
int orc_laplacian(const orc_grid *g, const double *u, double *out) {
    orc_grid gg = *g;
    gg.nb = 0;
    if (gg.nt < 1) gg.nt = 1;
    orc_model m;
    double *ones = (double *)malloc((size_t)g->nz * g->nx * sizeof(double));
    if (!ones) return ORC_ENOMEM;
    for (size_t i = 0; i < (size_t)g->nz * g->nx; i++) ones[i] = 1.0;
    int rc = model_init(&m, &gg, ones);
    free(ones);
    if (rc) return rc;
    for (int iz = 0; iz < m.nzp; iz++)
        for (int ix = 0; ix < m.nxp; ix++) out[(size_t)iz * m.nxp + ix] = lap_at(&m, u, iz, ix);
    model_free(&m);
    return ORC_OK;
}

/*
 * Forward modelling of the source wavefield (Eq. 4 with the wavelet as the
 * source term):  u^{-1} = u^0 = 0 (or the given initial state), then for
 * n = 0..nt-2,  u^{n+1} = G(2u^n + c(Lu^n + w^n e_s/(dx dz))) - G^2 u^{n-1}.
 *
 *   vel       [nz][nx]     physical velocity (m/s)
 *   wavelet   [nt]         w^n (may be NULL: no source)
 *   src       physical node (iz, ix); ignored when wavelet is NULL
 *   rec_iz/ix [nrec]       physical receiver nodes
 *   traces    [nt][nrec]   out, d[n][r] = u^n(r)         (nullable)
 *   snaps     [nt][nz][nx] out, physical u^n             (nullable)
 *   final2    [2][nz][nx]  out, (u^{nt-1}, u^{nt-2})     (nullable)
 *   init2     [2][nz][nx]  in, (u^{-1}, u^0) on the physical grid (nullable;
 *                          only meaningful with nb = 0)
 */
int orc_forward(const orc_grid *g, const double *vel, const double *wavelet, int src_iz,
                int src_ix, int nrec, const int *rec_iz, const int *rec_ix, double *traces,
                double *snaps, double *final2, const double *init2) {
    orc_model m;
    int rc = model_init(&m, g, vel);
    if (rc) return rc;
    if (wavelet && !in_phys(&m, src_iz, src_ix)) {
        model_free(&m);
        return ORC_EINVAL;
    }
    for (int r = 0; r < nrec; r++)
        if (!in_phys(&m, rec_iz[r], rec_ix[r])) {
            model_free(&m);
            return ORC_EINVAL;
        }
    size_t N = npad(&m), P = (size_t)m.nz * m.nx;
    double *a = (double *)calloc(N, sizeof(double)); /* u^{n-1} */
    double *b = (double *)calloc(N, sizeof(double)); /* u^n */
    if (!a || !b) {
        free(a);
        free(b);
        model_free(&m);
        return ORC_ENOMEM;
    }
    if (init2) {
        for (int iz = 0; iz < m.nz; iz++)
            for (int ix = 0; ix < m.nx; ix++) {
                a[pidx_of(&m, iz, ix)] = init2[(size_t)iz * m.nx + ix];
                b[pidx_of(&m, iz, ix)] = init2[P + (size_t)iz * m.nx + ix];
            }
    }
    long sidx = wavelet ? pidx_of(&m, src_iz, src_ix) : 0;
    double inv_cell = 1.0 / (m.dx * m.dz);
    /* n = 0 samples */
    for (int r = 0; r < nrec && traces; r++) traces[r] = b[pidx_of(&m, rec_iz[r], rec_ix[r])];
    if (snaps) phys_copy(&m, b, snaps);
    for (int n = 0; n + 1 < g->nt; n++) {
        double f = wavelet ? wavelet[n] * inv_cell : 0.0;
        leapfrog(&m, b, a, a, wavelet ? 1 : 0, &sidx, &f); /* a <- u^{n+1} */
        double *t = a;
        a = b;
        b = t; /* now a = u^n, b = u^{n+1} */
        if (traces)
            for (int r = 0; r < nrec; r++)
                traces[(size_t)(n + 1) * nrec + r] = b[pidx_of(&m, rec_iz[r], rec_ix[r])];
        if (snaps) phys_copy(&m, b, snaps + (size_t)(n + 1) * P);
    }
    if (final2) {
        phys_copy(&m, b, final2);     /* u^{nt-1} */
        phys_copy(&m, a, final2 + P); /* u^{nt-2} (u^{-1} when nt = 1) */
    }
    free(a);
    free(b);
    model_free(&m);
    return ORC_OK;
}

/*
 * Born (single-scattering) modelling, used for the adjoint (dot-product)
 * test only:  background u0 as in orc_forward, and
 *     du^{n+1} = G(2du^n + c(L du^n + mpert (.) u0^n)) - G^2 du^{n-1},
 * with dd[n][r] = du^n(r).  mpert [nz][nx] lives on the physical region.
 */
int orc_born(const orc_grid *g, const double *vel, const double *wavelet, int src_iz, int src_ix,
             const double *mpert, int nrec, const int *rec_iz, const int *rec_ix, double *dd) {
    orc_model m;
    int rc = model_init(&m, g, vel);
    if (rc) return rc;
    if (!in_phys(&m, src_iz, src_ix)) {
        model_free(&m);
        return ORC_EINVAL;
    }
    size_t N = npad(&m), P = (size_t)m.nz * m.nx;
    double *a = (double *)calloc(N, sizeof(double));
    double *b = (double *)calloc(N, sizeof(double));
    double *da = (double *)calloc(N, sizeof(double));
    double *db = (double *)calloc(N, sizeof(double));
    long *bidx = (long *)malloc(P * sizeof(long));
    double *bval = (double *)malloc(P * sizeof(double));
    if (!a || !b || !da || !db || !bidx || !bval) {
        free(a); free(b); free(da); free(db); free(bidx); free(bval);
        model_free(&m);
        return ORC_ENOMEM;
    }
    for (int iz = 0; iz < m.nz; iz++)
        for (int ix = 0; ix < m.nx; ix++) bidx[(size_t)iz * m.nx + ix] = pidx_of(&m, iz, ix);
    long sidx = pidx_of(&m, src_iz, src_ix);
    double inv_cell = 1.0 / (m.dx * m.dz);
    for (int r = 0; r < nrec; r++) dd[r] = 0.0;
    for (int n = 0; n + 1 < g->nt; n++) {
        /* Born source at step n uses the background at time n (b = u0^n) */
        for (size_t p = 0; p < P; p++) bval[p] = mpert[p] * b[bidx[p]];
        leapfrog(&m, db, da, da, (int)P, bidx, bval);
        double f = wavelet[n] * inv_cell;
        leapfrog(&m, b, a, a, 1, &sidx, &f);
        double *t = a; a = b; b = t;
        t = da; da = db; db = t;
        for (int r = 0; r < nrec; r++)
            dd[(size_t)(n + 1) * nrec + r] = db[pidx_of(&m, rec_iz[r], rec_ix[r])];
    }
    free(a); free(b); free(da); free(db); free(bidx); free(bval);
    model_free(&m);
    return ORC_OK;
}

/*
 * Reverse time migration of one shot (Sec. 2.2):
 *   source wavefield S^n = u^n of orc_forward;
 *   receiver wavefield R^m for m = nt-1..0 (see the header comment);
 *   image I = k sum_{n in N} Q(S^n) (.) R^{n+1},  illum = k sum Q(S^n)^2,
 * where Q is the identity (quant = 0) or the 16-bit emulation (1 bf16, 2 fp16).
 *
 * s_mode 0 keeps every physical S^n in memory.  s_mode 1 keeps checkpoints
 * (u^j, u^{j+1}) every ckpt steps and recomputes each segment forward before
 * it is consumed, which yields the same S^n bit for bit.
 *
 *   data  [nt][nrec]   receiver data (injected as c d, no 1/(dx dz))
 *   image [nz][nx]     out
 *   illum [nz][nx]     out (nullable)
 */
int orc_rtm(const orc_grid *g, const double *vel, const double *wavelet, int src_iz, int src_ix,
            int nrec, const int *rec_iz, const int *rec_ix, const double *data, int stride,
            int quant, int s_mode, int ckpt, double *image, double *illum) {
    if (stride < 1 || quant < 0 || quant > 2 || (s_mode == 1 && ckpt < 1)) return ORC_EINVAL;
    orc_model m;
    int rc = model_init(&m, g, vel);
    if (rc) return rc;
    if (!in_phys(&m, src_iz, src_ix)) {
        model_free(&m);
        return ORC_EINVAL;
    }
    for (int r = 0; r < nrec; r++)
        if (!in_phys(&m, rec_iz[r], rec_ix[r])) {
            model_free(&m);
            return ORC_EINVAL;
        }
    const int nt = g->nt;
    size_t N = npad(&m), P = (size_t)m.nz * m.nx;
    long sidx = pidx_of(&m, src_iz, src_ix);
    double inv_cell = 1.0 / (m.dx * m.dz);

    /* storage for S: either all steps, or checkpoints + one segment */
    int seg = s_mode == 1 ? ckpt : nt;
    int nck = s_mode == 1 ? (nt + ckpt - 1) / ckpt : 0;
    double *store = (double *)malloc((size_t)(s_mode == 1 ? seg + 1 : nt) * P * sizeof(double));
    double *ck = s_mode == 1 ? (double *)malloc((size_t)nck * 2 * N * sizeof(double)) : NULL;
    double *a = (double *)calloc(N, sizeof(double));
    double *b = (double *)calloc(N, sizeof(double));
    long *ridx = (long *)malloc((size_t)(nrec > 0 ? nrec : 1) * sizeof(long));
    double *rval = (double *)malloc((size_t)(nrec > 0 ? nrec : 1) * sizeof(double));
    double *Sn = (double *)malloc(P * sizeof(double));
    if (!store || (s_mode == 1 && !ck) || !a || !b || !ridx || !rval || !Sn) {
        free(store); free(ck); free(a); free(b); free(ridx); free(rval); free(Sn);
        model_free(&m);
        return ORC_ENOMEM;
    }
    for (int r = 0; r < nrec; r++) ridx[r] = pidx_of(&m, rec_iz[r], rec_ix[r]);

    /* ---- forward pass ---- */
    /* a = u^{n-1}, b = u^n */
    for (int n = 0; n < nt; n++) {
        if (s_mode == 0) {
            phys_copy(&m, b, store + (size_t)n * P);
        } else if (n % ckpt == 0) {
            memcpy(ck + (size_t)(n / ckpt) * 2 * N, a, N * sizeof(double));
            memcpy(ck + (size_t)(n / ckpt) * 2 * N + N, b, N * sizeof(double));
        }
        if (n + 1 < nt) {
            double f = wavelet[n] * inv_cell;
            leapfrog(&m, b, a, a, 1, &sidx, &f);
            double *t = a; a = b; b = t;
        }
    }

    /* ---- backward pass with imaging ---- */
    memset(image, 0, P * sizeof(double));
    if (illum) memset(illum, 0, P * sizeof(double));
    double *Rp = a, *Rc = b; /* reuse: R^{m+2}, R^{m+1} */
    memset(Rp, 0, N * sizeof(double));
    memset(Rc, 0, N * sizeof(double));
    int seg_lo = -1; /* first step held in store when s_mode == 1 */
    for (int mstep = nt - 1; mstep >= 0; mstep--) {
        /* imaging term S^m (.) R^{m+1}, m in N, m <= nt-2 (Rc holds R^{m+1}) */
        if (mstep <= nt - 2 && mstep % stride == 0) {
            const double *S;
            if (s_mode == 0) {
                S = store + (size_t)mstep * P;
            } else {
                if (seg_lo < 0 || mstep < seg_lo) {
                    /* recompute segment [j, min(j+ckpt, nt-1)] from its checkpoint */
                    int j = (mstep / ckpt) * ckpt;
                    double *ua = (double *)malloc(N * sizeof(double));
                    double *ub = (double *)malloc(N * sizeof(double));
                    if (!ua || !ub) {
                        free(ua); free(ub);
                        rc = ORC_ENOMEM;
                        goto done;
                    }
                    memcpy(ua, ck + (size_t)(j / ckpt) * 2 * N, N * sizeof(double));
                    memcpy(ub, ck + (size_t)(j / ckpt) * 2 * N + N, N * sizeof(double));
                    int hi = j + ckpt < nt ? j + ckpt : nt - 1;
                    for (int n = j; n <= hi; n++) {
                        phys_copy(&m, ub, store + (size_t)(n - j) * P);
                        if (n + 1 <= hi) {
                            double f = wavelet[n] * inv_cell;
                            leapfrog(&m, ub, ua, ua, 1, &sidx, &f);
                            double *t = ua; ua = ub; ub = t;
                        }
                    }
                    free(ua);
                    free(ub);
                    seg_lo = j;
                }
                S = store + (size_t)(mstep - seg_lo) * P;
            }
            memcpy(Sn, S, P * sizeof(double));
            if (quant) emulate_16bit(Sn, P, quant);
            for (int iz = 0; iz < m.nz; iz++)
                for (int ix = 0; ix < m.nx; ix++) {
                    size_t p = (size_t)iz * m.nx + ix;
                    double r1 = Rc[pidx_of(&m, iz, ix)];
                    image[p] += stride * Sn[p] * r1;
                    if (illum) illum[p] += stride * Sn[p] * Sn[p];
                }
        }
        /* R^m = G(2R^{m+1} + c(L R^{m+1} + sum_r d[m][r] e_r)) - G^2 R^{m+2} */
        for (int r = 0; r < nrec; r++) rval[r] = data[(size_t)mstep * nrec + r];
        leapfrog(&m, Rc, Rp, Rp, nrec, ridx, rval);
        double *t = Rp; Rp = Rc; Rc = t;
    }
done:
    free(store); free(ck); free(a); free(b); free(ridx); free(rval); free(Sn);
    model_free(&m);
    return rc;
}

/*
 * Source-wavefield reconstruction by time reversal (used only to pin that
 * reconstruction reproduces the stored wavefield).  The forward pass saves
 * the 4-cell ring inside the physical perimeter at every step and the last
 * two states; the backward pass runs, on physical nodes at distance >= 4
 * from the physical edge,
 *     S^n = 2 S^{n+1} - S^{n+2} + c (L S^{n+1} + w^{n+1} e_s/(dx dz)),
 * and restores the ring from storage.  Output: srec [nt][nz][nx].
 */
int orc_reconstruct(const orc_grid *g, const double *vel, const double *wavelet, int src_iz,
                    int src_ix, double *srec) {
    orc_model m;
    int rc = model_init(&m, g, vel);
    if (rc) return rc;
    if (!in_phys(&m, src_iz, src_ix) || m.nz < 9 || m.nx < 9 || g->nt < 2) {
        model_free(&m);
        return ORC_EINVAL;
    }
    const int nt = g->nt;
    size_t N = npad(&m), P = (size_t)m.nz * m.nx;
    /* ring membership on the physical grid */
    size_t nring = 0;
    for (int iz = 0; iz < m.nz; iz++)
        for (int ix = 0; ix < m.nx; ix++)
            if (iz < 4 || iz >= m.nz - 4 || ix < 4 || ix >= m.nx - 4) nring++;
    long *ridx = (long *)malloc(nring * sizeof(long));
    double *ring = (double *)malloc((size_t)nt * nring * sizeof(double));
    double *a = (double *)calloc(N, sizeof(double));
    double *b = (double *)calloc(N, sizeof(double));
    if (!ridx || !ring || !a || !b) {
        free(ridx); free(ring); free(a); free(b);
        model_free(&m);
        return ORC_ENOMEM;
    }
    size_t q = 0;
    for (int iz = 0; iz < m.nz; iz++)
        for (int ix = 0; ix < m.nx; ix++)
            if (iz < 4 || iz >= m.nz - 4 || ix < 4 || ix >= m.nx - 4) ridx[q++] = pidx_of(&m, iz, ix);
    long sidx = pidx_of(&m, src_iz, src_ix);
    double inv_cell = 1.0 / (m.dx * m.dz);
    for (int n = 0; n < nt; n++) {
        for (size_t j = 0; j < nring; j++) ring[(size_t)n * nring + j] = b[ridx[j]];
        if (n + 1 < nt) {
            double f = wavelet[n] * inv_cell;
            leapfrog(&m, b, a, a, 1, &sidx, &f);
            double *t = a; a = b; b = t;
        }
    }
    /* b = u^{nt-1}, a = u^{nt-2}; keep only the physical region */
    double *s1 = (double *)calloc(N, sizeof(double)); /* S^{n+1} */
    double *s2 = (double *)calloc(N, sizeof(double)); /* S^{n+2} */
    if (!s1 || !s2) {
        free(s1); free(s2); free(ridx); free(ring); free(a); free(b);
        model_free(&m);
        return ORC_ENOMEM;
    }
    for (int iz = 0; iz < m.nz; iz++)
        for (int ix = 0; ix < m.nx; ix++) {
            long i = pidx_of(&m, iz, ix);
            s1[i] = a[i];
            s2[i] = b[i];
        }
    phys_copy(&m, s2, srec + (size_t)(nt - 1) * P);
    if (nt >= 2) phys_copy(&m, s1, srec + (size_t)(nt - 2) * P);
    for (int n = nt - 3; n >= 0; n--) {
        /* s1 = S^{n+1}, s2 = S^{n+2}; write S^n into s2 */
#pragma omp parallel for schedule(static)
        for (int iz = 4; iz < m.nz - 4; iz++)
            for (int ix = 4; ix < m.nx - 4; ix++) {
                long i = pidx_of(&m, iz, ix);
                double L = lap_at(&m, s1, iz + m.nb, ix + m.nb);
                double f = (i == sidx) ? wavelet[n + 1] * inv_cell : 0.0;
                s2[i] = 2.0 * s1[i] - s2[i] + m.c[i] * (L + f);
            }
        for (size_t j = 0; j < nring; j++) s2[ridx[j]] = ring[(size_t)n * nring + j];
        phys_copy(&m, s2, srec + (size_t)n * P);
        double *t = s1; s1 = s2; s2 = t;
    }
    free(s1); free(s2); free(ridx); free(ring); free(a); free(b);
    model_free(&m);
    return ORC_OK;
}
