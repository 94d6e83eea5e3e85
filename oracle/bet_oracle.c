/* bet_oracle.c -- plain CPU oracle of Stage 1, Bayesian Eikonal tomography.
 *
 * TEST INFRASTRUCTURE ONLY: called by the tests, the smoke check and the
 * benchmark's CPU-baseline leg; nothing on the library's path links it.
 *
 * What it computes (Sec. 2.1, Eq. 1-3):
 *   - the forward operator F: first-arrival travel times from the Eikonal
 *     equation |grad T| = 1/v, discretised by the first-order Godunov upwind
 *     scheme on a square grid of spacing h and solved by fast marching (nodes
 *     finalised in increasing T from a heap; each trial value uses only
 *     finalised neighbours);
 *   - the model: Voronoi cells with a constant velocity in each; a grid node
 *     takes the velocity of the nearest nucleus (ties: lowest index);
 *   - the likelihood of Eq. 3 as exp(-Phi/2), Phi = sum ((F(m) - d)/sigma)^2;
 *   - reversible-jump Markov chains whose proposals add, delete or move one
 *     nucleus (with probabilities p_birth, p_death, 1 - both), a new nucleus
 *     drawing its position and velocity from the uniform prior, so that every
 *     acceptance ratio is the likelihood ratio;
 *   - pooled FP64 Welford mean and M2 of the sampled velocity grids after
 *     burn-in (the velocity uncertainty maps of Stage 3).
 * Random numbers: the counter form of splitmix64 (Steele, Lea and Flood,
 * 2014): output n of a stream seeded with s is mix(s + (n + 1) gamma).
 *
 * Travel times come from fast marching in double precision, or, for accept
 * decisions taken in the precision of the device solver, from fast sweeping
 * in single precision (in single precision the two algorithms reach fixed
 * points that can differ in the last bits; sweeps in the same directions
 * reach the same one).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define GAMMA 0x9E3779B97F4A7C15ull

/* ---- random numbers -------------------------------------------------- */
uint64_t orc_sm64_mix(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

/* output n of the splitmix64 stream seeded with s */
uint64_t orc_sm64_at(uint64_t s, uint64_t n) { return orc_sm64_mix(s + (n + 1) * GAMMA); }

/* draw k of iteration t (t = -1: the initial model) of chain c */
uint64_t orc_bet_draw(uint64_t seed, int c, int t, int k) {
    const uint64_t sc = orc_sm64_at(seed, (uint64_t)c);
    return orc_sm64_at(sc, (uint64_t)(t + 1) * 256u + (uint64_t)k);
}

static double unit_open0(uint64_t x) { return (double)(x >> 11) * 0x1.0p-53; }         /* [0, 1) */
static double unit_open1(uint64_t x) { return (double)((x >> 11) + 1) * 0x1.0p-53; }   /* (0, 1] */

/* ---- Voronoi model ------------------------------------------------- */
/* cell[i * nx + j] = index of the nucleus nearest to node (i h, j h) */
void orc_voronoi(int nz, int nx, double h, int k, const double* zs, const double* xs, int32_t* cell) {
    for (int i = 0; i < nz; ++i)
        for (int j = 0; j < nx; ++j) {
            const double z = (double)i * h, x = (double)j * h;
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
            cell[i * nx + j] = best;
        }
}

/* ---- Eikonal: fast marching ----------------------------------------- */
typedef struct {
    int* idx;
    double* key;
    int n, cap;
} Heap;

static void heap_push(Heap* hp, int idx, double key) {
    if (hp->n == hp->cap) {
        hp->cap = hp->cap ? 2 * hp->cap : 1024;
        hp->idx = (int*)realloc(hp->idx, sizeof(int) * hp->cap);
        hp->key = (double*)realloc(hp->key, sizeof(double) * hp->cap);
    }
    int c = hp->n++;
    while (c > 0) {
        int p = (c - 1) / 2;
        if (hp->key[p] <= key) break;
        hp->idx[c] = hp->idx[p];
        hp->key[c] = hp->key[p];
        c = p;
    }
    hp->idx[c] = idx;
    hp->key[c] = key;
}

static int heap_pop(Heap* hp, int* idx) {
    if (hp->n == 0) return 0;
    *idx = hp->idx[0];
    const int li = hp->idx[--hp->n];
    const double lk = hp->key[hp->n];
    int c = 0;
    for (;;) {
        int l = 2 * c + 1;
        if (l >= hp->n) break;
        if (l + 1 < hp->n && hp->key[l + 1] < hp->key[l]) ++l;
        if (hp->key[l] >= lk) break;
        hp->idx[c] = hp->idx[l];
        hp->key[c] = hp->key[l];
        c = l;
    }
    if (hp->n > 0) {
        hp->idx[c] = li;
        hp->key[c] = lk;
    }
    return 1;
}

/* Godunov upwind value from the smaller z-neighbour a, the smaller
 * x-neighbour b and sh = slowness * h:
 *   one-sided  a + sh                                   if |b - a| >= sh
 *   two-sided  ((a + b) + sqrt((q + q) - d d)) / 2      q = sh sh, d = b - a */
static double godunov_d(double a, double b, double sh) {
    if (a > b) {
        const double t = a;
        a = b;
        b = t;
    }
    const double d = b - a;
    if (!(d < sh)) return a + sh;
    const double q = sh * sh;
    return ((a + b) + sqrt((q + q) - d * d)) * 0.5;
}

static float godunov_f(float a, float b, float sh) {
    if (a > b) {
        const float t = a;
        a = b;
        b = t;
    }
    const float d = b - a;
    if (!(d < sh)) return a + sh;
    const float q = sh * sh;
    return ((a + b) + sqrtf((q + q) - d * d)) * 0.5f;
}

/* T[nz*nx] from a source node; s = slowness per node.  Returns the number of
 * finalised nodes. */
#define FMM_BODY(TYPE, GOD, INF_)                                                   \
    const int n = nz * nx;                                                          \
    char* known = (char*)calloc((size_t)n, 1);                                      \
    for (int q = 0; q < n; ++q) T[q] = INF_;                                        \
    Heap hp = {0};                                                                  \
    const int src = sz * nx + sx;                                                   \
    T[src] = 0;                                                                     \
    heap_push(&hp, src, 0.0);                                                       \
    int done = 0, cur;                                                              \
    while (heap_pop(&hp, &cur)) {                                                   \
        if (known[cur]) continue;                                                   \
        known[cur] = 1;                                                             \
        ++done;                                                                     \
        const int ci = cur / nx, cj = cur % nx;                                     \
        const int ni[4] = {ci - 1, ci + 1, ci, ci};                                 \
        const int nj[4] = {cj, cj, cj - 1, cj + 1};                                 \
        for (int e = 0; e < 4; ++e) {                                               \
            const int i = ni[e], j = nj[e];                                         \
            if (i < 0 || i >= nz || j < 0 || j >= nx) continue;                     \
            const int m = i * nx + j;                                               \
            if (known[m]) continue;                                                 \
            TYPE a = INF_, b = INF_;                                                \
            if (i > 0 && known[m - nx] && T[m - nx] < a) a = T[m - nx];             \
            if (i + 1 < nz && known[m + nx] && T[m + nx] < a) a = T[m + nx];        \
            if (j > 0 && known[m - 1] && T[m - 1] < b) b = T[m - 1];                \
            if (j + 1 < nx && known[m + 1] && T[m + 1] < b) b = T[m + 1];           \
            const TYPE t = GOD(a, b, s[m] * hh);                                    \
            if (t < T[m]) {                                                         \
                T[m] = t;                                                           \
                heap_push(&hp, m, (double)t);                                       \
            }                                                                       \
        }                                                                           \
    }                                                                               \
    free(hp.idx);                                                                   \
    free(hp.key);                                                                   \
    free(known);                                                                    \
    return done;

int orc_eikonal_f64(int nz, int nx, double hh, const double* s, int sz, int sx, double* T) {
    FMM_BODY(double, godunov_d, INFINITY)
}

int orc_eikonal_f32(int nz, int nx, float hh, const float* s, int sz, int sx, float* T) {
    FMM_BODY(float, godunov_f, INFINITY)
}

/* ---- Eikonal: fast sweeping (single precision) ----------------------
 * Gauss-Seidel sweeps of the same Godunov update in four orderings per pass
 * (i up / j up, i down / j up, i down / j down, i up / j down), every node
 * taking the current times of its four neighbours, repeated until a pass
 * changes nothing (Zhao 2005).  Within one ordering a node sees its two
 * upwind neighbours already swept and its two downwind neighbours from
 * before, whatever the order of independent nodes, so any sweep order that
 * respects the direction gives the same times.  Returns the passes used
 * (256: gave up). */
int orc_eikonal_fsm_f32(int nz, int nx, float hh, const float* s, int sz, int sx, float* T) {
    const int n = nz * nx;
    for (int q = 0; q < n; ++q) T[q] = INFINITY;
    T[sz * nx + sx] = 0.0f;
    int pass = 0;
    for (; pass < 256; ++pass) {
        int changed = 0;
        for (int o = 0; o < 4; ++o) {
            const int fi = (o == 0 || o == 3), fj = (o < 2);
            for (int ii = 0; ii < nz; ++ii) {
                const int i = fi ? ii : nz - 1 - ii;
                for (int jj = 0; jj < nx; ++jj) {
                    const int j = fj ? jj : nx - 1 - jj;
                    const int m = i * nx + j;
                    const float up = i > 0 ? T[m - nx] : INFINITY, dn = i + 1 < nz ? T[m + nx] : INFINITY;
                    const float lf = j > 0 ? T[m - 1] : INFINITY, rt = j + 1 < nx ? T[m + 1] : INFINITY;
                    const float t = godunov_f(up < dn ? up : dn, lf < rt ? lf : rt, s[m] * hh);
                    if (t < T[m]) {
                        T[m] = t;
                        changed = 1;
                    }
                }
            }
        }
        if (!changed) break;
    }
    return pass;
}

/* ---- the chains ----------------------------------------------------- */
typedef struct {
    int32_t nz, nx;
    double h;
    int32_t nsrc, nrec;
    int32_t chains, k_min, k_max, k_init;
    double v_min, v_max;
    double p_birth, p_death;
    double move_dz, move_dx;
    double sigma;
    uint64_t seed;
    int32_t burn_in, thin;
    int32_t single; /* 1: travel times by single-precision fast sweeping (the device's) */
    int32_t chain0; /* chains chain0 .. chain0 + chains - 1 */
} orc_bet_cfg;

typedef struct {
    int32_t k;
    double misfit;
    int64_t proposed[3], accepted[3]; /* birth, death, move */
} orc_chain_info;

/* travel times at the receivers for one model; returns Phi (or writes tt) */
static double model_misfit(const orc_bet_cfg* c, int k, const double* zs, const double* xs, const double* vs,
                           const int32_t* src, const int32_t* rec, const float* tt_obs, float* tt_out,
                           int32_t* cell, double* sd, float* sf, double* Td, float* Tf) {
    const int n = c->nz * c->nx;
    orc_voronoi(c->nz, c->nx, c->h, k, zs, xs, cell);
    for (int q = 0; q < n; ++q) {
        const double sl = 1.0 / vs[cell[q]];
        sd[q] = sl;
        sf[q] = (float)sl;
    }
    double phi = 0.0;
    for (int e = 0; e < c->nsrc; ++e) {
        if (c->single)
            orc_eikonal_fsm_f32(c->nz, c->nx, (float)c->h, sf, src[2 * e], src[2 * e + 1], Tf);
        else
            orc_eikonal_f64(c->nz, c->nx, c->h, sd, src[2 * e], src[2 * e + 1], Td);
        for (int r = 0; r < c->nrec; ++r) {
            const int m = rec[2 * r] * c->nx + rec[2 * r + 1];
            const double t = c->single ? (double)Tf[m] : Td[m];
            if (tt_out) tt_out[(size_t)e * c->nrec + r] = (float)t;
            if (tt_obs) {
                const double rr = (t - (double)tt_obs[(size_t)e * c->nrec + r]) / c->sigma;
                phi += rr * rr;
            }
        }
    }
    return phi;
}

/* Travel times [nsrc][nrec] of the velocity grid vel[nz][nx] (m/s). */
int orc_eikonal_table(const orc_bet_cfg* c, const double* vel, const int32_t* src, const int32_t* rec, double* tt) {
    const int n = c->nz * c->nx;
    double* sd = (double*)malloc(sizeof(double) * n);
    double* Td = (double*)malloc(sizeof(double) * n);
    float* sf = (float*)malloc(sizeof(float) * n);
    float* Tf = (float*)malloc(sizeof(float) * n);
    for (int q = 0; q < n; ++q) {
        sd[q] = 1.0 / vel[q];
        sf[q] = (float)sd[q];
    }
    for (int e = 0; e < c->nsrc; ++e) {
        if (c->single)
            orc_eikonal_fsm_f32(c->nz, c->nx, (float)c->h, sf, src[2 * e], src[2 * e + 1], Tf);
        else
            orc_eikonal_f64(c->nz, c->nx, c->h, sd, src[2 * e], src[2 * e + 1], Td);
        for (int r = 0; r < c->nrec; ++r) {
            const int m = rec[2 * r] * c->nx + rec[2 * r + 1];
            tt[(size_t)e * c->nrec + r] = c->single ? (double)Tf[m] : Td[m];
        }
    }
    free(sd);
    free(Td);
    free(sf);
    free(Tf);
    return 0;
}

/* Initial model of chain ch: k_init nuclei, position and velocity from the prior. */
static void init_model(const orc_bet_cfg* c, int ch, double* zs, double* xs, double* vs) {
    const double Z = (double)(c->nz - 1) * c->h, X = (double)(c->nx - 1) * c->h;
    for (int q = 0; q < c->k_init; ++q) {
        zs[q] = unit_open0(orc_bet_draw(c->seed, ch, -1, 3 * q)) * Z;
        xs[q] = unit_open0(orc_bet_draw(c->seed, ch, -1, 3 * q + 1)) * X;
        vs[q] = c->v_min + unit_open0(orc_bet_draw(c->seed, ch, -1, 3 * q + 2)) * (c->v_max - c->v_min);
    }
}

/* Runs `iters` iterations of every chain from its initial model.
 * state_z/x/v [chains][k_max], info [chains]; mean/m2 [nz*nx] (double) and
 * count (int) accumulate the pooled post-burn-in samples; accept_log
 * [iters][chains] (nullable) records 0 = rejected, 1 + move type = accepted,
 * -1 = invalid proposal. */
int orc_bet_run(const orc_bet_cfg* c, const int32_t* src, const int32_t* rec, const float* tt_obs, int iters,
                double* state_z, double* state_x, double* state_v, orc_chain_info* info, double* mean,
                double* m2, int64_t* count, int8_t* accept_log) {
    const int n = c->nz * c->nx, K = c->k_max;
    if (c->k_min < 1 || c->k_init < c->k_min || c->k_init > K || K > 64) return -1;
    int32_t* cell = (int32_t*)malloc(sizeof(int32_t) * n);
    double* sd = (double*)malloc(sizeof(double) * n);
    double* Td = (double*)malloc(sizeof(double) * n);
    float* sf = (float*)malloc(sizeof(float) * n);
    float* Tf = (float*)malloc(sizeof(float) * n);
    double pz[64], px[64], pv[64];
    const double Z = (double)(c->nz - 1) * c->h, X = (double)(c->nx - 1) * c->h;
    for (int ch = 0; ch < c->chains; ++ch) {
        double* zs = state_z + (size_t)ch * K;
        double* xs = state_x + (size_t)ch * K;
        double* vs = state_v + (size_t)ch * K;
        init_model(c, c->chain0 + ch, zs, xs, vs);
        memset(&info[ch], 0, sizeof info[ch]);
        info[ch].k = c->k_init;
        info[ch].misfit = model_misfit(c, c->k_init, zs, xs, vs, src, rec, tt_obs, NULL, cell, sd, sf, Td, Tf);
    }
    for (int q = 0; q < n; ++q) {
        mean[q] = 0.0;
        m2[q] = 0.0;
    }
    *count = 0;
    for (int t = 0; t < iters; ++t) {
        for (int ch = 0; ch < c->chains; ++ch) {
            double* zs = state_z + (size_t)ch * K;
            double* xs = state_x + (size_t)ch * K;
            double* vs = state_v + (size_t)ch * K;
            const int k = info[ch].k;
            const double u0 = unit_open0(orc_bet_draw(c->seed, c->chain0 + ch, t, 0));
            const double u1 = unit_open0(orc_bet_draw(c->seed, c->chain0 + ch, t, 1));
            const double u2 = unit_open0(orc_bet_draw(c->seed, c->chain0 + ch, t, 2));
            const double u3 = unit_open0(orc_bet_draw(c->seed, c->chain0 + ch, t, 3));
            const double ua = unit_open1(orc_bet_draw(c->seed, c->chain0 + ch, t, 4));
            const int type = u0 < c->p_birth ? 0 : (u0 < c->p_birth + c->p_death ? 1 : 2);
            int kk = k, valid = 1;
            memcpy(pz, zs, sizeof(double) * k);
            memcpy(px, xs, sizeof(double) * k);
            memcpy(pv, vs, sizeof(double) * k);
            if (type == 0) {
                if (k >= K) {
                    valid = 0;
                } else {
                    pz[k] = u1 * Z;
                    px[k] = u2 * X;
                    pv[k] = c->v_min + u3 * (c->v_max - c->v_min);
                    kk = k + 1;
                }
            } else if (type == 1) {
                if (k <= c->k_min) {
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
                const double nzp = pz[i] + (2.0 * u2 - 1.0) * c->move_dz;
                const double nxp = px[i] + (2.0 * u3 - 1.0) * c->move_dx;
                if (nzp < 0.0 || nzp > Z || nxp < 0.0 || nxp > X) {
                    valid = 0;
                } else {
                    pz[i] = nzp;
                    px[i] = nxp;
                }
            }
            int8_t logv = -1;
            if (valid) {
                ++info[ch].proposed[type];
                const double phi = model_misfit(c, kk, pz, px, pv, src, rec, tt_obs, NULL, cell, sd, sf, Td, Tf);
                logv = 0;
                if (phi - info[ch].misfit < -2.0 * log(ua)) {
                    memcpy(zs, pz, sizeof(double) * kk);
                    memcpy(xs, px, sizeof(double) * kk);
                    memcpy(vs, pv, sizeof(double) * kk);
                    info[ch].k = kk;
                    info[ch].misfit = phi;
                    ++info[ch].accepted[type];
                    logv = (int8_t)(1 + type);
                }
            }
            if (accept_log) accept_log[(size_t)t * c->chains + ch] = logv;
        }
        if (t >= c->burn_in && (t - c->burn_in) % c->thin == 0) {
            for (int ch = 0; ch < c->chains; ++ch) {
                const double* zs = state_z + (size_t)ch * K;
                const double* xs = state_x + (size_t)ch * K;
                const double* vs = state_v + (size_t)ch * K;
                orc_voronoi(c->nz, c->nx, c->h, info[ch].k, zs, xs, cell);
                ++*count;
                for (int q = 0; q < n; ++q) {
                    const double x = vs[cell[q]];
                    const double d = x - mean[q];
                    mean[q] += d / (double)*count;
                    m2[q] += d * (x - mean[q]);
                }
            }
        }
    }
    free(cell);
    free(sd);
    free(Td);
    free(sf);
    free(Tf);
    return 0;
}
