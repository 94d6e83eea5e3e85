/* Sanitizer driver of the Stage-1 oracle (oracle/bet_oracle.c, compiled
 * into this file): the travel-time solvers on small and degenerate grids
 * (one row, one column, 2 x 2, sources on corners) and short chain runs in
 * both travel-time modes, built by tests/test_host_logic.py with ASan +
 * UBSan.  Checks that the times are finite and non-negative. */
#include "../../oracle/bet_oracle.c"

#include <stdio.h>
#include <stdlib.h>

static void need(int ok, const char *what) {
    if (!ok) {
        fprintf(stderr, "FAIL: %s\n", what);
        exit(1);
    }
}

static void grid_case(int nz, int nx, int sz, int sx) {
    size_t n = (size_t)nz * nx;
    double *s = (double *)malloc(n * sizeof(double)), *T = (double *)malloc(n * sizeof(double));
    float *sf = (float *)malloc(n * sizeof(float)), *Tf = (float *)malloc(n * sizeof(float));
    need(s && T && sf && Tf, "malloc");
    for (size_t i = 0; i < n; ++i) s[i] = 1.0 / (1500.0 + 100.0 * (double)(i % 7)), sf[i] = (float)s[i];
    need(orc_eikonal_f64(nz, nx, 100.0, s, sz, sx, T) == nz * nx, "fast marching f64 accepts every node");
    for (size_t i = 0; i < n; ++i) need(isfinite(T[i]) && T[i] >= 0, "f64 times");
    need(orc_eikonal_f32(nz, nx, 100.0f, sf, sz, sx, Tf) == nz * nx, "fast marching f32 accepts every node");
    const int passes = orc_eikonal_fsm_f32(nz, nx, 100.0f, sf, sz, sx, Tf);
    need(passes > 0 && passes < 256, "fast sweeping f32 converges");
    for (size_t i = 0; i < n; ++i) need(isfinite(Tf[i]) && Tf[i] >= 0, "f32 times");
    free(s); free(T); free(sf); free(Tf);
}

static void chain_case(int single) {
    orc_bet_cfg c;
    memset(&c, 0, sizeof c);
    c.nz = 6; c.nx = 9; c.h = 100.0; c.nsrc = 2; c.nrec = 9; c.chains = 3; c.k_min = 1; c.k_max = 8;
    c.k_init = 3; c.v_min = 1400.0; c.v_max = 5000.0; c.p_birth = 0.3; c.p_death = 0.3; c.move_dz = 100.0;
    c.move_dx = 300.0; c.sigma = 0.01; c.seed = 42; c.burn_in = 5; c.thin = 2; c.single = single; c.chain0 = 1;
    int32_t src[4] = {0, 0, 0, 8}, rec[18];
    for (int r = 0; r < 9; ++r) rec[2 * r] = 0, rec[2 * r + 1] = r;
    float tt[18];
    for (int i = 0; i < 18; ++i) tt[i] = 0.05f * (float)(i % 9);
    double z[24], x[24], v[24], mean[54] = {0}, m2[54] = {0};
    orc_chain_info info[3];
    int64_t count = 0;
    int8_t log[3 * 40];
    need(orc_bet_run(&c, src, rec, tt, 40, z, x, v, info, mean, m2, &count, log) == 0, "chain run");
    for (int k = 0; k < 3; ++k) need(info[k].k >= c.k_min && info[k].k <= c.k_max, "k in bounds");
    need(count > 0, "pooled samples");
}

int main(void) {
    grid_case(1, 40, 0, 0);
    grid_case(40, 1, 39, 0);
    grid_case(2, 2, 1, 1);
    grid_case(12, 17, 0, 16);
    grid_case(30, 30, 15, 15);
    chain_case(1);
    chain_case(0);
    printf("oracle bet: ok\n");
    return 0;
}
