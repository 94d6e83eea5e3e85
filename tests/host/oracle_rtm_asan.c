/* Sanitizer driver of the RTM oracle (oracle/rtm_oracle.c, compiled into
 * this file): every entry point on small grids, including the edge cases
 * the tests use (no sponge, a 9 x 9 window, nt = 2, strides, 16-bit
 * emulation, checkpoint segments shorter and longer than nt, receivers on
 * the grid edges), built by tests/test_host_logic.py with ASan + UBSan.
 * Checks that checkpointed and stored source wavefields give the same image
 * bit for bit and that the results are finite. */
#include "../../oracle/rtm_oracle.c"

#include <stdio.h>
#include <stdlib.h>

static void need(int ok, const char *what) {
    if (!ok) {
        fprintf(stderr, "FAIL: %s\n", what);
        exit(1);
    }
}

static double *vec(size_t n, double v) {
    double *p = (double *)malloc(n * sizeof(double));
    need(p != NULL, "malloc");
    for (size_t i = 0; i < n; ++i) p[i] = v;
    return p;
}

static void finite(const double *a, size_t n, const char *what) {
    for (size_t i = 0; i < n; ++i) need(isfinite(a[i]), what);
}

static void case_rtm(int nz, int nx, int nb, int nt, int stride, int quant, int ckpt) {
    orc_grid g = {nz, nx, nb, nt, 10.0, 12.5, 1e-3, 0.0, 0, 0};
    size_t N = (size_t)nz * nx;
    double *vel = vec(N, 0.0), *w = vec((size_t)nt, 0.0);
    for (size_t i = 0; i < N; ++i) vel[i] = 1500.0 + 7.0 * (double)(i % 13);
    for (int n = 0; n < nt; ++n) w[n] = sin(0.3 * n) * exp(-0.01 * n);
    int nrec = nx;
    int *riz = (int *)malloc(sizeof(int) * nrec), *rix = (int *)malloc(sizeof(int) * nrec);
    for (int r = 0; r < nrec; ++r) riz[r] = r % 2 ? 0 : nz - 1, rix[r] = r;  /* both edge rows */
    double *tr = vec((size_t)nt * nrec, 0.0), *fin = vec(2 * N, 0.0);
    need(orc_forward(&g, vel, w, nz / 2, nx / 2, nrec, riz, rix, tr, NULL, fin, NULL) == 0, "forward");
    finite(tr, (size_t)nt * nrec, "forward traces");
    double *img = vec(N, 0.0), *ill = vec(N, 0.0), *img2 = vec(N, 0.0);
    need(orc_rtm(&g, vel, w, nz / 2, nx / 2, nrec, riz, rix, tr, stride, quant, 0, 1, img, ill) == 0, "rtm store");
    need(orc_rtm(&g, vel, w, nz / 2, nx / 2, nrec, riz, rix, tr, stride, quant, 1, ckpt, img2, NULL) == 0,
         "rtm checkpoint");
    for (size_t i = 0; i < N; ++i) need(img[i] == img2[i], "checkpoint image equals store image");
    finite(img, N, "image");
    finite(ill, N, "illumination");
    double *m = vec(N, 1e-3), *dd = vec((size_t)nt * nrec, 0.0);
    need(orc_born(&g, vel, w, nz / 2, nx / 2, m, nrec, riz, rix, dd) == 0, "born");
    finite(dd, (size_t)nt * nrec, "born traces");
    double *lap = vec(N, 0.0);
    need(orc_laplacian(&g, vel, lap) == 0, "laplacian");
    if (nz >= 9 && nx >= 9) {
        double *srec = vec((size_t)nt * N, 0.0);
        need(orc_reconstruct(&g, vel, w, nz / 2, nx / 2, srec) == 0, "reconstruct");
        finite(srec, (size_t)nt * N, "reconstructed source wavefield");
        free(srec);
    }
    free(vel); free(w); free(riz); free(rix); free(tr); free(fin); free(img); free(ill); free(img2);
    free(m); free(dd); free(lap);
}

int main(void) {
    case_rtm(20, 24, 6, 40, 1, 0, 7);    /* checkpoint segments shorter than nt */
    case_rtm(20, 24, 6, 40, 3, 1, 64);   /* one segment longer than nt; bf16, stride 3 */
    case_rtm(9, 9, 0, 2, 1, 0, 1);       /* no sponge, nt = 2 */
    case_rtm(9, 9, 0, 3, 2, 2, 2);       /* fp16, stride 2 */
    case_rtm(13, 70, 20, 33, 4, 2, 5);   /* sponge wider than the grid */
    /* periodic test mode (nb = 0) and rejected arguments */
    orc_grid gp = {16, 16, 0, 4, 1.0, 1.0, 1e-3, 0.0, 1, 0};
    double *u = vec(256, 1.0), *out = vec(256, 0.0);
    need(orc_laplacian(&gp, u, out) == 0, "periodic laplacian");
    for (int i = 0; i < 256; ++i) need(fabs(out[i]) < 1e-12, "periodic laplacian of a constant");
    orc_grid bad = {16, 16, 0, 4, 1.0, 1.0, 1e-3, 0.0, 0, 0};
    double *w = vec(4, 0.0), *img = vec(256, 0.0);
    int r0 = 0;
    need(orc_rtm(&bad, u, w, 1, 1, 1, &r0, &r0, w, 0, 0, 0, 1, img, NULL) != 0, "stride 0 rejected");
    need(orc_rtm(&bad, u, w, 1, 1, 1, &r0, &r0, w, 1, 3, 0, 1, img, NULL) != 0, "quant 3 rejected");
    need(orc_rtm(&bad, u, w, 1, 1, 1, &r0, &r0, w, 1, 0, 1, 0, img, NULL) != 0, "checkpoint 0 rejected");
    free(u); free(out); free(w); free(img);
    printf("oracle rtm: ok\n");
    return 0;
}
