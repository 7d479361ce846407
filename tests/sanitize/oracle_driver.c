/* Runs every function of the FP64 oracle (oracle/joseph64.c) on small seeded problems,
 * including its edge cases (no rays, non-finite and zero-length rays, rays missing the grid,
 * listmode bins out of range, unusable per-ray TOF parameters, a tabulated kernel), for a build
 * with AddressSanitizer and UndefinedBehaviorSanitizer.  Exit status 0 and no sanitizer report
 * = clean; it also checks the adjoint identity of each projector pair as a sanity check. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

void orc_fwd(const float*, const float*, int64_t, const float*, const float*, const int32_t*, const double*, double*);
void orc_back(const float*, const float*, int64_t, const float*, const float*, const int32_t*, double*, const double*);
#define TOFARGS float, float, float, float, int32_t, const float*, int32_t, double, double, const float*, const float*
void orc_fwd_tof_sino(const float*, const float*, int64_t, const float*, const float*, const int32_t*, TOFARGS,
                      const double*, double*);
void orc_back_tof_sino(const float*, const float*, int64_t, const float*, const float*, const int32_t*, TOFARGS,
                       double*, const double*);
void orc_fwd_tof_lm(const float*, const float*, int64_t, const float*, const float*, const int32_t*, TOFARGS,
                    const int16_t*, const double*, double*);
void orc_back_tof_lm(const float*, const float*, int64_t, const float*, const float*, const int32_t*, TOFARGS,
                     const int16_t*, double*, const double*);
int64_t orc_count_samples(const float*, const float*, int64_t, const float*, const float*, const int32_t*, TOFARGS,
                          const int16_t*, int64_t*);
void orc_tof_kernel(const double*, int64_t, float, float, float, const float*, int32_t, double, double, double*);
void orc_gauss3d(const double*, double*, const int32_t*, const float*, const double*);
void orc_lm_osem(const float*, const float*, const int16_t*, int64_t, const float*, const float*, const int32_t*,
                 TOFARGS, const double*, double, int32_t, int32_t, double*, const double*);
void orc_tof_sino_osem(const float*, const float*, int64_t, const int32_t*, int32_t, const float*, const float*,
                       const int32_t*, float, float, float, float, int32_t, const double*, double, int32_t, double*);

static uint64_t rng = 88172645463325252ull;
static double urand(void) { /* xorshift64 */
    rng ^= rng << 13;
    rng ^= rng >> 7;
    rng ^= rng << 17;
    return (double)(rng >> 11) * (1.0 / 9007199254740992.0);
}

static int fails = 0;
static void check_adj(const char* what, const double* a, const double* b, int64_t n, const double* c,
                      const double* d, int64_t m) {
    double l = 0, r = 0;
    for (int64_t i = 0; i < n; ++i) l += a[i] * b[i];
    for (int64_t i = 0; i < m; ++i) r += c[i] * d[i];
    if (!(fabs(l - r) <= 1e-10 * fabs(l) + 1e-300)) {
        fprintf(stderr, "%s: adjoint mismatch %.17g vs %.17g\n", what, l, r);
        ++fails;
    }
}

int main(void) {
    enum { N = 400, NB = 7 };
    const int32_t dim[3] = {9, 7, 5};
    const float vs[3] = {2.0f, 1.5f, 2.5f}, origin[3] = {-8.0f, -4.5f, -5.0f};
    const int64_t nv = 9 * 7 * 5;
    float* xs = malloc(3 * N * sizeof(float));
    float* xe = malloc(3 * N * sizeof(float));
    for (int i = 0; i < N; ++i) {
        double u[3], s = 0;
        for (int a = 0; a < 3; ++a) s += (u[a] = urand() - 0.5) * u[a];
        s = sqrt(s);
        for (int a = 0; a < 3; ++a) {
            double off = (urand() - 0.5) * 10.0;
            xs[3 * i + a] = (float)(off + 25.0 * u[a] / s);
            xe[3 * i + a] = (float)(off - 25.0 * u[a] / s + 3.0 * (urand() - 0.5));
        }
    }
    xs[0] = NAN;                                                            /* non-finite */
    memcpy(xe + 3, xs + 3, 3 * sizeof(float));                              /* zero length */
    xs[6] = 500.0f; xe[6] = 600.0f;                                         /* misses the grid */
    xs[9] = 0.5f; xs[10] = 0.25f; xs[11] = 0.0f;                            /* starts inside */
    double *img = malloc(nv * sizeof(double)), *img2 = calloc(nv, sizeof(double));
    for (int64_t v = 0; v < nv; ++v) img[v] = urand();
    double *p = malloc(N * NB * sizeof(double)), *y = malloc(N * NB * sizeof(double));
    for (int i = 0; i < N * NB; ++i) y[i] = urand();
    int16_t* bins = malloc(N * sizeof(int16_t));
    for (int i = 0; i < N; ++i) bins[i] = (int16_t)((int)(urand() * (NB + 2)) - 1); /* some out of range */
    const float bw = 4.0f, sig = 3.0f, ns = 3.0f;

    orc_fwd(xs, xe, N, origin, vs, dim, img, p);
    orc_back(xs, xe, N, origin, vs, dim, img2, y);
    check_adj("non-TOF", p, y, N, img, img2, nv);
    orc_fwd(xs, xe, 0, origin, vs, dim, img, p);

    memset(img2, 0, nv * sizeof(double));
    orc_fwd_tof_sino(xs, xe, N, origin, vs, dim, bw, sig, ns, 0.5f, NB, NULL, 0, 0, 1, NULL, NULL, img, p);
    orc_back_tof_sino(xs, xe, N, origin, vs, dim, bw, sig, ns, 0.5f, NB, NULL, 0, 0, 1, NULL, NULL, img2, y);
    check_adj("TOF sino", p, y, (int64_t)N * NB, img, img2, nv);

    memset(img2, 0, nv * sizeof(double));
    orc_fwd_tof_lm(xs, xe, N, origin, vs, dim, bw, sig, ns, 0.0f, NB, NULL, 0, 0, 1, NULL, NULL, bins, img, p);
    orc_back_tof_lm(xs, xe, N, origin, vs, dim, bw, sig, ns, 0.0f, NB, NULL, 0, 0, 1, NULL, NULL, bins, img2, y);
    check_adj("TOF LM", p, y, N, img, img2, nv);

    /* per-ray sigma / offset, some unusable */
    float *sr = malloc(N * sizeof(float)), *orr = malloc(N * sizeof(float));
    for (int i = 0; i < N; ++i) { sr[i] = (float)(sig * (0.8 + 0.4 * urand())); orr[i] = (float)(urand() - 0.5); }
    sr[1] = 0.0f; sr[2] = -1.0f; sr[3] = NAN; orr[4] = INFINITY;
    memset(img2, 0, nv * sizeof(double));
    orc_fwd_tof_sino(xs, xe, N, origin, vs, dim, bw, sig, ns, 0.0f, NB, NULL, 0, 0, 1, sr, orr, img, p);
    orc_back_tof_sino(xs, xe, N, origin, vs, dim, bw, sig, ns, 0.0f, NB, NULL, 0, 0, 1, sr, orr, img2, y);
    check_adj("TOF sino per ray", p, y, (int64_t)N * NB, img, img2, nv);

    /* tabulated kernel (a triangle) */
    float lut[41];
    for (int i = 0; i < 41; ++i) lut[i] = (float)(1.0 - fabs(i - 20) / 20.0);
    memset(img2, 0, nv * sizeof(double));
    orc_fwd_tof_lm(xs, xe, N, origin, vs, dim, bw, sig, ns, 0.0f, NB, lut, 41, -10.0, 0.5, NULL, orr, bins, img, p);
    orc_back_tof_lm(xs, xe, N, origin, vs, dim, bw, sig, ns, 0.0f, NB, lut, 41, -10.0, 0.5, NULL, orr, bins, img2, y);
    check_adj("TOF LM table", p, y, N, img, img2, nv);

    int64_t* per = malloc(N * sizeof(int64_t));
    orc_count_samples(xs, xe, N, origin, vs, dim, bw, sig, ns, 0.0f, NB, NULL, 0, 0, 1, NULL, NULL, NULL, per);
    orc_count_samples(xs, xe, N, origin, vs, dim, bw, sig, ns, 0.0f, NB, NULL, 0, 0, 1, sr, orr, bins, per);
    orc_count_samples(xs, xe, N, origin, vs, dim, bw, sig, ns, 0.0f, NB, lut, 41, -10.0, 0.5, NULL, NULL, bins, per);

    double xk[64], wk[64];
    for (int i = 0; i < 64; ++i) xk[i] = (i - 32) * 0.5;
    orc_tof_kernel(xk, 64, bw, sig, ns, NULL, 0, 0, 1, wk);
    orc_tof_kernel(xk, 64, bw, sig, ns, lut, 41, -10.0, 0.5, wk);

    const double fwhm[3] = {4.5, 3.0, 0.0};
    orc_gauss3d(img, img2, dim, vs, fwhm);

    double* sens = calloc(nv, sizeof(double));
    double* ones = malloc(N * sizeof(double));
    for (int i = 0; i < N; ++i) ones[i] = 1.0;
    orc_back(xs, xe, N, origin, vs, dim, sens, ones);
    double* x = malloc(nv * sizeof(double));
    for (int64_t v = 0; v < nv; ++v) x[v] = sens[v] > 0 ? 1.0 : 0.0;
    orc_lm_osem(xs, xe, bins, N, origin, vs, dim, bw, sig, ns, 0.0f, NB, NULL, 0, 0, 1, NULL, NULL, sens, 0.1, 2, 3,
                x, NULL);
    orc_lm_osem(xs, xe, bins, N, origin, vs, dim, bw, sig, ns, 0.0f, NB, NULL, 0, 0, 1, NULL, NULL, sens, 0.1, 1, 4,
                x, fwhm);

    int32_t* sub = malloc(N * sizeof(int32_t));
    for (int i = 0; i < N; ++i) sub[i] = (i % 5) - 1; /* some LORs in no subset */
    for (int64_t v = 0; v < nv; ++v) x[v] = 1.0;
    orc_tof_sino_osem(xs, xe, N, sub, 3, origin, vs, dim, bw, sig, ns, 0.0f, NB, y, 0.1, 2, x);

    for (int64_t v = 0; v < nv; ++v)
        if (!isfinite(x[v]) || x[v] < 0) { fprintf(stderr, "OSEM image not finite/non-negative\n"); ++fails; break; }
    free(xs); free(xe); free(img); free(img2); free(p); free(y); free(bins); free(sr); free(orr); free(per);
    free(sens); free(ones); free(x); free(sub);
    printf("oracle driver: %s\n", fails ? "FAILED" : "ok");
    return fails ? 1 : 0;
}
