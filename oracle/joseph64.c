/*
 * FP64 reference ("oracle") for Joseph's ray-driven projector, its TOF
 * extensions and listmode OSEM.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
 * call this file; it exists so that tests, the smoke check and the CPU
 * baseline of the benchmark have an independent, obviously-correct result to
 * compare the GPU kernels with.  It shares no code with the HIP sources.
 *
 * Method (Sec. 2.1 and Fig. 1 of the paper, Joseph 1982):
 *   - pick the principal axis p: the image axis most parallel to the ray;
 *   - visit the image planes perpendicular to p one by one; in each, take the
 *     ray/plane intersection and bilinearly interpolate the four voxel centres
 *     around it;
 *   - add the plane contributions and multiply by the ray length per plane
 *     step (the incidence-angle correction).
 * TOF (Sec. 2.1, Sec. 2.6): every plane sample gets, for TOF bin t, the
 * weight of a Gaussian (truncated at n_sigmas) convolved with a rect of the
 * bin width, i.e. a difference of two error functions evaluated at the
 * distance between the sample and the bin centre.  TOF sinogram projection
 * fills all bins of a LOR, TOF listmode projection only the event's bin
 * (Sec. 2.2).  Back projections are the exact adjoints (Sec. 2.2).
 *
 * Readings of points the paper leaves open (each also listed in the design
 * notes):
 *   - principal axis = argmax_a |e_a - s_a| in mm, first axis on ties, the
 *     comparison taken on the float32 differences the GPU also forms;
 *   - the ray is the segment from start to end: plane k is visited iff its
 *     parameter t_k = (k - S_p)/D_p lies in [0, 1];
 *   - voxels outside the grid read as 0 (zero padding of the 2x2 stencil);
 *   - voxel (i,j,k) has its centre at origin + (i,j,k) * voxsize;
 *   - TOF position of a sample: signed mm from the LOR midpoint towards the
 *     end point, s = (t - 1/2) |e - s|; one TOF weight per plane sample;
 *   - TOF bin centre c_t = (t - (n_bins - 1)/2) * bin_width + center_offset;
 *   - truncation clips the Gaussian before the convolution:
 *       w_t(s) = G(s - c_t + bw/2) - G(s - c_t - bw/2),
 *       G(x)   = erf(clip(x, -n_sigmas*sigma, n_sigmas*sigma) / (sqrt(2) sigma)) / 2,
 *     not renormalised;
 *   - the alternative kernel of Sec. 4 (a tabulated, possibly non-Gaussian,
 *     TOF kernel): a table of the bin weight w(x) as a function of the
 *     signed distance x of the sample from the bin centre, at
 *     x_i = x0 + i dx (i = 0 .. n-1), linearly interpolated, 0 outside
 *     [x0, x_{n-1}]; sigma and n_sigmas are then unused;
 *   - per-ray TOF parameters (a generalisation of the single kernel of
 *     Sec. 2.2, where every LOR shares one Gaussian width and one bin-centre
 *     convention): where an array of one sigma or one centre offset per ray
 *     is given, ray l uses sigma[l] (with the same n_sigmas) or offset[l]
 *     in place of the scalar; a ray whose sigma is not a positive finite
 *     number, or whose offset is not finite, contributes nothing;
 *   - listmode bins outside [0, n_bins) and non-finite or zero-length LORs
 *     contribute nothing;
 *   - listmode OSEM: subset j holds the events with index e mod n_sub == j;
 *     an event whose expectation a_e x + bg is not positive contributes
 *     nothing; voxels with zero sensitivity are set to 0.
 *
 * All arithmetic is double; inputs are the float32 arrays the GPU sees,
 * widened.  Back projections use one private image per OpenMP thread, summed
 * in thread order, so results are deterministic for a fixed thread count.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef struct {
    double o[3];  /* centre of voxel (0,0,0), mm */
    double h[3];  /* voxel size, mm */
    int64_t n[3]; /* dimensions, axis 2 fastest in memory */
} grid64;

typedef struct {
    double bw;     /* bin width, mm */
    double sig;    /* Gaussian sigma, mm */
    double trunc;  /* n_sigmas * sigma, mm */
    double off;    /* centre offset, mm */
    double nsig;   /* truncation in units of sigma */
    int nb;        /* number of bins */
    const float* sig_l; /* sigma of each ray, or NULL (all rays: sig) */
    const float* off_l; /* centre offset of each ray, or NULL (all rays: off) */
    const float* lut; /* tabulated bin weight w(x_i), or NULL (Gaussian) */
    int64_t lut_n;
    double lut_x0, lut_dx;
} tof64;

typedef struct {
    int ok;          /* 0: the ray contributes nothing */
    int p, u, w;     /* principal axis, in-plane axes (u < w) */
    double S[3];     /* start point in voxel-index units */
    double D[3];     /* end - start in voxel-index units */
    double len;      /* |end - start|, mm */
    double ell;      /* ray length per plane step, mm */
} ray64;

static grid64 mkgrid(const float* origin, const float* vs, const int32_t* dim) {
    grid64 g;
    for (int a = 0; a < 3; ++a) {
        g.o[a] = origin[a];
        g.h[a] = vs[a];
        g.n[a] = dim[a];
    }
    return g;
}

static tof64 mktof(float bw, float sig, float nsig, float off, int32_t nb, const float* lut, int32_t lut_n,
                   double lut_x0, double lut_dx, const float* sig_l, const float* off_l) {
    tof64 t;
    t.bw = bw;
    t.sig = sig;
    t.nsig = nsig;
    t.trunc = (double)nsig * (double)sig;
    t.off = off;
    t.sig_l = sig_l;
    t.off_l = off_l;
    t.nb = nb;
    t.lut = lut;
    t.lut_n = lut_n;
    t.lut_x0 = lut_x0;
    t.lut_dx = lut_dx;
    return t;
}

#define NOTOF(name) tof64 name = mktof(1.f, 1.f, 1.f, 0.f, 1, NULL, 0, 0.0, 1.0, NULL, NULL)

/* TOF parameters of ray l: its own sigma and centre offset where per-ray
 * arrays are given.  Returns 0 if they are unusable (the ray contributes
 * nothing). */
static int ray_tof(const tof64* tf, int64_t l, tof64* out) {
    *out = *tf;
    if (tf->sig_l) {
        double s = tf->sig_l[l];
        if (!(s > 0.0) || !isfinite(s)) return 0;
        out->sig = s;
        out->trunc = tf->nsig * s;
    }
    if (tf->off_l) {
        double o = tf->off_l[l];
        if (!isfinite(o)) return 0;
        out->off = o;
    }
    return 1;
}

static ray64 ray_setup(const float* xs, const float* xe, const grid64* g) {
    ray64 r;
    memset(&r, 0, sizeof r);
    float df[3];
    for (int a = 0; a < 3; ++a) {
        if (!isfinite(xs[a]) || !isfinite(xe[a])) return r;
        df[a] = xe[a] - xs[a]; /* float32 difference: the axis decision */
    }
    int p = 0;
    for (int a = 1; a < 3; ++a)
        if (fabsf(df[a]) > fabsf(df[p])) p = a;
    if (df[p] == 0.0f) return r;
    double d[3];
    for (int a = 0; a < 3; ++a) d[a] = (double)xe[a] - (double)xs[a];
    r.len = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
    for (int a = 0; a < 3; ++a) {
        r.S[a] = ((double)xs[a] - g->o[a]) / g->h[a];
        r.D[a] = d[a] / g->h[a];
    }
    r.p = p;
    r.u = (p == 0) ? 1 : 0;
    r.w = (p == 2) ? 1 : 2;
    r.ell = g->h[p] * r.len / fabs(d[p]);
    r.ok = 1;
    return r;
}

/* The 2x2 stencil of plane k.  Returns 0 if the plane is not on the segment;
 * otherwise fills t and, for each of the 4 neighbours, the flat voxel index
 * (-1 if outside the grid) and the bilinear weight. */
static int plane_stencil(const grid64* g, const ray64* r, int64_t k, double* t_out, int64_t idx[4],
                         double wt[4]) {
    double t = ((double)k - r->S[r->p]) / r->D[r->p];
    if (!(t >= 0.0 && t <= 1.0)) return 0;
    double U = r->S[r->u] + t * r->D[r->u];
    double W = r->S[r->w] + t * r->D[r->w];
    double fi = floor(U), fj = floor(W);
    double fu = U - fi, fw = W - fj;
    int64_t i0 = (int64_t)fi, j0 = (int64_t)fj;
    int q = 0;
    for (int a = 0; a < 2; ++a) {
        for (int b = 0; b < 2; ++b, ++q) {
            int64_t iu = i0 + a, jw = j0 + b;
            wt[q] = (a ? fu : 1.0 - fu) * (b ? fw : 1.0 - fw);
            if (iu < 0 || iu >= g->n[r->u] || jw < 0 || jw >= g->n[r->w]) {
                idx[q] = -1;
                continue;
            }
            int64_t c[3];
            c[r->p] = k;
            c[r->u] = iu;
            c[r->w] = jw;
            idx[q] = (c[0] * g->n[1] + c[1]) * g->n[2] + c[2];
        }
    }
    *t_out = t;
    return 1;
}

static double tof_G(double x, const tof64* tf) {
    if (x > tf->trunc) x = tf->trunc;
    if (x < -tf->trunc) x = -tf->trunc;
    return 0.5 * erf(x / (sqrt(2.0) * tf->sig));
}

/* tabulated kernel: linear interpolation between the table entries around x */
static double tof_lut(double x, const tof64* tf) {
    double u = (x - tf->lut_x0) / tf->lut_dx;
    if (!(u >= 0.0) || u > (double)(tf->lut_n - 1)) return 0.0;
    int64_t i = (int64_t)floor(u);
    if (i >= tf->lut_n - 1) return (double)tf->lut[tf->lut_n - 1];
    double f = u - (double)i;
    return (1.0 - f) * (double)tf->lut[i] + f * (double)tf->lut[i + 1];
}

/* weight of TOF bin `bin` for a sample at signed position s (mm from the midpoint) */
static double tof_weight(double s, int bin, const tof64* tf) {
    double c = ((double)bin - 0.5 * (double)(tf->nb - 1)) * tf->bw + tf->off;
    if (tf->lut) return tof_lut(s - c, tf);
    return tof_G(s - c + 0.5 * tf->bw, tf) - tof_G(s - c - 0.5 * tf->bw, tf);
}

/* whether a sample at s lies inside the support of bin `bin` (work counter): the
 * Gaussian's weight is non-zero exactly there, a table's support is its open range */
static int tof_inside(double s, int bin, const tof64* tf) {
    if (!tf->lut) return tof_weight(s, bin, tf) != 0.0;
    double c = ((double)bin - 0.5 * (double)(tf->nb - 1)) * tf->bw + tf->off;
    double x = s - c;
    return x > tf->lut_x0 && x < tf->lut_x0 + (double)(tf->lut_n - 1) * tf->lut_dx;
}

/* interpolated image value of one stencil */
static double stencil_value(const double* img, const int64_t idx[4], const double wt[4]) {
    double v = 0.0;
    for (int q = 0; q < 4; ++q)
        if (idx[q] >= 0) v += wt[q] * img[idx[q]];
    return v;
}

static void stencil_scatter(double* img, const int64_t idx[4], const double wt[4], double val) {
    for (int q = 0; q < 4; ++q)
        if (idx[q] >= 0) img[idx[q]] += wt[q] * val;
}

/* forward of one ray; mode 0 non-TOF, 1 TOF sinogram (out[nb]), 2 TOF listmode (bin) */
static void ray_forward(const float* xs, const float* xe, const grid64* g, const tof64* tf, int mode,
                        int bin, const double* img, double* out) {
    int nout = (mode == 1) ? tf->nb : 1;
    for (int q = 0; q < nout; ++q) out[q] = 0.0;
    if (mode == 2 && (bin < 0 || bin >= tf->nb)) return;
    ray64 r = ray_setup(xs, xe, g);
    if (!r.ok) return;
    int64_t idx[4];
    double wt[4], t;
    for (int64_t k = 0; k < g->n[r.p]; ++k) {
        if (!plane_stencil(g, &r, k, &t, idx, wt)) continue;
        double v = stencil_value(img, idx, wt);
        if (mode == 0) {
            out[0] += v;
        } else {
            double s = (t - 0.5) * r.len;
            if (mode == 1)
                for (int b = 0; b < tf->nb; ++b) out[b] += tof_weight(s, b, tf) * v;
            else
                out[0] += tof_weight(s, bin, tf) * v;
        }
    }
    for (int q = 0; q < nout; ++q) out[q] *= r.ell;
}

/* back projection of one ray into img: exact transpose of ray_forward */
static void ray_back(const float* xs, const float* xe, const grid64* g, const tof64* tf, int mode, int bin,
                     double* img, const double* in) {
    if (mode == 2 && (bin < 0 || bin >= tf->nb)) return;
    ray64 r = ray_setup(xs, xe, g);
    if (!r.ok) return;
    int64_t idx[4];
    double wt[4], t;
    for (int64_t k = 0; k < g->n[r.p]; ++k) {
        if (!plane_stencil(g, &r, k, &t, idx, wt)) continue;
        double c;
        if (mode == 0) {
            c = in[0];
        } else {
            double s = (t - 0.5) * r.len;
            if (mode == 1) {
                c = 0.0;
                for (int b = 0; b < tf->nb; ++b) c += tof_weight(s, b, tf) * in[b];
            } else {
                c = tof_weight(s, bin, tf) * in[0];
            }
        }
        stencil_scatter(img, idx, wt, r.ell * c);
    }
}

static int64_t nvox(const grid64* g) { return g->n[0] * g->n[1] * g->n[2]; }

static int nthreads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

static int thread_id(void) {
#ifdef _OPENMP
    return omp_get_thread_num();
#else
    return 0;
#endif
}

static void forward_all(const float* xs, const float* xe, int64_t n, const grid64* g, const tof64* tf, int mode,
                        const int16_t* bins, const double* img, double* p) {
    int nout = (mode == 1) ? tf->nb : 1;
#pragma omp parallel for schedule(static)
    for (int64_t l = 0; l < n; ++l) {
        tof64 tl;
        if (!ray_tof(tf, l, &tl)) {
            for (int q = 0; q < nout; ++q) p[(int64_t)nout * l + q] = 0.0;
            continue;
        }
        ray_forward(xs + 3 * l, xe + 3 * l, g, &tl, mode, bins ? bins[l] : 0, img, p + (int64_t)nout * l);
    }
}

/* events l with l % stride == phase only (stride 1: all) */
static void back_all(const float* xs, const float* xe, int64_t n, const grid64* g, const tof64* tf, int mode,
                     const int16_t* bins, double* img, const double* p) {
    int nout = (mode == 1) ? tf->nb : 1;
    int nt = nthreads();
    int64_t nv = nvox(g);
    double* priv = (double*)calloc((size_t)nt * (size_t)nv, sizeof(double));
    if (!priv) abort();
#pragma omp parallel
    {
        double* mine = priv + (size_t)thread_id() * (size_t)nv;
#pragma omp for schedule(static)
        for (int64_t l = 0; l < n; ++l) {
            tof64 tl;
            if (!ray_tof(tf, l, &tl)) continue;
            ray_back(xs + 3 * l, xe + 3 * l, g, &tl, mode, bins ? bins[l] : 0, mine, p + (int64_t)nout * l);
        }
    }
#pragma omp parallel for schedule(static)
    for (int64_t v = 0; v < nv; ++v) {
        double s = 0.0;
        for (int th = 0; th < nt; ++th) s += priv[(size_t)th * (size_t)nv + (size_t)v];
        img[v] += s;
    }
    free(priv);
}

/* ------------------------------------------------------------------ API -- */

int orc_max_threads(void) { return nthreads(); }

void orc_fwd(const float* xs, const float* xe, int64_t n, const float* origin, const float* vs, const int32_t* dim,
             const double* img, double* p) {
    grid64 g = mkgrid(origin, vs, dim);
    NOTOF(tf);
    forward_all(xs, xe, n, &g, &tf, 0, NULL, img, p);
}

void orc_back(const float* xs, const float* xe, int64_t n, const float* origin, const float* vs, const int32_t* dim,
              double* img, const double* p) {
    grid64 g = mkgrid(origin, vs, dim);
    NOTOF(tf);
    back_all(xs, xe, n, &g, &tf, 0, NULL, img, p);
}

void orc_fwd_tof_sino(const float* xs, const float* xe, int64_t n, const float* origin, const float* vs,
                      const int32_t* dim, float bin_width, float sigma, float n_sigmas, float center_offset,
                      int32_t n_bins, const float* lut, int32_t lut_n, double lut_x0, double lut_dx,
                      const float* sigma_per_ray, const float* offset_per_ray,
                      const double* img, double* p) {
    grid64 g = mkgrid(origin, vs, dim);
    tof64 tf = mktof(bin_width, sigma, n_sigmas, center_offset, n_bins, lut, lut_n, lut_x0, lut_dx, sigma_per_ray,
                     offset_per_ray);
    forward_all(xs, xe, n, &g, &tf, 1, NULL, img, p);
}

void orc_back_tof_sino(const float* xs, const float* xe, int64_t n, const float* origin, const float* vs,
                       const int32_t* dim, float bin_width, float sigma, float n_sigmas, float center_offset,
                       int32_t n_bins, const float* lut, int32_t lut_n, double lut_x0, double lut_dx,
                       const float* sigma_per_ray, const float* offset_per_ray,
                       double* img, const double* p) {
    grid64 g = mkgrid(origin, vs, dim);
    tof64 tf = mktof(bin_width, sigma, n_sigmas, center_offset, n_bins, lut, lut_n, lut_x0, lut_dx, sigma_per_ray,
                     offset_per_ray);
    back_all(xs, xe, n, &g, &tf, 1, NULL, img, p);
}

void orc_fwd_tof_lm(const float* xs, const float* xe, int64_t n, const float* origin, const float* vs,
                    const int32_t* dim, float bin_width, float sigma, float n_sigmas, float center_offset,
                    int32_t n_bins, const float* lut, int32_t lut_n, double lut_x0, double lut_dx,
                    const float* sigma_per_ray, const float* offset_per_ray,
                    const int16_t* bins, const double* img, double* p) {
    grid64 g = mkgrid(origin, vs, dim);
    tof64 tf = mktof(bin_width, sigma, n_sigmas, center_offset, n_bins, lut, lut_n, lut_x0, lut_dx, sigma_per_ray,
                     offset_per_ray);
    forward_all(xs, xe, n, &g, &tf, 2, bins, img, p);
}

void orc_back_tof_lm(const float* xs, const float* xe, int64_t n, const float* origin, const float* vs,
                     const int32_t* dim, float bin_width, float sigma, float n_sigmas, float center_offset,
                     int32_t n_bins, const float* lut, int32_t lut_n, double lut_x0, double lut_dx,
                     const float* sigma_per_ray, const float* offset_per_ray,
                     const int16_t* bins, double* img, const double* p) {
    grid64 g = mkgrid(origin, vs, dim);
    tof64 tf = mktof(bin_width, sigma, n_sigmas, center_offset, n_bins, lut, lut_n, lut_x0, lut_dx, sigma_per_ray,
                     offset_per_ray);
    back_all(xs, xe, n, &g, &tf, 2, bins, img, p);
}

/* Work counter: per ray, the number of plane samples whose 2x2 stencil has at
 * least one neighbour inside the grid; with bins != NULL only samples whose
 * TOF weight for the event's bin is non-zero are counted.  Returns the sum;
 * per_ray (nullable) receives the per-ray counts. */
int64_t orc_count_samples(const float* xs, const float* xe, int64_t n, const float* origin, const float* vs,
                          const int32_t* dim, float bin_width, float sigma, float n_sigmas, float center_offset,
                          int32_t n_bins, const float* lut, int32_t lut_n, double lut_x0, double lut_dx,
                          const float* sigma_per_ray, const float* offset_per_ray,
                          const int16_t* bins, int64_t* per_ray) {
    grid64 g = mkgrid(origin, vs, dim);
    tof64 tf = mktof(bin_width, sigma, n_sigmas, center_offset, n_bins, lut, lut_n, lut_x0, lut_dx, sigma_per_ray,
                     offset_per_ray);
    int64_t total = 0;
#pragma omp parallel for schedule(static) reduction(+ : total)
    for (int64_t l = 0; l < n; ++l) {
        int64_t cnt = 0;
        tof64 tl;
        int ok = (!bins || (bins[l] >= 0 && bins[l] < tf.nb)) && ray_tof(&tf, l, &tl);
        ray64 r = ray_setup(xs + 3 * l, xe + 3 * l, &g);
        if (ok && r.ok) {
            int64_t idx[4];
            double wt[4], t;
            for (int64_t k = 0; k < g.n[r.p]; ++k) {
                if (!plane_stencil(&g, &r, k, &t, idx, wt)) continue;
                if (idx[0] < 0 && idx[1] < 0 && idx[2] < 0 && idx[3] < 0) continue;
                if (bins && !tof_inside((t - 0.5) * r.len, bins[l], &tl)) continue;
                ++cnt;
            }
        }
        if (per_ray) per_ray[l] = cnt;
        total += cnt;
    }
    return total;
}

/* The TOF bin weight w(x) of a single bin centred at x = 0 (Gaussian or table), at n points:
 * the function every TOF projection evaluates at each plane sample. */
void orc_tof_kernel(const double* x, int64_t n, float bin_width, float sigma, float n_sigmas, const float* lut,
                    int32_t lut_n, double lut_x0, double lut_dx, double* w) {
    tof64 tf = mktof(bin_width, sigma, n_sigmas, 0.0f, 1, lut, lut_n, lut_x0, lut_dx, NULL, NULL);
    for (int64_t i = 0; i < n; ++i) w[i] = tof_weight(x[i], 0, &tf);
}

/* Image-based resolution model (the Gaussian blur the paper's listmode OSEM
 * reconstructions include, Sec. 2.6): a shift-invariant 3D Gaussian of the
 * given FWHM per axis (mm), applied as a discrete convolution on the voxel
 * grid.  Readings: sigma_a = FWHM_a / (2 sqrt(2 ln 2)) / h_a in voxels; the
 * kernel of axis a is exp(-i^2 / (2 sigma_a^2)) for |i| <= r_a =
 * floor(4 sigma_a + 1/2), normalised to sum 1 (FWHM_a == 0: identity); the
 * 3D kernel is the product of the three; voxels outside the grid read as 0.
 * With these readings the operator is symmetric, so it is its own adjoint.
 * Evaluated as one 1D convolution per axis (the product kernel factorises). */
static int gauss_taps(double fwhm, float h, double* w, int max_r) {
    if (!(fwhm > 0.0)) {
        w[0] = 1.0;
        return 0;
    }
    double sig = fwhm / (2.0 * sqrt(2.0 * log(2.0))) / (double)h;
    int r = (int)floor(4.0 * sig + 0.5);
    if (r > max_r) abort();
    double sum = 0.0;
    for (int i = -r; i <= r; ++i) sum += (w[i + r] = exp(-(double)i * i / (2.0 * sig * sig)));
    for (int i = -r; i <= r; ++i) w[i + r] /= sum;
    return r;
}

void orc_gauss3d(const double* src, double* dst, const int32_t* dim, const float* vs, const double* fwhm) {
    enum { MAXR = 64 };
    int64_t n0 = dim[0], n1 = dim[1], n2 = dim[2], nv = n0 * n1 * n2;
    double* a = (double*)malloc((size_t)nv * sizeof(double));
    double* b = (double*)malloc((size_t)nv * sizeof(double));
    if (!a || !b) abort();
    memcpy(a, src, (size_t)nv * sizeof(double));
    const int64_t stride[3] = {n1 * n2, n2, 1};
    for (int ax = 0; ax < 3; ++ax) {
        double w[2 * MAXR + 1];
        int r = gauss_taps(fwhm[ax], vs[ax], w, MAXR);
        int64_t len = dim[ax];
#pragma omp parallel for schedule(static)
        for (int64_t v = 0; v < nv; ++v) {
            int64_t pos = (v / stride[ax]) % len;  /* index along this axis */
            double acc = 0.0;
            for (int i = -r; i <= r; ++i) {
                int64_t q = pos + i;
                if (q < 0 || q >= len) continue;
                acc += w[i + r] * a[v + (int64_t)i * stride[ax]];
            }
            b[v] = acc;
        }
        double* t = a;
        a = b;
        b = t;
    }
    memcpy(dst, a, (size_t)nv * sizeof(double));
    free(a);
    free(b);
}

/* Listmode OSEM with TOF (ordered subsets EM, the paper's Sec. 2.6 iteration):
 * for it in [0, n_iter), subset j in [0, n_sub):
 *     acc = sum over events e with e % n_sub == j of a_e / (a_e . x' + bg)
 *     x_v <- x_v * acc'_v / (sens_v / n_sub)   if sens_v > 0, else 0,
 * where without a resolution model (fwhm == NULL) x' = x and acc' = acc, and
 * with one x' = G x and acc' = G acc (G = orc_gauss3d with that FWHM: the
 * system model is the projector after the blur, its adjoint the blur after
 * the back projection; sens must then be G applied to the back projection of
 * ones).  x holds the initial image on entry and the result on return. */
void orc_lm_osem(const float* xs, const float* xe, const int16_t* bins, int64_t n, const float* origin,
                 const float* vs, const int32_t* dim, float bin_width, float sigma, float n_sigmas,
                 float center_offset, int32_t n_bins, const float* lut, int32_t lut_n, double lut_x0,
                 double lut_dx, const float* sigma_per_ray, const float* offset_per_ray, const double* sens,
                 double bg, int32_t n_iter,
                 int32_t n_sub, double* x, const double* fwhm) {
    grid64 g = mkgrid(origin, vs, dim);
    tof64 tf = mktof(bin_width, sigma, n_sigmas, center_offset, n_bins, lut, lut_n, lut_x0, lut_dx, sigma_per_ray,
                     offset_per_ray);
    int64_t nv = nvox(&g);
    int nt = nthreads();
    double* priv = (double*)malloc((size_t)nt * (size_t)nv * sizeof(double));
    double* acc = (double*)malloc((size_t)nv * sizeof(double));
    double* xf = fwhm ? (double*)malloc((size_t)nv * sizeof(double)) : x;
    if (!priv || !acc || !xf) abort();
    for (int it = 0; it < n_iter; ++it) {
        for (int j = 0; j < n_sub; ++j) {
            if (fwhm) orc_gauss3d(x, xf, dim, vs, fwhm);
            memset(priv, 0, (size_t)nt * (size_t)nv * sizeof(double));
            int64_t n_j = (n > j) ? (n - j + n_sub - 1) / n_sub : 0;
#pragma omp parallel
            {
                double* mine = priv + (size_t)thread_id() * (size_t)nv;
#pragma omp for schedule(static)
                for (int64_t q = 0; q < n_j; ++q) {
                    int64_t e = (int64_t)j + q * n_sub;
                    tof64 tl;
                    if (!ray_tof(&tf, e, &tl)) continue;
                    double ybar;
                    ray_forward(xs + 3 * e, xe + 3 * e, &g, &tl, 2, bins[e], xf, &ybar);
                    ybar += bg;
                    if (!(ybar > 0.0)) continue;
                    double r = 1.0 / ybar;
                    ray_back(xs + 3 * e, xe + 3 * e, &g, &tl, 2, bins[e], mine, &r);
                }
            }
#pragma omp parallel for schedule(static)
            for (int64_t v = 0; v < nv; ++v) {
                double s = 0.0;
                for (int th = 0; th < nt; ++th) s += priv[(size_t)th * (size_t)nv + (size_t)v];
                acc[v] = s;
            }
            if (fwhm) orc_gauss3d(acc, acc, dim, vs, fwhm);
#pragma omp parallel for schedule(static)
            for (int64_t v = 0; v < nv; ++v)
                x[v] = (sens[v] > 0.0) ? x[v] * acc[v] / (sens[v] / (double)n_sub) : 0.0;
        }
    }
    free(priv);
    free(acc);
    if (fwhm) free(xf);
}


/* TOF sinogram OSEM: the sinogram counterpart of the listmode OSEM above (the paper's Sec. 4
 * discusses the memory such a reconstruction needs and chunk-wise processing for long axial
 * fields of view).  LOR l belongs to subset sub[l] (LORs with sub[l] outside [0, n_sub) take no
 * part); y holds the measured counts [n][n_bins], bg the additive expectation of every bin.
 * For it in [0, n_iter), subset j in [0, n_sub):
 *     sens_j = A_j^T 1                 (all LORs of subset j, all bins)
 *     acc    = A_j^T (y / (A_j x + bg)), a (LOR, bin) whose expectation is not positive
 *              contributing nothing
 *     x_v   <- x_v acc_v / sens_j,v   if sens_j,v > 0, else 0.
 * x holds the initial image on entry and the result on return. */
void orc_tof_sino_osem(const float* xs, const float* xe, int64_t n, const int32_t* sub, int32_t n_sub,
                       const float* origin, const float* vs, const int32_t* dim, float bin_width, float sigma,
                       float n_sigmas, float center_offset, int32_t n_bins, const double* y, double bg,
                       int32_t n_iter, double* x) {
    grid64 g = mkgrid(origin, vs, dim);
    tof64 tf = mktof(bin_width, sigma, n_sigmas, center_offset, n_bins, NULL, 0, 0.0, 1.0, NULL, NULL);
    const int64_t nv = nvox(&g), nb = n_bins;
    int64_t* cnt = (int64_t*)calloc((size_t)n_sub + 1, sizeof(int64_t));
    if (!cnt) abort();
    for (int64_t l = 0; l < n; ++l)
        if (sub[l] >= 0 && sub[l] < n_sub) ++cnt[sub[l] + 1];
    for (int j = 0; j < n_sub; ++j) cnt[j + 1] += cnt[j];
    /* the LORs of each subset, copied out in their original order */
    float* sxs = (float*)malloc((size_t)(3 * cnt[n_sub] + 3) * sizeof(float));
    float* sxe = (float*)malloc((size_t)(3 * cnt[n_sub] + 3) * sizeof(float));
    double* sy = (double*)malloc((size_t)(nb * cnt[n_sub] + 1) * sizeof(double));
    double* q = (double*)malloc((size_t)(nb * cnt[n_sub] + 1) * sizeof(double));
    double* sens = (double*)calloc((size_t)(nv * n_sub), sizeof(double));
    double* acc = (double*)malloc((size_t)nv * sizeof(double));
    int64_t* fill = (int64_t*)malloc((size_t)(n_sub + 1) * sizeof(int64_t));
    if (!sxs || !sxe || !sy || !q || !sens || !acc || !fill) abort();
    memcpy(fill, cnt, (size_t)(n_sub + 1) * sizeof(int64_t));
    for (int64_t l = 0; l < n; ++l) {
        if (sub[l] < 0 || sub[l] >= n_sub) continue;
        int64_t d = fill[sub[l]]++;
        memcpy(sxs + 3 * d, xs + 3 * l, 3 * sizeof(float));
        memcpy(sxe + 3 * d, xe + 3 * l, 3 * sizeof(float));
        memcpy(sy + nb * d, y + nb * l, (size_t)nb * sizeof(double));
    }
    for (int j = 0; j < n_sub; ++j) {
        int64_t a = cnt[j], m = cnt[j + 1] - cnt[j];
        for (int64_t i = 0; i < nb * m; ++i) q[nb * a + i] = 1.0;
        back_all(sxs + 3 * a, sxe + 3 * a, m, &g, &tf, 1, NULL, sens + nv * j, q + nb * a);
    }
    for (int it = 0; it < n_iter; ++it) {
        for (int j = 0; j < n_sub; ++j) {
            int64_t a = cnt[j], m = cnt[j + 1] - cnt[j];
            forward_all(sxs + 3 * a, sxe + 3 * a, m, &g, &tf, 1, NULL, x, q + nb * a);
            for (int64_t i = nb * a; i < nb * (a + m); ++i) {
                double e = q[i] + bg;
                q[i] = (e > 0.0) ? sy[i] / e : 0.0;
            }
            memset(acc, 0, (size_t)nv * sizeof(double));
            back_all(sxs + 3 * a, sxe + 3 * a, m, &g, &tf, 1, NULL, acc, q + nb * a);
            const double* sj = sens + nv * j;
            for (int64_t v = 0; v < nv; ++v) x[v] = (sj[v] > 0.0) ? x[v] * acc[v] / sj[v] : 0.0;
        }
    }
    free(cnt);
    free(sxs);
    free(sxe);
    free(sy);
    free(q);
    free(sens);
    free(acc);
    free(fill);
}
