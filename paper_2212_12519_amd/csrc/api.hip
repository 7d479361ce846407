// C ABI of libppmi.so: argument checks, kernel-side geometry, dispatch.
// The declarations, conventions and error codes are documented in ppmi.h.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstdio>

#include "joseph.hpp"
#include "launch.hpp"

using namespace ppmi;

static_assert(sizeof(pp_tof_t) == 64, "pp_tof_t layout");
static_assert(sizeof(pp_frame_desc_t) == 120, "pp_frame_desc_t layout");

namespace {

thread_local char g_hip_msg[256] = "";

int hip_status(hipError_t e) {
    if (e == hipSuccess) return PP_OK;
    std::snprintf(g_hip_msg, sizeof g_hip_msg, "HIP error %d: %s", (int)e, hipGetErrorString(e));
    return PP_EHIP;
}

bool finite3(const float* v) { return std::isfinite(v[0]) && std::isfinite(v[1]) && std::isfinite(v[2]); }

int make_geom(const pp_image_t* gi, GeomK& g) {
    if (!gi) return PP_EINVAL_PTR;
    if (!finite3(gi->origin) || !finite3(gi->voxsize)) return PP_EINVAL_GEOM;
    int64_t nv = 1;
    for (int a = 0; a < 3; ++a) {
        if (gi->dim[a] <= 0 || !(gi->voxsize[a] > 0.0f)) return PP_EINVAL_GEOM;
        nv *= gi->dim[a];
        if (nv >= (int64_t(1) << 30)) return PP_EINVAL_GEOM;  // byte offsets of the image fit 32 bits
    }
    for (int a = 0; a < 3; ++a) {
        g.o[a] = gi->origin[a];
        g.h[a] = gi->voxsize[a];
        g.n[a] = gi->dim[a];
    }
    g.stride[2] = 1;
    g.stride[1] = gi->dim[2];
    g.stride[0] = gi->dim[1] * gi->dim[2];
    return PP_OK;
}

// The Gaussian bin weight of ppmi.h in float64 (the exact function the polynomial approximates).
double tof_w_exact(double x, double hbw, double trunc, double inv_s2) {
    const double a = std::fmin(std::fmax(x + hbw, -trunc), trunc);
    const double b = std::fmin(std::fmax(x - hbw, -trunc), trunc);
    return 0.5 * (std::erf(a * inv_s2) - std::erf(b * inv_s2));
}

// Chebyshev interpolant of f on [-1, 1] through the N + 1 Chebyshev points (the zeros of T_{N+1}),
// returned as the coefficients c[i] of s^i: c_j = 2/(N+1) sum_k f(s_k) T_j(s_k) (c_0 halved), and
// the T_j expanded in powers by T_{j+1} = 2 s T_j - T_{j-1}.
constexpr int kChebMax = 16;
template <class F>
void cheb_powers(F f, int N, double* c) {
    const double pi = 3.14159265358979323846;
    double fv[kChebMax], ch[kChebMax], T[kChebMax][kChebMax] = {};
    for (int k = 0; k <= N; ++k) fv[k] = f(std::cos(pi * (k + 0.5) / (N + 1)));
    for (int j = 0; j <= N; ++j) {
        double a = 0.0;
        for (int k = 0; k <= N; ++k) a += fv[k] * std::cos(pi * j * (k + 0.5) / (N + 1));
        ch[j] = a * 2.0 / (N + 1);
    }
    ch[0] *= 0.5;
    T[0][0] = 1.0;
    if (N >= 1) T[1][1] = 1.0;
    for (int j = 1; j < N; ++j)
        for (int i = 0; i <= j + 1; ++i) T[j + 1][i] = (i > 0 ? 2.0 * T[j][i - 1] : 0.0) - T[j - 1][i];
    for (int i = 0; i <= N; ++i) {
        c[i] = 0.0;
        for (int j = i; j <= N; ++j) c[i] += ch[j] * T[j][i];
    }
}

// The device's tof_poly, evaluated on the host in the same float32 operations.
float tof_poly_host(float x, const TofK& t) {
    const float y = std::fabs(x), u = y * t.pq1;
    const float s1 = std::fmaf(u, u, -1.0f), s2 = std::fmaf(y, t.pa2, t.pb2);
    float a = t.pc[kPolyCentral], b = t.pt[kPolyTail];
    for (int i = kPolyCentral - 1; i >= 0; --i) {
        a = std::fmaf(a, s1, t.pc[i]);
        if (i < kPolyTail) b = std::fmaf(b, s2, t.pt[i]);
    }
    return y < t.pk1 ? a : (y < t.pk2 ? b : 0.0f);
}

// Fits the polynomial form of the Gaussian bin weight (tof_poly in joseph.hpp) and keeps it
// (t.poly = 1) if its float32 evaluation stays within 5e-7 of the peak weight of the exact
// weight everywhere (checked on a grid 1/4096 of the support apart, up to 2% past its end);
// otherwise the kernels use the erf form.
void fit_tof_poly(TofK& t, double sig, double ns, double bw) {
    t.poly = 0;
    const double hbw = 0.5 * bw, trunc = ns * sig, inv_s2 = 1.0 / (std::sqrt(2.0) * sig);
    const double k1 = std::fabs(trunc - hbw), k2 = trunc + hbw;
    if (!(k1 > 1e-3 * k2) || !(k2 - k1 > 1e-3 * k2)) return;  // a piece too short to fit
    auto w = [&](double x) { return tof_w_exact(x, hbw, trunc, inv_s2); };
    double c1[kPolyCentral + 1], c2[kPolyTail + 1];
    cheb_powers([&](double s) { return w(k1 * std::sqrt(0.5 * (s + 1.0))); }, kPolyCentral, c1);
    cheb_powers([&](double s) { return w(0.5 * (k1 + k2) + 0.5 * (k2 - k1) * s); }, kPolyTail, c2);
    for (int i = 0; i <= kPolyCentral; ++i) t.pc[i] = (float)c1[i];
    for (int i = 0; i <= kPolyTail; ++i) t.pt[i] = (float)c2[i];
    t.pk1 = (float)k1;
    t.pk2 = (float)k2;
    t.pq1 = (float)(std::sqrt(2.0) / k1);
    t.pa2 = (float)(2.0 / (k2 - k1));
    t.pb2 = (float)(-(k1 + k2) / (k2 - k1));
    const double peak = w(0.0);
    double err = 0.0;
    const int m = 4096;
    for (int i = 0; i <= m + m / 50; ++i) {
        const float x = (float)(k2 * i / m);
        err = std::fmax(err, std::fabs((double)tof_poly_host(x, t) - w((double)x)));
    }
    if (err <= 5e-7 * peak) t.poly = 1;
}

int make_tof(const pp_tof_t* ti, TofK& t) {
    if (!ti) return PP_EINVAL_PTR;
    if (ti->n_bins < 1 || ti->n_bins > 256) return PP_EINVAL_TOF;
    if (!std::isfinite(ti->bin_width) || !(ti->bin_width > 0.0f) || !std::isfinite(ti->center_offset))
        return PP_EINVAL_TOF;
    t.sig_ray = ti->sigma_per_ray;
    t.off_ray = ti->offset_per_ray;
    // with per-ray offsets, c0 is the centre of bin 0 before the offset (each ray adds its own)
    const double offset = ti->offset_per_ray ? 0.0 : (double)ti->center_offset;
    if (ti->lut) {  // tabulated kernel: sigma and n_sigmas are not used
        const double x0 = ti->lut_x0, dx = ti->lut_dx, x1 = x0 + (double)(ti->lut_n - 1) * dx;
        if (ti->lut_n < 2 || ti->lut_n > (1 << 24) || !std::isfinite(ti->lut_x0) || !std::isfinite(ti->lut_dx) ||
            !(ti->lut_dx > 0.0f) || !(std::fabs(x1) <= 3.0e38) ||  // the table's end must be a float
            ti->sigma_per_ray)                                      // the table fixes the kernel's shape
            return PP_EINVAL_TOF;
        t.bw = ti->bin_width;
        t.inv_bw = 1.0 / t.bw;
        t.c0 = -0.5 * (double)(ti->n_bins - 1) * t.bw + offset;
        t.hbw = (float)(0.5 * t.bw);
        t.u_per_mm = 1.0f;
        t.u_max = 1.0f;
        t.nsig = 1.0f;
        t.nb = ti->n_bins;
        t.lo = x0;
        t.hi = x1;
        t.win = std::fmax(std::fabs(x0), std::fabs(x1));
        t.lut = ti->lut;
        t.lut_n = ti->lut_n;
        t.lut_inv_dx = (float)(1.0 / dx);
        t.poly = 0;
        t.wpeak = 0.0f;
        return PP_OK;
    }
    if (!std::isfinite(ti->sigma) || !(ti->sigma > 0.0f) || !std::isfinite(ti->n_sigmas) || !(ti->n_sigmas > 0.0f))
        return PP_EINVAL_TOF;
    const double bw = ti->bin_width, sig = ti->sigma, ns = ti->n_sigmas;
    t.bw = bw;
    t.inv_bw = 1.0 / bw;
    t.c0 = -0.5 * (double)(ti->n_bins - 1) * bw + offset;
    t.hbw = (float)(0.5 * bw);
    const double erf_c = std::sqrt(1.0 / std::log(2.0));  // sqrt(log2 e), kErfC
    t.u_max = (float)(erf_c * ns / std::sqrt(2.0));
    t.nsig = ti->n_sigmas;
    t.win = ns * sig + 0.5 * bw;
    t.u_per_mm = (float)(erf_c / (std::sqrt(2.0) * sig));
    t.wpeak = (float)std::erf(std::fmin(0.5 * bw, ns * sig) / (std::sqrt(2.0) * sig));
    t.nb = ti->n_bins;
    t.lo = -t.win;
    t.hi = t.win;
    t.lut = nullptr;
    t.lut_n = 0;
    t.lut_inv_dx = 0.0f;
    fit_tof_poly(t, sig, ns, bw);
    return PP_OK;
}

// Resolution-model taps (definition in ppmi.h at pp_gauss3d); fwhm == NULL: no blur.
int make_gauss(const float* fwhm, const GeomK& g, GaussK& k) {
    for (int a = 0; a < 3; ++a) {
        const double f = fwhm ? (double)fwhm[a] : 0.0;
        if (!std::isfinite(f) || f < 0.0) return PP_EINVAL_RES;
        for (int i = 0; i < 2 * kGaussMaxR + 1; ++i) k.w[a][i] = 0.0f;
        if (f == 0.0) {
            k.r[a] = 0;
            k.w[a][kGaussMaxR] = 1.0f;
            continue;
        }
        const double sig = f / (2.0 * std::sqrt(2.0 * std::log(2.0))) / g.h[a];
        const double rr = std::floor(4.0 * sig + 0.5);
        if (!(rr <= kGaussMaxR)) return PP_EINVAL_RES;
        const int r = (int)rr;
        double w[2 * kGaussMaxR + 1], sum = 0.0;
        for (int i = -r; i <= r; ++i) sum += (w[i + r] = std::exp(-(double)i * i / (2.0 * sig * sig)));
        for (int i = 0; i <= 2 * r; ++i) k.w[a][kGaussMaxR - r + i] = (float)(w[i] / sum);
        k.r[a] = r;
    }
    return PP_OK;
}

bool overlap(const void* a, const void* b, int64_t bytes) {
    const char* p = static_cast<const char*>(a);
    const char* q = static_cast<const char*>(b);
    return p < q + bytes && q < p + bytes;
}

// [a, a + a_bytes) and [b, b + b_bytes) share a byte
bool overlap2(const void* a, int64_t a_bytes, const void* b, int64_t b_bytes) {
    const char* p = static_cast<const char*>(a);
    const char* q = static_cast<const char*>(b);
    return p < q + b_bytes && q < p + a_bytes;
}

// grid limit: 2^31 - 1 workgroups of >= 64 threads
constexpr int64_t kMaxRays = ((int64_t(1) << 31) - 1) * 64;

int check_n(int64_t n) { return (n < 0 || n > kMaxRays) ? PP_EINVAL_N : PP_OK; }

// TOF sinogram calls: the sheet back projection carries ray indices in 32 bits
int check_n_sino(int64_t n) { return (n < 0 || n >= (int64_t(1) << 31)) ? PP_EINVAL_N : PP_OK; }

hipStream_t as_stream(void* s) { return reinterpret_cast<hipStream_t>(s); }

RaySrc coords(const float* xs, const float* xe) { return RaySrc{xs, xe, nullptr, 0}; }

// Crystal-index events: table and pairs checked (pointers when n > 0, alignment of the pairs).
int crystals(const float* xyz, int32_t n_crystals, const int32_t* pair, int64_t n, RaySrc& src) {
    if (n_crystals < 1) return PP_EINVAL_N;
    if (n > 0 && (!xyz || !pair || (reinterpret_cast<uintptr_t>(pair) & 7u) != 0)) return PP_EINVAL_PTR;
    src = RaySrc{xyz, nullptr, reinterpret_cast<const int2*>(pair), n_crystals};
    return PP_OK;
}

int device_cus() {
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 256;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0) return 256;
    return cus;
}

}  // namespace

#define PP_TRY(expr)                   \
    do {                               \
        int _rc = (expr);              \
        if (_rc != PP_OK) return _rc;  \
    } while (0)

extern "C" {

int pp_abi_version(void) { return PP_ABI_VERSION; }

const char* pp_strerror(int code) {
    switch (code) {
        case PP_OK: return "ok";
        case PP_EINVAL_PTR: return "a required pointer is NULL";
        case PP_EINVAL_GEOM: return "invalid image geometry (dim <= 0, >= 2^30 voxels, voxsize <= 0 or non-finite)";
        case PP_EINVAL_TOF:
            return "invalid TOF parameters (n_bins not in [1,256], width/sigma/n_sigmas <= 0, bad table, or per-ray "
                   "parameters where unsupported)";
        case PP_EINVAL_N: return "count or slot argument out of range";
        case PP_EHIP: return g_hip_msg[0] ? g_hip_msg : "HIP launch error";
        case PP_EINVAL_RES: return "invalid resolution model (FWHM < 0 or non-finite, or radius > 31 voxels)";
        default: return "unknown status code";
    }
}

int pp_fwd(const float* xstart, const float* xend, int64_t n, const pp_image_t* geom, const float* img, float* p,
           const int32_t* order, void* stream) {
    GeomK g;
    PP_TRY(make_geom(geom, g));
    PP_TRY(check_n(n));
    if (n == 0) return PP_OK;
    if (!xstart || !xend || !img || !p) return PP_EINVAL_PTR;
    return hip_status(launch_fwd(coords(xstart, xend), n, g, img, p, order, as_stream(stream)));
}

int pp_back(const float* xstart, const float* xend, int64_t n, const pp_image_t* geom, float* img, const float* p,
            const int32_t* order, void* stream) {
    GeomK g;
    PP_TRY(make_geom(geom, g));
    PP_TRY(check_n(n));
    if (n == 0) return PP_OK;
    if (!xstart || !xend || !img || !p) return PP_EINVAL_PTR;
    return hip_status(launch_back(coords(xstart, xend), n, g, img, p, order, as_stream(stream)));
}

int pp_fwd_tof_sino(const float* xstart, const float* xend, int64_t n, const pp_image_t* geom, const pp_tof_t* tof,
                    const float* img, float* p, void* stream) {
    GeomK g;
    TofK t;
    PP_TRY(make_geom(geom, g));
    PP_TRY(make_tof(tof, t));
    PP_TRY(check_n_sino(n));
    if (n == 0) return PP_OK;
    if (!xstart || !xend || !img || !p) return PP_EINVAL_PTR;
    return hip_status(launch_fwd_tof_sino(coords(xstart, xend), n, g, t, img, p, as_stream(stream)));
}

int pp_back_tof_sino(const float* xstart, const float* xend, int64_t n, const pp_image_t* geom, const pp_tof_t* tof,
                     float* img, const float* p, void* stream) {
    GeomK g;
    TofK t;
    PP_TRY(make_geom(geom, g));
    PP_TRY(make_tof(tof, t));
    PP_TRY(check_n_sino(n));
    if (n == 0) return PP_OK;
    if (!xstart || !xend || !img || !p) return PP_EINVAL_PTR;
    return hip_status(launch_back_tof_sino(coords(xstart, xend), n, g, t, img, p, as_stream(stream)));
}

int pp_fwd_tof_lm(const float* xstart, const float* xend, const int16_t* tof_bin, int64_t n, const pp_image_t* geom,
                  const pp_tof_t* tof, const float* img, float* p, const int32_t* order, void* stream) {
    GeomK g;
    TofK t;
    PP_TRY(make_geom(geom, g));
    PP_TRY(make_tof(tof, t));
    PP_TRY(check_n(n));
    if (n == 0) return PP_OK;
    if (!xstart || !xend || !tof_bin || !img || !p) return PP_EINVAL_PTR;
    return hip_status(launch_fwd_tof_lm(coords(xstart, xend), tof_bin, n, g, t, img, p, order, as_stream(stream)));
}

int pp_fwd_tof_lm_gather(const float* xstart, const float* xend, const int16_t* tof_bin, int64_t n,
                         const pp_image_t* geom, const pp_tof_t* tof, const float* img, float* p, const int32_t* order,
                         float* xstart_out, float* xend_out, int16_t* tof_bin_out, float* p_out, void* stream) {
    GeomK g;
    TofK t;
    PP_TRY(make_geom(geom, g));
    PP_TRY(make_tof(tof, t));
    PP_TRY(check_n(n));
    if (t.sig_ray || t.off_ray) return PP_EINVAL_TOF;  // per-event TOF arrays are not reordered
    if (n == 0) return PP_OK;
    if (!xstart || !xend || !tof_bin || !img || !p || !order || !xstart_out || !xend_out || !tof_bin_out || !p_out)
        return PP_EINVAL_PTR;
    return hip_status(launch_fwd_tof_lm_gather(coords(xstart, xend), tof_bin, n, g, t, img, p, order,
                                               EventsOut{xstart_out, xend_out, tof_bin_out, p_out}, as_stream(stream)));
}

int pp_fwd_tof_lm_batch(const float* xstart, const float* xend, const int16_t* tof_bin, int64_t n,
                        const pp_image_t* geom, const pp_tof_t* tof, const float* imgs, int32_t n_img, float* p,
                        const int32_t* order, void* stream) {
    GeomK g;
    TofK t;
    PP_TRY(make_geom(geom, g));
    PP_TRY(make_tof(tof, t));
    PP_TRY(check_n(n));
    if (n_img < 0 || n_img > (1 << 20)) return PP_EINVAL_N;
    if (n == 0 || n_img == 0) return PP_OK;
    if (!xstart || !xend || !tof_bin || !imgs || !p) return PP_EINVAL_PTR;
    return hip_status(
        launch_fwd_tof_lm_batch(coords(xstart, xend), tof_bin, n, g, t, imgs, n_img, p, order, as_stream(stream)));
}

int pp_back_tof_lm_batch(const float* xstart, const float* xend, const int16_t* tof_bin, int64_t n,
                         const pp_image_t* geom, const pp_tof_t* tof, float* imgs, int32_t n_img, const float* p,
                         const int32_t* order, void* stream) {
    GeomK g;
    TofK t;
    PP_TRY(make_geom(geom, g));
    PP_TRY(make_tof(tof, t));
    PP_TRY(check_n(n));
    if (n_img < 0 || n_img > (1 << 20)) return PP_EINVAL_N;
    if (n == 0 || n_img == 0) return PP_OK;
    if (!xstart || !xend || !tof_bin || !imgs || !p) return PP_EINVAL_PTR;
    return hip_status(
        launch_back_tof_lm_batch(coords(xstart, xend), tof_bin, n, g, t, imgs, n_img, p, order, as_stream(stream)));
}

int pp_back_tof_lm(const float* xstart, const float* xend, const int16_t* tof_bin, int64_t n, const pp_image_t* geom,
                   const pp_tof_t* tof, float* img, const float* p, const int32_t* order, void* stream) {
    GeomK g;
    TofK t;
    PP_TRY(make_geom(geom, g));
    PP_TRY(make_tof(tof, t));
    PP_TRY(check_n(n));
    if (n == 0) return PP_OK;
    if (!xstart || !xend || !tof_bin || !img || !p) return PP_EINVAL_PTR;
    return hip_status(launch_back_tof_lm(coords(xstart, xend), tof_bin, n, g, t, img, p, order, as_stream(stream)));
}

int pp_count_samples(const float* xstart, const float* xend, const int16_t* tof_bin, int64_t n, const pp_image_t* geom,
                     const pp_tof_t* tof, int32_t* counts, void* stream) {
    GeomK g;
    TofK t{};
    PP_TRY(make_geom(geom, g));
    if (tof_bin) PP_TRY(make_tof(tof, t));
    PP_TRY(check_n(n));
    if (n == 0) return PP_OK;
    if (!xstart || !xend || !counts) return PP_EINVAL_PTR;
    return hip_status(launch_count(coords(xstart, xend), tof_bin, n, g, t, counts, as_stream(stream)));
}

int pp_tof_gaussian_table(const pp_tof_t* tof, float dx_max, float* lut, int32_t capacity, int32_t* n_out,
                          float* x0_out, float* dx_out, void* stream) {
    if (!tof) return PP_EINVAL_PTR;
    const double bw = tof->bin_width, sig = tof->sigma, ns = tof->n_sigmas;
    if (!(std::isfinite(bw) && bw > 0.0 && std::isfinite(sig) && sig > 0.0 && std::isfinite(ns) && ns > 0.0))
        return PP_EINVAL_TOF;
    if (!(std::isfinite(dx_max) && dx_max > 0.0f)) return PP_EINVAL_N;
    const double win = ns * sig + 0.5 * bw;
    const double cells = std::ceil(2.0 * win / (double)dx_max);
    if (!(cells + 1.0 <= (double)(1 << 24))) return PP_EINVAL_N;
    const int n = (int)cells + 1;
    // the nodes are placed where the projectors will interpolate them: at the float32 origin and
    // spacing that pp_tof_t carries
    const float x0 = (float)(-win), dx = (float)(2.0 * win / (double)(n - 1));
    if (n_out) *n_out = n;
    if (x0_out) *x0_out = x0;
    if (dx_out) *dx_out = dx;
    if (!lut) return PP_OK;
    if (capacity < n) return PP_EINVAL_N;
    return hip_status(launch_tof_gauss_table(lut, n, (double)x0, (double)dx, bw, sig, ns, as_stream(stream)));
}

int pp_tof_weight_form(const pp_tof_t* tof, int32_t* form) {
    TofK t;
    PP_TRY(make_tof(tof, t));
    if (!form) return PP_EINVAL_PTR;
    *form = tof_form(t);
    return PP_OK;
}

int pp_fwd_crystals(const float* crystal_xyz, int32_t n_crystals, const int32_t* pair, int64_t n,
                    const pp_image_t* geom, const float* img, float* p, const int32_t* order, void* stream) {
    GeomK g;
    RaySrc src;
    PP_TRY(make_geom(geom, g));
    PP_TRY(check_n(n));
    PP_TRY(crystals(crystal_xyz, n_crystals, pair, n, src));
    if (n == 0) return PP_OK;
    if (!img || !p) return PP_EINVAL_PTR;
    return hip_status(launch_fwd(src, n, g, img, p, order, as_stream(stream)));
}

int pp_back_crystals(const float* crystal_xyz, int32_t n_crystals, const int32_t* pair, int64_t n,
                     const pp_image_t* geom, float* img, const float* p, const int32_t* order, void* stream) {
    GeomK g;
    RaySrc src;
    PP_TRY(make_geom(geom, g));
    PP_TRY(check_n(n));
    PP_TRY(crystals(crystal_xyz, n_crystals, pair, n, src));
    if (n == 0) return PP_OK;
    if (!img || !p) return PP_EINVAL_PTR;
    return hip_status(launch_back(src, n, g, img, p, order, as_stream(stream)));
}

int pp_fwd_tof_lm_crystals(const float* crystal_xyz, int32_t n_crystals, const int32_t* pair, const int16_t* tof_bin,
                           int64_t n, const pp_image_t* geom, const pp_tof_t* tof, const float* img, float* p,
                           const int32_t* order, void* stream) {
    GeomK g;
    TofK t;
    RaySrc src;
    PP_TRY(make_geom(geom, g));
    PP_TRY(make_tof(tof, t));
    PP_TRY(check_n(n));
    PP_TRY(crystals(crystal_xyz, n_crystals, pair, n, src));
    if (n == 0) return PP_OK;
    if (!tof_bin || !img || !p) return PP_EINVAL_PTR;
    return hip_status(launch_fwd_tof_lm(src, tof_bin, n, g, t, img, p, order, as_stream(stream)));
}

int pp_back_tof_lm_crystals(const float* crystal_xyz, int32_t n_crystals, const int32_t* pair, const int16_t* tof_bin,
                            int64_t n, const pp_image_t* geom, const pp_tof_t* tof, float* img, const float* p,
                            const int32_t* order, void* stream) {
    GeomK g;
    TofK t;
    RaySrc src;
    PP_TRY(make_geom(geom, g));
    PP_TRY(make_tof(tof, t));
    PP_TRY(check_n(n));
    PP_TRY(crystals(crystal_xyz, n_crystals, pair, n, src));
    if (n == 0) return PP_OK;
    if (!tof_bin || !img || !p) return PP_EINVAL_PTR;
    return hip_status(launch_back_tof_lm(src, tof_bin, n, g, t, img, p, order, as_stream(stream)));
}

int pp_count_samples_crystals(const float* crystal_xyz, int32_t n_crystals, const int32_t* pair,
                              const int16_t* tof_bin, int64_t n, const pp_image_t* geom, const pp_tof_t* tof,
                              int32_t* counts, void* stream) {
    GeomK g;
    TofK t{};
    RaySrc src;
    PP_TRY(make_geom(geom, g));
    if (tof_bin) PP_TRY(make_tof(tof, t));
    PP_TRY(check_n(n));
    PP_TRY(crystals(crystal_xyz, n_crystals, pair, n, src));
    if (n == 0) return PP_OK;
    if (!counts) return PP_EINVAL_PTR;
    return hip_status(launch_count(src, tof_bin, n, g, t, counts, as_stream(stream)));
}

int pp_lm_presort_crystals(const float* crystal_xyz, int32_t n_crystals, const int32_t* pair, const int16_t* tof_bin,
                           int64_t n, const pp_image_t* geom, const pp_tof_t* tof, int32_t n_sub, int32_t* order,
                           void* workspace, size_t workspace_bytes, void* stream) {
    GeomK g;
    TofK t{};
    RaySrc src;
    PP_TRY(make_geom(geom, g));
    if (tof_bin) PP_TRY(make_tof(tof, t));
    if (n < 0 || n > INT32_MAX || n_sub < 1 || n_sub > 4096) return PP_EINVAL_N;
    PP_TRY(crystals(crystal_xyz, n_crystals, pair, n, src));
    if (n == 0) return PP_OK;
    if (!order || !workspace) return PP_EINVAL_PTR;
    if (workspace_bytes < presort_workspace_bytes(n)) return PP_EINVAL_N;
    return hip_status(launch_presort(src, tof_bin, n, g, tof_bin ? t.nb : 1, n_sub, order, workspace, workspace_bytes,
                                     as_stream(stream)));
}

int pp_gather_crystal_events(const int32_t* pair, const int16_t* tof_bin, const int32_t* order, int64_t n,
                             int32_t* pair_out, int16_t* tof_bin_out, void* stream) {
    if (n < 0 || n > INT32_MAX) return PP_EINVAL_N;
    if (n == 0) return PP_OK;
    if (!pair || !order || !pair_out || (tof_bin && !tof_bin_out)) return PP_EINVAL_PTR;
    if (((reinterpret_cast<uintptr_t>(pair) | reinterpret_cast<uintptr_t>(pair_out)) & 7u) != 0) return PP_EINVAL_PTR;
    return hip_status(launch_gather_pairs(pair, tof_bin, order, n, pair_out, tof_bin_out, as_stream(stream)));
}

size_t pp_lm_presort_workspace_bytes(int64_t n) {
    if (n <= 0 || n > INT32_MAX) return 0;
    return presort_workspace_bytes(n);
}

int pp_lm_presort(const float* xstart, const float* xend, const int16_t* tof_bin, int64_t n, const pp_image_t* geom,
                  const pp_tof_t* tof, int32_t n_sub, int32_t* order, void* workspace, size_t workspace_bytes,
                  void* stream) {
    GeomK g;
    TofK t{};
    PP_TRY(make_geom(geom, g));
    if (tof_bin) PP_TRY(make_tof(tof, t));
    if (n < 0 || n > INT32_MAX || n_sub < 1 || n_sub > 4096) return PP_EINVAL_N;
    if (n == 0) return PP_OK;
    if (!xstart || !xend || !order || !workspace) return PP_EINVAL_PTR;
    if (workspace_bytes < presort_workspace_bytes(n)) return PP_EINVAL_N;
    return hip_status(launch_presort(coords(xstart, xend), tof_bin, n, g, tof_bin ? t.nb : 1, n_sub, order, workspace,
                                     workspace_bytes, as_stream(stream)));
}

int pp_lm_presort_noalloc(const float* xstart, const float* xend, const int16_t* tof_bin, int64_t n,
                          const pp_image_t* geom, const pp_tof_t* tof, int32_t n_sub, int32_t* order, void* stream) {
    GeomK g;
    TofK t{};
    PP_TRY(make_geom(geom, g));
    if (tof_bin) PP_TRY(make_tof(tof, t));
    if (n < 0 || n > INT32_MAX || n_sub < 1 || n_sub > 4096) return PP_EINVAL_N;
    if (n == 0) return PP_OK;
    if (!xstart || !xend || !order) return PP_EINVAL_PTR;
    const size_t need = presort_workspace_bytes(n);
    if (need == 0 || need > kPresortScratchBytes) return PP_EINVAL_N;
    void* ws = nullptr;
    hipError_t e = presort_scratch(&ws);
    if (e != hipSuccess) return hip_status(e);
    return hip_status(launch_presort(coords(xstart, xend), tof_bin, n, g, tof_bin ? t.nb : 1, n_sub, order, ws,
                                     kPresortScratchBytes, as_stream(stream)));
}

int pp_gather_events(const float* xstart, const float* xend, const int16_t* tof_bin, const int32_t* order, int64_t n,
                     float* xstart_out, float* xend_out, int16_t* tof_bin_out, void* stream) {
    if (n < 0 || n > INT32_MAX) return PP_EINVAL_N;
    if (n == 0) return PP_OK;
    if (!xstart || !xend || !order || !xstart_out || !xend_out || (tof_bin && !tof_bin_out)) return PP_EINVAL_PTR;
    return hip_status(launch_gather_events(xstart, xend, tof_bin, order, n, xstart_out, xend_out, tof_bin_out,
                                           as_stream(stream)));
}

int pp_osem_init(float* x, const float* sens, int64_t n_vox, void* stream) {
    if (n_vox < 0 || n_vox > (int64_t(1) << 30)) return PP_EINVAL_N;
    if (n_vox == 0) return PP_OK;
    if (!x || !sens) return PP_EINVAL_PTR;
    return hip_status(launch_osem_init(x, sens, n_vox, as_stream(stream)));
}

int64_t pp_osem_chunks(int64_t n_events, int32_t n_sub) { return osem_chunks(n_events, n_sub); }

int pp_lm_osem_subset_batched(const pp_frame_desc_t* d_slots, int32_t n_slots, const pp_image_t* geom,
                          const pp_tof_t* tof, void* stream) {
    GeomK g;
    TofK t;
    PP_TRY(make_geom(geom, g));
    PP_TRY(make_tof(tof, t));
    if (t.sig_ray || t.off_ray) return PP_EINVAL_TOF;  // one kernel for every slot
    if (n_slots < 0 || n_slots > (1 << 20)) return PP_EINVAL_N;
    if (n_slots == 0) return PP_OK;
    if (!d_slots) return PP_EINVAL_PTR;
    return hip_status(launch_osem_accumulate(d_slots, n_slots, g, t, device_cus(), as_stream(stream)));
}

int pp_osem_update_batched(pp_frame_desc_t* d_slots, int32_t n_slots, const pp_image_t* geom, const float* res_fwhm,
                      void* stream) {
    GeomK g;
    GaussK k;
    PP_TRY(make_geom(geom, g));
    PP_TRY(make_gauss(res_fwhm, g, k));
    if (n_slots < 0 || n_slots > (1 << 20)) return PP_EINVAL_N;
    if (n_slots == 0) return PP_OK;
    if (!d_slots) return PP_EINVAL_PTR;
    const int64_t n_vox = (int64_t)g.n[0] * g.n[1] * g.n[2];
    int64_t blocks = (n_vox + 255) / 256;  // per slot
    const int cus = device_cus();
    const int64_t cap = (int64_t)cus * 4;
    if (blocks > cap) blocks = cap;
    hipStream_t s = as_stream(stream);
    // slots without the model: plain update; slots with it: the blur passes with the fused update;
    // then every updated slot advances
    hipError_t e = launch_osem_update(d_slots, n_slots, n_vox, (int)blocks, s);
    if (e == hipSuccess) e = launch_osem_res_update(d_slots, n_slots, g, k, cus, s);
    if (e == hipSuccess) e = launch_osem_advance(d_slots, n_slots, s);
    return hip_status(e);
}

int pp_tof_sino_sensitivity(const float* xstart, const float* xend, int64_t n_lors, const pp_image_t* geom,
                            const pp_tof_t* tof, float* sens, float* work, int64_t work_lors, void* stream) {
    GeomK g;
    TofK t;
    PP_TRY(make_geom(geom, g));
    PP_TRY(make_tof(tof, t));
    if (t.sig_ray || t.off_ray) return PP_EINVAL_TOF;
    PP_TRY(check_n(n_lors));
    if (work_lors < 1 || work_lors >= (int64_t(1) << 31)) return PP_EINVAL_N;
    if (n_lors == 0) return PP_OK;
    if (!xstart || !xend || !sens || !work) return PP_EINVAL_PTR;
    return hip_status(launch_tof_sino_sensitivity(xstart, xend, n_lors, g, t, sens, work, work_lors, as_stream(stream)));
}

int pp_tof_sino_osem_subset(const float* xstart, const float* xend, const float* y, int64_t n_lors,
                            const pp_image_t* geom, const pp_tof_t* tof, float bg, float* x, float* acc,
                            int32_t n_shards, const float* sens, float* work, int64_t work_lors, void* stream) {
    GeomK g;
    TofK t;
    PP_TRY(make_geom(geom, g));
    PP_TRY(make_tof(tof, t));
    if (t.sig_ray || t.off_ray) return PP_EINVAL_TOF;
    PP_TRY(check_n(n_lors));
    if (n_shards < 1 || n_shards > 1024 || work_lors < 1 || work_lors >= (int64_t(1) << 31) || !std::isfinite(bg))
        return PP_EINVAL_N;
    if (!x || !acc || !sens || (n_lors > 0 && (!xstart || !xend || !y || !work))) return PP_EINVAL_PTR;
    const int64_t vb = (int64_t)g.n[0] * g.n[1] * g.n[2] * (int64_t)sizeof(float), ab = vb * n_shards;
    const int64_t wb = work_lors * t.nb * (int64_t)sizeof(float);
    if (overlap2(x, vb, acc, ab) || overlap2(x, vb, sens, vb) || overlap2(acc, ab, sens, vb) ||
        (n_lors > 0 && (overlap2(work, wb, x, vb) || overlap2(work, wb, acc, ab) || overlap2(work, wb, sens, vb))))
        return PP_EINVAL_PTR;
    return hip_status(launch_tof_sino_osem_subset(xstart, xend, y, n_lors, g, t, bg, x, acc, n_shards, sens, work,
                                                  work_lors, device_cus(), as_stream(stream)));
}

int pp_gauss3d(const float* src, float* dst, float* tmp, const pp_image_t* geom, const float* fwhm, void* stream) {
    GeomK g;
    GaussK k;
    PP_TRY(make_geom(geom, g));
    if (!src || !dst || !tmp || !fwhm) return PP_EINVAL_PTR;
    PP_TRY(make_gauss(fwhm, g, k));
    const int64_t bytes = (int64_t)g.n[0] * g.n[1] * g.n[2] * (int64_t)sizeof(float);
    if (overlap(src, dst, bytes) || overlap(src, tmp, bytes) || overlap(dst, tmp, bytes)) return PP_EINVAL_PTR;
    return hip_status(launch_gauss3d(src, dst, tmp, g, k, device_cus(), as_stream(stream)));
}

int pp_poisson_nll(const float* p, float bg, const float* y, int64_t n, float* grad, double* partial,
                   int32_t n_partial, void* stream) {
    if (n < 0 || n_partial < 1 || n_partial > 65536) return PP_EINVAL_N;
    if (!std::isfinite(bg)) return PP_EINVAL_N;
    if (!partial || (n > 0 && (!p || !y || !grad))) return PP_EINVAL_PTR;
    return hip_status(launch_poisson_nll(p, bg, y, n, grad, partial, n_partial, as_stream(stream)));
}

int pp_fill(float* dst, int64_t n, float value, void* stream) {
    if (n < 0) return PP_EINVAL_N;
    if (n == 0) return PP_OK;
    if (!dst) return PP_EINVAL_PTR;
    return hip_status(launch_fill(dst, n, value, as_stream(stream)));
}

}  // extern "C"
