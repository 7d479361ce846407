// Device-side Joseph traversal shared by every projector kernel.
//
// Forward and back projection kernels call the same setup and stencil code,
// so each back projection is the exact transpose of its forward projection
// (the matched pair of Sec. 2.2 of the paper).
//
// Precision: image values, interpolation weights, TOF weights and sums are
// float32.  The ray geometry (plane range, intersection point of every plane,
// TOF position of every sample) is float64: positions reach ~250 voxel units
// at clinical sizes, where float32 would put ~2e-5 voxel of error into every
// interpolation weight; in float64 a single FMA per plane gives the
// intersection directly (no running sums), exact to ~1e-13 voxel.
#pragma once

#include <hip/hip_runtime.h>
#include <float.h>
#include <limits.h>
#include <stdint.h>

namespace ppmi {

struct GeomK {
    double o[3];   // centre of voxel (0,0,0), mm
    double h[3];   // voxel size, mm
    int n[3];      // voxels per axis
    int stride[3]; // element strides (n1*n2, n2, 1)
};

// Degrees of the two polynomial pieces of the Gaussian bin weight (tof_poly).
constexpr int kPolyCentral = 8;
constexpr int kPolyTail = 7;

struct TofK {
    double bw;            // bin width, mm
    double inv_bw;        // 1 / bw
    double c0;            // centre of bin 0, mm: -(n_bins - 1)/2 * bw + offset
    double win;           // half support of a bin's weight: n_sigmas * sigma + bw / 2
    double lo, hi;        // support of a bin's weight relative to its centre (table: its range)
    const float* lut;     // tabulated bin weight at lo + i * dx, or nullptr (Gaussian)
    int lut_n;
    float lut_inv_dx;
    float hbw;            // bw / 2, mm
    float u_per_mm;       // kErfC / (sqrt(2) sigma): the scaled erf argument (erf_scaled) per mm
    float u_max;          // kErfC n_sigmas / sqrt(2): the truncation in units of that argument
    float nsig;           // n_sigmas
    float wpeak;          // the Gaussian bin weight's largest value, w(0) (0 with a table)
    int nb;               // bins
    const float* sig_ray; // sigma of each ray (mm), or nullptr: every ray has sigma
    const float* off_ray; // centre offset of each ray (mm), or nullptr: c0 holds the offset
    // The Gaussian bin weight w(x) as two polynomials of y = |x| (tof_poly), fitted on the host;
    // poly == 0 when the fit missed its error bound (the erf form is used then).
    int poly;
    float pk1, pk2;            // pieces: y < pk1 central, pk1 <= y < pk2 tail, 0 beyond
    float pq1;                 // central variable (y pq1)^2 - 1 = 2 y^2 / k1^2 - 1 (pq1 = sqrt(2) / k1)
    float pa2, pb2;            // tail variable y pa2 + pb2; both variables in [-1, 1] on their piece
    float pc[kPolyCentral + 1];  // central polynomial, pc[i] the coefficient of the i-th power
    float pt[kPolyTail + 1];     // tail polynomial
};

constexpr float kErfC = 1.2011224087864498f;  // sqrt(log2(e)): scale of the erf argument (erf_scaled)

// Resolution-model blur taps per axis: tap i of axis a at w[a][i + kGaussMaxR] (centred, so that a
// tap's offset is a compile-time index when i is), 0 for |i| > r[a].
constexpr int kGaussMaxR = 31;
struct GaussK {
    int r[3];
    float w[3][2 * kGaussMaxR + 1];
};

// A ray prepared for plane stepping along its principal axis p.
struct RayK {
    double U0, dU;  // in-plane voxel coordinate along axis u at plane k: U0 + k dU
    double W0, dW;  // same along axis w
    double s0, ds;  // TOF position (mm from midpoint, towards end) at plane k: s0 + k ds
    int k_lo, k_hi; // planes to visit, inclusive (empty if k_lo > k_hi)
    int sp, su, sw; // element strides of axes p, u, w
    int nu, nw;     // grid size along u, w
    int p;          // principal axis
    float ell;      // ray length per plane step, mm (incidence-angle correction)
};

__device__ __forceinline__ int clamp_plane(double v, int lo, int hi) {
    // conservative conversion of a real plane bound to an int in [lo - 1, hi + 1]
    v = fmin(fmax(v, (double)lo - 1.0), (double)hi + 1.0);
    return (int)v;
}

// Restrict [lo, hi] to the planes k whose coordinate a0 + k da lies in (amin, amax).
// Conservative by one plane on each side; exact filtering happens per sample.
__device__ __forceinline__ void clip_affine(double a0, double da, double amin, double amax, int& lo, int& hi) {
    if (da == 0.0) {
        if (!(a0 > amin && a0 < amax)) hi = lo - 1;
        return;
    }
    double k1 = (amin - a0) / da;
    double k2 = (amax - a0) / da;
    double kmin = fmin(k1, k2), kmax = fmax(k1, k2);
    int a = clamp_plane(floor(kmin), lo, hi);
    int b = clamp_plane(ceil(kmax), lo, hi);
    lo = max(lo, a);
    hi = min(hi, b);
}

// Set up ray (xs -> xe).  Returns false if it contributes nothing.
__device__ __forceinline__ bool ray_setup(const float* __restrict__ xs, const float* __restrict__ xe,
                                          const GeomK& g, RayK& r) {
    float s32[3], e32[3], d32[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        s32[a] = xs[a];
        e32[a] = xe[a];
        d32[a] = e32[a] - s32[a];
    }
    bool finite = true;
#pragma unroll
    for (int a = 0; a < 3; ++a) finite &= isfinite(s32[a]) && isfinite(e32[a]);
    if (!finite) return false;
    // principal axis: largest |d| in mm, first axis on ties (float32 comparison)
    int p = 0;
    if (fabsf(d32[1]) > fabsf(d32[p])) p = 1;
    if (fabsf(d32[2]) > fabsf(d32[p])) p = 2;
    if (d32[p] == 0.0f) return false;
    const int u = (p == 0) ? 1 : 0;
    const int w = (p == 2) ? 1 : 2;
    double d[3], S[3], D[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        d[a] = (double)e32[a] - (double)s32[a];
        S[a] = ((double)s32[a] - g.o[a]) / g.h[a];
        D[a] = d[a] / g.h[a];
    }
    const double len = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
    const double Sp = S[p], Dp = D[p];
    r.dU = D[u] / Dp;
    r.dW = D[w] / Dp;
    r.U0 = S[u] - Sp * r.dU;
    r.W0 = S[w] - Sp * r.dW;
    r.ds = len / Dp;
    r.s0 = -Sp * r.ds - 0.5 * len;
    r.ell = (float)(g.h[p] * len / fabs(d[p]));
    r.sp = g.stride[p];
    r.su = g.stride[u];
    r.sw = g.stride[w];
    r.nu = g.n[u];
    r.nw = g.n[w];
    r.p = p;
    // planes on the segment: t = (k - Sp) / Dp in [0, 1]
    const double ka = fmin(Sp, Sp + Dp), kb = fmax(Sp, Sp + Dp);
    int lo = 0, hi = g.n[p] - 1;
    lo = max(lo, clamp_plane(ceil(ka), 0, g.n[p] - 1));
    hi = min(hi, clamp_plane(floor(kb), 0, g.n[p] - 1));
    // planes whose 2x2 stencil can touch the grid: U in [-1, nu), W in [-1, nw)
    clip_affine(r.U0, r.dU, -1.0 - 1e-9, (double)r.nu + 1e-9, lo, hi);
    clip_affine(r.W0, r.dW, -1.0 - 1e-9, (double)r.nw + 1e-9, lo, hi);
    r.k_lo = lo;
    r.k_hi = hi;
    return lo <= hi;
}

// Where the rays' end points come from: lists of coordinates (xs, xe: [n][3] mm), or pairs of
// crystal indices (pair: [n] of (start, end)) into a table of crystal positions (xs = the table
// [nc][3], xe unused).  A crystal index outside [0, nc) makes its ray contribute nothing.
struct RaySrc {
    const float* xs;
    const float* xe;
    const int2* pair;
    int nc;
    __device__ __forceinline__ bool ends(int64_t l, const float*& s, const float*& e) const {
        if (!pair) {
            s = xs + 3 * l;
            e = xe + 3 * l;
            return true;
        }
        const int2 ab = pair[l];
        if ((unsigned)ab.x >= (unsigned)nc || (unsigned)ab.y >= (unsigned)nc) return false;
        s = xs + 3 * (int64_t)ab.x;
        e = xs + 3 * (int64_t)ab.y;
        return true;
    }
    // the rays from position k on
    __host__ __device__ RaySrc from(int64_t k) const {
        return pair ? RaySrc{xs, xe, pair + k, nc} : RaySrc{xs + 3 * k, xe + 3 * k, nullptr, 0};
    }
};

__device__ __forceinline__ bool ray_setup(const RaySrc& src, int64_t l, const GeomK& g, RayK& r) {
    const float *s, *e;
    return src.ends(l, s, e) && ray_setup(s, e, g, r);
}

// The TOF parameters of one ray.  Without per-ray arrays these are the kernel's; with them
// ray l has its own width (sigma_l, same n_sigmas) and/or its own centre offset, which is
// folded into the ray's TOF coordinate (s0 -= shift) so that bin centres stay c0 + b bw.
struct TofRay {
    double shift;   // the ray's centre offset (0 without per-ray offsets: c0 holds it)
    double lo, hi;  // support of a bin's weight relative to its centre
    float inv;      // kErfC / (sqrt(2) sigma_l), the erf argument per mm
};

// kErfC / (sqrt(2) sigma) of a per-ray sigma (sigma below 1e-30 mm taken as 1e-30 mm, a kernel far
// narrower than any voxel, so that the product never overflows)
__device__ __forceinline__ float tof_inv_sigma(float sigma) {
    return kErfC / (1.41421356f * fmaxf(sigma, 1e-30f));
}

// Parameters of ray l; false if its per-ray entries are unusable (sigma not a positive
// finite number, offset not finite): the ray contributes nothing.
template <bool PerRay>
__device__ __forceinline__ bool tof_ray(const TofK& t, int64_t l, TofRay& q) {
    q.shift = 0.0;
    q.lo = t.lo;
    q.hi = t.hi;
    q.inv = t.u_per_mm;
    if (!PerRay) return true;
    if (t.sig_ray) {
        const float sg = t.sig_ray[l];
        if (!(sg > 0.0f && sg <= FLT_MAX)) return false;
        q.inv = tof_inv_sigma(sg);
        q.hi = (double)t.nsig * (double)sg + 0.5 * t.bw;
        q.lo = -q.hi;
    }
    if (t.off_ray) {
        const float o = t.off_ray[l];
        if (!(fabsf(o) <= FLT_MAX)) return false;
        q.shift = o;
    }
    return true;
}

// Plane range of the ray restricted to the support of one bin (centre + [lo, hi]).
__device__ __forceinline__ bool tof_window(RayK& r, double centre, double lo_x, double hi_x) {
    int lo = r.k_lo, hi = r.k_hi;
    clip_affine(r.s0, r.ds, centre + lo_x, centre + hi_x, lo, hi);
    r.k_lo = lo;
    r.k_hi = hi;
    return lo <= hi;
}

// The same, then s(k) made relative to the bin centre (s0 -= centre): fma(k, ds, s0) is
// the signed distance of plane sample k from the centre, the argument of tof_weight.
__device__ __forceinline__ bool tof_window_rel(RayK& r, double centre, double lo_x, double hi_x) {
    const bool any = tof_window(r, centre, lo_x, hi_x);
    r.s0 -= centre;
    return any;
}

struct Stencil {
    int base;      // flat index of voxel (k, i0, j0)
    float fu, fw;  // fractional position inside the 2x2 cell
    bool i0ok, i1ok, j0ok, j1ok;
};

__device__ __forceinline__ Stencil stencil_at(const RayK& r, int k) {
    const double U = fma((double)k, r.dU, r.U0);
    const double W = fma((double)k, r.dW, r.W0);
    const double fi = floor(U), fj = floor(W);
    const int i0 = (int)fi, j0 = (int)fj;
    Stencil st;
    st.fu = (float)(U - fi);
    st.fw = (float)(W - fj);
    st.i0ok = (unsigned)i0 < (unsigned)r.nu;
    st.i1ok = (unsigned)(i0 + 1) < (unsigned)r.nu;
    st.j0ok = (unsigned)j0 < (unsigned)r.nw;
    st.j1ok = (unsigned)(j0 + 1) < (unsigned)r.nw;
    st.base = k * r.sp + i0 * r.su + j0 * r.sw;
    return st;
}

// The image as a raw buffer: loads take 32-bit byte offsets, and an offset at or beyond the
// image's end reads 0 (the hardware range check).  Neighbours outside the grid are given the
// offset 0xFFFFFFFF, so the zero padding of the stencil costs a select instead of a branch per
// neighbour.  Byte offsets fit 32 bits: grids hold fewer than 2^30 voxels.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t img_buffer(const float* img, const GeomK& g) {
    const unsigned bytes = (unsigned)g.n[0] * (unsigned)g.n[1] * (unsigned)g.n[2] * 4u;
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<float*>(img), (short)0, (int)bytes, 0x00020000);
}

__device__ __forceinline__ float img_load(__amdgpu_buffer_rsrc_t ib, bool ok, int idx) {
    return __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(ib, ok ? (unsigned)idx * 4u : 0xFFFFFFFFu, 0, 0));
}

// A raw buffer over `count` consecutive images of the grid (count * voxels * 4 < 2^32, checked on the
// host): stencil_gather_at reads image b of them at the offset b * image bytes.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t img_buffer_n(const float* img, const GeomK& g, int count) {
    const unsigned bytes = (unsigned)g.n[0] * (unsigned)g.n[1] * (unsigned)g.n[2] * 4u * (unsigned)count;
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<float*>(img), (short)0, (int)bytes, 0x00020000);
}

// The four neighbours of a sample, zero outside the grid.  When axis w is the contiguous one
// (stride 1: every ray whose principal axis is 0 or 1) and the grid has at least two voxels along
// it, each pair (j0, j0 + 1) of a row is read with one 8-byte load: at j0 when both are inside,
// one voxel earlier when only j0 is (the last voxel of the row), one later when only j0 + 1 is (the
// first), so that the load never leaves its row; four 4-byte loads otherwise.  Same values either
// way.  `base` is the flat index of voxel (k, i0, j0) in the buffer.  Pairs = false: always the four
// loads (kernels bound by arithmetic, where the per-sample choice costs more than the loads save).
template <bool Pairs = true>
__device__ __forceinline__ void stencil_load(__amdgpu_buffer_rsrc_t ib, const RayK& r, const Stencil& st, int base,
                                             float& v00, float& v01, float& v10, float& v11) {
    // the neighbours' indices as additions to the base (an empty asm keeps the compiler from
    // turning them back into products, which are quarter-rate instructions)
    asm volatile("" : "+v"(base));
    const int b10 = base + r.su;
    if (Pairs && r.sw == 1 && r.nw >= 2) {
        const int sh = st.j0ok ? (st.j1ok ? 0 : -1) : 1;
        const auto a = __builtin_amdgcn_raw_buffer_load_b64(ib, st.i0ok ? (unsigned)(base + sh) * 4u : 0xFFFFFFF0u, 0, 0);
        const auto c = __builtin_amdgcn_raw_buffer_load_b64(ib, st.i1ok ? (unsigned)(b10 + sh) * 4u : 0xFFFFFFF0u, 0, 0);
        v00 = st.i0ok && st.j0ok ? __uint_as_float(st.j1ok ? a[0] : a[1]) : 0.0f;
        v01 = st.i0ok && st.j1ok ? __uint_as_float(st.j0ok ? a[1] : a[0]) : 0.0f;
        v10 = st.i1ok && st.j0ok ? __uint_as_float(st.j1ok ? c[0] : c[1]) : 0.0f;
        v11 = st.i1ok && st.j1ok ? __uint_as_float(st.j0ok ? c[1] : c[0]) : 0.0f;
    } else {
        v00 = img_load(ib, st.i0ok && st.j0ok, base);
        v01 = img_load(ib, st.i0ok && st.j1ok, base + r.sw);
        v10 = img_load(ib, st.i1ok && st.j0ok, b10);
        v11 = img_load(ib, st.i1ok && st.j1ok, b10 + r.sw);
    }
}

// bilinear interpolation with zero padding
template <bool Pairs = true>
__device__ __forceinline__ float stencil_gather(__amdgpu_buffer_rsrc_t ib, const RayK& r, const Stencil& st) {
    float v00, v01, v10, v11;
    stencil_load<Pairs>(ib, r, st, st.base, v00, v01, v10, v11);
    const float gu = 1.0f - st.fu, gw = 1.0f - st.fw;
    return gu * (gw * v00 + st.fw * v01) + st.fu * (gw * v10 + st.fw * v11);
}

// stencil_gather of the image that starts `img_off` voxels into the buffer (same arithmetic)
template <bool Pairs = true>
__device__ __forceinline__ float stencil_gather_at(__amdgpu_buffer_rsrc_t ib, const RayK& r, const Stencil& st,
                                                   int img_off) {
    float v00, v01, v10, v11;
    stencil_load<Pairs>(ib, r, st, st.base + img_off, v00, v01, v10, v11);
    const float gu = 1.0f - st.fu, gw = 1.0f - st.fw;
    return gu * (gw * v00 + st.fw * v01) + st.fu * (gw * v10 + st.fw * v11);
}

// Transpose of stencil_gather for the direct path: img[...] += weight * c with hardware float
// atomics, wave-cooperative; every lane of the wave must call it (inactive lanes with
// active == false).  Float atomics that hit the
// same address within one instruction are serialised by the memory system,
// which is exactly what nearly coincident rays of a wave produce.  Lanes are
// therefore grouped into runs of equal stencil (same base voxel and principal
// axis, adjacent in lane order); a segmented reduction over each run sums the
// four weighted values into the run's first lane, and only that lane issues
// the atomic adds.  Only the order of float additions changes.
__device__ __forceinline__ void wave_stencil_scatter(float* __restrict__ img, bool active, const RayK& r,
                                                     const Stencil& st, float c) {
    const int lane = (int)__lane_id();
    const float gu = 1.0f - st.fu, gw = 1.0f - st.fw;
    float v00 = (active && st.i0ok && st.j0ok) ? gu * gw * c : 0.0f;
    float v01 = (active && st.i0ok && st.j1ok) ? gu * st.fw * c : 0.0f;
    float v10 = (active && st.i1ok && st.j0ok) ? st.fu * gw * c : 0.0f;
    float v11 = (active && st.i1ok && st.j1ok) ? st.fu * st.fw * c : 0.0f;
    active = active && (st.i0ok || st.i1ok) && (st.j0ok || st.j1ok);
    const int kb = active ? st.base : (INT_MIN + lane);  // inactive lanes never match
    const int kp = active ? r.p : -1;
    const int pb = __shfl_up(kb, 1, 64), pp = __shfl_up(kp, 1, 64);
    const bool head = lane == 0 || kb != pb || kp != pp;
    const unsigned long long heads = __ballot(head);
    const unsigned long long later = (lane == 63) ? 0ull : (heads & (~0ull << (lane + 1)));
    const int run_end = later ? (__ffsll((long long)later) - 1) : 64;  // first lane of the next run
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const float a = __shfl_down(v00, off, 64), b = __shfl_down(v01, off, 64);
        const float d = __shfl_down(v10, off, 64), e = __shfl_down(v11, off, 64);
        if (lane + off < run_end) {
            v00 += a;
            v01 += b;
            v10 += d;
            v11 += e;
        }
    }
    if (head && active) {
        if (v00 != 0.0f) unsafeAtomicAdd(img + st.base, v00);
        if (v01 != 0.0f) unsafeAtomicAdd(img + st.base + r.sw, v01);
        if (v10 != 0.0f) unsafeAtomicAdd(img + st.base + r.su, v10);
        if (v11 != 0.0f) unsafeAtomicAdd(img + st.base + r.su + r.sw, v11);
    }
}

// erf by Hastings' rational approximation (Abramowitz & Stegun 7.1.26):
// erf(u) = 1 - t P(t) exp(-u^2), t = 1 / (1 + p u), u >= 0, |error| <= 1.5e-7; about
// 6e-7 when evaluated in float32 (the cancellation in 1 - t P e near u = 0).  Branch-free,
// so the plane loops keep several rays' dependency chains interleaved (a library erf
// with a branch per range serialises them), and about a third of the instructions.
// erf_scaled takes v = kErfC u, kErfC = sqrt(log2 e), so that exp(-u^2) = exp2(-v^2) costs one
// multiply; the callers fold kErfC into the factor that forms the argument.

__device__ __forceinline__ float erf_scaled(float v) {
    const float a = fabsf(v);
    const float t = __builtin_amdgcn_rcpf(fmaf(0.3275911f / kErfC, a, 1.0f));
    float P = fmaf(1.061405429f, t, -1.453152027f);
    P = fmaf(P, t, 1.421413741f);
    P = fmaf(P, t, -0.284496736f);
    P = fmaf(P, t, 0.254829592f);
    const float e = __builtin_amdgcn_exp2f(-(a * a));  // exp(-u^2)
    return copysignf(fmaf(-(t * P), e, 1.0f), v);
}

// erf(clip(x, -n_sigmas sigma, n_sigmas sigma) / (sqrt(2) sigma)), x in mm, with inv =
// kErfC / (sqrt(2) sigma): the clip is taken on the scaled argument (at +-u_max), so a ray with
// its own sigma needs nothing but its own inv
__device__ __forceinline__ float tof_erf(float x, float inv, const TofK& t) {
    return erf_scaled(__builtin_amdgcn_fmed3f(x * inv, -t.u_max, t.u_max));
}


// Tabulated kernel (the lookup-table alternative of Sec. 4, which also admits non-Gaussian
// TOF kernels): linear interpolation of the table at u = (x - lo) / dx, 0 outside it.
__device__ __forceinline__ float tof_lut(double x, const TofK& t) {
    const float u = (float)(x - t.lo) * t.lut_inv_dx;
    if (!(u >= 0.0f) || u > (float)(t.lut_n - 1)) return 0.0f;
    const int i = min((int)u, t.lut_n - 2);
    const float f = u - (float)i, a = t.lut[i], b = t.lut[i + 1];
    return fmaf(f, b - a, a);
}

// The Gaussian bin weight w(x) = G(x + bw/2) - G(x - bw/2) as a piecewise polynomial of y = |x|
// (w is even).  w is smooth except where one of the clipped G starts or stops moving: at
// y = |n_sigmas sigma - bw/2| and at the end of the support y = n_sigmas sigma + bw/2.  Between
// those points it is analytic, so each piece is a Chebyshev interpolant (fitted on the host in
// float64 from the exact erf, converted to powers of a variable in [-1, 1]): the central piece in
// y^2, the tail piece in y.  Both pieces are evaluated (two independent Horner chains, no
// transcendental instruction) and the one for y selected; 0 beyond the support.  The host checks
// the float32 evaluation against the exact weight and falls back to the erf form if it misses
// its bound.
// The polynomial constants that meet a second scalar operand in one instruction (the first
// coefficients of the two Horner chains, the tail variable's offset), moved to vector registers once
// before a plane loop: an instruction reads at most one scalar register, so otherwise the compiler
// may copy them to vector registers again in every step.
__device__ __forceinline__ void tof_poly_to_vgprs(TofK& t) {
    asm volatile("" : "+v"(t.pc[kPolyCentral]), "+v"(t.pt[kPolyTail]), "+v"(t.pb2));
}

__device__ __forceinline__ float tof_poly(float x, const TofK& t) {
    const float y = fabsf(x), u = y * t.pq1;
    const float s1 = fmaf(u, u, -1.0f), s2 = fmaf(y, t.pa2, t.pb2);
    float a = t.pc[kPolyCentral], b = t.pt[kPolyTail];
#pragma unroll
    for (int i = kPolyCentral - 1; i >= 0; --i) {
        a = fmaf(a, s1, t.pc[i]);
        if (i < kPolyTail) b = fmaf(b, s2, t.pt[i]);
    }
    return y < t.pk1 ? a : (y < t.pk2 ? b : 0.0f);
}

// tof_poly with the piece chosen for the whole wave when every active lane is on the same one: only
// that polynomial is evaluated (presorted events of a wave walk through their windows in step, so in
// the forward loops most steps are uniform).  The same operations per lane, so the same values.
__device__ __forceinline__ float tof_poly_wave(float x, const TofK& t) {
    const float y = fabsf(x);
    const bool central = y < t.pk1;
    if (__ballot(!central) == 0ull) {
        const float u = y * t.pq1, s1 = fmaf(u, u, -1.0f);
        float a = t.pc[kPolyCentral];
#pragma unroll
        for (int i = kPolyCentral - 1; i >= 0; --i) a = fmaf(a, s1, t.pc[i]);
        return a;
    }
    if (__ballot(central) == 0ull) {
        const float s2 = fmaf(y, t.pa2, t.pb2);
        float b = t.pt[kPolyTail];
#pragma unroll
        for (int i = kPolyTail - 1; i >= 0; --i) b = fmaf(b, s2, t.pt[i]);
        return y < t.pk2 ? b : 0.0f;
    }
    return tof_poly(x, t);
}

// How a kernel evaluates the TOF bin weight: the two clipped erf (any sigma, also per ray), the
// table, or the fitted polynomial (one sigma for all rays).
enum TofForm : int { kFormErf = 0, kFormLut = 1, kFormPoly = 2 };

// The form a call uses for listmode kernels: the table when given, else the polynomial when its
// fit is valid and every ray shares sigma, else the erf.
__host__ __device__ inline int tof_form(const TofK& t) {
    if (t.lut) return kFormLut;
    return (t.poly && !t.sig_ray) ? kFormPoly : kFormErf;
}

// Weight of a bin for a plane sample at signed distance x (mm) from the bin centre, up to the
// factor kTofScale<Form>: for the erf form (inv = kErfC / (sqrt(2) sigma)) 2 w(x) = 2 (G(x + bw/2) -
// G(x - bw/2)), the difference of the two clipped erf; table and polynomial give w(x).  Every
// caller folds kTofScale into its per-ray constant (ell, or ell times the ray's value); a
// power-of-two factor commutes with float rounding, so the weights are applied exactly as if
// scaled per sample.
template <int Form>
constexpr float kTofScale = Form == kFormErf ? 0.5f : 1.0f;

// Wave: the polynomial's piece chosen per wave where uniform (tof_poly_wave; any lane pattern is
// allowed, the ballots see the active lanes)
template <int Form, bool Wave = false>
__device__ __forceinline__ float tof_weight_unscaled(double x, const TofK& t, float inv) {
    if (Form == kFormLut) return tof_lut(x, t);
    if (Form == kFormPoly) return Wave ? tof_poly_wave((float)x, t) : tof_poly((float)x, t);
    const float xf = (float)x, h = t.hbw * inv;
    return erf_scaled(__builtin_amdgcn_fmed3f(fmaf(xf, inv, h), -t.u_max, t.u_max)) -
           erf_scaled(__builtin_amdgcn_fmed3f(fmaf(xf, inv, -h), -t.u_max, t.u_max));
}

// TOF bins whose support [lo_x, hi_x] (relative to the bin centre) contains a sample at TOF
// position s (clamped to [0, n_bins)).
__device__ __forceinline__ void tof_bin_range(double s, const TofK& t, double lo_x, double hi_x, int& b_lo,
                                              int& b_hi) {
    // bins b with c_b in (s - hi, s - lo); a rounding of the products can only drop a bin whose
    // centre sits exactly on the open end, whose weight is 0
    const double lo = floor((s - hi_x - t.c0) * t.inv_bw);
    const double hi = ceil((s - lo_x - t.c0) * t.inv_bw);
    b_lo = (int)fmax(lo, 0.0);
    b_hi = (int)fmin(hi, (double)(t.nb - 1));
}

// Wave-wide min / max (wave64; every lane of the wave must call it).
__device__ __forceinline__ int wave_min(int v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v = min(v, __shfl_xor(v, off, 64));
    return v;
}

__device__ __forceinline__ int wave_max(int v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v = max(v, __shfl_xor(v, off, 64));
    return v;
}

}  // namespace ppmi
