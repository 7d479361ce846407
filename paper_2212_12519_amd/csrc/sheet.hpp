// Run/sheet back projection for ordered ray lists (presorted listmode events,
// radial-view-plane sinograms).
//
// Float atomic adds on this GPU are priced per cache-line request at the
// memory side, so the direct scatter (4 atomics per plane sample) is bound by
// request count.  In an ordered ray list, consecutive rays very often lie on
// the same transaxial line: same principal axis p (0 or 1) and identical
// in-plane coordinate U(k) = U0 + k dU at every plane k -- they differ only in
// their axial coordinate W(k) and in their value.  All contributions of such a
// run then fall into a "sheet" of the image: at plane k the two columns
// (k, i0(k), :) and (k, i0(k) + 1, :) along the fastest axis (2).
//
// A workgroup takes 256 consecutive rays of the processing order and splits
// them into runs (bitwise-equal p, U0, dU).  The rays of every run of >=
// kRunMin rays are spread over the workgroup's eight half-waves (32 lanes),
// one ray per half-wave, whose lanes walk the ray's plane window 32 planes at a
// time and add the W-interpolated values into an LDS image of the sheet
// (planes x z, one column per plane) with LDS atomics; then the waves flush
// the sheet with contiguous, duplicate-free atomics -- one memory request per
// ~16 values instead of one per value.  The column stride is the grid's
// longest line + 1, so that two workgroups fit a CU's LDS on clinical grids.
// The u-weights (1 - fu, fu) are shared by the run and applied at the flush.
// Rays in short runs (or with p == 2, or grids whose axis 2 exceeds the LDS
// column) take the direct wave-synchronous, run-combined scatter.  The
// arithmetic per (ray, plane) sample is the same as in the direct path; only
// the order of float additions differs.
#pragma once

#include <type_traits>

#include "joseph.hpp"

namespace ppmi {

constexpr int kSheetBlock = 256;
constexpr int kRunMin = 2;
constexpr int kSheetMaxW = 128;  // largest axis-2 size with an LDS sheet
constexpr int kSheetGroups = 8;  // groups of 256 rays per workgroup (a sheet persists across them)
// Largest sum of value bounds a sheet takes, in its fixed-point units: 2^31 less room for the
// rounding of every added value (at most kSheetGroups * 256 additions to one entry, 1.5 units each)
// and of the coarsenings (half a unit each).
constexpr float kSheetCap = 2147483648.0f - 1048576.0f;
// Fewest bits a ray's largest value keeps in a sheet's fixed point (an added value is off by at most
// 1.5 units, 1.5 * 2^-kSheetBits of the ray's largest at worst, and the carried remainders keep sums
// unbiased); rays with smaller values take the direct scatter.
constexpr int kSheetBits = 8;

// A value in fixed-point units rounded to the nearest integer, halves up: floor(x + 1/2) in one
// instruction (v_cvt_rpi_i32_f32; the compiler's round-to-nearest-even conversion takes two).  |x|
// stays below 2^31 in the sheet by construction.
__device__ __forceinline__ int round_half_up(float x) {
    int r;
    asm("v_cvt_rpi_i32_f32 %0, %1" : "=v"(r) : "v"(x));
    return r;
}

// LDS layout of k_back_runs (bytes): per-ray arrays, then the column buffer.
struct SheetLayout {
    static constexpr int kDoubles = 6;  // W0 dW s0 ds U0 dU
    static constexpr int kWords = 6;    // cv, lohi, start, cnt, list, aux; + 24 words
    static size_t ray_bytes() { return (size_t)kSheetBlock * (kDoubles * 8 + kWords * 4) + 24 * 4; }
    // column stride: the longest line a sheet can hold (planes along axis 0 or 1, at most 256),
    // rounded up to an odd count, so that the 64 consecutive z entries of one plane that a wave
    // reads in the flush fall in 64 different LDS banks; sized to the grid so that two workgroups
    // share a CU's LDS on the clinical grid (215 planes, 71 z entries: 79.1 KB)
    __host__ __device__ static int col_stride(const GeomK& g) {
        const int np = g.n[0] > g.n[1] ? g.n[0] : g.n[1];
        return (np < kSheetBlock ? np : kSheetBlock) | 1;
    }
    // nw rows of the sheet plus one spare row that absorbs the out-of-grid entries of a z pair
    // (217-entry rows on the clinical grid: 81,024 bytes, two workgroups per CU)
    static size_t bytes(int nw, const GeomK& g) { return ray_bytes() + (size_t)(nw + 1) * col_stride(g) * 4; }
};

// Largest |x| over a table of n floats (every thread of the workgroup calls it; red: 4 floats of
// LDS).  A linear interpolation of the table never exceeds it.
__device__ inline float table_abs_max(const float* __restrict__ tab, int n, float* red) {
    float v = 0.0f;
    for (int i = threadIdx.x; i < n; i += kSheetBlock) v = fmaxf(v, fabsf(tab[i]));
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v = fmaxf(v, __shfl_xor(v, off, 64));
    __syncthreads();  // red[] may still be read by a previous call
    if (__lane_id() == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    return fmaxf(fmaxf(red[0], red[1]), fmaxf(red[2], red[3]));
}

// Upper bound of |tof_weight_unscaled<Form>|: the Gaussian bin weight peaks at w(0) (at most 1 with
// per-ray sigma), the erf form gives 2 w (its erf within 1e-6), the polynomial is within 5e-7 w(0)
// of w (margin: the caller's), and a table's interpolation stays within its largest entry.
template <int Form>
__device__ inline float tof_weight_bound(const TofK& t, float* red) {
    if (Form == kFormLut) return table_abs_max(t.lut, t.lut_n, red);
    const float w0 = t.sig_ray ? 1.0f : t.wpeak + 1e-6f;
    return Form == kFormErf ? 2.0f * w0 : w0;
}

// Per-ray value hooks:
//   setup(l, r, cv, aux): prepare ray l (false = no contribution); cv = ell * p (the constant
//                    factor of every sample); for listmode TOF, r.s0 is made relative to the bin
//                    centre; aux: a per-ray word the mode keeps (kAux)
//   sample(x, cv, aux): the value scattered at the plane sample with TOF coordinate
//                    x = fma(k, r.ds, r.s0); linear in cv
//   mag(cv, aux):    an upper bound of |sample(x, cv, aux)| / weight_bound() over all x
//   weight_bound(red): the largest |TOF weight| a sample can take (1 without TOF); every thread of
//                    the workgroup calls it (a table is reduced with red[4] of LDS)
struct ModeNonTof {
    static constexpr bool kAux = false;
    static constexpr bool kBatch = false;
    const float* __restrict__ p;
    __device__ bool setup(int64_t l, const RaySrc& src, const GeomK& g, RayK& r, float& cv,
                          int& /*aux*/) const {
        const float pl = p[l];
        const bool geo = ray_setup(src, l, g, r);  // evaluated in any case: all loads issue together
        if (pl == 0.0f || !geo) return false;
        cv = r.ell * pl;
        return true;
    }
    __device__ float sample(double /*x*/, float cv, int /*aux*/) const { return cv; }
    __device__ void to_vgprs() {}
    __device__ float mag(float cv, int /*aux*/) const { return fabsf(cv); }
    __device__ float weight_bound(float* /*red*/) const { return 1.0f; }
};

// Listmode TOF, the weight in form Form (TofForm).  With per-ray TOF parameters (PerRay) the ray's
// offset is folded into its TOF coordinate at setup and aux carries the bits of its erf argument
// per mm (TofRay::inv).  Batch: several value arrays (p[b][l], value()) for one set of rays; setup
// then gives the value-free constant (cv for a value of 1) and keeps rays of any value.
template <int Form, bool PerRay = false, bool Batch = false>
struct ModeTofLm {
    static constexpr bool kAux = PerRay;
    static constexpr bool kBatch = Batch;
    const float* __restrict__ p;
    const int16_t* __restrict__ bins;
    TofK t;
    __device__ float value(int64_t l, int b, int64_t n) const { return p[(int64_t)b * n + l]; }
    __device__ bool setup(int64_t l, const RaySrc& src, const GeomK& g, RayK& r, float& cv,
                          int& aux) const {
        const int b = bins[l];
        const float pl = Batch ? 1.0f : p[l];
        TofRay q;
        // every condition evaluated (no short circuit), so that all of the ray's loads issue together
        const bool geo = ray_setup(src, l, g, r);
        const bool tr = tof_ray<PerRay>(t, l, q);
        if (b < 0 || b >= t.nb || pl == 0.0f || !tr || !geo) return false;
        if (PerRay) r.s0 -= q.shift;
        if (!tof_window_rel(r, t.c0 + b * t.bw, q.lo, q.hi)) return false;
        cv = r.ell * pl * kTofScale<Form>;
        if (PerRay) aux = __float_as_int(q.inv);
        return true;
    }
    __device__ float sample(double x, float cv, int aux) const {
        return tof_weight_unscaled<Form>(x, t, PerRay ? __int_as_float(aux) : t.u_per_mm) * cv;
    }
    __device__ void to_vgprs() {
        if constexpr (Form == kFormPoly) tof_poly_to_vgprs(t);
    }
    __device__ float mag(float cv, int /*aux*/) const { return fabsf(cv); }
    __device__ float weight_bound(float* red) const { return tof_weight_bound<Form>(t, red); }
};

// Sinogram TOF: the value at a plane sample is ell * sum over the bins b of its TOF window of
// w_b(s) p[l][b] (neighbouring bins share their erf edge).  aux carries the ray index l (the
// sheet path is used for fewer than 2^31 rays); all lanes of a wave read the same ray's bin
// values, so those loads hit one or two cache lines.  With per-ray TOF parameters (PerRay) the
// ray's offset is folded into its TOF coordinate at setup and its sigma is read per sample.
template <bool Lut, bool PerRay = false>
struct ModeTofSino {
    static constexpr bool kAux = true;
    static constexpr bool kBatch = false;
    const float* __restrict__ p;  // [n][n_bins]
    TofK t;
    __device__ bool setup(int64_t l, const RaySrc& src, const GeomK& g, RayK& r, float& cv,
                          int& aux) const {
        const float* pr = p + l * t.nb;
        bool any = false;
        for (int b = 0; b < t.nb; ++b) any |= (pr[b] != 0.0f);
        TofRay q;
        if (!any || !tof_ray<PerRay>(t, l, q) || !ray_setup(src, l, g, r)) return false;
        if (PerRay) r.s0 -= q.shift;
        cv = r.ell;
        aux = (int)l;
        return true;
    }
    __device__ float sample(double s, float cv, int aux) const {
        const float* pr = p + (int64_t)aux * t.nb;
        TofRay q;
        tof_ray<PerRay>(t, aux, q);  // usable: checked at setup
        int b_lo, b_hi;
        tof_bin_range(s, t, q.lo, q.hi, b_lo, b_hi);
        float c = 0.0f;
        if (Lut) {
            for (int b = b_lo; b <= b_hi; ++b) c += tof_lut(s - (t.c0 + b * t.bw), t) * pr[b];
        } else {
            const float x_hi0 = (float)(s - (t.c0 + b_lo * t.bw) + 0.5 * t.bw), bwf = (float)t.bw;
            float e_hi = tof_erf(x_hi0, q.inv, t);
            for (int b = b_lo; b <= b_hi; ++b) {
                const float e_lo = tof_erf(x_hi0 - (float)(b - b_lo + 1) * bwf, q.inv, t);
                c += 0.5f * (e_hi - e_lo) * pr[b];
                e_hi = e_lo;
            }
        }
        return c * cv;
    }
    // a bin weight is at most w(0) (1 with per-ray sigma) or the table's largest entry
    __device__ void to_vgprs() {}
    __device__ float mag(float cv, int aux) const {
        const float* pr = p + (int64_t)aux * t.nb;
        float a = 0.0f;
        for (int b = 0; b < t.nb; ++b) a += fabsf(pr[b]);
        return fabsf(cv) * a;
    }
    __device__ float weight_bound(float* red) const {
        return Lut ? table_abs_max(t.lut, t.lut_n, red) : (t.sig_ray ? 1.0f : t.wpeak + 1e-6f);
    }
};

// The rectangle [k0, k1] x [z0, z1] (planes, z entries) of the sheet that the workgroup's lanes
// added to since the last flush (each lane passes its own klo, khi, zlo, zhi; empty: k0 > k1 or
// z0 > z1).  Every thread of the workgroup calls it; part[] takes 4 words; it synchronises once.
__device__ __forceinline__ void sheet_rect(int klo, int khi, int zlo, int zhi, int nw, int* part, int& k0, int& k1,
                                           int& z0, int& z1) {
    constexpr int B = kSheetBlock;
    const int lane = (int)__lane_id(), wave = (int)threadIdx.x >> 6;
    // per wave, packed in one word: lowest plane (bits 0-7), highest plane (8-15), lowest z
    // (16-23), highest z (24-31); planes < 256 and nw <= 128.  A lane that added nothing passes
    // klo > khi; z is clamped to the grid per lane (a lane whose pairs were all out of the grid, as
    // at the conservative end plane of a window, has zhi < 0 or zlo >= nw).
    const bool any = klo <= khi;
    const int a = wave_min(any ? klo : 255), b = wave_max(any ? khi : 0);
    const int c = wave_min(any ? min(max(zlo, 0), nw - 1) : 255);
    const int d = wave_max(any ? max(min(zhi, nw - 1), 0) : 0);
    if (lane == 0) part[wave] = a | (b << 8) | (c << 16) | (d << 24);
    __syncthreads();
    k0 = 255, k1 = 0, z0 = 255, z1 = 0;
    for (int w = 0; w < B / 64; ++w) {
        const unsigned q = (unsigned)part[w];
        k0 = min(k0, (int)(q & 0xff));
        k1 = max(k1, (int)((q >> 8) & 0xff));
        z0 = min(z0, (int)((q >> 16) & 0xff));
        z1 = max(z1, (int)(q >> 24));
    }
}

// Coarsen the sheet's fixed point by 2^sft (1 <= sft <= 24): every entry of the written rectangle
// is divided by 2^sft and rounded, each thread carrying its rounding remainder (exact, in the old
// units) into its next entry, so that the entries' sum is kept to within half a new unit per
// thread: no systematic loss of the many small entries.  Every thread of the workgroup calls it; the
// caller synchronises after it.
__device__ __forceinline__ void sheet_rescale(int* col, int cs, int sft, int klo, int khi, int zlo, int zhi, int nw,
                                              int* part) {
    constexpr int B = kSheetBlock;
    int k0, k1, z0, z1;
    sheet_rect(klo, khi, zlo, zhi, nw, part, k0, k1, z0, z1);
    const int nk = max(k1 - k0 + 1, 0), nz = max(z1 - z0 + 1, 0);
    const int total = nk * nz;
    const float inv_nz = 1.0f / (float)max(nz, 1);
    long long rem = 0;
    for (int e = (int)threadIdx.x; e < total; e += B) {
        const int pi = (int)(((float)e + 0.5f) * inv_nz), j = z0 + e - pi * nz;
        int* cp = col + j * cs + k0 + pi;
        const long long t = (long long)*cp + rem;
        const long long q = (t + (1ll << (sft - 1))) >> sft;
        rem = t - (q << sft);
        *cp = (int)q;
    }
}

// Flush the sheet of line (p, U0, dU) with contiguous atomics and clear it: the entries that hold a
// value, in the rectangle the workgroup's lanes wrote (sheet_rect), times inv_scale (the fixed
// point's unit) and the in-plane weights.  Every thread of the workgroup calls it; part[] takes 4
// words; the caller synchronises after it.
__device__ __forceinline__ void sheet_flush(float* __restrict__ img, int* col, const GeomK& g, int p, double U0,
                                            double dU, float inv_scale, int klo, int khi, int zlo, int zhi, int nw,
                                            int cs, int* part) {
    constexpr int B = kSheetBlock;
    const int tid = threadIdx.x;
    int k0, k1, z0, z1;
    sheet_rect(klo, khi, zlo, zhi, nw, part, k0, k1, z0, z1);
    const int su = (p == 0) ? g.stride[1] : g.stride[0];
    const int sp = g.stride[p];
    const int nu = (p == 0) ? g.n[1] : g.n[0];
    const int nk = max(k1 - k0 + 1, 0), nz = max(z1 - z0 + 1, 0);
    const int total = nk * nz;
    const float inv_nz = 1.0f / (float)max(nz, 1);
    // the entries spread over all threads, consecutive threads on consecutive z of a plane (64
    // contiguous image addresses per atomic instruction; the odd column stride puts them in 64 banks)
    for (int e = tid; e < total; e += B) {
        // e / nz: (e + 1/2) / nz stays >= 1/(2 nz) away from an integer, far above float error
        const int pi = (int)(((float)e + 0.5f) * inv_nz), j = z0 + e - pi * nz;
        const int k = k0 + pi;
        int* cp = col + j * cs + k;
        const int q = *cp;
        if (q != 0) {
            *cp = 0;
            const float v = (float)q * inv_scale;
            const double U = fma((double)k, dU, U0);
            const double fi = floor(U);
            const int i0 = (int)fi;
            const float fu = (float)(U - fi);
            const int base = k * sp + i0 * su;
            if ((unsigned)i0 < (unsigned)nu) unsafeAtomicAdd(img + base + j, (1.0f - fu) * v);
            if ((unsigned)(i0 + 1) < (unsigned)nu) unsafeAtomicAdd(img + base + su + j, fu * v);
        }
    }
}

// One workgroup walks `groups` consecutive groups of 256 rays of the processing
// order.  The sheet of the current line (one column per absolute plane, so lines
// need n_p <= 256) persists across groups; it is flushed when a run of another
// line starts, when the line's values outgrow its fixed-point range, and at the end.
template <class Mode>
__device__ void back_runs_chunk(const Mode& m, RaySrc src, int64_t n,
                                const GeomK& g, float* __restrict__ img, const int32_t* __restrict__ order,
                                int nw_lds, int groups, int64_t chunk0, double* smem, int n_img = 1,
                                int64_t img_stride = 0) {
    constexpr int B = kSheetBlock;
    double* W0 = smem;
    double* dW = W0 + B;
    double* s0 = dW + B;
    double* ds = s0 + B;
    double* U0 = ds + B;
    double* dU = U0 + B;
    float* cvs = reinterpret_cast<float*>(dU + B);
    // k_lo | k_hi << 8 | p << 16 (the plane range is read for sheet rays only, whose planes are < 256)
    int* lohi = reinterpret_cast<int*>(cvs + B);
    auto pax = [&](int e) { return lohi[e] >> 16; };
    int* start = lohi + B;
    int* cnt = start + B;
    int* masks = cnt + B;  // 8 words: run-boundary ballots of the 4 waves
    int* list = masks + 8;  // sheet-run heads; count at list[B]; per-wave counts at list[B + 4 ..]
    int* aux = list + B + 8;  // per-ray word of the mode (sinogram TOF: the ray index)
    // the flush's per-wave words reuse masks[], which only the run detection before the sheet
    // loop uses
    // free words: aux[B .. B + 3] the per-wave sums of the bound prefix, aux[B + 4 .. B + 7] reductions
    float* wsum = reinterpret_cast<float*>(aux + B);
    float* red = wsum + 4;
    int* col = aux + B + 8;  // [nw + 1][cs], 32-bit fixed point
    const int cs = SheetLayout::col_stride(g);

    const int tid = threadIdx.x;
    const int lane = (int)__lane_id();
    const int wave = tid >> 6;
    const int nw = g.n[2];
    const bool sheets = nw_lds > 0 && nw <= nw_lds;
    if (sheets)
        for (int q = tid; q < nw * cs; q += B) col[q] = 0;
    // bound of |an added value| per unit of a ray's mag() (margin for float rounding in the bounds)
    const float wb = m.weight_bound(red) * (1.0f + 0x1p-8f);
    // the mode as the plane loops use it (constants they need in vector registers moved there once)
    Mode ms = m;
    ms.to_vgprs();
    // current sheet (block-uniform copies in registers, updated after barriers)
    bool sh_on = false;
    float sh_scale = 1.0f, sh_used = 0.0f;  // fixed-point scale of the sheet; bounds added (scaled)
    // this lane's rounding remainder, carried from one of its samples to the next (sheet units)
    float res = 0.0f;
    // planes and z entries this lane added to since the last flush (empty: klo > khi)
    int t_klo = 255, t_khi = 0, t_zlo = INT_MAX, t_zhi = INT_MIN;
    int sh_p = -1;
    double sh_U0 = 0.0, sh_dU = 0.0;
    for (int grp = 0; grp < groups; ++grp) {
        const int64_t i = chunk0 + (int64_t)grp * B + tid;
        if (chunk0 + (int64_t)grp * B >= n) break;  // block-uniform
        int64_t l = -1;
        if (i < n) {
            l = order ? (int64_t)order[i] : i;
            if (l < 0 || l >= n) l = -1;
        }
        RayK r;
        float cv = 0.0f;
        int ax = 0;
        const bool ok = l >= 0 && ms.setup(l, src, g, r, cv, ax);
        // compact the valid rays to the front of the group (stable order), so that rays
        // without a contribution do not break runs
        const unsigned long long vb = __ballot(ok);
        // inclusive prefix sum, in ray order, of the valid rays' bounds of |an added value| (a run's
        // bound is the difference of two of them)
        float pm = ok ? m.mag(cv, ax) * wb : 0.0f;
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
            const float o = __shfl_up(pm, off, 64);
            if (lane >= off) pm += o;
        }
        __syncthreads();  // previous group's LDS readers are done
        if (lane == 0) list[B + 4 + wave] = __popcll(vb);
        if (lane == 63) wsum[wave] = pm;
        __syncthreads();
        int voff = 0, nvalid = 0;
        for (int w = 0; w < B / 64; ++w) {
            const int c_w = list[B + 4 + w];
            voff += (w < wave) ? c_w : 0;
            nvalid += c_w;
            pm += (w < wave) ? wsum[w] : 0.0f;
        }
        const int cp = ok ? voff + __popcll(vb & ((1ull << lane) - 1ull)) : -1;
        if (ok) {
            W0[cp] = r.W0;
            dW[cp] = r.dW;
            s0[cp] = r.s0;
            ds[cp] = r.ds;
            U0[cp] = r.U0;
            dU[cp] = r.dU;
            cvs[cp] = cv;
            aux[cp] = ax;
            lohi[cp] = (r.k_lo & 0xff) | ((r.k_hi & 0xff) << 8) | (r.p << 16);
        }
        __syncthreads();
        // runs over the compacted entries (thread t examines entry t): maximal stretches with
        // bitwise-equal (p, U0, dU)
        const bool e_ok = tid < nvalid;
        const bool same =
            e_ok && tid > 0 && pax(tid - 1) == pax(tid) && U0[tid - 1] == U0[tid] && dU[tid - 1] == dU[tid];
        int st = (e_ok && !same) ? tid : -1;
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
            const int o = __shfl_up(st, off, 64);
            if (lane >= off) st = max(st, o);
        }
        // carry across waves: latest head position of each earlier wave; boundary masks for lengths
        const bool bnd = !(e_ok && same);  // a run head, or an entry past the valid ones
        const unsigned long long bmask = __ballot(bnd);
        if (lane == 63) start[wave] = st;
        if (lane == 0) {
            masks[2 * wave] = (int)(bmask & 0xffffffffull);
            masks[2 * wave + 1] = (int)(bmask >> 32);
        }
        __syncthreads();
        int carry = -1;
        for (int w = 0; w < wave; ++w) carry = max(carry, start[w]);
        // run length of a head: distance to the next boundary after it
        int len = 0;
        if (e_ok && !same) {
            int w = wave;
            unsigned long long mk = (lane == 63) ? 0ull : (bmask & (~0ull << (lane + 1)));
            int nxt = B;
            while (true) {
                if (mk) {
                    nxt = w * 64 + __ffsll((long long)mk) - 1;
                    break;
                }
                if (++w >= B / 64) break;
                mk = ((unsigned long long)(unsigned)masks[2 * w + 1] << 32) | (unsigned)masks[2 * w];
            }
            len = nxt - tid;
        }
        __syncthreads();
        if (e_ok && same && st < 0) st = carry;
        if (!e_ok) st = -1;
        start[tid] = st;
        cnt[tid] = len;
        __syncthreads();
        // a run goes to the sheet if it is long, or if it continues the current sheet's line
        auto sheet_run = [&](int h) {
            if (!sheets || cnt[h] == 0 || pax(h) == 2 || g.n[pax(h)] > B) return false;
            if (cnt[h] >= kRunMin) return true;
            return sh_on && pax(h) == sh_p && U0[h] == sh_U0 && dU[h] == sh_dU;
        };
        const bool in_sheet = ok && sheet_run(start[cp]);
        // start[] now takes the bound prefix of the compacted entries (each thread rewrites only the
        // entry it just read; the loop reads them after the barriers below)
        if (ok) start[cp] = __float_as_int(pm);
        // parallel compaction of the sheet-run heads (in order): ballot + prefix popcount
        {
            const bool f = sheet_run(tid);
            const unsigned long long bal = __ballot(f);
            if (lane == 0) list[B + 4 + wave] = __popcll(bal);
            __syncthreads();
            int off = 0, total = 0;
            for (int w = 0; w < B / 64; ++w) {
                const int c_w = list[B + 4 + w];
                off += (w < wave) ? c_w : 0;
                total += c_w;
            }
            if (f) list[off + __popcll(bal & ((1ull << lane) - 1ull))] = tid;
            if (tid == 0) list[B] = total;
        }
        // the images of the call: one, or (batch modes) n_img, each with its own values, sharing the
        // rays' setup, compaction and runs; a batch flushes its sheet at the end of every image's pass
        for (int bi = 0; bi < (Mode::kBatch ? n_img : 1); ++bi) {
            float* const imgb = img + (int64_t)bi * img_stride;
            float cvb = cv;
            if constexpr (Mode::kBatch) {
                // this image's values and the inclusive prefix of their bounds (as at the group's start)
                cvb = ok ? cv * m.value(l, bi, n) : 0.0f;
                float pb = ok ? m.mag(cvb, ax) * wb : 0.0f;
#pragma unroll
                for (int off = 1; off < 64; off <<= 1) {
                    const float o = __shfl_up(pb, off, 64);
                    if (lane >= off) pb += o;
                }
                if (lane == 63) wsum[wave] = pb;
                __syncthreads();  // also: the previous image's readers of cvs[] and start[] are done
                for (int w = 0; w < wave; ++w) pb += wsum[w];
                if (ok) {
                    cvs[cp] = cvb;
                    start[cp] = __float_as_int(pb);
                }
            }
            // direct path for the other rays: wave-synchronous, run-combined atomics
            {
                const bool d = ok && !in_sheet;
                const int dlo = d ? r.k_lo : (1 << 30), dhi = d ? r.k_hi : -(1 << 30);
                const int k0 = wave_min(dlo), k1 = wave_max(dhi);
                for (int k = k0; k <= k1; ++k) {
                    const bool act = k >= dlo && k <= dhi;
                    Stencil stn{};
                    float v = 0.0f;
                    if (act) {
                        stn = stencil_at(r, k);
                        v = ms.sample(fma((double)k, r.ds, r.s0), cvb, ax);
                    }
                    wave_stencil_scatter(imgb, act && v != 0.0f, r, stn, v);
                }
            }
            __syncthreads();
            const int n_long = list[B];
            for (int li = 0; li < n_long; ++li) {
                const int h = list[li];
                const int len = cnt[h], hend = h + len;
                // bound of the run's added values (margin for the rounding of the two prefix sums)
                const float pb1 = __int_as_float(start[hend - 1]), pb0 = h > 0 ? __int_as_float(start[h - 1]) : 0.0f;
                const float bnd = (pb1 - pb0) + pb1 * 0x1p-14f;
                const bool same_line = sh_on && pax(h) == sh_p && U0[h] == sh_U0 && dU[h] == sh_dU;
                // the run continues the sheet if its values fit the sheet's fixed-point range, else after
                // a coarsening of the sheet's fixed point that makes them fit (a flush instead when that
                // would cost the sheet more than 24 bits or leave the float range of the scale)
                bool fits = same_line && sh_used + bnd * sh_scale <= kSheetCap;
                if (same_line && !fits) {
                    int e = 0;
                    frexpf(sh_used + bnd * sh_scale, &e);  // the sum of the bounds < 2^e
                    const int sft = max(e - 30, 1);       // then below 2^30 after the coarsening
                    if (sft <= 24 && sh_scale >= 0x1p-96f) {
                        sheet_rescale(col, cs, sft, t_klo, t_khi, t_zlo, t_zhi, nw, masks);
                        __syncthreads();
                        sh_scale = ldexpf(sh_scale, -sft);
                        sh_used = ldexpf(sh_used, -sft) + 1.0f;  // each entry's rounding adds at most 1/2
                        res = ldexpf(res, -sft);                  // the lanes' remainders in the new unit
                        fits = true;
                    }
                }
                if (sh_on && !fits) {
                    sheet_flush(imgb, col, g, sh_p, sh_U0, sh_dU, 1.0f / sh_scale, t_klo, t_khi, t_zlo, t_zhi, nw, cs,
                                masks);
                    t_klo = 255;
                    t_khi = 0;
                    t_zlo = INT_MAX;
                    t_zhi = INT_MIN;
                    __syncthreads();
                    sh_on = false;
                }
                if (!sh_on) {
                    sh_on = true;
                    sh_p = pax(h);
                    sh_U0 = U0[h];
                    sh_dU = dU[h];
                    // a power of two that puts the run's bound below 2^30 (later runs of the line coarsen
                    // it when they do not fit)
                    int e = 0;
                    frexpf(bnd, &e);  // bnd < 2^e
                    sh_scale = ldexpf(1.0f, min(max(30 - e, -126), 126));
                    sh_used = 0.0f;
                    res = 0.0f;
                }
                sh_used += bnd * sh_scale;
                // The eight half-waves of the workgroup take the run's rays in turn (half-wave q: rays
                // h + q, h + q + 8, ...); a half-wave walks its ray's plane window 32 planes per step,
                // lane i at plane k_lo + i + 32 c, and adds the two W-interpolated values of each sample
                // to the column entries (j0, k) and (j0 + 1, k) with LDS atomics.  A ray's window fills
                // its steps up to the last one (about 95% of the lanes carry a sample on clinical TOF
                // windows), and the waves share no plane ownership, so they need no barrier until the
                // flush.  Entries outside the grid (j = -1, j = nw, the conservative end planes) go to
                // the spare row nw, which is never flushed.
                const int half = lane >> 5, hl = lane & 31;
                typedef __attribute__((address_space(3))) int lds_int;
                // LDS byte addresses: row j of plane k at col + 4 (j cs + k)
                const unsigned cs4 = 4u * (unsigned)cs;
                const unsigned colb = (unsigned)(uintptr_t)(__attribute__((address_space(3))) char*)col;
                auto at = [&](unsigned addr) { return (lds_int*)(uintptr_t)addr; };
                // a half-wave's ray: its records, read one ray ahead of its steps (a ray index past the
                // run reads the run head's records and gets an empty window)
                struct Rec {
                    double W0, dW, s0, ds;
                    float cv, mg;  // mg: the ray's bound of |an added value| (a difference of the prefix)
                    int ax, lh;
                };
                auto load = [&](int ra) {
                    const int r = ra + half < hend ? ra + half : h;
                    const float pr0 = r > 0 ? __int_as_float(start[r - 1]) : 0.0f;
                    Rec q{W0[r], dW[r], s0[r], ds[r], cvs[r], __int_as_float(start[r]) - pr0, Mode::kAux ? aux[r] : 0,
                          lohi[r]};
                    if (ra + half >= hend) q.lh = 0xff;  // k_lo 255 > k_hi 0: no planes
                    return q;
                };
                // the line's in-plane stencil terms, for rays that add to the image directly
                const int sp = g.stride[sh_p], su = g.stride[sh_p == 0 ? 1 : 0], nu = g.n[sh_p == 0 ? 1 : 0];
                const float inv_scale = 1.0f / sh_scale;
                Rec cur = load(h + 2 * wave);
                // wait for these reads here: the loop then sees them complete on every path and its steps
                // carry no LDS wait (which, LDS operations completing in order, would also wait for the
                // previous step's adds)
                __builtin_amdgcn_s_waitcnt(0xc07f);  // lgkmcnt(0)
                for (int ra = h + 2 * wave; ra < hend; ra += 8) {  // wave-uniform
                    const Rec nxt = load(ra + 8);
                    // a compiler-only barrier: keeps the prefetch here rather than next to its use
                    asm volatile("" ::: "memory");
                    const int klo = cur.lh & 0xff, khi = (cur.lh >> 8) & 0xff;
                    const float cvs_ = cur.cv * sh_scale;  // the sample values in fixed-point units
                    // a ray whose values would keep fewer than kSheetBits bits in the sheet's fixed point
                    // (far smaller values than the run's others) adds them to the image directly, with the
                    // direct path's float atomics
                    const bool direct = cur.mg * sh_scale < (float)(1 << kSheetBits);
                    if (klo <= khi) {
                        t_klo = min(t_klo, klo);
                        t_khi = max(t_khi, khi);
                    }
                    // planes - 1 of the longer of the two rays (wave-uniform)
                    const int span = max(__builtin_amdgcn_readlane(khi - klo, 0), __builtin_amdgcn_readlane(khi - klo, 32));
                    // the samples of the two rays, 32 planes per step; Mixed: some lane adds directly
                    auto steps = [&](auto mixed) {
                        for (int c = 0; c <= span; c += 32) {
                            const int k = klo + hl + c;
                            if (k <= khi) {
                                const double W = fma((double)k, cur.dW, cur.W0);
                                const double fj = floor(W);
                                const int j0 = (int)fj;
                                const float fw = (float)(W - fj);
                                const float v = ms.sample(fma((double)k, cur.ds, cur.s0), cvs_, cur.ax);
                                if (!decltype(mixed)::value || !direct) {
                                    const unsigned kb = 4u * (unsigned)k + colb;
                                    const unsigned a0 = __umul24(min((unsigned)j0, (unsigned)nw), cs4) + kb;
                                    const unsigned a1 = __umul24(min((unsigned)(j0 + 1), (unsigned)nw), cs4) + kb;
                                    // the sample's value with the carried remainder, rounded; the first
                                    // entry gets its own share rounded, the second the rest, so that the
                                    // lane's added integers track the exact running sum of its values
                                    const float tv = v + res;
                                    const float qt = rintf(tv);
                                    res = tv - qt;
                                    const int q0 = round_half_up(fmaf(-fw, v, v));
                                    const int q1 = (int)qt - q0;
                                    __hip_atomic_fetch_add(at(a0), q0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
                                    __hip_atomic_fetch_add(at(a1), q1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
                                    t_zlo = min(t_zlo, j0);
                                    t_zhi = max(t_zhi, j0 + 1);
                                } else {
                                    const float vf = v * inv_scale;  // exact: the scale is a power of two
                                    const double U = fma((double)k, sh_dU, sh_U0);
                                    const double fi = floor(U);
                                    const int i0 = (int)fi;
                                    const float fu = (float)(U - fi), gu = 1.0f - fu, gw = 1.0f - fw;
                                    const int base = k * sp + i0 * su + j0;
                                    const bool i0ok = (unsigned)i0 < (unsigned)nu, i1ok = (unsigned)(i0 + 1) < (unsigned)nu;
                                    const bool j0ok = (unsigned)j0 < (unsigned)nw, j1ok = (unsigned)(j0 + 1) < (unsigned)nw;
                                    if (i0ok && j0ok) unsafeAtomicAdd(imgb + base, gu * gw * vf);
                                    if (i0ok && j1ok) unsafeAtomicAdd(imgb + base + 1, gu * fw * vf);
                                    if (i1ok && j0ok) unsafeAtomicAdd(imgb + base + su, fu * gw * vf);
                                    if (i1ok && j1ok) unsafeAtomicAdd(imgb + base + su + 1, fu * fw * vf);
                                }
                            }
                        }
                    };
                    if (__ballot(direct && klo <= khi))
                        steps(std::integral_constant<bool, true>{});
                    else
                        steps(std::integral_constant<bool, false>{});
                    cur = nxt;
                }
                // no barrier between runs of one line: the adds are atomic, and the columns are read
                // only in a flush, whose first barrier follows every wave's last add
            }
            if (Mode::kBatch && sh_on) {
                sheet_flush(imgb, col, g, sh_p, sh_U0, sh_dU, 1.0f / sh_scale, t_klo, t_khi, t_zlo, t_zhi, nw, cs,
                            masks);
                t_klo = 255;
                t_khi = 0;
                t_zlo = INT_MAX;
                t_zhi = INT_MIN;
                __syncthreads();
                sh_on = false;
            }
        }
    }
    if (sh_on) sheet_flush(img, col, g, sh_p, sh_U0, sh_dU, 1.0f / sh_scale, t_klo, t_khi, t_zlo, t_zhi, nw, cs, masks);
    __syncthreads();  // the LDS may be reused by the caller
}

// (batch modes: n_img images at img + b * img_stride, values p[b][l])
template <class Mode>
__global__ void __launch_bounds__(kSheetBlock) k_back_runs(Mode m, RaySrc src, int64_t n, GeomK g,
                                                          float* __restrict__ img, const int32_t* __restrict__ order,
                                                          int nw_lds, int groups, int n_img, int64_t img_stride) {
    extern __shared__ double smem[];
    const int64_t chunk0 = (int64_t)blockIdx.x * groups * kSheetBlock;
    back_runs_chunk(m, src, n, g, img, order, nw_lds, groups, chunk0, smem, n_img, img_stride);
}

}  // namespace ppmi
