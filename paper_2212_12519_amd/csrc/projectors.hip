// Joseph forward / back projection kernels for gfx950 (non-TOF, TOF sinogram,
// TOF listmode).  One thread per ray; 256-thread workgroups (4 wave64s) in
// plain workgroup order.  See joseph.hpp for the traversal itself.
#include <hip/hip_runtime.h>

#include "joseph.hpp"
#include "launch.hpp"
#include "sheet.hpp"

namespace ppmi {

constexpr int kBlock = 256;

// ------------------------------------------------------------- non-TOF ----

// Ray processed by this thread: position i of the processing order (identity,
// or a permutation such as the one pp_lm_presort produces).  Entries outside
// [0, n) are skipped.
__device__ __forceinline__ int64_t ray_index(const int32_t* __restrict__ order, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return -1;
    if (!order) return i;
    const int64_t l = order[i];
    return (l >= 0 && l < n) ? l : -1;
}

__global__ void __launch_bounds__(kBlock) k_fwd(RaySrc src,
                                                int64_t n, GeomK g, const float* __restrict__ img,
                                                float* __restrict__ p, const int32_t* __restrict__ order) {
    const int64_t l = ray_index(order, n);
    if (l < 0) return;
    const __amdgpu_buffer_rsrc_t ib = img_buffer(img, g);
    RayK r;
    float acc = 0.0f;
    if (ray_setup(src, l, g, r)) {
        for (int k = r.k_lo; k <= r.k_hi; ++k) acc += stencil_gather(ib, r, stencil_at(r, k));
        acc *= r.ell;
    }
    p[l] = acc;
}

// ------------------------------------------------------- TOF listmode ----

// PerRay: per-ray sigma / centre offset arrays are set (TofRay in joseph.hpp).  Presorted
// events of one wave share their TOF bin, so their plane windows nearly coincide and the lanes
// of a wave gather from the same planes at each step; with per-ray parameters the windows start
// at different planes, so the loop runs over absolute planes instead (wave-synchronous: all
// lanes at plane k, each active inside its own window), keeping the gathers of a step coherent.
// Emit: also write the events and their projections in processing order (thread i: the event order[i];
// an order entry outside [0, n) gives event i with the value 0), for a back projection that then walks
// them without an order array.
template <int Form, bool PerRay, bool Emit = false>
__global__ void __launch_bounds__(kBlock) k_fwd_tof_lm(RaySrc src,
                                                       const int16_t* __restrict__ bins, int64_t n, GeomK g,
                                                       TofK t, const float* __restrict__ img,
                                                       float* __restrict__ p, const int32_t* __restrict__ order,
                                                       EventsOut eo) {
    constexpr bool kWaveSync = PerRay;
    const __amdgpu_buffer_rsrc_t ib = img_buffer(img, g);
    const int64_t l = ray_index(order, n);
    // every load of the ray issued together (no short circuit); a thread past the end reads ray 0
    const int64_t lc = l >= 0 ? l : 0;
    const int b = bins[lc];
    float acc = 0.0f;
    RayK r;
    TofRay q;
    // Emit: the event is copied from the registers of its setup, before the plane loop (coordinate
    // events only; an order entry outside [0, n) copies event i)
    bool geo;
    if constexpr (Emit) {
        float ev[6];
        const float *ps = src.xs + 3 * lc, *pe = src.xe + 3 * lc;
        ev[0] = ps[0], ev[1] = ps[1], ev[2] = ps[2], ev[3] = pe[0], ev[4] = pe[1], ev[5] = pe[2];
        geo = ray_setup(ev, ev + 3, g, r);
        const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
        if (i < n) {
            if (l < 0) {
                const float *qs = src.xs + 3 * i, *qe = src.xe + 3 * i;
                ev[0] = qs[0], ev[1] = qs[1], ev[2] = qs[2], ev[3] = qe[0], ev[4] = qe[1], ev[5] = qe[2];
            }
            eo.xs[3 * i] = ev[0];
            eo.xs[3 * i + 1] = ev[1];
            eo.xs[3 * i + 2] = ev[2];
            eo.xe[3 * i] = ev[3];
            eo.xe[3 * i + 1] = ev[4];
            eo.xe[3 * i + 2] = ev[5];
            eo.bins[i] = l >= 0 ? (int16_t)b : bins[i];
        }
    } else {
        geo = ray_setup(src, lc, g, r);
    }
    const bool tr = tof_ray<PerRay>(t, lc, q);
    bool on = l >= 0 && b >= 0 && b < t.nb && tr && geo;
    if (on) {
        if (PerRay) r.s0 -= q.shift;
        on = tof_window_rel(r, t.c0 + b * t.bw, q.lo, q.hi);
    }
    if (kWaveSync) {  // every lane of the wave reaches this point
        const int lo = on ? r.k_lo : (1 << 30), hi = on ? r.k_hi : -(1 << 30);
        const int k0 = wave_min(lo), k1 = wave_max(hi);
        for (int k = k0; k <= k1; ++k) {
            if (k >= lo && k <= hi) {
                const float w = tof_weight_unscaled<Form, true>(fma((double)k, r.ds, r.s0), t, q.inv);
                acc += w * stencil_gather<!PerRay>(ib, r, stencil_at(r, k));  // per-ray: arithmetic-bound
            }
        }
    } else if (on) {
        for (int k = r.k_lo; k <= r.k_hi; ++k) {
            const float w = tof_weight_unscaled<Form, true>(fma((double)k, r.ds, r.s0), t, q.inv);
            acc += w * stencil_gather<!PerRay>(ib, r, stencil_at(r, k));
        }
    }
    if (on) acc *= r.ell * kTofScale<Form>;
    if (l >= 0) p[l] = acc;
    if constexpr (Emit) {
        const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
        if (i < n) eo.p[i] = l >= 0 ? acc : 0.0f;
    }
}

// Batched listmode forward: the same events through `nimg` images of the grid (imgs[b] at b * voxels,
// at most kFwdBatch per launch), p[b * n + l] for image b.  Ray setup, TOF window, plane positions,
// stencils and TOF weights are computed once per sample for all images; only the four gathers and the
// accumulation are per image, in the order of k_fwd_tof_lm, so each image's result is that kernel's.
constexpr int kFwdBatch = 8;

template <int Form, bool PerRay>
__global__ void __launch_bounds__(kBlock) k_fwd_tof_lm_batch(RaySrc src, const int16_t* __restrict__ bins, int64_t n,
                                                             GeomK g, TofK t, const float* __restrict__ imgs,
                                                             int nimg, float* __restrict__ p,
                                                             const int32_t* __restrict__ order) {
    constexpr bool kWaveSync = PerRay;
    const __amdgpu_buffer_rsrc_t ib = img_buffer_n(imgs, g, nimg);
    const int nv = g.n[0] * g.n[1] * g.n[2];
    const int64_t l = ray_index(order, n);
    // every load of the ray issued together (no short circuit); a thread past the end reads ray 0
    const int64_t lc = l >= 0 ? l : 0;
    const int b = bins[lc];
    float acc[kFwdBatch];
#pragma unroll
    for (int q = 0; q < kFwdBatch; ++q) acc[q] = 0.0f;
    RayK r;
    TofRay tq;
    const bool geo = ray_setup(src, lc, g, r);
    const bool tr = tof_ray<PerRay>(t, lc, tq);
    bool on = l >= 0 && b >= 0 && b < t.nb && tr && geo;
    if (on) {
        if (PerRay) r.s0 -= tq.shift;
        on = tof_window_rel(r, t.c0 + b * t.bw, tq.lo, tq.hi);
    }
    auto sample = [&](int k) {
        const float w = tof_weight_unscaled<Form, true>(fma((double)k, r.ds, r.s0), t, tq.inv);
        const Stencil st = stencil_at(r, k);
#pragma unroll
        for (int q = 0; q < kFwdBatch; ++q)
            if (q < nimg) acc[q] += w * stencil_gather_at<!PerRay>(ib, r, st, q * nv);  // nimg: uniform
    };
    if (kWaveSync) {  // every lane of the wave reaches this point
        const int lo = on ? r.k_lo : (1 << 30), hi = on ? r.k_hi : -(1 << 30);
        const int k0 = wave_min(lo), k1 = wave_max(hi);
        for (int k = k0; k <= k1; ++k)
            if (k >= lo && k <= hi) sample(k);
    } else if (on) {
        for (int k = r.k_lo; k <= r.k_hi; ++k) sample(k);
    }
    if (l < 0) return;
    const float scale = on ? r.ell * kTofScale<Form> : 0.0f;
#pragma unroll
    for (int q = 0; q < kFwdBatch; ++q)
        if (q < nimg) p[(int64_t)q * n + l] = on ? acc[q] * scale : 0.0f;
}

// ------------------------------------------------------- TOF sinogram ----
//
// Each thread keeps its n_bins accumulators in LDS (column per thread, so a
// wave touching the same bin hits 64 distinct banks).  Per plane sample only
// the bins inside the TOF window are evaluated; neighbouring bins share their
// edge, so a window of m bins costs m + 1 erf evaluations.  The block's
// [rays][bins] output tile is contiguous in memory and is written with
// coalesced stores at the end.  PerRay: per-ray sigma / centre offset arrays are set.

template <bool PerRay>
__global__ void k_fwd_tof_sino(RaySrc src, int64_t n, GeomK g,
                               TofK t, const float* __restrict__ img, float* __restrict__ p) {
    extern __shared__ float lds[];  // [nb][blockDim]
    const int nt = blockDim.x;
    const int64_t l0 = (int64_t)blockIdx.x * nt;
    const int64_t l = l0 + threadIdx.x;
    for (int b = 0; b < t.nb; ++b) lds[b * nt + threadIdx.x] = 0.0f;
    const __amdgpu_buffer_rsrc_t ib = img_buffer(img, g);
    RayK r;
    TofRay q;
    if (l < n && tof_ray<PerRay>(t, l, q) && ray_setup(src, l, g, r)) {
        if (PerRay) r.s0 -= q.shift;
        float* mine = lds + threadIdx.x;
        for (int k = r.k_lo; k <= r.k_hi; ++k) {
            const float v = stencil_gather<false>(ib, r, stencil_at(r, k));  // arithmetic-bound
            if (v == 0.0f) continue;
            const double s = fma((double)k, r.ds, r.s0);
            int b_lo, b_hi;
            tof_bin_range(s, t, q.lo, q.hi, b_lo, b_hi);
            if (t.lut) {
                for (int b = b_lo; b <= b_hi; ++b) mine[b * nt] += tof_lut(s - (t.c0 + b * t.bw), t) * v;
                continue;
            }
            // upper edge argument of bin b_lo; the next edges follow in float steps of bw
            const float x_hi0 = (float)(s - (t.c0 + b_lo * t.bw) + 0.5 * t.bw), bwf = (float)t.bw;
            float e_hi = tof_erf(x_hi0, q.inv, t);
            for (int b = b_lo; b <= b_hi; ++b) {
                const float e_lo = tof_erf(x_hi0 - (float)(b - b_lo + 1) * bwf, q.inv, t);
                mine[b * nt] += 0.5f * (e_hi - e_lo) * v;
                e_hi = e_lo;
            }
        }
        const float ell = r.ell;
        for (int b = 0; b < t.nb; ++b) mine[b * nt] *= ell;
    }
    __syncthreads();
    const int64_t nrays = (n - l0 < nt) ? (n - l0) : nt;
    const int64_t total = nrays * t.nb;
    float* out = p + l0 * t.nb;
    for (int64_t i = threadIdx.x; i < total; i += nt) {
        const int ray = (int)(i / t.nb), b = (int)(i - (int64_t)ray * t.nb);
        out[i] = lds[b * nt + ray];
    }
}

// ------------------------------------------------------- work counter ----
//
// Plane samples per ray whose 2x2 stencil has at least one voxel inside the
// grid; for TOF listmode (bins != nullptr) only samples strictly inside the
// event's TOF window (non-zero weight).  Same traversal as the projectors.

__global__ void __launch_bounds__(kBlock) k_count(RaySrc src,
                                                  const int16_t* __restrict__ bins, int64_t n, GeomK g, TofK t,
                                                  int32_t* __restrict__ counts) {
    const int64_t l = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (l >= n) return;
    int cnt = 0;
    RayK r;
    TofRay q{};
    bool ok = ray_setup(src, l, g, r);
    double centre = 0.0;
    if (ok && bins) {
        const int b = bins[l];
        ok = b >= 0 && b < t.nb && tof_ray<true>(t, l, q);
        r.s0 -= q.shift;
        centre = t.c0 + b * t.bw;
        ok = ok && tof_window(r, centre, q.lo, q.hi);
    }
    if (ok) {
        for (int k = r.k_lo; k <= r.k_hi; ++k) {
            const Stencil st = stencil_at(r, k);
            if (!((st.i0ok || st.i1ok) && (st.j0ok || st.j1ok))) continue;
            if (bins) {
                const double x = fma((double)k, r.ds, r.s0) - centre;
                if (!(x > q.lo && x < q.hi)) continue;
            }
            ++cnt;
        }
    }
    counts[l] = cnt;
}

// --------------------------------------------------------------- launch ----

static unsigned grid_for(int64_t n, int block) { return (unsigned)((n + block - 1) / block); }

hipError_t launch_fwd(const RaySrc& src, int64_t n, const GeomK& g, const float* img, float* p,
                      const int32_t* order, hipStream_t s) {
    hipLaunchKernelGGL(k_fwd, dim3(grid_for(n, kBlock)), dim3(kBlock), 0, s, src, n, g, img, p, order);
    return hipGetLastError();
}

// Back projections of ray lists go through the run/sheet kernel (sheet.hpp).
template <class Mode>
static hipError_t launch_runs(const Mode& m, const RaySrc& src, int64_t n, const GeomK& g, float* img,
                              const int32_t* order, hipStream_t s, int n_img = 1, int64_t img_stride = 0) {
    const int nw = (g.n[2] <= kSheetMaxW) ? g.n[2] : 0;
    const size_t lds = SheetLayout::bytes(nw, g);
    hipError_t e = hipFuncSetAttribute((const void*)k_back_runs<Mode>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)lds);
    if (e != hipSuccess) return e;
    // enough workgroups for about 4 per CU (small subsets), at most kSheetGroups groups each
    int dev = 0, cus = 256;
    if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) !=
                                                 hipSuccess || cus <= 0)
        cus = 256;
    int64_t groups = (n + (int64_t)kSheetBlock * 4 * cus - 1) / ((int64_t)kSheetBlock * 4 * cus);
    groups = groups < 1 ? 1 : (groups > kSheetGroups ? kSheetGroups : groups);
    hipLaunchKernelGGL(k_back_runs<Mode>, dim3(grid_for(n, kSheetBlock * groups)), dim3(kSheetBlock), lds, s, m, src, n,
                       g, img, order, nw, (int)groups, n_img, img_stride);
    return hipGetLastError();
}

hipError_t launch_back(const RaySrc& src, int64_t n, const GeomK& g, float* img, const float* p,
                       const int32_t* order, hipStream_t s) {
    ModeNonTof m{p};
    return launch_runs(m, src, n, g, img, order, s);
}

hipError_t launch_fwd_tof_lm(const RaySrc& src, const int16_t* bins, int64_t n, const GeomK& g,
                             const TofK& t, const float* img, float* p, const int32_t* order, hipStream_t s) {
    const bool per = t.sig_ray || t.off_ray;
    const int form = tof_form(t);
    auto* k = form == kFormLut    ? (per ? k_fwd_tof_lm<kFormLut, true> : k_fwd_tof_lm<kFormLut, false>)
              : form == kFormPoly ? (per ? k_fwd_tof_lm<kFormPoly, true> : k_fwd_tof_lm<kFormPoly, false>)
                                  : (per ? k_fwd_tof_lm<kFormErf, true> : k_fwd_tof_lm<kFormErf, false>);
    hipLaunchKernelGGL(k, dim3(grid_for(n, kBlock)), dim3(kBlock), 0, s, src, bins, n, g, t, img, p, order,
                       EventsOut{});
    return hipGetLastError();
}

hipError_t launch_fwd_tof_lm_gather(const RaySrc& src, const int16_t* bins, int64_t n, const GeomK& g,
                                    const TofK& t, const float* img, float* p, const int32_t* order,
                                    const EventsOut& eo, hipStream_t s) {
    const int form = tof_form(t);
    auto* k = form == kFormLut    ? k_fwd_tof_lm<kFormLut, false, true>
              : form == kFormPoly ? k_fwd_tof_lm<kFormPoly, false, true>
                                  : k_fwd_tof_lm<kFormErf, false, true>;
    hipLaunchKernelGGL(k, dim3(grid_for(n, kBlock)), dim3(kBlock), 0, s, src, bins, n, g, t, img, p, order, eo);
    return hipGetLastError();
}

hipError_t launch_fwd_tof_lm_batch(const RaySrc& src, const int16_t* bins, int64_t n, const GeomK& g, const TofK& t,
                                   const float* imgs, int n_img, float* p, const int32_t* order, hipStream_t s) {
    const bool per = t.sig_ray || t.off_ray;
    const int form = tof_form(t);
    auto* k = form == kFormLut    ? (per ? k_fwd_tof_lm_batch<kFormLut, true> : k_fwd_tof_lm_batch<kFormLut, false>)
              : form == kFormPoly ? (per ? k_fwd_tof_lm_batch<kFormPoly, true> : k_fwd_tof_lm_batch<kFormPoly, false>)
                                  : (per ? k_fwd_tof_lm_batch<kFormErf, true> : k_fwd_tof_lm_batch<kFormErf, false>);
    // images per launch: at most kFwdBatch, and their bytes within the 32-bit buffer range
    const int64_t nv = (int64_t)g.n[0] * g.n[1] * g.n[2];
    int64_t per_launch = ((int64_t(1) << 32) - 1) / (nv * 4);
    if (per_launch > kFwdBatch) per_launch = kFwdBatch;
    for (int b0 = 0; b0 < n_img; b0 += (int)per_launch) {
        const int cnt = (n_img - b0 < per_launch) ? (n_img - b0) : (int)per_launch;
        hipLaunchKernelGGL(k, dim3(grid_for(n, kBlock)), dim3(kBlock), 0, s, src, bins, n, g, t, imgs + b0 * nv, cnt,
                           p + b0 * n, order);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t launch_back_tof_lm(const RaySrc& src, const int16_t* bins, int64_t n, const GeomK& g,
                              const TofK& t, float* img, const float* p, const int32_t* order, hipStream_t s) {
    const int form = tof_form(t);
    if (t.sig_ray || t.off_ray) {
        if (form == kFormLut) return launch_runs(ModeTofLm<kFormLut, true>{p, bins, t}, src, n, g, img, order, s);
        if (form == kFormPoly) return launch_runs(ModeTofLm<kFormPoly, true>{p, bins, t}, src, n, g, img, order, s);
        return launch_runs(ModeTofLm<kFormErf, true>{p, bins, t}, src, n, g, img, order, s);
    }
    if (form == kFormLut) return launch_runs(ModeTofLm<kFormLut>{p, bins, t}, src, n, g, img, order, s);
    if (form == kFormPoly) return launch_runs(ModeTofLm<kFormPoly>{p, bins, t}, src, n, g, img, order, s);
    return launch_runs(ModeTofLm<kFormErf>{p, bins, t}, src, n, g, img, order, s);
}

// Images per launch of the batched listmode back projection (each launch walks the events once)
constexpr int kBackBatch = 16;

hipError_t launch_back_tof_lm_batch(const RaySrc& src, const int16_t* bins, int64_t n, const GeomK& g,
                                    const TofK& t, float* imgs, int n_img, const float* p, const int32_t* order,
                                    hipStream_t s) {
    const int64_t nv = (int64_t)g.n[0] * g.n[1] * g.n[2];
    const int form = tof_form(t);
    const bool per = t.sig_ray || t.off_ray;
    for (int b0 = 0; b0 < n_img; b0 += kBackBatch) {
        const int cnt = (n_img - b0 < kBackBatch) ? (n_img - b0) : kBackBatch;
        float* im = imgs + (int64_t)b0 * nv;
        const float* pb = p + (int64_t)b0 * n;
        hipError_t e;
        if (per) {
            if (form == kFormLut) e = launch_runs(ModeTofLm<kFormLut, true, true>{pb, bins, t}, src, n, g, im, order, s, cnt, nv);
            else if (form == kFormPoly) e = launch_runs(ModeTofLm<kFormPoly, true, true>{pb, bins, t}, src, n, g, im, order, s, cnt, nv);
            else e = launch_runs(ModeTofLm<kFormErf, true, true>{pb, bins, t}, src, n, g, im, order, s, cnt, nv);
        } else {
            if (form == kFormLut) e = launch_runs(ModeTofLm<kFormLut, false, true>{pb, bins, t}, src, n, g, im, order, s, cnt, nv);
            else if (form == kFormPoly) e = launch_runs(ModeTofLm<kFormPoly, false, true>{pb, bins, t}, src, n, g, im, order, s, cnt, nv);
            else e = launch_runs(ModeTofLm<kFormErf, false, true>{pb, bins, t}, src, n, g, im, order, s, cnt, nv);
        }
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

static int sino_block(int nb) { return nb <= 64 ? 256 : 64; }  // LDS tile <= 64 KiB

hipError_t launch_fwd_tof_sino(const RaySrc& src, int64_t n, const GeomK& g, const TofK& t,
                               const float* img, float* p, hipStream_t s) {
    const int blk = sino_block(t.nb);
    const size_t lds = (size_t)t.nb * blk * sizeof(float);
    hipLaunchKernelGGL((t.sig_ray || t.off_ray) ? k_fwd_tof_sino<true> : k_fwd_tof_sino<false>, dim3(grid_for(n, blk)),
                       dim3(blk), lds, s, src, n, g, t, img, p);
    return hipGetLastError();
}

hipError_t launch_back_tof_sino(const RaySrc& src, int64_t n, const GeomK& g, const TofK& t,
                                float* img, const float* p, hipStream_t s) {
    // the run/sheet kernel carries ray indices in 32 bits: the C ABI takes n < 2^31
    if (t.sig_ray || t.off_ray) {
        if (t.lut) return launch_runs(ModeTofSino<true, true>{p, t}, src, n, g, img, nullptr, s);
        return launch_runs(ModeTofSino<false, true>{p, t}, src, n, g, img, nullptr, s);
    }
    if (t.lut) return launch_runs(ModeTofSino<true>{p, t}, src, n, g, img, nullptr, s);
    return launch_runs(ModeTofSino<false>{p, t}, src, n, g, img, nullptr, s);
}

// The Gaussian bin weight w(x) = (erf(clip(x + bw/2) / (sqrt2 sigma)) - erf(clip(x - bw/2) /
// (sqrt2 sigma))) / 2, clip at +-trunc, at x_i = x0 + i dx, in float64 (the device library's erf).
__global__ void __launch_bounds__(kBlock) k_tof_gauss_table(float* __restrict__ lut, int n, double x0, double dx,
                                                           double hbw, double trunc, double inv_s2) {
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    const double x = fma((double)i, dx, x0);
    const double a = fmin(fmax(x + hbw, -trunc), trunc), b = fmin(fmax(x - hbw, -trunc), trunc);
    lut[i] = (float)(0.5 * (erf(a * inv_s2) - erf(b * inv_s2)));
}

hipError_t launch_tof_gauss_table(float* lut, int n, double x0, double dx, double bw, double sigma, double n_sigmas,
                                  hipStream_t s) {
    hipLaunchKernelGGL(k_tof_gauss_table, dim3(grid_for(n, kBlock)), dim3(kBlock), 0, s, lut, n, x0, dx, 0.5 * bw,
                       n_sigmas * sigma, 1.0 / (sqrt(2.0) * sigma));
    return hipGetLastError();
}

hipError_t launch_count(const RaySrc& src, const int16_t* bins, int64_t n, const GeomK& g,
                        const TofK& t, int32_t* counts, hipStream_t s) {
    hipLaunchKernelGGL(k_count, dim3(grid_for(n, kBlock)), dim3(kBlock), 0, s, src, bins, n, g, t, counts);
    return hipGetLastError();
}

}  // namespace ppmi
