// Batched listmode TOF OSEM on device-resident frames (the paper's listmode
// OSEM of Sec. 2.6, run for many frames at once).
//
// Event storage of a frame is subset-major: subset j (the events whose index
// in the frame is j mod n_sub) occupies the contiguous range
// [off_j, off_j + n_j) with n_j = n / n_sub + (j < n mod n_sub) and
// off_j = j * (n / n_sub) + min(j, n mod n_sub); inside a subset the events
// may be in any order (pp_lm_presort with n_sub groups them by LOR).
//
// k_osem_accumulate: one persistent grid walks the work chunks of all live
// slots (a chunk = 1024 consecutive events of one slot's current subset); each
// lane projects its event forward through the slot's image, forms
// ell / ybar and back projects it into the slot's accumulator -- forward,
// ratio and back projection fused, the event set up once.  The scatter is the
// run/sheet back projection of sheet.hpp (LDS sheets for runs of events on one
// transaxial line, run-combined atomics for the rest).
// k_osem_update: x <- x * acc / (sens / n_sub) (0 where sens == 0), acc <- 0, for
// the slots without the resolution model (blur.hip updates the others).
// k_osem_advance: next subset, one step fewer.
#include <hip/hip_runtime.h>

#include "joseph.hpp"
#include "launch.hpp"
#include "sheet.hpp"

namespace ppmi {

constexpr int kOsemBlock = 256;
constexpr int kOsemGroups = 4;
constexpr int64_t kOsemChunk = (int64_t)kSheetBlock * kOsemGroups;  // events of one work chunk

// live: active with steps to run, a well-formed subset state (n_sub >= 1, 0 <= subset < n_sub,
// n_events >= 0: anything else would place the subset's range outside the events), and (without
// the resolution model, or with its scratch image) (coordinates, or a usable crystal table)
__device__ __forceinline__ bool slot_live(const pp_frame_desc_t& s) {
    return s.active && s.steps_left > 0 && s.n_sub >= 1 && s.subset >= 0 && s.subset < s.n_sub &&
           s.n_events >= 0 && (s.x_fwd == nullptr || s.tmp != nullptr) &&
           (s.crystal_pair == nullptr || (s.crystal_xyz != nullptr && s.n_crystals > 0));
}

__host__ __device__ inline int64_t slot_chunks(int64_t n_events, int32_t n_sub) {
    if (n_events <= 0 || n_sub <= 0) return 0;
    const int64_t per_subset = (n_events + n_sub - 1) / n_sub;  // largest subset
    return (per_subset + kOsemChunk - 1) / kOsemChunk;
}

// Per event: forward project through the frame's current image (setup), then scatter
// ell / ybar times the TOF weight (sample) -- the run/sheet back projection of sheet.hpp.
template <int Form>
struct ModeOsem {
    static constexpr bool kAux = false;
    static constexpr bool kBatch = false;
    const float* __restrict__ x;
    const int16_t* __restrict__ bins;
    float bg;
    TofK t;
    __device__ bool setup(int64_t l, const RaySrc& src, const GeomK& g, RayK& r, float& cv,
                          int& /*aux*/) const {
        const int b = bins[l];
        if (b < 0 || b >= t.nb || !ray_setup(src, l, g, r)) return false;
        if (!tof_window_rel(r, t.c0 + b * t.bw, t.lo, t.hi)) return false;
        const __amdgpu_buffer_rsrc_t ib = img_buffer(x, g);
        float fwd = 0.0f;
        for (int k = r.k_lo; k <= r.k_hi; ++k) {
            const float w = tof_weight_unscaled<Form, true>(fma((double)k, r.ds, r.s0), t, t.u_per_mm);
            fwd += w * stencil_gather(ib, r, stencil_at(r, k));
        }
        const float ybar = r.ell * kTofScale<Form> * fwd + bg;
        if (!(ybar > 0.0f)) return false;
        cv = r.ell / ybar * kTofScale<Form>;
        return true;
    }
    __device__ float sample(double x, float cv, int /*aux*/) const {
        return tof_weight_unscaled<Form>(x, t, t.u_per_mm) * cv;
    }
    __device__ void to_vgprs() {
        if constexpr (Form == kFormPoly) tof_poly_to_vgprs(t);
    }
    __device__ float mag(float cv, int /*aux*/) const { return fabsf(cv); }
    __device__ float weight_bound(float* red) const { return tof_weight_bound<Form>(t, red); }
};

template <int Form>
__global__ void __launch_bounds__(kSheetBlock) k_osem_accumulate(const pp_frame_desc_t* __restrict__ slots,
                                                                 int n_slots, GeomK g, TofK t, int nw_lds) {
    extern __shared__ double smem[];
    const pp_frame_desc_t& last = slots[n_slots - 1];
    const int64_t total = last.chunk_begin + (last.active ? slot_chunks(last.n_events, last.n_sub) : 0);
    for (int64_t c = blockIdx.x; c < total; c += gridDim.x) {
        // largest slot index whose first chunk is <= c (block-uniform)
        int lo_s = 0, hi_s = n_slots - 1;
        while (lo_s < hi_s) {
            const int mid = (lo_s + hi_s + 1) >> 1;
            if (slots[mid].chunk_begin <= c) lo_s = mid; else hi_s = mid - 1;
        }
        const pp_frame_desc_t& s = slots[lo_s];
        if (!slot_live(s)) continue;  // block-uniform
        const int64_t n = s.n_events, ns = s.n_sub, j = s.subset;
        const int64_t base_n = n / ns, rem = n - base_n * ns;
        const int64_t n_j = base_n + (j < rem ? 1 : 0);
        const int64_t off_j = j * base_n + (j < rem ? j : rem);
        const int64_t q0 = (c - s.chunk_begin) * kOsemChunk;
        if (q0 < 0 || q0 >= n_j) continue;  // chunk offsets not from pp_osem_chunks: nothing to do
        ModeOsem<Form> m{s.x_fwd ? s.x_fwd : s.x, s.tof_bin + off_j, s.bg, t};
        const RaySrc src = s.crystal_pair ? RaySrc{s.crystal_xyz, nullptr, reinterpret_cast<const int2*>(s.crystal_pair),
                                                   s.n_crystals}
                                          : RaySrc{s.xstart, s.xend, nullptr, 0};
        back_runs_chunk(m, src.from(off_j), n_j, g, s.acc, nullptr, nw_lds, kOsemGroups, q0, smem);
    }
}

// grid: (blocks per slot, slots); a workgroup of a slot that is not live (or has the resolution
// model: blur.hip updates it) returns at once, so empty slots of a large table cost almost nothing
__global__ void __launch_bounds__(kOsemBlock) k_osem_update(const pp_frame_desc_t* __restrict__ slots, int64_t n_vox) {
    const pp_frame_desc_t& s = slots[blockIdx.y];
    if (!slot_live(s) || s.x_fwd != nullptr) return;  // block-uniform
    const float scale = 1.0f / (float)s.n_sub;
    const int64_t stride = (int64_t)gridDim.x * kOsemBlock;
    for (int64_t v = (int64_t)blockIdx.x * kOsemBlock + threadIdx.x; v < n_vox; v += stride) {
        const float sv = s.sens[v];
        const float a = s.acc[v];
        s.x[v] = (sv > 0.0f) ? s.x[v] * a / (sv * scale) : 0.0f;
        s.acc[v] = 0.0f;
    }
}

__global__ void k_osem_advance(pp_frame_desc_t* slots, int n_slots) {
    for (int i = threadIdx.x; i < n_slots; i += blockDim.x) {
        pp_frame_desc_t& s = slots[i];
        if (!slot_live(s)) continue;
        s.subset = (s.subset + 1) % s.n_sub;
        s.steps_left -= 1;
    }
}

__global__ void k_osem_init(float* __restrict__ x, const float* __restrict__ sens, int64_t n_vox) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n_vox; i += stride)
        x[i] = sens[i] > 0.0f ? 1.0f : 0.0f;
}

__global__ void k_fill(float* __restrict__ dst, int64_t n, float value) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) dst[i] = value;
}

int64_t osem_chunks(int64_t n_events, int32_t n_sub) { return slot_chunks(n_events, n_sub); }

template <int Form>
static hipError_t launch_accumulate(const pp_frame_desc_t* slots, int n_slots, const GeomK& g, const TofK& t, int cus,
                                   hipStream_t s) {
    const int nw = (g.n[2] <= kSheetMaxW) ? g.n[2] : 0;
    const size_t lds = SheetLayout::bytes(nw, g);
    hipError_t e = hipFuncSetAttribute((const void*)k_osem_accumulate<Form>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    // persistent grid: as many workgroups as can be resident at once (LDS-limited)
    int per_cu = 0;
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void*)k_osem_accumulate<Form>, kSheetBlock, lds);
    if (e != hipSuccess) return e;
    if (per_cu < 1) per_cu = 1;
    hipLaunchKernelGGL(k_osem_accumulate<Form>, dim3(cus * per_cu), dim3(kSheetBlock), lds, s, slots, n_slots, g, t,
                       nw);
    return hipGetLastError();
}

hipError_t launch_osem_accumulate(const pp_frame_desc_t* slots, int n_slots, const GeomK& g, const TofK& t, int cus,
                                  hipStream_t s) {
    const int form = tof_form(t);
    if (form == kFormLut) return launch_accumulate<kFormLut>(slots, n_slots, g, t, cus, s);
    if (form == kFormPoly) return launch_accumulate<kFormPoly>(slots, n_slots, g, t, cus, s);
    return launch_accumulate<kFormErf>(slots, n_slots, g, t, cus, s);
}

hipError_t launch_osem_update(pp_frame_desc_t* slots, int n_slots, int64_t n_vox, int n_blocks, hipStream_t s) {
    constexpr int kMaxY = 65535;  // grid limit along y: tables beyond it go in several launches
    for (int first = 0; first < n_slots; first += kMaxY) {
        const int count = (n_slots - first < kMaxY) ? (n_slots - first) : kMaxY;
        hipLaunchKernelGGL(k_osem_update, dim3((unsigned)n_blocks, (unsigned)count), dim3(kOsemBlock), 0, s,
                           slots + first, n_vox);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t launch_osem_advance(pp_frame_desc_t* slots, int n_slots, hipStream_t s) {
    hipLaunchKernelGGL(k_osem_advance, dim3(1), dim3(256), 0, s, slots, n_slots);
    return hipGetLastError();
}

static unsigned fill_blocks(int64_t n) {
    int64_t blocks = (n + 255) / 256;
    return (unsigned)(blocks > 8192 ? 8192 : blocks);
}

hipError_t launch_osem_init(float* x, const float* sens, int64_t n_vox, hipStream_t s) {
    hipLaunchKernelGGL(k_osem_init, dim3(fill_blocks(n_vox)), dim3(256), 0, s, x, sens, n_vox);
    return hipGetLastError();
}

hipError_t launch_fill(float* dst, int64_t n, float value, hipStream_t s) {
    hipLaunchKernelGGL(k_fill, dim3(fill_blocks(n)), dim3(256), 0, s, dst, n, value);
    return hipGetLastError();
}

}  // namespace ppmi
