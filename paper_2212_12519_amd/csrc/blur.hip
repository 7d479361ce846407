// Image-based resolution model: a shift-invariant 3-D Gaussian blur G of the
// image (the paper's listmode OSEM reconstructions include one, Sec. 2.6).
//
// G is the product of three 1-D kernels: along axis a the taps
// exp(-i^2 / (2 s_a^2)), |i| <= r_a, normalised to sum 1, with
// s_a = FWHM_a / (2 sqrt(2 ln 2)) / h_a voxels and r_a = floor(4 s_a + 1/2)
// (FWHM_a == 0: the single tap 1); voxels outside the grid read as 0.  The
// kernel is symmetric, so G is its own adjoint.  It is applied as one pass per
// axis.  A pass is bound by HBM (read + write of the image, 8 B per voxel; the
// 2 r + 1 neighbours along the axis come from L2): each thread produces one
// voxel, consecutive threads consecutive voxels along axis 2 (fastest), so
// every tap of every pass is a coalesced load of a contiguous row.
//
// In batched OSEM with the model the system matrix is A G: the forward
// projects x_fwd = G x and the update uses G acc.  Per step and frame:
//   acc -> tmp (axis 0), tmp -> acc (axis 1),
//   acc -> (axis 2) G acc, fused with x <- x * G acc / (sens / n_sub);
//   x -> acc (axis 0), acc -> tmp (axis 1), tmp -> x_fwd (axis 2) with acc <- 0.
#include <hip/hip_runtime.h>

#include "joseph.hpp"
#include "launch.hpp"

namespace ppmi {

constexpr int kBlurBlock = 256;

struct GridDims {
    int n0, n1, n2;
};

// One output voxel of the pass along Axis.  The tap loop is wave-uniform (the
// tap index never depends on the lane), so the weights are scalar loads.
template <int Axis>
__device__ __forceinline__ float blur_at(const float* __restrict__ src, int64_t v, const GaussK& k, GridDims d) {
    int pos, len;
    int64_t stride;
    if (Axis == 2) {
        pos = (int)(v % d.n2);
        len = d.n2;
        stride = 1;
    } else if (Axis == 1) {
        pos = (int)((v / d.n2) % d.n1);
        len = d.n1;
        stride = d.n2;
    } else {
        stride = (int64_t)d.n1 * d.n2;
        pos = (int)(v / stride);
        len = d.n0;
    }
    const int r = k.r[Axis];
    float acc = 0.0f;
    for (int i = -r; i <= r; ++i) {
        const int q = pos + i;
        const float s = (q >= 0 && q < len) ? src[v + (int64_t)i * stride] : 0.0f;
        acc = fmaf(k.w[Axis][i + r], s, acc);
    }
    return acc;
}

template <int Axis>
__global__ void __launch_bounds__(kBlurBlock) k_blur(const float* __restrict__ src, float* __restrict__ dst,
                                                     int64_t n_vox, GaussK k, GridDims d) {
    const int64_t stride = (int64_t)gridDim.x * kBlurBlock;
    for (int64_t v = (int64_t)blockIdx.x * kBlurBlock + threadIdx.x; v < n_vox; v += stride)
        dst[v] = blur_at<Axis>(src, v, k, d);
}

// ---------------------------------------------------------------- batched OSEM

enum SlotField { kFieldX = 0, kFieldXFwd = 1, kFieldAcc = 2, kFieldTmp = 3 };
enum BlurOp {
    kOpCopy = 0,    // dst = blur(src)
    kOpUpdate = 1,  // x = x * blur(src) / (sens / n_sub), 0 where sens <= 0
    kOpZero = 2     // dst = blur(src) and acc = 0
};

__device__ __forceinline__ float* slot_field(const pp_frame_desc_t& s, int f) {
    return f == kFieldX ? s.x : f == kFieldXFwd ? s.x_fwd : f == kFieldAcc ? s.acc : s.tmp;
}

__device__ __forceinline__ bool slot_res_live(const pp_frame_desc_t& s) {
    return s.active && s.steps_left > 0 && s.n_sub >= 1 && s.subset >= 0 && s.subset < s.n_sub &&
           s.n_events >= 0 && s.x_fwd != nullptr && s.tmp != nullptr;
}

template <int Axis, int Op>
__global__ void __launch_bounds__(kBlurBlock) k_osem_blur(const pp_frame_desc_t* __restrict__ slots, int n_slots,
                                                          int64_t n_vox, GaussK k, GridDims d, int src_f,
                                                          int dst_f) {
    const int64_t total = (int64_t)n_slots * n_vox;
    const int64_t stride = (int64_t)gridDim.x * kBlurBlock;
    for (int64_t i = (int64_t)blockIdx.x * kBlurBlock + threadIdx.x; i < total; i += stride) {
        const int si = (int)(i / n_vox);
        const int64_t v = i - (int64_t)si * n_vox;
        const pp_frame_desc_t& s = slots[si];
        if (!slot_res_live(s)) continue;
        const float b = blur_at<Axis>(slot_field(s, src_f), v, k, d);
        if (Op == kOpUpdate) {
            const float sv = s.sens[v];
            s.x[v] = (sv > 0.0f) ? s.x[v] * b / (sv / (float)s.n_sub) : 0.0f;
        } else {
            slot_field(s, dst_f)[v] = b;
            if (Op == kOpZero) s.acc[v] = 0.0f;
        }
    }
}

static unsigned blur_blocks(int64_t total, int cus) {
    int64_t blocks = (total + kBlurBlock - 1) / kBlurBlock;
    const int64_t cap = (int64_t)cus * 16;
    return (unsigned)(blocks > cap ? cap : blocks);
}

static GridDims dims_of(const GeomK& g) { return GridDims{g.n[0], g.n[1], g.n[2]}; }

hipError_t launch_gauss3d(const float* src, float* dst, float* tmp, const GeomK& g, const GaussK& k, int cus,
                          hipStream_t s) {
    const int64_t nv = (int64_t)g.n[0] * g.n[1] * g.n[2];
    const GridDims d = dims_of(g);
    const unsigned nb = blur_blocks(nv, cus);
    hipLaunchKernelGGL(k_blur<0>, dim3(nb), dim3(kBlurBlock), 0, s, src, dst, nv, k, d);
    hipLaunchKernelGGL(k_blur<1>, dim3(nb), dim3(kBlurBlock), 0, s, dst, tmp, nv, k, d);
    hipLaunchKernelGGL(k_blur<2>, dim3(nb), dim3(kBlurBlock), 0, s, tmp, dst, nv, k, d);
    return hipGetLastError();
}

hipError_t launch_osem_res_update(pp_frame_desc_t* slots, int n_slots, const GeomK& g, const GaussK& k, int cus,
                                  hipStream_t s) {
    const int64_t nv = (int64_t)g.n[0] * g.n[1] * g.n[2];
    const GridDims d = dims_of(g);
    const unsigned nb = blur_blocks((int64_t)n_slots * nv, cus);
    const dim3 grid(nb), block(kBlurBlock);
    hipLaunchKernelGGL((k_osem_blur<0, kOpCopy>), grid, block, 0, s, slots, n_slots, nv, k, d, kFieldAcc, kFieldTmp);
    hipLaunchKernelGGL((k_osem_blur<1, kOpCopy>), grid, block, 0, s, slots, n_slots, nv, k, d, kFieldTmp, kFieldAcc);
    hipLaunchKernelGGL((k_osem_blur<2, kOpUpdate>), grid, block, 0, s, slots, n_slots, nv, k, d, kFieldAcc, kFieldX);
    hipLaunchKernelGGL((k_osem_blur<0, kOpCopy>), grid, block, 0, s, slots, n_slots, nv, k, d, kFieldX, kFieldAcc);
    hipLaunchKernelGGL((k_osem_blur<1, kOpCopy>), grid, block, 0, s, slots, n_slots, nv, k, d, kFieldAcc, kFieldTmp);
    hipLaunchKernelGGL((k_osem_blur<2, kOpZero>), grid, block, 0, s, slots, n_slots, nv, k, d, kFieldTmp, kFieldXFwd);
    return hipGetLastError();
}

}  // namespace ppmi
