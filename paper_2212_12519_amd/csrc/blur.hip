// Image-based resolution model: a shift-invariant 3-D Gaussian blur G of the
// image (the paper's listmode OSEM reconstructions include one, Sec. 2.6).
//
// G is the product of three 1-D kernels: along axis a the taps
// exp(-i^2 / (2 s_a^2)), |i| <= r_a, normalised to sum 1, with
// s_a = FWHM_a / (2 sqrt(2 ln 2)) / h_a voxels and r_a = floor(4 s_a + 1/2)
// (FWHM_a == 0: the single tap 1); voxels outside the grid read as 0.  The
// kernel is symmetric, so G is its own adjoint, and the three 1-D passes
// commute (each acts on its own index, with the zero padding of its own axis).
//
// Two kernels per blur:
//   k_blur21: a workgroup takes one plane i (axis 0) and a tile of rows j
//     (axis 1); it blurs the tile's rows plus r_1 halo rows on each side along
//     axis 2 straight from global memory (the 2 r_2 + 1 taps of a row are one
//     contiguous, cached line) into LDS, then blurs the tile along axis 1 out
//     of LDS and writes it: one HBM read and one write per voxel for two axes.
//   k_blur0: one thread per voxel, consecutive threads consecutive voxels of a
//     plane, the 2 r_0 + 1 taps along axis 0 as coalesced rows of the planes
//     around it; the batched OSEM update (or the copy to G x with the
//     accumulator cleared) is fused into this last pass.
// Grids whose tile would not fit the LDS budget (very long axis 2 with a wide
// kernel along axis 1) take three plain per-axis passes instead.
//
// In batched OSEM with the model the system matrix is A G: the forward
// projects x_fwd = G x and the update uses G acc.  Per step and frame:
//   acc -> tmp (axes 2, 1), tmp -> (axis 0) G acc fused with
//   x <- x * G acc / (sens / n_sub);
//   x -> tmp (axes 2, 1), tmp -> (axis 0) x_fwd, fused with acc <- 0.
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
        acc = fmaf(k.w[Axis][i + kGaussMaxR], s, acc);
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

// ------------------------------------------------- tiled passes (axes 2+1, axis 0)
//
// R: compile-time tap bound (every radius up to 8, then 16 and kGaussMaxR), covering the largest
// radius of the three axes.  The taps are unrolled to R with no branches: weights beyond an axis'
// own radius are 0 in the centred table, and taps outside the grid read a valid address whose value
// is replaced by 0, so the loads of all taps are in flight together.

constexpr int kBlurTileRows = 32;              // rows j of a k_blur21 tile
constexpr size_t kBlurLdsBudget = 64 * 1024;   // LDS of one k_blur21 workgroup (two buffers)
constexpr int kBlurUnroll = 4;                 // row elements a thread loads at once

// rows of a k_blur21 tile for this grid and kernel, 0 if even one row does not fit the budget (the
// raw rows carry kGaussMaxR zeros of padding on each side: the budget holds for any tap bound)
static int blur_tile_rows(const GridDims& d, const GaussK& k) {
    const int64_t per_row = ((int64_t)d.n2 * 2 + 2 * kGaussMaxR) * 4;
    const int64_t fit = (int64_t)kBlurLdsBudget / per_row - 2 * k.r[1];
    if (fit < 1) return 0;
    int tj = kBlurTileRows < d.n1 ? kBlurTileRows : d.n1;
    return (int)(fit < tj ? fit : tj);
}

template <int R>
static size_t blur21_lds(const GridDims& d, const GaussK& k, int tj) {
    return (size_t)(tj + 2 * k.r[1]) * (2 * d.n2 + 2 * R) * sizeof(float);
}

// e / n for 0 <= e < 2^22 by a float reciprocal: (e + 1/2) / n stays at least 1/(2n) away from
// an integer, far more than the float error
__device__ __forceinline__ int div_small(int e, float inv_n) { return (int)(((float)e + 0.5f) * inv_n); }

// Tile (plane i, rows j0 .. j0 + tj - 1) of dst = G_1 G_2 src.  The tile's rows plus r_1 halo rows on
// each side are contiguous in memory: they are read once, coalesced, into LDS rows padded with R
// zeros on each side (rows outside the grid all zeros), blurred along axis 2 into a second LDS
// buffer (each tap a read at a fixed offset), and blurred along axis 1 from there.
template <int R>
__device__ __forceinline__ void blur21_tile(const float* __restrict__ src, float* __restrict__ dst, const GaussK& k,
                                            GridDims d, int i, int j0, int tj, float* lds) {
    const int r1 = k.r[1], n1 = d.n1, n2 = d.n2;
    const int rows = tj + 2 * r1, ne = rows * n2, ps = n2 + 2 * R;  // padded row stride
    float* A = lds;               // [rows][R zeros, n2 values, R zeros]
    float* B = lds + rows * ps;   // [rows][n2]
    const int64_t top = (int64_t)i * n1 * n2 + (int64_t)(j0 - r1) * n2;  // element 0 of the tile's first row
    // the elements of rows inside the grid: [e_lo, e_hi) (never empty: row r1 is the tile's first row)
    const int e_lo = max(r1 - j0, 0) * n2, e_hi = min(rows, n1 - j0 + r1) * n2;
    const float inv_n2 = 1.0f / (float)n2;
    for (int e0 = threadIdx.x; e0 < ne; e0 += kBlurBlock * kBlurUnroll) {
        float v[kBlurUnroll];
#pragma unroll
        for (int u = 0; u < kBlurUnroll; ++u) {
            const int e = e0 + u * kBlurBlock;
            v[u] = src[top + min(max(e, e_lo), e_hi - 1)];
        }
#pragma unroll
        for (int u = 0; u < kBlurUnroll; ++u) {
            const int e = e0 + u * kBlurBlock;
            const int row = div_small(e, inv_n2);
            if (e < ne) A[row * ps + R + (e - row * n2)] = (e >= e_lo && e < e_hi) ? v[u] : 0.0f;
        }
    }
    if (R > 0) {
        for (int q = threadIdx.x; q < rows * 2 * R; q += kBlurBlock) {
            const int row = q / (2 * R), c = q - row * 2 * R;
            A[row * ps + (c < R ? c : n2 + c)] = 0.0f;
        }
    }
    __syncthreads();
    for (int e = threadIdx.x; e < ne; e += kBlurBlock) {
        const int row = div_small(e, inv_n2);
        const float* a = A + row * ps + (e - row * n2);  // a[R + t]: tap t of element e
        float acc = 0.0f;
#pragma unroll
        for (int t = -R; t <= R; ++t) acc = fmaf(k.w[2][t + kGaussMaxR], a[R + t], acc);
        B[e] = acc;
    }
    __syncthreads();
    const int e_out = min(tj, n1 - j0) * n2;
    float* out = dst + top + (int64_t)r1 * n2;
    for (int e = threadIdx.x; e < e_out; e += kBlurBlock) {
        float acc = 0.0f;
#pragma unroll
        for (int t = -R; t <= R; ++t) {
            const int row = min(max(r1 + t, 0), 2 * r1);  // |t| <= r1 rows exist; beyond, the weight is 0
            acc = fmaf(k.w[1][t + kGaussMaxR], B[e + row * n2], acc);
        }
        out[e] = acc;
    }
}

template <int R>
__global__ void __launch_bounds__(kBlurBlock) k_blur21(const float* __restrict__ src, float* __restrict__ dst, GaussK k,
                                                       GridDims d, int tj) {
    extern __shared__ float lds[];
    const int ntj = (d.n1 + tj - 1) / tj;
    const int i = blockIdx.x / ntj, jt = blockIdx.x - i * ntj;
    blur21_tile<R>(src, dst, k, d, i, jt * tj, tj, lds);
}

// Axis 0 over a chunk of planes: a thread takes one position pos of the planes and the planes
// [i0, i1) of a chunk (at most kBlurChunk); it loads the chunk's planes and R on each side into
// registers at once (all loads in flight together), so each input plane is read
// (kBlurChunk + 2R) / kBlurChunk times instead of 2R + 1.  Planes outside the grid read as 0 (a
// uniform condition; the load goes to plane i0).  emit(v, value) stores the output of voxel v.
constexpr int kBlurChunk = 16;  // planes per chunk of the axis-0 pass

template <int R, class Emit>
__device__ __forceinline__ void blur0_walk(const float* __restrict__ src, const GaussK& k, GridDims d, int i0, int i1,
                                           int64_t pos, int64_t pstride, Emit emit) {
    float col[kBlurChunk + 2 * R];
#pragma unroll
    for (int u = 0; u < kBlurChunk + 2 * R; ++u) {
        const int q = i0 - R + u;
        const bool in = q >= 0 && q < d.n0;  // uniform
        const float a = src[(int64_t)(in ? q : i0) * pstride + pos];
        col[u] = in ? a : 0.0f;
    }
#pragma unroll
    for (int u = 0; u < kBlurChunk; ++u) {
        if (i0 + u >= i1) break;  // uniform
        float acc = 0.0f;
#pragma unroll
        for (int t = -R; t <= R; ++t) acc = fmaf(k.w[0][t + kGaussMaxR], col[u + R + t], acc);
        emit((int64_t)(i0 + u) * pstride + pos, acc);
    }
}

template <int R>
__global__ void __launch_bounds__(kBlurBlock) k_blur0(const float* __restrict__ src, float* __restrict__ dst, GaussK k,
                                                      GridDims d) {
    const int64_t pstride = (int64_t)d.n1 * d.n2;
    const int npb = (int)((pstride + kBlurBlock - 1) / kBlurBlock);
    const int c = blockIdx.x / npb, pb = blockIdx.x - c * npb;
    const int64_t pos = (int64_t)pb * kBlurBlock + threadIdx.x;
    if (pos >= pstride) return;
    const int i0 = c * kBlurChunk, i1 = min(i0 + kBlurChunk, d.n0);
    blur0_walk<R>(src, k, d, i0, i1, pos, pstride, [&](int64_t v, float b) { dst[v] = b; });
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

// batched tiled passes: workgroup b = (slot, plane i, tile / block of the plane)
template <int R>
__global__ void __launch_bounds__(kBlurBlock) k_osem_blur21(const pp_frame_desc_t* __restrict__ slots, GaussK k,
                                                            GridDims d, int tj, int src_f, int dst_f) {
    extern __shared__ float lds[];
    const int ntj = (d.n1 + tj - 1) / tj;
    const int per_slot = d.n0 * ntj;
    const int si = blockIdx.x / per_slot, rest = blockIdx.x - si * per_slot;
    const int i = rest / ntj, jt = rest - i * ntj;
    const pp_frame_desc_t& s = slots[si];
    if (!slot_res_live(s)) return;  // block-uniform
    blur21_tile<R>(slot_field(s, src_f), slot_field(s, dst_f), k, d, i, jt * tj, tj, lds);
}

template <int R, int Op>
__global__ void __launch_bounds__(kBlurBlock) k_osem_blur0(const pp_frame_desc_t* __restrict__ slots, GaussK k,
                                                           GridDims d, int src_f, int dst_f) {
    const int64_t pstride = (int64_t)d.n1 * d.n2;
    const int npb = (int)((pstride + kBlurBlock - 1) / kBlurBlock);
    const int nch = (d.n0 + kBlurChunk - 1) / kBlurChunk;
    const int per_slot = nch * npb;
    const int si = blockIdx.x / per_slot, rest = blockIdx.x - si * per_slot;
    const int c = rest / npb, pb = rest - c * npb;
    const pp_frame_desc_t& s = slots[si];
    if (!slot_res_live(s)) return;  // block-uniform
    const int64_t pos = (int64_t)pb * kBlurBlock + threadIdx.x;
    if (pos >= pstride) return;
    const int i0 = c * kBlurChunk, i1 = min(i0 + kBlurChunk, d.n0);
    float* dst = slot_field(s, dst_f);
    blur0_walk<R>(slot_field(s, src_f), k, d, i0, i1, pos, pstride, [&](int64_t v, float b) {
        if (Op == kOpUpdate) {
            const float sv = s.sens[v];
            s.x[v] = (sv > 0.0f) ? s.x[v] * b / (sv / (float)s.n_sub) : 0.0f;
        } else {
            dst[v] = b;
            if (Op == kOpZero) s.acc[v] = 0.0f;
        }
    });
}

static unsigned blur_blocks(int64_t total, int cus) {
    int64_t blocks = (total + kBlurBlock - 1) / kBlurBlock;
    const int64_t cap = (int64_t)cus * 16;
    return (unsigned)(blocks > cap ? cap : blocks);
}

static GridDims dims_of(const GeomK& g) { return GridDims{g.n[0], g.n[1], g.n[2]}; }

// workgroups of the tiled passes over `copies` images (0 if their count does not fit the grid)
static int64_t tiled_blocks21(const GridDims& d, int tj, int copies) {
    return (int64_t)copies * d.n0 * ((d.n1 + tj - 1) / tj);
}
static int64_t tiled_blocks0(const GridDims& d, int copies) {
    return (int64_t)copies * ((d.n0 + kBlurChunk - 1) / kBlurChunk) *
           (((int64_t)d.n1 * d.n2 + kBlurBlock - 1) / kBlurBlock);
}
static bool tiled_ok(const GridDims& d, int tj, int copies) {
    return tj > 0 && tiled_blocks21(d, tj, copies) < INT32_MAX && tiled_blocks0(d, copies) < INT32_MAX;
}

template <int R>
static void launch_tiled(const float* src, float* dst, float* tmp, const GaussK& k, const GridDims& d, int tj,
                         hipStream_t s) {
    const size_t lds = blur21_lds<R>(d, k, tj);
    hipLaunchKernelGGL(k_blur21<R>, dim3((unsigned)tiled_blocks21(d, tj, 1)), dim3(kBlurBlock), lds, s, src, tmp, k, d,
                       tj);
    hipLaunchKernelGGL(k_blur0<R>, dim3((unsigned)tiled_blocks0(d, 1)), dim3(kBlurBlock), 0, s, tmp, dst, k, d);
}

template <int R>
static void launch_osem_tiled(pp_frame_desc_t* slots, int n_slots, const GaussK& k, const GridDims& d, int tj,
                              hipStream_t s) {
    const size_t lds = blur21_lds<R>(d, k, tj);
    const dim3 g21((unsigned)tiled_blocks21(d, tj, n_slots)), g0((unsigned)tiled_blocks0(d, n_slots));
    const dim3 block(kBlurBlock);
    hipLaunchKernelGGL(k_osem_blur21<R>, g21, block, lds, s, slots, k, d, tj, (int)kFieldAcc, (int)kFieldTmp);
    hipLaunchKernelGGL((k_osem_blur0<R, kOpUpdate>), g0, block, 0, s, slots, k, d, (int)kFieldTmp, (int)kFieldX);
    hipLaunchKernelGGL(k_osem_blur21<R>, g21, block, lds, s, slots, k, d, tj, (int)kFieldX, (int)kFieldTmp);
    hipLaunchKernelGGL((k_osem_blur0<R, kOpZero>), g0, block, 0, s, slots, k, d, (int)kFieldTmp, (int)kFieldXFwd);
}

// the smallest tap bound covering every axis' radius
static int tap_bound(const GaussK& k) {
    const int r = max(k.r[0], max(k.r[1], k.r[2]));
    return r <= 8 ? r : r <= 16 ? 16 : kGaussMaxR;
}

hipError_t launch_gauss3d(const float* src, float* dst, float* tmp, const GeomK& g, const GaussK& k, int cus,
                          hipStream_t s) {
    const int64_t nv = (int64_t)g.n[0] * g.n[1] * g.n[2];
    const GridDims d = dims_of(g);
    const int tj = blur_tile_rows(d, k);
    if (tiled_ok(d, tj, 1)) {
        switch (tap_bound(k)) {
            case 0: launch_tiled<0>(src, dst, tmp, k, d, tj, s); break;
            case 1: launch_tiled<1>(src, dst, tmp, k, d, tj, s); break;
            case 2: launch_tiled<2>(src, dst, tmp, k, d, tj, s); break;
            case 3: launch_tiled<3>(src, dst, tmp, k, d, tj, s); break;
            case 4: launch_tiled<4>(src, dst, tmp, k, d, tj, s); break;
            case 5: launch_tiled<5>(src, dst, tmp, k, d, tj, s); break;
            case 6: launch_tiled<6>(src, dst, tmp, k, d, tj, s); break;
            case 7: launch_tiled<7>(src, dst, tmp, k, d, tj, s); break;
            case 8: launch_tiled<8>(src, dst, tmp, k, d, tj, s); break;
            case 16: launch_tiled<16>(src, dst, tmp, k, d, tj, s); break;
            default: launch_tiled<kGaussMaxR>(src, dst, tmp, k, d, tj, s); break;
        }
        return hipGetLastError();
    }
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
    const int tj = blur_tile_rows(d, k);
    if (tiled_ok(d, tj, n_slots)) {
        switch (tap_bound(k)) {
            case 0: launch_osem_tiled<0>(slots, n_slots, k, d, tj, s); break;
            case 1: launch_osem_tiled<1>(slots, n_slots, k, d, tj, s); break;
            case 2: launch_osem_tiled<2>(slots, n_slots, k, d, tj, s); break;
            case 3: launch_osem_tiled<3>(slots, n_slots, k, d, tj, s); break;
            case 4: launch_osem_tiled<4>(slots, n_slots, k, d, tj, s); break;
            case 5: launch_osem_tiled<5>(slots, n_slots, k, d, tj, s); break;
            case 6: launch_osem_tiled<6>(slots, n_slots, k, d, tj, s); break;
            case 7: launch_osem_tiled<7>(slots, n_slots, k, d, tj, s); break;
            case 8: launch_osem_tiled<8>(slots, n_slots, k, d, tj, s); break;
            case 16: launch_osem_tiled<16>(slots, n_slots, k, d, tj, s); break;
            default: launch_osem_tiled<kGaussMaxR>(slots, n_slots, k, d, tj, s); break;
        }
        return hipGetLastError();
    }
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
