// TOF sinogram OSEM in LOR chunks (the sinogram counterpart of the listmode
// OSEM of Sec. 2.6; Sec. 4 of the paper notes that a TOF sinogram
// reconstruction needs tens of GB for the data and its expectation, and that
// scanners with long axial fields of view need chunk-wise processing).
//
// One subset update, x <- x * A_j^T (y / (A_j x + bg)) / A_j^T 1, runs over
// the subset's LORs in chunks of a caller-sized workspace: the forward TOF
// sinogram projection of a chunk into the workspace, the ratio y / (q + bg)
// in place (k_sino_ratio), the back projection of the ratio into an
// accumulator image.  Only the counts y and the LOR geometry are resident in
// full; the expectation never is.
//
// Shards: the subset's LORs are split into K contiguous ranges, each back
// projected into its own accumulator image -- what K GPUs would do, each on
// its share of the LORs with its own image -- and one pass (k_sino_update)
// sums the K images (the sum-reduction that would cross the GPUs) and applies
// the multiplicative update, clearing the accumulators for the next subset.
#include <hip/hip_runtime.h>

#include "joseph.hpp"
#include "launch.hpp"

namespace ppmi {

constexpr int kSinoBlock = 256;

// q <- y / (q + bg) where q + bg > 0, else 0 (a bin with no positive expectation contributes nothing)
__global__ void __launch_bounds__(kSinoBlock) k_sino_ratio(const float* __restrict__ y, float* __restrict__ q,
                                                          int64_t n, float bg) {
    const int64_t stride = (int64_t)gridDim.x * kSinoBlock;
    for (int64_t i = (int64_t)blockIdx.x * kSinoBlock + threadIdx.x; i < n; i += stride) {
        const float e = q[i] + bg;
        q[i] = (e > 0.0f) ? y[i] / e : 0.0f;
    }
}

// acc_sum = sum over the K shard images; x <- x * acc_sum / sens where sens > 0, else 0; every
// shard image <- 0
__global__ void __launch_bounds__(kSinoBlock) k_sino_update(float* __restrict__ x, float* __restrict__ acc,
                                                           int n_shards, const float* __restrict__ sens,
                                                           int64_t n_vox) {
    const int64_t stride = (int64_t)gridDim.x * kSinoBlock;
    for (int64_t v = (int64_t)blockIdx.x * kSinoBlock + threadIdx.x; v < n_vox; v += stride) {
        float a = 0.0f;
        for (int s = 0; s < n_shards; ++s) {
            a += acc[(int64_t)s * n_vox + v];
            acc[(int64_t)s * n_vox + v] = 0.0f;
        }
        const float sv = sens[v];
        x[v] = (sv > 0.0f) ? x[v] * a / sv : 0.0f;
    }
}

static unsigned stream_blocks(int64_t n, int cus) {
    const int64_t want = (n + kSinoBlock - 1) / kSinoBlock, cap = (int64_t)cus * 8;
    return (unsigned)(want < 1 ? 1 : (want > cap ? cap : want));
}

hipError_t launch_tof_sino_osem_subset(const float* xs, const float* xe, const float* y, int64_t n, const GeomK& g,
                                       const TofK& t, float bg, float* x, float* acc, int n_shards,
                                       const float* sens, float* work, int64_t work_lors, int cus, hipStream_t s) {
    const int64_t nb = t.nb;
    const int64_t n_vox = (int64_t)g.n[0] * g.n[1] * g.n[2];
    for (int sh = 0; sh < n_shards; ++sh) {
        const int64_t lo = n * sh / n_shards, hi = n * (sh + 1) / n_shards;
        float* acc_s = acc + (int64_t)sh * n_vox;
        for (int64_t c0 = lo; c0 < hi; c0 += work_lors) {
            const int64_t m = (hi - c0 < work_lors) ? (hi - c0) : work_lors;
            const RaySrc src{xs + 3 * c0, xe + 3 * c0, nullptr, 0};
            hipError_t e = launch_fwd_tof_sino(src, m, g, t, x, work, s);
            if (e != hipSuccess) return e;
            hipLaunchKernelGGL(k_sino_ratio, dim3(stream_blocks(m * nb, cus)), dim3(kSinoBlock), 0, s, y + c0 * nb,
                               work, m * nb, bg);
            e = hipGetLastError();
            if (e != hipSuccess) return e;
            e = launch_back_tof_sino(src, m, g, t, acc_s, work, s);
            if (e != hipSuccess) return e;
        }
    }
    hipLaunchKernelGGL(k_sino_update, dim3(stream_blocks(n_vox, cus)), dim3(kSinoBlock), 0, s, x, acc, n_shards, sens,
                       n_vox);
    return hipGetLastError();
}

hipError_t launch_tof_sino_sensitivity(const float* xs, const float* xe, int64_t n, const GeomK& g, const TofK& t,
                                       float* sens, float* work, int64_t work_lors, hipStream_t s) {
    const int64_t first = (n < work_lors) ? n : work_lors;
    hipError_t e = launch_fill(work, first * t.nb, 1.0f, s);
    if (e != hipSuccess) return e;
    for (int64_t c0 = 0; c0 < n; c0 += work_lors) {
        const int64_t m = (n - c0 < work_lors) ? (n - c0) : work_lors;
        e = launch_back_tof_sino(RaySrc{xs + 3 * c0, xe + 3 * c0, nullptr, 0}, m, g, t, sens, work, s);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace ppmi
