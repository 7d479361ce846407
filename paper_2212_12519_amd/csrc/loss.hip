// Poisson data fidelity of the projections (the loss of the differentiable projectors, Sec. 1 and 4):
// with the expectation ybar_e = p_e + bg (added in float32, as the projection's caller would),
//   L = sum_e (ybar_e - y_e log ybar_e)        (the negative log-likelihood up to a constant),
//   dL/dp_e = 1 - y_e / ybar_e,
// both in float64 per element; the gradient is stored as float32.  One pass over p and y: each
// workgroup of the grid-stride launch sums its elements in float64 and stores one partial sum (the
// caller adds the partials, so the result does not depend on the order of atomics).
#include <hip/hip_runtime.h>

#include "launch.hpp"

namespace ppmi {

constexpr int kLossBlock = 256;

__global__ void __launch_bounds__(kLossBlock) k_poisson_nll(const float* __restrict__ p, float bg,
                                                           const float* __restrict__ y, int64_t n,
                                                           float* __restrict__ grad, double* __restrict__ partial) {
    double acc = 0.0;
    const int64_t stride = (int64_t)gridDim.x * kLossBlock;
    for (int64_t i = (int64_t)blockIdx.x * kLossBlock + threadIdx.x; i < n; i += stride) {
        const double yb = (double)(p[i] + bg), yv = (double)y[i];
        acc += yb - yv * log(yb);
        grad[i] = (float)(1.0 - yv / yb);
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_down(acc, off, 64);
    __shared__ double wsum[kLossBlock / 64];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0) wsum[wave] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        double s = 0.0;
        for (int w = 0; w < kLossBlock / 64; ++w) s += wsum[w];
        partial[blockIdx.x] = s;
    }
}

hipError_t launch_poisson_nll(const float* p, float bg, const float* y, int64_t n, float* grad, double* partial,
                              int n_partial, hipStream_t s) {
    hipLaunchKernelGGL(k_poisson_nll, dim3((unsigned)n_partial), dim3(kLossBlock), 0, s, p, bg, y, n, grad, partial);
    return hipGetLastError();
}

}  // namespace ppmi
