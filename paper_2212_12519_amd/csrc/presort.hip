// Listmode event presorting: a processing order that groups events lying on
// the same or neighbouring lines of response, so that the 64 lanes of a wave
// project nearly parallel, nearly coincident rays.  Their image gathers and
// atomic adds then fall into the same cache lines: float atomics on this GPU
// cost per cache-line request, not per value, so an unsorted listmode back
// projection (one line per lane) runs ~15x below the rate of a wave-coherent
// one.  The paper's discussion suggests presorting listmode events to reduce
// races in the back projection; the order changes nothing but the summation
// order of floats.
//
// Key (64 bits, most significant first):
//   32 bits  OSEM subset of the event (index mod n_sub; 0 when n_sub == 1)
//   10 bits  transaxial direction angle of the LOR in [0, pi)   (axes 0, 1)
//   10 bits  signed transaxial distance of the LOR from the grid centre
//    5 bits  TOF bin (scaled to 32 levels)
//    7 bits  axial (axis 2) position of the LOR midpoint
// Events on one crystal pair share the first 20 bits.  Non-finite rays sort last.  Without subsets
// (n_sub == 1) the upper word is zero and the keys are sorted as 32-bit words (a third less memory
// traffic per radix pass; the sort is stable, so the order is the same).
#include <hip/hip_runtime.h>

#include <hipcub/hipcub.hpp>

#include <mutex>

#include "joseph.hpp"
#include "launch.hpp"

namespace ppmi {

struct KeyGeom {
    float cx, cy;        // grid centre (axes 0, 1), mm
    float inv_rmax;      // 1 / (half diagonal of the transaxial grid extent)
    float z0, inv_zext;  // axial grid start and 1 / extent
};

// Key: uint64_t, or uint32_t when n_sub == 1
template <class Key>
__global__ void __launch_bounds__(256) k_lm_keys(RaySrc src, const int16_t* __restrict__ bins, int64_t n,
                                                 KeyGeom kg, int nb, int n_sub, Key* __restrict__ keys,
                                                 int32_t* __restrict__ idx) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    idx[i] = (int32_t)i;
    const uint64_t sub = sizeof(Key) == 8 ? (uint64_t)(i % n_sub) << 32 : 0;
    const float *ps, *pe;
    if (!src.ends(i, ps, pe)) {  // crystal index out of range: no contribution, sorted last
        keys[i] = (Key)(sub | 0xffffffffull);
        return;
    }
    const float sx = ps[0], sy = ps[1], sz = ps[2];
    const float ex = pe[0], ey = pe[1], ez = pe[2];
    if (!(isfinite(sx) && isfinite(sy) && isfinite(sz) && isfinite(ex) && isfinite(ey) && isfinite(ez))) {
        keys[i] = (Key)(sub | 0xffffffffull);
        return;
    }
    const float pi = 3.14159265358979f;
    float phi = atan2f(ey - sy, ex - sx);
    if (phi < 0.0f) phi += pi;
    if (phi >= pi) phi -= pi;
    float sn, cs;
    sincosf(phi, &sn, &cs);
    const float rho = -(sx - kg.cx) * sn + (sy - kg.cy) * cs;
    const uint32_t qphi = min(1023u, (uint32_t)(phi * (1024.0f / pi)));
    const float fr = fminf(fmaxf((rho * kg.inv_rmax + 1.0f) * 512.0f, 0.0f), 1023.0f);
    const uint32_t qrho = (uint32_t)fr;
    uint32_t qt = 31u;
    if (bins) {
        const int b = bins[i];
        if (b >= 0 && b < nb) qt = (uint32_t)((b * 32) / nb);
    }
    const float fz = fminf(fmaxf((0.5f * (sz + ez) - kg.z0) * kg.inv_zext * 128.0f, 0.0f), 127.0f);
    keys[i] = (Key)(sub | (uint64_t)((qphi << 22) | (qrho << 12) | (qt << 7) | (uint32_t)fz));
}

static size_t align256(size_t b) { return (b + 255) & ~size_t(255); }

static int key_bits(int n_sub) {
    int b = 32;
    while (n_sub > 1 && (1 << (b - 32)) < n_sub) ++b;
    return b;
}

// temporary storage of the radix sort, the larger of the 64- and 32-bit key sorts (a size query: no
// launch); 0 if a query fails, which makes the sort itself report the error
static size_t sort_temp_bytes(int64_t n) {
    size_t b64 = 0, b32 = 0;
    if (hipcub::DeviceRadixSort::SortPairs(nullptr, b64, (const uint64_t*)nullptr, (uint64_t*)nullptr,
                                           (const int32_t*)nullptr, (int32_t*)nullptr, (int)n, 0, 64,
                                           (hipStream_t)0) != hipSuccess ||
        hipcub::DeviceRadixSort::SortPairs(nullptr, b32, (const uint32_t*)nullptr, (uint32_t*)nullptr,
                                           (const int32_t*)nullptr, (int32_t*)nullptr, (int)n, 0, 32,
                                           (hipStream_t)0) != hipSuccess)
        return 0;
    return b64 > b32 ? b64 : b32;
}

size_t presort_workspace_bytes(int64_t n) {
    if (n <= 0) return 0;
    return 2 * align256((size_t)n * 8) + align256((size_t)n * 4) + align256(sort_temp_bytes(n));
}

// Workspace of the presort for callers that cannot allocate device memory: one array per GPU,
// resident from the library's load on that GPU until the process ends.  Host code never passes
// the array's name to a kernel or a copy (on the host it names a stand-in, not device memory):
// it uses the device address that hipGetSymbolAddress returns for the current GPU, resolved
// once per GPU and kept.
static __device__ __align__(256) unsigned char scratch[kPresortScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mutex;
void* g_scratch_ptr[kMaxDevices] = {};
}  // namespace

hipError_t presort_scratch(void** ptr) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mutex);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        g_scratch_ptr[dev] = p;
    }
    *ptr = g_scratch_ptr[dev];
    return hipSuccess;
}

hipError_t launch_presort(const RaySrc& src, const int16_t* bins, int64_t n, const GeomK& g, int nb,
                          int n_sub, int32_t* order, void* ws, size_t ws_bytes, hipStream_t s) {
    const size_t a8 = align256((size_t)n * 8), a4 = align256((size_t)n * 4);
    char* base = static_cast<char*>(ws);
    uint64_t* keys = reinterpret_cast<uint64_t*>(base);
    uint64_t* keys_sorted = reinterpret_cast<uint64_t*>(base + a8);
    int32_t* idx = reinterpret_cast<int32_t*>(base + 2 * a8);
    void* temp = base + 2 * a8 + a4;
    size_t temp_bytes = ws_bytes - (2 * a8 + a4);
    KeyGeom kg;
    const double ext0 = g.n[0] * g.h[0], ext1 = g.n[1] * g.h[1];
    kg.cx = (float)(g.o[0] + 0.5 * (g.n[0] - 1) * g.h[0]);
    kg.cy = (float)(g.o[1] + 0.5 * (g.n[1] - 1) * g.h[1]);
    kg.inv_rmax = (float)(1.0 / (0.5 * sqrt(ext0 * ext0 + ext1 * ext1) + 1e-3));
    kg.z0 = (float)(g.o[2] - 0.5 * g.h[2]);
    kg.inv_zext = (float)(1.0 / (g.n[2] * g.h[2]));
    const dim3 grid((unsigned)((n + 255) / 256));
    if (n_sub <= 1) {  // 32-bit keys in the same workspace
        uint32_t* k32 = reinterpret_cast<uint32_t*>(keys);
        uint32_t* k32s = reinterpret_cast<uint32_t*>(keys_sorted);
        hipLaunchKernelGGL(k_lm_keys<uint32_t>, grid, dim3(256), 0, s, src, bins, n, kg, nb, 1, k32, idx);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        return hipcub::DeviceRadixSort::SortPairs(temp, temp_bytes, k32, k32s, idx, order, (int)n, 0, 32, s);
    }
    hipLaunchKernelGGL(k_lm_keys<uint64_t>, grid, dim3(256), 0, s, src, bins, n, kg, nb, n_sub, keys, idx);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return hipcub::DeviceRadixSort::SortPairs(temp, temp_bytes, keys, keys_sorted, idx, order, (int)n, 0,
                                              key_bits(n_sub), s);
}

// out[i] = in[order[i]] for the three event arrays (bins optional)
__global__ void __launch_bounds__(256) k_gather_events(const float* __restrict__ xs, const float* __restrict__ xe,
                                                       const int16_t* __restrict__ bins,
                                                       const int32_t* __restrict__ order, int64_t n,
                                                       float* __restrict__ xs_out, float* __restrict__ xe_out,
                                                       int16_t* __restrict__ bins_out) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    int64_t j = order[i];
    if (j < 0 || j >= n) j = i;  // not a permutation entry: keep the event in place
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        xs_out[3 * i + a] = xs[3 * j + a];
        xe_out[3 * i + a] = xe[3 * j + a];
    }
    if (bins) bins_out[i] = bins[j];
}

hipError_t launch_gather_events(const float* xs, const float* xe, const int16_t* bins, const int32_t* order, int64_t n,
                                float* xs_out, float* xe_out, int16_t* bins_out, hipStream_t s) {
    hipLaunchKernelGGL(k_gather_events, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, xs, xe, bins, order, n,
                       xs_out, xe_out, bins_out);
    return hipGetLastError();
}

// out[i] = in[order[i]] for crystal-index events (pairs as int2; bins optional)
__global__ void __launch_bounds__(256) k_gather_pairs(const int2* __restrict__ pair, const int16_t* __restrict__ bins,
                                                      const int32_t* __restrict__ order, int64_t n,
                                                      int2* __restrict__ pair_out, int16_t* __restrict__ bins_out) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const int64_t o = order[i];
    const int64_t j = (o >= 0 && o < n) ? o : i;
    pair_out[i] = pair[j];
    if (bins) bins_out[i] = bins[j];
}

hipError_t launch_gather_pairs(const int32_t* pair, const int16_t* bins, const int32_t* order, int64_t n,
                               int32_t* pair_out, int16_t* bins_out, hipStream_t s) {
    hipLaunchKernelGGL(k_gather_pairs, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s,
                       reinterpret_cast<const int2*>(pair), bins, order, n, reinterpret_cast<int2*>(pair_out),
                       bins_out);
    return hipGetLastError();
}

}  // namespace ppmi
