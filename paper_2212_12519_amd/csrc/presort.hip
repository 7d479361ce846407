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
// Key (32 bits, most significant first):
//   10 bits  transaxial direction angle of the LOR in [0, pi)   (axes 0, 1)
//   10 bits  signed transaxial distance of the LOR from the grid centre
//    5 bits  TOF bin (scaled to 32 levels)
//    7 bits  axial (axis 2) position of the LOR midpoint
// Events on one crystal pair share the first 20 bits.  Non-finite rays sort last.
#include <hip/hip_runtime.h>

#include <hipcub/hipcub.hpp>

#include "joseph.hpp"
#include "launch.hpp"

namespace ppmi {

struct KeyGeom {
    float cx, cy;        // grid centre (axes 0, 1), mm
    float inv_rmax;      // 1 / (half diagonal of the transaxial grid extent)
    float z0, inv_zext;  // axial grid start and 1 / extent
};

__global__ void __launch_bounds__(256) k_lm_keys(const float* __restrict__ xs, const float* __restrict__ xe,
                                                 const int16_t* __restrict__ bins, int64_t n, KeyGeom kg, int nb,
                                                 uint32_t* __restrict__ keys, int32_t* __restrict__ idx) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    idx[i] = (int32_t)i;
    const float sx = xs[3 * i], sy = xs[3 * i + 1], sz = xs[3 * i + 2];
    const float ex = xe[3 * i], ey = xe[3 * i + 1], ez = xe[3 * i + 2];
    if (!(isfinite(sx) && isfinite(sy) && isfinite(sz) && isfinite(ex) && isfinite(ey) && isfinite(ez))) {
        keys[i] = 0xffffffffu;
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
    keys[i] = (qphi << 22) | (qrho << 12) | (qt << 7) | (uint32_t)fz;
}

static size_t align256(size_t b) { return (b + 255) & ~size_t(255); }

static size_t sort_temp_bytes(int64_t n) {
    size_t bytes = 0;
    hipcub::DeviceRadixSort::SortPairs(nullptr, bytes, (const uint32_t*)nullptr, (uint32_t*)nullptr,
                                       (const int32_t*)nullptr, (int32_t*)nullptr, (int)n, 0, 32, (hipStream_t)0);
    return bytes;
}

size_t presort_workspace_bytes(int64_t n) {
    if (n <= 0) return 0;
    return 3 * align256((size_t)n * 4) + align256(sort_temp_bytes(n));
}

hipError_t launch_presort(const float* xs, const float* xe, const int16_t* bins, int64_t n, const GeomK& g, int nb,
                          int32_t* order, void* ws, size_t ws_bytes, hipStream_t s) {
    const size_t a = align256((size_t)n * 4);
    char* base = static_cast<char*>(ws);
    uint32_t* keys = reinterpret_cast<uint32_t*>(base);
    uint32_t* keys_sorted = reinterpret_cast<uint32_t*>(base + a);
    int32_t* idx = reinterpret_cast<int32_t*>(base + 2 * a);
    void* temp = base + 3 * a;
    size_t temp_bytes = ws_bytes - 3 * a;
    KeyGeom kg;
    const double ext0 = g.n[0] * g.h[0], ext1 = g.n[1] * g.h[1];
    kg.cx = (float)(g.o[0] + 0.5 * (g.n[0] - 1) * g.h[0]);
    kg.cy = (float)(g.o[1] + 0.5 * (g.n[1] - 1) * g.h[1]);
    kg.inv_rmax = (float)(1.0 / (0.5 * sqrt(ext0 * ext0 + ext1 * ext1) + 1e-3));
    kg.z0 = (float)(g.o[2] - 0.5 * g.h[2]);
    kg.inv_zext = (float)(1.0 / (g.n[2] * g.h[2]));
    hipLaunchKernelGGL(k_lm_keys, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, xs, xe, bins, n, kg, nb, keys,
                       idx);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return hipcub::DeviceRadixSort::SortPairs(temp, temp_bytes, keys, keys_sorted, idx, order, (int)n, 0, 32, s);
}

}  // namespace ppmi
