// Internal launch interface between the C ABI (api.cpp) and the kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/ppmi.h"

namespace ppmi {

struct GeomK;
struct TofK;
struct RaySrc;

// Events and projections written in processing order by launch_fwd_tof_lm_gather
struct EventsOut {
    float* xs;
    float* xe;
    int16_t* bins;
    float* p;
};

hipError_t launch_fwd(const RaySrc& src, int64_t n, const GeomK& g, const float* img, float* p,
                      const int32_t* order, hipStream_t s);
hipError_t launch_back(const RaySrc& src, int64_t n, const GeomK& g, float* img, const float* p,
                       const int32_t* order, hipStream_t s);
hipError_t launch_fwd_tof_sino(const RaySrc& src, int64_t n, const GeomK& g, const TofK& t,
                               const float* img, float* p, hipStream_t s);
hipError_t launch_back_tof_sino(const RaySrc& src, int64_t n, const GeomK& g, const TofK& t,
                                float* img, const float* p, hipStream_t s);
hipError_t launch_tof_gauss_table(float* lut, int n, double x0, double dx, double bw, double sigma, double n_sigmas,
                                  hipStream_t s);
hipError_t launch_fwd_tof_lm(const RaySrc& src, const int16_t* bins, int64_t n, const GeomK& g,
                             const TofK& t, const float* img, float* p, const int32_t* order, hipStream_t s);
hipError_t launch_fwd_tof_lm_gather(const RaySrc& src, const int16_t* bins, int64_t n, const GeomK& g,
                                    const TofK& t, const float* img, float* p, const int32_t* order,
                                    const EventsOut& eo, hipStream_t s);
hipError_t launch_fwd_tof_lm_batch(const RaySrc& src, const int16_t* bins, int64_t n, const GeomK& g, const TofK& t,
                                   const float* imgs, int n_img, float* p, const int32_t* order, hipStream_t s);
hipError_t launch_back_tof_lm(const RaySrc& src, const int16_t* bins, int64_t n, const GeomK& g,
                              const TofK& t, float* img, const float* p, const int32_t* order, hipStream_t s);
hipError_t launch_back_tof_lm_batch(const RaySrc& src, const int16_t* bins, int64_t n, const GeomK& g,
                                    const TofK& t, float* imgs, int n_img, const float* p, const int32_t* order,
                                    hipStream_t s);
hipError_t launch_poisson_nll(const float* p, float bg, const float* y, int64_t n, float* grad, double* partial,
                              int n_partial, hipStream_t s);
size_t presort_workspace_bytes(int64_t n);
// capacity of the library-owned presort workspace (one per GPU) and its device address on the
// current GPU
constexpr size_t kPresortScratchBytes = size_t(64) << 20;
hipError_t presort_scratch(void** ptr);
hipError_t launch_presort(const RaySrc& src, const int16_t* bins, int64_t n, const GeomK& g, int nb,
                          int n_sub, int32_t* order, void* ws, size_t ws_bytes, hipStream_t s);
hipError_t launch_gather_events(const float* xs, const float* xe, const int16_t* bins, const int32_t* order, int64_t n,
                                float* xs_out, float* xe_out, int16_t* bins_out, hipStream_t s);
hipError_t launch_gather_pairs(const int32_t* pair, const int16_t* bins, const int32_t* order, int64_t n,
                               int32_t* pair_out, int16_t* bins_out, hipStream_t s);
hipError_t launch_osem_init(float* x, const float* sens, int64_t n_vox, hipStream_t s);

hipError_t launch_count(const RaySrc& src, const int16_t* bins, int64_t n, const GeomK& g,
                        const TofK& t, int32_t* counts, hipStream_t s);

int64_t osem_chunks(int64_t n_events, int32_t n_sub);
hipError_t launch_osem_accumulate(const pp_frame_desc_t* slots, int n_slots, const GeomK& g, const TofK& t, int cus,
                                  hipStream_t s);
hipError_t launch_osem_update(pp_frame_desc_t* slots, int n_slots, int64_t n_vox, int n_blocks, hipStream_t s);
hipError_t launch_osem_advance(pp_frame_desc_t* slots, int n_slots, hipStream_t s);
hipError_t launch_fill(float* dst, int64_t n, float value, hipStream_t s);
hipError_t launch_tof_sino_osem_subset(const float* xs, const float* xe, const float* y, int64_t n, const GeomK& g,
                                       const TofK& t, float bg, float* x, float* acc, int n_shards,
                                       const float* sens, float* work, int64_t work_lors, int cus, hipStream_t s);
hipError_t launch_tof_sino_sensitivity(const float* xs, const float* xe, int64_t n, const GeomK& g, const TofK& t,
                                       float* sens, float* work, int64_t work_lors, hipStream_t s);

struct GaussK;
hipError_t launch_gauss3d(const float* src, float* dst, float* tmp, const GeomK& g, const GaussK& k, int cus,
                          hipStream_t s);
hipError_t launch_osem_res_update(pp_frame_desc_t* slots, int n_slots, const GeomK& g, const GaussK& k, int cus,
                                  hipStream_t s);

}  // namespace ppmi
