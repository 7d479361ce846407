/*
 * ppmi.h -- C ABI of libppmi.so: Joseph ray-driven forward and back
 * projection (non-TOF, TOF sinogram, TOF listmode) and a batched, fused
 * listmode-OSEM subset update, as hand-written HIP kernels for gfx950.
 *
 * The operations are those of Schramm & Thielemans, "PARALLELPROJ - An
 * open-source framework for fast calculation of projections in tomography"
 * (arXiv 2212.12519):
 *   - Sec. 2.1 and Fig. 1: Joseph's method -- step plane by plane along the
 *     image axis most parallel to the ray, bilinearly interpolate the four
 *     voxels around each ray/plane intersection, sum, and correct for the
 *     incidence angle; TOF weights from a Gaussian convolved with the bin
 *     rect (a difference of two error functions) evaluated at the distance
 *     to the TOF-bin centre;
 *   - Sec. 2.2: generic lists of ray start/end points as input; TOF
 *     sinogram projections fill every bin of a ray in one traversal, TOF
 *     listmode projections only the event's bin; back projections are the
 *     exact adjoints and scatter with atomic adds;
 *   - Sec. 2.6: the TOF Gaussian is truncated beyond +-n_sigmas sigma (3 in
 *     the paper); listmode OSEM with ordered subsets.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *   Coordinates: float32, array of structures [n][3] = (x, y, z) in mm.
 *   Image: float32, C order [dim[0]][dim[1]][dim[2]] (axis 2 fastest); the
 *     centre of voxel (i, j, k) is origin + (i, j, k) * voxsize.  Voxels
 *     outside the grid read as zero.  dim[0]*dim[1]*dim[2] < 2^30.
 *   Principal axis: argmax_a |end_a - start_a| in mm (float32 differences,
 *     first axis on ties).  The ray is the segment start -> end: plane k is
 *     visited iff its ray parameter t in [0, 1].
 *   TOF: a plane sample at ray parameter t sits at s = (t - 1/2) |end - start|
 *     mm from the LOR midpoint (positive towards `end`).  Bin b has centre
 *     c_b = (b - (n_bins - 1)/2) * bin_width + center_offset and weight
 *       w_b(s) = G(s - c_b + bin_width/2) - G(s - c_b - bin_width/2),
 *       G(x)   = erf(clip(x, -n_sigmas*sigma, n_sigmas*sigma) / (sqrt(2) sigma)) / 2
 *     (the Gaussian is truncated before the convolution; no renormalisation),
 *     or a tabulated kernel (pp_tof_t.lut).
 *   Pointers: every array argument is a DEVICE pointer owned by the caller;
 *     the geometry / TOF structs are HOST pointers read during the call.
 *     The library allocates nothing and keeps no state between calls (one
 *     exception: the per-GPU workspace of pp_lm_presort_noalloc).
 *   Streams: `stream` is a hipStream_t (NULL = the default stream).  Calls
 *     are asynchronous: they enqueue kernels and return.  Calls on different
 *     streams are independent.  Every call may be captured into a HIP graph.
 *   Forward projections overwrite their output.  Back projections ADD into
 *     the image (the caller zeroes it), which allows chunked / subset calls.
 *     Their result depends on the order of floating-point atomic adds.
 *     Ray lists in an order that puts rays of one transaxial line next to
 *     each other (presorted listmode, sinograms) are accumulated per line in
 *     32-bit fixed point in on-chip memory first: each line's scale is a
 *     power of two fitted to the largest values its rays can add (coarsened
 *     when more rays of the line arrive), every value is rounded to the unit
 *     with the rounding remainder carried to the next value, so that sums
 *     over many values lose nothing systematically; an added value is off by
 *     at most 1.5 units, and every ray in the fixed point adds values of at
 *     least 2^8 units at its largest.  Rays whose values are too small for
 *     that beside the line's others are added in float directly.  Values
 *     must be finite: with an infinite or NaN value the result of a back
 *     projection is unspecified (no memory outside the image is touched).
 *   Zero-length or non-finite rays, and listmode bins outside [0, n_bins),
 *     contribute nothing (no error: they are data).  n == 0 is a no-op.
 *
 * Errors: every function returns PP_OK (0) or a PP_E* code; nothing is
 *   launched when an argument check fails.  PP_EHIP reports a failed launch;
 *   faults during kernel execution surface at the caller's next
 *   synchronisation.  pp_strerror() describes a code.
 */
#ifndef PPMI_H
#define PPMI_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define PP_ABI_VERSION 9

enum pp_status {
    PP_OK = 0,
    PP_EINVAL_PTR = 1,  /* a required pointer is NULL */
    PP_EINVAL_GEOM = 2, /* dim <= 0, voxel count >= 2^30, voxsize <= 0 or non-finite, origin non-finite */
    PP_EINVAL_TOF = 3,  /* n_bins not in [1, 256], bin_width/sigma/n_sigmas <= 0 or non-finite, bad table,
                         * per-ray sigma with a table, per-ray parameters where unsupported */
    PP_EINVAL_N = 4,    /* negative count, or a count/slot argument out of range */
    PP_EHIP = 5,        /* the HIP runtime rejected a launch */
    PP_EINVAL_RES = 6   /* resolution model: FWHM negative or non-finite, or wider than 31 voxels of radius */
};

typedef struct pp_image {
    float origin[3];  /* mm: centre of voxel (0, 0, 0) */
    float voxsize[3]; /* mm, > 0 (non-isotropic allowed) */
    int32_t dim[3];   /* voxels per axis, > 0 */
} pp_image_t;

/* TOF kernel.  Bin b of a LOR is centred at c_b = (b - (n_bins - 1)/2) bin_width +
 * center_offset (mm from the LOR midpoint towards its end point).  The weight of bin b for
 * a plane sample at TOF position s is w(x), x = s - c_b:
 *   lut == NULL: the Gaussian of the given sigma, truncated at n_sigmas, convolved with the
 *     bin's rect: G(x + bw/2) - G(x - bw/2), G(x) = erf(clip(x, +-n_sigmas sigma) /
 *     (sqrt(2) sigma)) / 2 (Sec. 2.1; truncation Sec. 2.6);
 *   lut != NULL: the tabulated kernel that Sec. 4 proposes (which also allows non-Gaussian
 *     kernels): lut[i] = w(lut_x0 + i lut_dx), i in [0, lut_n), linearly interpolated and 0
 *     outside [lut_x0, lut_x0 + (lut_n - 1) lut_dx]; sigma and n_sigmas are ignored.  The
 *     table is DEVICE memory owned by the caller and must stay valid until the calls that
 *     use it have run (it is read at run time, also by captured graphs).
 * Per-ray parameters (a generalisation of the single kernel of Sec. 2.2, for scanners whose
 * timing resolution or timing offset varies with the LOR or the event): sigma_per_ray and
 * offset_per_ray are optional DEVICE float32 arrays with one entry per ray (per LOR of a
 * sinogram call, per event of a listmode call, indexed like xstart), owned by the caller and
 * read at run time.  Ray l then uses sigma_per_ray[l] in place of sigma (truncation at
 * n_sigmas * sigma_per_ray[l]) and offset_per_ray[l] in place of center_offset.  A ray whose
 * sigma is not a positive finite number, or whose offset is not finite, contributes nothing
 * (data, not an error; a sigma below 1e-30 mm is taken as 1e-30 mm).  A table kernel takes
 * offset_per_ray but not sigma_per_ray (PP_EINVAL_TOF).  Accepted by the projectors and
 * pp_count_samples; pp_lm_osem_subset_batched returns PP_EINVAL_TOF when either is set. */
typedef struct pp_tof {
    float bin_width;     /* mm, > 0 */
    float sigma;         /* mm, > 0 (FWHM / 2.355) */
    float n_sigmas;      /* truncation in sigmas, > 0 */
    float center_offset; /* mm, shift of every bin centre along the LOR */
    int32_t n_bins;      /* 1 .. 256 */
    const float* lut;    /* DEVICE [lut_n] tabulated bin weight, or NULL (Gaussian) */
    int32_t lut_n;       /* 2 .. 2^24 when lut is set */
    float lut_x0;        /* mm, position of lut[0] relative to the bin centre; finite */
    float lut_dx;        /* mm, table spacing, > 0 */
    const float* sigma_per_ray;  /* DEVICE [n] sigma of each ray (mm), or NULL */
    const float* offset_per_ray; /* DEVICE [n] centre offset of each ray (mm), or NULL */
} pp_tof_t;

/* Non-TOF forward projection (Sec. 2.1, Fig. 1).
 * p[l] = ell_l * sum_k bilinear(img, plane k of ray l), l in [0, n_lors).
 * xstart, xend: [n_lors][3]; img: [dim0][dim1][dim2]; p: [n_lors] (overwritten).
 * order: NULL, or int32 [n_lors] -- the order in which rays are processed (a
 * permutation of [0, n_lors), e.g. from pp_lm_presort; entries outside the
 * range are skipped).  It changes speed, not results: outputs stay indexed
 * by ray. */
int pp_fwd(const float* xstart, const float* xend, int64_t n_lors, const pp_image_t* geom, const float* img,
           float* p, const int32_t* order, void* stream);

/* Non-TOF back projection, the exact adjoint of pp_fwd (Sec. 2.2): img += A^T p. */
int pp_back(const float* xstart, const float* xend, int64_t n_lors, const pp_image_t* geom, float* img,
            const float* p, const int32_t* order, void* stream);

/* TOF sinogram forward projection (Sec. 2.1, 2.2): all n_bins of every ray in
 * one traversal.  p: [n_lors][n_bins] (bin fastest), overwritten.
 * Both TOF sinogram calls take n_lors < 2^31 (else PP_EINVAL_N); larger LOR
 * sets are projected in chunks of consecutive LORs (xstart + 3 c, xend + 3 c,
 * p + c n_bins), back projections accumulating into the same image. */
int pp_fwd_tof_sino(const float* xstart, const float* xend, int64_t n_lors, const pp_image_t* geom,
                    const pp_tof_t* tof, const float* img, float* p, void* stream);

/* TOF sinogram back projection, adjoint of pp_fwd_tof_sino: img += A^T p, p: [n_lors][n_bins]. */
int pp_back_tof_sino(const float* xstart, const float* xend, int64_t n_lors, const pp_image_t* geom,
                     const pp_tof_t* tof, float* img, const float* p, void* stream);

/* TOF listmode forward projection (Sec. 2.2): only bin tof_bin[e] of event e.
 * Only the planes within n_sigmas*sigma + bin_width/2 of the bin centre are
 * visited (the weight is exactly zero elsewhere).  tof_bin: int16 [n_events];
 * p: [n_events], overwritten (0 for out-of-range bins). */
int pp_fwd_tof_lm(const float* xstart, const float* xend, const int16_t* tof_bin, int64_t n_events,
                  const pp_image_t* geom, const pp_tof_t* tof, const float* img, float* p, const int32_t* order,
                  void* stream);

/* pp_fwd_tof_lm (p[e] for every event e, the same values) that also writes
 * the events and their projections in processing order -- pp_gather_events
 * fused into the projection, which reads every event anyway:
 *   xstart_out[i] = xstart[order[i]], xend_out[i] = xend[order[i]]  ([n][3]),
 *   tof_bin_out[i] = tof_bin[order[i]], p_out[i] = p[order[i]]      ([n]),
 * so that a following pp_back_tof_lm(xstart_out, xend_out, tof_bin_out, ...,
 * p_out or other values in that order, order = NULL) walks the events in
 * the same order without gathering them (Sec. 4's presorting, kept for the
 * rest of an iteration).  order is required (e.g. from pp_lm_presort); an
 * entry outside [0, n) gives event i and the value 0 at position i.  All
 * pointers DEVICE; outputs must not overlap the inputs.  Errors as
 * pp_fwd_tof_lm, and PP_EINVAL_PTR for a NULL order or output,
 * PP_EINVAL_TOF with per-event TOF arrays (which are not reordered). */
int pp_fwd_tof_lm_gather(const float* xstart, const float* xend, const int16_t* tof_bin, int64_t n_events,
                         const pp_image_t* geom, const pp_tof_t* tof, const float* img, float* p, const int32_t* order,
                         float* xstart_out, float* xend_out, int16_t* tof_bin_out, float* p_out, void* stream);

/* pp_fwd_tof_lm of the same events through n_img images of the grid at once
 * (a batch of images, as in networks that project several images per step,
 * Sec. 1 and 4 of the paper): imgs float32 [n_img][dim0][dim1][dim2],
 * p float32 [n_img][n_events], p[b][e] the projection of event e through
 * image b -- equal to pp_fwd_tof_lm of image b alone (the same arithmetic in
 * the same order).  The ray setup, the TOF window, plane positions,
 * stencils and TOF weights are computed once for all images; the library
 * projects up to 8 images per launch.  n_img in [0, 2^20] (else
 * PP_EINVAL_N); n_img == 0 or n_events == 0 is a no-op.  Other arguments
 * and errors as pp_fwd_tof_lm. */
int pp_fwd_tof_lm_batch(const float* xstart, const float* xend, const int16_t* tof_bin, int64_t n_events,
                        const pp_image_t* geom, const pp_tof_t* tof, const float* imgs, int32_t n_img, float* p,
                        const int32_t* order, void* stream);

/* pp_back_tof_lm of the same events for n_img value arrays at once (the
 * adjoint of pp_fwd_tof_lm_batch, Sec. 2.2): imgs float32
 * [n_img][dim0][dim1][dim2] += the back projection of p[b] (float32
 * [n_img][n_events]) into image b.  The rays' setup, compaction and runs are
 * done once per group of events for all images; each image then gets its own
 * pass of the sheet (flushed at the end of every group, as the sheet cannot
 * hold several images), 16 images per launch.  Each image's result equals
 * pp_back_tof_lm of that image alone up to the rounding of the fixed point
 * and the order of float atomic adds.  n_img in [0, 2^20] (else
 * PP_EINVAL_N); n_img == 0 or n_events == 0 is a no-op.  Other arguments and
 * errors as pp_back_tof_lm. */
int pp_back_tof_lm_batch(const float* xstart, const float* xend, const int16_t* tof_bin, int64_t n_events,
                         const pp_image_t* geom, const pp_tof_t* tof, float* imgs, int32_t n_img, const float* p,
                         const int32_t* order, void* stream);

/* TOF listmode back projection, adjoint of pp_fwd_tof_lm: img += A^T p. */
int pp_back_tof_lm(const float* xstart, const float* xend, const int16_t* tof_bin, int64_t n_events,
                   const pp_image_t* geom, const pp_tof_t* tof, float* img, const float* p, const int32_t* order,
                   void* stream);

/* Listmode presort (Sec. 4 of the paper suggests presorting listmode events
 * to cut back-projection races): writes to `order` (int32 [n]) a permutation
 * of [0, n) that groups events on the same or neighbouring LORs -- key:
 * OSEM subset (event index mod n_sub; use n_sub = 1 for none), transaxial
 * direction (axes 0, 1), transaxial distance from the grid centre, TOF bin
 * (when tof_bin != NULL; tof then required), axial midpoint (axis 2); GPU
 * radix sort.  Passing it as `order` to the listmode projections makes a
 * wave's rays nearly coincident, so their gathers and atomic adds share cache
 * lines.  With n_sub > 1 the order is subset-major (see the OSEM section).
 * workspace: device memory of pp_lm_presort_workspace_bytes(n) bytes, caller
 * owned.  n <= 2^31 - 1, 1 <= n_sub <= 4096. */
size_t pp_lm_presort_workspace_bytes(int64_t n);
int pp_lm_presort(const float* xstart, const float* xend, const int16_t* tof_bin, int64_t n,
                  const pp_image_t* geom, const pp_tof_t* tof, int32_t n_sub, int32_t* order, void* workspace,
                  size_t workspace_bytes, void* stream);

/* pp_lm_presort for callers that cannot allocate device memory (code under
 * HIP graph capture, serving loops that forbid allocation): the same key,
 * sort and output, with the workspace taken from a buffer the library holds
 * on each GPU (64 MiB, allocated when the library is loaded on that GPU and
 * kept until the process ends) instead of a caller argument.  The call
 * itself allocates nothing.  n is limited to the counts whose
 * pp_lm_presort_workspace_bytes(n) fits 64 MiB (about 2 million events);
 * larger n returns PP_EINVAL_N with nothing launched.  Every call on one GPU
 * uses that GPU's one buffer: calls that overlap in time on one GPU (on
 * different streams, or from different host threads without ordering) race
 * on it and must be serialised by the caller; calls on one stream are
 * ordered.  Every other argument and error code is that of pp_lm_presort. */
int pp_lm_presort_noalloc(const float* xstart, const float* xend, const int16_t* tof_bin, int64_t n,
                          const pp_image_t* geom, const pp_tof_t* tof, int32_t n_sub, int32_t* order, void* stream);

/* Reorders event arrays: out[i] = in[order[i]] (tof_bin / tof_bin_out may be
 * NULL together).  In and out must not overlap.  Entries of order outside
 * [0, n) copy event i unchanged. */
int pp_gather_events(const float* xstart, const float* xend, const int16_t* tof_bin, const int32_t* order,
                     int64_t n, float* xstart_out, float* xend_out, int16_t* tof_bin_out, void* stream);

/* Work counter (for throughput accounting, not part of the method): counts[l]
 * = plane samples of ray l whose 2x2 stencil has at least one voxel inside
 * the grid -- the samples a projection of that ray touches memory for.  With
 * tof_bin != NULL (listmode; tof required) only samples strictly inside the
 * event's TOF window count; out-of-range bins count 0.  counts: int32 [n]. */
int pp_count_samples(const float* xstart, const float* xend, const int16_t* tof_bin, int64_t n,
                     const pp_image_t* geom, const pp_tof_t* tof, int32_t* counts, void* stream);

/* The Gaussian kernel of `tof` (sigma, n_sigmas, bin_width; its lut and
 * per-ray fields are ignored) as a table for pp_tof_t.lut: the bin weight
 * w(x) = G(x + bin_width/2) - G(x - bin_width/2) of Sec. 2.1 (G truncated at
 * n_sigmas as in Sec. 2.6) over its support [-win, win], win = n_sigmas
 * sigma + bin_width/2, at x_i = -win + i dx, i in [0, n), with
 * n = ceil(2 win / dx_max) + 1 and dx = 2 win / (n - 1) (the largest spacing
 * <= dx_max whose last entry lands on +win).  Evaluated in float64 on the
 * device, stored as float32.
 *   lut:      DEVICE float32 [capacity], or NULL to query the size only;
 *   n_out, x0_out, dx_out: HOST outputs n, -win, dx (each may be NULL);
 *             pass x0_out / dx_out as pp_tof_t.lut_x0 / lut_dx.
 * Errors: PP_EINVAL_TOF (sigma, n_sigmas or bin_width not positive-finite),
 * PP_EINVAL_N (dx_max not positive-finite, n > 2^24, or capacity < n with
 * lut set). */
int pp_tof_gaussian_table(const pp_tof_t* tof, float dx_max, float* lut, int32_t capacity, int32_t* n_out,
                          float* x0_out, float* dx_out, void* stream);

/* How the listmode kernels (pp_*_tof_lm*, pp_lm_osem_subset_batched) evaluate
 * the bin weight of `tof` (host-only, nothing launched): *form = 1 for a
 * table (lut set); 2 for a piecewise polynomial of |x| fitted by the library
 * to the Gaussian weight (two Chebyshev pieces split where the truncation
 * makes w non-smooth, accepted only if its float32 evaluation stays within
 * 5e-7 of the peak weight of the exact weight); 0 for the two clipped erf
 * (per-ray sigma, or a fit that missed that bound).  The sinogram kernels
 * always use the erf (or the table).  Errors: those of the TOF checks;
 * PP_EINVAL_PTR if form is NULL. */
int pp_tof_weight_form(const pp_tof_t* tof, int32_t* form);

/* ------------------------------------------------------------------------
 * Crystal-index events (index-based LOR geometry).  A scanner identifies a
 * listmode event by the two crystals that detected it; the entry points
 * above take the rays' end points as coordinates (the generic ray lists of
 * Sec. 2.2).  The _crystals variants take them as indices into a table of
 * crystal positions: event e runs from crystal_xyz[pair[e][0]] to
 * crystal_xyz[pair[e][1]], exactly the ray the coordinate entry point
 * computes for those coordinates, at 8 instead of 24 bytes per event.
 *   crystal_xyz: DEVICE float32 [n_crystals][3], mm, caller owned;
 *   pair:        DEVICE int32 [n][2] (start crystal, end crystal), 8-byte
 *                aligned (else PP_EINVAL_PTR);
 *   n_crystals:  >= 1 (else PP_EINVAL_N).  A pair entry outside
 *                [0, n_crystals) makes its event contribute nothing (p = 0,
 *                sorted last by the presort): data, not an error.
 * Every other argument, the order and the error codes are those of the
 * coordinate entry point of the same name.
 * ------------------------------------------------------------------------ */
int pp_fwd_crystals(const float* crystal_xyz, int32_t n_crystals, const int32_t* pair, int64_t n_events,
                    const pp_image_t* geom, const float* img, float* p, const int32_t* order, void* stream);
int pp_back_crystals(const float* crystal_xyz, int32_t n_crystals, const int32_t* pair, int64_t n_events,
                     const pp_image_t* geom, float* img, const float* p, const int32_t* order, void* stream);
int pp_fwd_tof_lm_crystals(const float* crystal_xyz, int32_t n_crystals, const int32_t* pair,
                           const int16_t* tof_bin, int64_t n_events, const pp_image_t* geom, const pp_tof_t* tof,
                           const float* img, float* p, const int32_t* order, void* stream);
int pp_back_tof_lm_crystals(const float* crystal_xyz, int32_t n_crystals, const int32_t* pair,
                            const int16_t* tof_bin, int64_t n_events, const pp_image_t* geom, const pp_tof_t* tof,
                            float* img, const float* p, const int32_t* order, void* stream);
int pp_lm_presort_crystals(const float* crystal_xyz, int32_t n_crystals, const int32_t* pair,
                           const int16_t* tof_bin, int64_t n, const pp_image_t* geom, const pp_tof_t* tof,
                           int32_t n_sub, int32_t* order, void* workspace, size_t workspace_bytes, void* stream);
int pp_count_samples_crystals(const float* crystal_xyz, int32_t n_crystals, const int32_t* pair,
                              const int16_t* tof_bin, int64_t n, const pp_image_t* geom, const pp_tof_t* tof,
                              int32_t* counts, void* stream);
/* out[i] = in[order[i]] for pair (int32 [n][2]) and tof_bin (int16 [n], may be
 * NULL together with tof_bin_out), as pp_gather_events. */
int pp_gather_crystal_events(const int32_t* pair, const int16_t* tof_bin, const int32_t* order, int64_t n,
                             int32_t* pair_out, int16_t* tof_bin_out, void* stream);

/* ------------------------------------------------------------------------
 * Batched listmode TOF OSEM (the paper's listmode OSEM of Sec. 2.6, run for
 * many short frames at once).  One "step" of a frame is one ordered-subset
 * update with subset j = {events e : e mod n_sub == j}:
 *     acc  = sum_{e in subset j} a_e / (a_e . x' + bg)     (pp_lm_osem_subset_batched)
 *     x_v <- x_v * acc'_v / (sens_v / n_sub) if sens_v > 0, else 0;  acc <- 0
 *                                                           (pp_osem_update_batched)
 * An event whose expectation a_e . x' + bg is not positive contributes nothing.
 * Without the resolution model (x_fwd == NULL) x' = x and acc' = acc.  With it
 * (x_fwd and tmp set) the system model is the projector after the Gaussian
 * blur G of pp_gauss3d (the paper's OSEM includes such an image-based model):
 * x' = x_fwd = G x, acc' = G acc, and sens must be G applied to the back
 * projection of ones; before the first step x_fwd must hold G x
 * (pp_gauss3d(x, x_fwd, tmp, ...)).  pp_osem_update_batched keeps x_fwd = G x.
 * Event storage of a frame is SUBSET-MAJOR: subset j occupies the contiguous
 * range [off_j, off_j + n_j), n_j = n / n_sub + (j < n mod n_sub),
 * off_j = j (n / n_sub) + min(j, n mod n_sub), in any order inside the range
 * (pp_lm_presort with n_sub, then pp_gather_events, produces exactly this).
 * The slot table lives in DEVICE memory and is read by the kernels at run
 * time, so one captured graph of steps serves any mix of frames: the host
 * rewrites slots between replays.  pp_osem_update_batched advances `subset`
 * ((subset + 1) mod n_sub) and decrements `steps_left` of every slot it
 * updates; slots with active == 0 or steps_left <= 0 are skipped by both
 * calls, and so are malformed slots (n_sub < 1, subset outside [0, n_sub),
 * n_events < 0), which the library cannot reject on the host because the
 * table is device memory.  All frames of one call share the image grid and TOF parameters.
 * Each frame owns its x, acc (zero before its first step) and events, so a
 * frame's result does not depend on the other frames of the batch (up to
 * the order of atomic adds).
 * ------------------------------------------------------------------------ */
/* One frame of the batch (a "slot" of the table). */
typedef struct pp_frame_desc {
    const float* xstart;     /* [n_events][3] (unused with crystal_pair) */
    const float* xend;       /* [n_events][3] (unused with crystal_pair) */
    const int16_t* tof_bin;  /* [n_events] */
    float* x;                /* [n_vox] current image, updated in place */
    float* acc;              /* [n_vox] accumulator, zero between steps */
    const float* sens;       /* [n_vox] sensitivity image */
    int64_t n_events;
    int64_t chunk_begin;     /* first work chunk of this slot (pp_osem_chunks prefix sum) */
    float bg;                /* additive expectation per event (contamination) */
    int32_t n_sub;           /* subsets of this frame, >= 1 */
    int32_t subset;          /* subset of the next step, in [0, n_sub) */
    int32_t steps_left;      /* steps still to run; 0 = finished */
    int32_t active;          /* 0 = empty slot */
    int32_t n_crystals;      /* entries of crystal_xyz (with crystal_pair) */
    float* x_fwd;            /* [n_vox] G x for the resolution model, or NULL (no model) */
    float* tmp;              /* [n_vox] scratch of the resolution model; required when x_fwd is set
                              * (a slot with x_fwd but no tmp is skipped by every call) */
    const int32_t* crystal_pair; /* [n_events][2] crystal-index events (8-byte aligned), or NULL */
    const float* crystal_xyz;    /* [n_crystals][3] crystal table, used with crystal_pair (a slot with
                                  * crystal_pair but no table or n_crystals < 1 is skipped by every call) */
} pp_frame_desc_t;

/* Work chunks a slot needs per step (events of the largest subset / 1024,
 * rounded up).  The host sets chunk_begin of slot s to the sum over slots
 * r < s of pp_osem_chunks(n_events_r, n_sub_r) (0 for inactive slots). */
int64_t pp_osem_chunks(int64_t n_events, int32_t n_sub);

/* Fused forward -> 1/(ybar) -> back projection of the current subset of
 * every live slot into its acc.  d_slots: DEVICE array of n_slots entries.
 * tof: one kernel for all slots (per-ray parameters: PP_EINVAL_TOF). */
int pp_lm_osem_subset_batched(const pp_frame_desc_t* d_slots, int32_t n_slots, const pp_image_t* geom,
                              const pp_tof_t* tof, void* stream);

/* Multiplicative image update of every live slot, then acc <- 0, subset
 * advanced, steps_left decremented.  geom: the slots' common image grid.
 * res_fwhm: host array of 3 FWHM values in mm (per image axis) of the
 * resolution model, applied to the slots that have x_fwd set; NULL = FWHM 0
 * (G = identity).  Errors: PP_EINVAL_RES as for pp_gauss3d. */
int pp_osem_update_batched(pp_frame_desc_t* d_slots, int32_t n_slots, const pp_image_t* geom,
                           const float* res_fwhm, void* stream);

/* OSEM start image: x_v = 1 where sens_v > 0, else 0. */
int pp_osem_init(float* x, const float* sens, int64_t n_vox, void* stream);

/* ------------------------------------------------------------------------
 * TOF sinogram OSEM in LOR chunks.  The sinogram counterpart of the listmode
 * OSEM above: x <- x * A_j^T (y / (A_j x + bg)) / A_j^T 1 per subset j (0
 * where A_j^T 1 == 0; a (LOR, bin) whose expectation A_j x + bg is not
 * positive contributes nothing).  The paper's Sec. 4 discusses the memory a
 * TOF sinogram reconstruction needs (the data and its expectation, tens of
 * GB) and chunk-wise processing for long axial fields of view: here only the
 * counts y and the LOR end points are resident; the expectation of at most
 * work_lors LORs at a time lives in a caller workspace.
 * The caller stores each subset's LORs contiguously (e.g. subset j = views
 * with view mod n_sub == j) and calls once per subset.
 * ------------------------------------------------------------------------ */

/* Subset sensitivity: sens += A^T 1 over the n_lors LORs (all n_bins bins),
 * back projected in chunks of work_lors LORs through work (DEVICE float32
 * [work_lors][n_bins], overwritten).  Errors: PP_EINVAL_TOF also for
 * per-ray TOF parameters; PP_EINVAL_N for work_lors not in [1, 2^31). */
int pp_tof_sino_sensitivity(const float* xstart, const float* xend, int64_t n_lors, const pp_image_t* geom,
                            const pp_tof_t* tof, float* sens, float* work, int64_t work_lors, void* stream);

/* One subset update of the n_lors LORs of subset j (xstart, xend [n][3];
 * y [n][n_bins] counts; sens = A_j^T 1 from pp_tof_sino_sensitivity over the
 * same LORs).  For each chunk of at most work_lors LORs: forward TOF sinogram
 * projection of x into work, work <- y / (work + bg) (0 where work + bg <=
 * 0), back projection of work into an accumulator.  Shards: the LORs are
 * split into n_shards contiguous ranges, shard s back projected into its own
 * image acc + s n_vox -- the private images K GPUs would fill, each with its
 * share of the LORs -- and one final pass sums the shard images, applies
 * x <- x * sum / sens (0 where sens == 0) and zeroes every shard image.
 *   x:    DEVICE [n_vox], updated in place;
 *   acc:  DEVICE [n_shards][n_vox], zero on entry, zero on return;
 *   work: DEVICE float32 [work_lors][n_bins] workspace.
 * x, acc, sens and work must not overlap (PP_EINVAL_PTR).  n_lors == 0 still
 * applies the update (an empty subset has sens == 0: x becomes 0).
 * Errors: PP_EINVAL_TOF also for per-ray TOF parameters; PP_EINVAL_N for
 * n_shards not in [1, 1024], work_lors not in [1, 2^31) or bg non-finite. */
int pp_tof_sino_osem_subset(const float* xstart, const float* xend, const float* y, int64_t n_lors,
                            const pp_image_t* geom, const pp_tof_t* tof, float bg, float* x, float* acc,
                            int32_t n_shards, const float* sens, float* work, int64_t work_lors, void* stream);

/* Image-based resolution model (the paper's listmode OSEM uses a 3D Gaussian
 * of 4.5 mm FWHM, Sec. 2.6): dst = G src, G the discrete Gaussian blur with,
 * along image axis a, taps exp(-i^2 / (2 s_a^2)) for |i| <= floor(4 s_a + 1/2),
 * normalised to sum 1, where s_a = fwhm[a] / (2 sqrt(2 ln 2)) / voxsize[a]
 * voxels (fwhm[a] == 0: no blur along a); voxels outside the grid count as 0.
 * G is symmetric (its own adjoint).  src, dst, tmp: DEVICE float arrays of
 * the grid's voxel count, pairwise non-overlapping (tmp is overwritten).
 * fwhm: host array of 3 values in mm.  Errors: PP_EINVAL_PTR (NULL or
 * overlapping arrays), PP_EINVAL_GEOM, PP_EINVAL_RES. */
int pp_gauss3d(const float* src, float* dst, float* tmp, const pp_image_t* geom, const float* fwhm, void* stream);

/* Poisson data fidelity of listmode or sinogram projections p with a constant
 * background bg and data y (the loss whose gradient the differentiable
 * projectors back-project, Sec. 1 and 4): with ybar_e = p_e + bg (float32
 * addition), in float64 per element
 *   L = sum_e (ybar_e - y_e log ybar_e),   grad_e = 1 - y_e / ybar_e,
 * grad stored as float32 [n].  One pass: workgroup b of the n_partial
 * workgroups (grid-stride over the elements) writes its float64 partial sum
 * to partial[b]; L = sum_b partial[b] (left to the caller, so the result
 * does not depend on atomic order).  ybar_e <= 0 gives what the formula
 * gives in IEEE arithmetic (infinite or NaN terms).  p, y, grad: DEVICE
 * float32 [n]; partial: DEVICE float64 [n_partial].  Errors: PP_EINVAL_N
 * (n < 0, n_partial outside [1, 65536], bg not finite), PP_EINVAL_PTR.
 * n == 0 writes zero partial sums. */
int pp_poisson_nll(const float* p, float bg, const float* y, int64_t n, float* grad, double* partial,
                   int32_t n_partial, void* stream);

/* Sets n floats at dst to value (a kernel, safe inside captured graphs). */
int pp_fill(float* dst, int64_t n, float value, void* stream);

const char* pp_strerror(int code);
int pp_abi_version(void);

#ifdef __cplusplus
}
#endif

#endif /* PPMI_H */
