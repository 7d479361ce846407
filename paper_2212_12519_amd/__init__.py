"""MI355X-native Joseph projector (non-TOF, TOF sinogram, TOF listmode) and
batched listmode OSEM, after Schramm & Thielemans, arXiv 2212.12519.

The compute path is libppmi.so (hand-written HIP for gfx950, C ABI in
include/ppmi.h); this package is its Python binding plus the autograd
wrappers and the OSEM serving loop built on it.
"""
from ._lib import ImageGeom, PPError, TofParams, load
from .projectors import (back, back_crystals, fwd_tof_lm_batch, pp_fwd_tof_lm_batch, fwd_tof_lm_gather, pp_fwd_tof_lm_gather, back_tof_lm_batch, pp_back_tof_lm_batch, back_tof_lm, back_tof_lm_crystals, back_tof_sino, count_samples,
                         count_samples_crystals, fwd, fwd_crystals, fwd_tof_lm, fwd_tof_lm_crystals, fwd_tof_sino,
                         gather_crystal_events, gather_events, gauss3d, gaussian_tof_table, pp_tof_gaussian_table, pp_back, pp_back_crystals,
                         pp_back_tof_lm, pp_back_tof_lm_crystals, pp_back_tof_sino, pp_count_samples, pp_fill, pp_poisson_nll, pp_fwd,
                         pp_fwd_crystals, pp_fwd_tof_lm, pp_fwd_tof_lm_crystals, pp_fwd_tof_sino, pp_gather_events,
                         pp_gauss3d, pp_lm_presort, pp_lm_presort_crystals, pp_lm_presort_noalloc, presort, presort_crystals,
                         presort_workspace)

__all__ = [
    "ImageGeom", "TofParams", "PPError", "load",
    "pp_fwd", "pp_back", "pp_fwd_tof_sino", "pp_back_tof_sino", "pp_fwd_tof_lm", "pp_back_tof_lm", "pp_fill", "pp_poisson_nll",
    "pp_count_samples", "count_samples", "pp_lm_presort", "pp_lm_presort_noalloc", "presort", "presort_workspace", "pp_gather_events",
    "gather_events", "pp_gauss3d", "gauss3d", "gaussian_tof_table", "pp_tof_gaussian_table",
    "fwd", "back", "fwd_tof_lm_batch", "pp_fwd_tof_lm_batch", "fwd_tof_lm_gather", "pp_fwd_tof_lm_gather", "back_tof_lm_batch", "pp_back_tof_lm_batch", "fwd_tof_sino", "back_tof_sino", "fwd_tof_lm", "back_tof_lm",
    "pp_fwd_crystals", "pp_back_crystals", "pp_fwd_tof_lm_crystals", "pp_back_tof_lm_crystals", "pp_lm_presort_crystals", "presort_crystals",
    "count_samples_crystals", "gather_crystal_events", "fwd_crystals", "back_crystals", "fwd_tof_lm_crystals",
    "back_tof_lm_crystals",
]
