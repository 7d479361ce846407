"""ctypes binding of libppmi.so (declared in include/ppmi.h).

Argument marshalling only: torch tensors are checked (device, dtype, shape,
contiguity) and passed as raw device pointers together with torch's current
HIP stream.  Every computation happens in the library's HIP kernels; there is
no CPU fallback -- if the library is missing, loading raises.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass, field

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libppmi.so")
_lib = None

PP_OK, PP_EINVAL_PTR, PP_EINVAL_GEOM, PP_EINVAL_TOF, PP_EINVAL_N, PP_EHIP, PP_EINVAL_RES = range(7)


class PPError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"ppmi error {code}: {msg}")
        self.code = code


class CImage(ctypes.Structure):
    _fields_ = [("origin", ctypes.c_float * 3), ("voxsize", ctypes.c_float * 3), ("dim", ctypes.c_int32 * 3)]


class CTof(ctypes.Structure):
    _fields_ = [("bin_width", ctypes.c_float), ("sigma", ctypes.c_float), ("n_sigmas", ctypes.c_float),
                ("center_offset", ctypes.c_float), ("n_bins", ctypes.c_int32), ("lut", ctypes.c_void_p),
                ("lut_n", ctypes.c_int32), ("lut_x0", ctypes.c_float), ("lut_dx", ctypes.c_float),
                ("sigma_per_ray", ctypes.c_void_p), ("offset_per_ray", ctypes.c_void_p)]


assert ctypes.sizeof(CTof) == 64, ctypes.sizeof(CTof)


class COsemSlot(ctypes.Structure):
    _fields_ = [("xstart", ctypes.c_void_p), ("xend", ctypes.c_void_p), ("tof_bin", ctypes.c_void_p),
                ("x", ctypes.c_void_p), ("acc", ctypes.c_void_p), ("sens", ctypes.c_void_p),
                ("n_events", ctypes.c_int64), ("chunk_begin", ctypes.c_int64), ("bg", ctypes.c_float),
                ("n_sub", ctypes.c_int32), ("subset", ctypes.c_int32), ("steps_left", ctypes.c_int32),
                ("active", ctypes.c_int32), ("n_crystals", ctypes.c_int32),
                ("x_fwd", ctypes.c_void_p), ("tmp", ctypes.c_void_p),
                ("crystal_pair", ctypes.c_void_p), ("crystal_xyz", ctypes.c_void_p)]


assert ctypes.sizeof(COsemSlot) == 120, ctypes.sizeof(COsemSlot)


@dataclass(frozen=True)
class ImageGeom:
    """dim (n0, n1, n2), voxsize mm, origin = centre of voxel (0,0,0) in mm (default: centred grid)."""
    dim: tuple
    voxsize: tuple
    origin: tuple = None

    def __post_init__(self):
        object.__setattr__(self, "dim", tuple(int(v) for v in self.dim))
        object.__setattr__(self, "voxsize", tuple(float(v) for v in self.voxsize))
        if self.origin is None:
            object.__setattr__(self, "origin", tuple(-(n - 1) / 2.0 * h for n, h in zip(self.dim, self.voxsize)))
        else:
            object.__setattr__(self, "origin", tuple(float(v) for v in self.origin))

    @property
    def n_vox(self):
        return self.dim[0] * self.dim[1] * self.dim[2]

    def c(self):
        return CImage((ctypes.c_float * 3)(*self.origin), (ctypes.c_float * 3)(*self.voxsize),
                      (ctypes.c_int32 * 3)(*self.dim))


@dataclass(frozen=True)
class TofParams:
    """TOF bins and kernel.  With `lut` (a float32 CUDA tensor: the bin weight at distances
    lut_x0 + i * lut_dx mm from the bin centre, linearly interpolated, 0 outside) the kernel is
    the table and sigma / n_sigmas are ignored.  `sigma_per_ray` / `offset_per_ray` (float32
    CUDA tensors [n], one entry per ray of the calls they are used with) replace sigma /
    center_offset ray by ray.  Tensors must outlive the calls using them."""
    bin_width: float
    sigma: float
    n_sigmas: float
    n_bins: int
    center_offset: float = 0.0
    lut: object = field(default=None, compare=False)
    lut_x0: float = 0.0
    lut_dx: float = 0.0
    sigma_per_ray: object = field(default=None, compare=False)
    offset_per_ray: object = field(default=None, compare=False)

    def __post_init__(self):
        if self.lut is not None:
            t = self.lut
            if not (isinstance(t, torch.Tensor) and t.device.type == "cuda" and t.dtype == torch.float32
                    and t.is_contiguous() and t.dim() == 1 and t.numel() >= 2):
                raise ValueError("lut must be a contiguous 1-D float32 CUDA tensor of >= 2 entries")
        for name in ("sigma_per_ray", "offset_per_ray"):
            t = getattr(self, name)
            if t is not None and not (isinstance(t, torch.Tensor) and t.device.type == "cuda"
                                      and t.dtype == torch.float32 and t.is_contiguous() and t.dim() == 1):
                raise ValueError(f"{name} must be a contiguous 1-D float32 CUDA tensor")

    @property
    def per_ray(self):
        return self.sigma_per_ray is not None or self.offset_per_ray is not None

    def c(self, n=None):
        """The C struct; `n` = the call's ray count, checked against the per-ray arrays."""
        per = []
        for t in (self.sigma_per_ray, self.offset_per_ray):
            if t is not None and (n is None or t.numel() != n):
                raise ValueError("per-ray TOF parameters need one entry per ray of the call")
            per.append(t.data_ptr() if t is not None else None)
        if self.lut is None:
            return CTof(self.bin_width, self.sigma, self.n_sigmas, self.center_offset, int(self.n_bins), None, 0,
                        0.0, 0.0, *per)
        return CTof(self.bin_width, self.sigma, self.n_sigmas, self.center_offset, int(self.n_bins),
                    self.lut.data_ptr(), int(self.lut.numel()), float(self.lut_x0), float(self.lut_dx), *per)


def as_geom(g) -> ImageGeom:
    if isinstance(g, ImageGeom):
        return g
    return ImageGeom(tuple(g.dim), tuple(g.voxsize), tuple(g.origin))


def as_tof(t) -> TofParams:
    if isinstance(t, TofParams):
        return t
    return TofParams(float(t.bin_width), float(t.sigma), float(t.n_sigmas), int(t.n_bins),
                     float(getattr(t, "center_offset", 0.0)), getattr(t, "lut", None),
                     float(getattr(t, "lut_x0", 0.0)), float(getattr(t, "lut_dx", 0.0)),
                     getattr(t, "sigma_per_ray", None), getattr(t, "offset_per_ray", None))


def load():
    """Load libppmi.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_2212_12519_amd.build`")
    lib = ctypes.CDLL(LIB_PATH)
    P, I64, I32, INT = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_int
    G = ctypes.POINTER(CImage)
    T = ctypes.POINTER(CTof)
    sig = {
        "pp_fwd": [P, P, I64, G, P, P, P, P],
        "pp_back": [P, P, I64, G, P, P, P, P],
        "pp_fwd_tof_sino": [P, P, I64, G, T, P, P, P],
        "pp_back_tof_sino": [P, P, I64, G, T, P, P, P],
        "pp_fwd_tof_lm": [P, P, P, I64, G, T, P, P, P, P],
        "pp_back_tof_lm": [P, P, P, I64, G, T, P, P, P, P],
        "pp_fwd_tof_lm_batch": [P, P, P, I64, G, T, P, I32, P, P, P],
        "pp_fwd_tof_lm_gather": [P, P, P, I64, G, T, P, P, P, P, P, P, P, P],
        "pp_back_tof_lm_batch": [P, P, P, I64, G, T, P, I32, P, P, P],
        "pp_lm_presort": [P, P, P, I64, G, T, I32, P, P, ctypes.c_size_t, P],
        "pp_lm_presort_noalloc": [P, P, P, I64, G, T, I32, P, P],
        "pp_gather_events": [P, P, P, P, I64, P, P, P, P],
        "pp_osem_init": [P, P, I64, P],
        "pp_lm_osem_subset_batched": [P, I32, G, T, P],
        "pp_osem_update_batched": [P, I32, G, P, P],
        "pp_gauss3d": [P, P, P, G, P, P],
        "pp_fill": [P, I64, ctypes.c_float, P],
        "pp_poisson_nll": [P, ctypes.c_float, P, I64, P, P, I32, P],
        "pp_count_samples": [P, P, P, I64, G, T, P, P],
        "pp_fwd_crystals": [P, I32, P, I64, G, P, P, P, P],
        "pp_back_crystals": [P, I32, P, I64, G, P, P, P, P],
        "pp_fwd_tof_lm_crystals": [P, I32, P, P, I64, G, T, P, P, P, P],
        "pp_back_tof_lm_crystals": [P, I32, P, P, I64, G, T, P, P, P, P],
        "pp_lm_presort_crystals": [P, I32, P, P, I64, G, T, I32, P, P, ctypes.c_size_t, P],
        "pp_count_samples_crystals": [P, I32, P, P, I64, G, T, P, P],
        "pp_gather_crystal_events": [P, P, P, I64, P, P, P],
        "pp_tof_weight_form": [T, ctypes.POINTER(I32)],
        "pp_tof_sino_sensitivity": [P, P, I64, G, T, P, P, I64, P],
        "pp_tof_sino_osem_subset": [P, P, P, I64, G, T, ctypes.c_float, P, P, I32, P, P, I64, P],
        "pp_tof_gaussian_table": [T, ctypes.c_float, P, I32, ctypes.POINTER(I32), ctypes.POINTER(ctypes.c_float),
                                  ctypes.POINTER(ctypes.c_float), P],
    }
    for name, argt in sig.items():
        f = getattr(lib, name)
        f.argtypes = argt
        f.restype = INT
    lib.pp_lm_presort_workspace_bytes.argtypes = [I64]
    lib.pp_lm_presort_workspace_bytes.restype = ctypes.c_size_t
    lib.pp_osem_chunks.argtypes = [I64, I32]
    lib.pp_osem_chunks.restype = I64
    lib.pp_strerror.argtypes = [INT]
    lib.pp_strerror.restype = ctypes.c_char_p
    lib.pp_abi_version.restype = INT
    _lib = lib
    return lib


def check(code):
    if code != PP_OK:
        raise PPError(code, load().pp_strerror(code).decode())


def stream_of(t: torch.Tensor):
    return ctypes.c_void_p(torch.cuda.current_stream(t.device).cuda_stream)


def ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(0)


def _dev(*ts):
    dev = None
    for t in ts:
        if t is None:
            continue
        if not isinstance(t, torch.Tensor) or t.device.type != "cuda":
            raise TypeError("libppmi takes GPU tensors only")
        if not t.is_contiguous():
            raise ValueError("tensors must be contiguous")
        if dev is None:
            dev = t.device
        elif t.device != dev:
            raise ValueError("tensors on different devices")
    return dev


def _rays(xstart, xend):
    if xstart.dtype != torch.float32 or xend.dtype != torch.float32:
        raise TypeError("ray endpoints must be float32")
    if xstart.dim() != 2 or xstart.shape[1] != 3 or xend.shape != xstart.shape:
        raise ValueError("ray endpoints must be [n, 3] each")
    return xstart.shape[0]


def _img(img, geom):
    if img.dtype != torch.float32 or img.numel() != geom.n_vox:
        raise ValueError(f"image must be float32 with {geom.n_vox} voxels")


def _order(order, n):
    if order is None:
        return
    if order.dtype != torch.int32 or order.numel() != n:
        raise ValueError("order must be int32 [n]")


def _crystal_events(crystal_xyz, pair):
    """(n events, n crystals) of a crystal table [n_crystals, 3] float32 and pairs [n, 2] int32."""
    if crystal_xyz.dtype != torch.float32 or crystal_xyz.dim() != 2 or crystal_xyz.shape[1] != 3:
        raise ValueError("crystal_xyz must be float32 [n_crystals, 3]")
    if not 1 <= crystal_xyz.shape[0] < 2**31:
        raise ValueError("crystal table size out of range")
    if pair.dtype != torch.int32 or pair.dim() != 2 or pair.shape[1] != 2:
        raise ValueError("pair must be int32 [n, 2]")
    if pair.numel() and pair.data_ptr() % 8:
        raise ValueError("pair must be 8-byte aligned")
    return pair.shape[0], crystal_xyz.shape[0]


def _bins(bins, n):
    if bins.dtype != torch.int16 or bins.numel() != n:
        raise ValueError("tof_bin must be int16 [n]")
