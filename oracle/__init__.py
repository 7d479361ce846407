"""FP64 CPU oracle for the Joseph projector (TEST INFRASTRUCTURE ONLY).

Only the tests, the smoke check and the benchmark's CPU-baseline leg may use
this package.  The GPU product path never imports it and shares no code with
it.  The arithmetic lives in ``joseph64.c`` (plain C, double precision,
OpenMP over rays); this module builds it with gcc and wraps it with ctypes
for numpy arrays.

Every function takes the same float32 ray endpoints (``[n, 3]``) and image
geometry the GPU library takes, the image / projections in float64, and
returns float64 results.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "joseph64.c")
_LIB = os.path.join(_HERE, "liboracle64.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile ``joseph64.c`` into ``liboracle64.so`` (gcc, -O2, OpenMP, IEEE math)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp", "-fno-fast-math",
               "-Wall", "-Wextra", "-o", tmp, _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        build(force=True)
    lib = ctypes.CDLL(_LIB)
    P = ctypes.c_void_p
    I64 = ctypes.c_int64
    F = ctypes.c_float
    I32 = ctypes.c_int32
    geo = [P, P, I64, P, P, P]
    tof = [F, F, F, F, I32, P, I32, ctypes.c_double, ctypes.c_double, P, P]
    lib.orc_fwd.argtypes = geo + [P, P]
    lib.orc_back.argtypes = geo + [P, P]
    lib.orc_fwd_tof_sino.argtypes = geo + tof + [P, P]
    lib.orc_back_tof_sino.argtypes = geo + tof + [P, P]
    lib.orc_fwd_tof_lm.argtypes = geo + tof + [P, P, P]
    lib.orc_back_tof_lm.argtypes = geo + tof + [P, P, P]
    lib.orc_count_samples.argtypes = geo + tof + [P, P]
    lib.orc_count_samples.restype = I64
    lib.orc_lm_osem.argtypes = [P, P, P, I64, P, P, P] + tof + [P, ctypes.c_double, I32, I32, P, P]
    lib.orc_gauss3d.argtypes = [P, P, P, P, P]
    lib.orc_tof_sino_osem.argtypes = [P, P, I64, P, I32, P, P, P, F, F, F, F, I32, P, ctypes.c_double, I32, P]
    lib.orc_tof_kernel.argtypes = [P, I64, F, F, F, P, I32, ctypes.c_double, ctypes.c_double, P]
    lib.orc_max_threads.restype = ctypes.c_int
    _lib = lib
    return lib


def _f32(a, shape_last=None):
    a = np.ascontiguousarray(np.asarray(a, dtype=np.float32))
    if shape_last is not None and (a.ndim != 2 or a.shape[1] != shape_last):
        raise ValueError("expected an array of shape [n, %d]" % shape_last)
    return a


def _geom(origin, voxsize, dim):
    o = np.ascontiguousarray(np.asarray(origin, dtype=np.float32).reshape(3))
    h = np.ascontiguousarray(np.asarray(voxsize, dtype=np.float32).reshape(3))
    d = np.ascontiguousarray(np.asarray(dim, dtype=np.int32).reshape(3))
    return o, h, d


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def _tofargs(tof, n=None):
    """tof: object/dict with bin_width, sigma, n_sigmas, n_bins, (center_offset) and, for a
    tabulated kernel, lut (float32 array of the bin weight at lut_x0 + i * lut_dx), lut_x0, lut_dx;
    optionally sigma_per_ray / offset_per_ray (float32 [n]: ray l's sigma / centre offset in place
    of the scalar).  The returned tuple keeps the arrays alive for the call."""
    g = (lambda k, d=None: tof.get(k, d)) if isinstance(tof, dict) else (lambda k, d=None: getattr(tof, k, d))
    per = []
    for key in ("sigma_per_ray", "offset_per_ray"):
        a = g(key)
        if a is not None:
            a = np.ascontiguousarray(np.asarray(a, dtype=np.float32).ravel())
            if n is None or a.size != n:
                raise ValueError(f"{key} needs one entry per ray")
        per.append(a)
    lut = g("lut")
    if lut is not None:
        lut = np.ascontiguousarray(np.asarray(lut, dtype=np.float32).ravel())
        if lut.size < 2 or not float(g("lut_dx")) > 0:
            raise ValueError("lut needs >= 2 entries and lut_dx > 0")
        lp, ln, x0, dx = _ptr(lut), lut.size, float(g("lut_x0")), float(g("lut_dx"))
    else:
        lp, ln, x0, dx = None, 0, 0.0, 1.0
    return _TofArgs((ctypes.c_float(g("bin_width")), ctypes.c_float(g("sigma")), ctypes.c_float(g("n_sigmas")),
                     ctypes.c_float(g("center_offset", 0.0)), ctypes.c_int32(int(g("n_bins"))), lp,
                     ctypes.c_int32(ln), ctypes.c_double(x0), ctypes.c_double(dx),
                     *[None if a is None else _ptr(a) for a in per]), (lut, per))


class _TofArgs(tuple):
    """The C arguments of a TOF kernel; holds references to the arrays they point into."""

    def __new__(cls, args, keep):
        t = super().__new__(cls, args)
        t._keep = keep
        return t


def max_threads() -> int:
    return int(_load().orc_max_threads())


def fwd(xstart, xend, origin, voxsize, dim, img):
    """Non-TOF forward projection. Returns float64 [n]."""
    lib = _load()
    xs, xe = _f32(xstart, 3), _f32(xend, 3)
    o, h, d = _geom(origin, voxsize, dim)
    x = np.ascontiguousarray(np.asarray(img, dtype=np.float64).reshape(tuple(d)))
    out = np.zeros(xs.shape[0], dtype=np.float64)
    lib.orc_fwd(_ptr(xs), _ptr(xe), xs.shape[0], _ptr(o), _ptr(h), _ptr(d), _ptr(x), _ptr(out))
    return out


def back(xstart, xend, origin, voxsize, dim, p):
    """Non-TOF back projection (adjoint). Returns float64 image ``dim``."""
    lib = _load()
    xs, xe = _f32(xstart, 3), _f32(xend, 3)
    o, h, d = _geom(origin, voxsize, dim)
    y = np.ascontiguousarray(np.asarray(p, dtype=np.float64).reshape(xs.shape[0]))
    out = np.zeros(tuple(d), dtype=np.float64)
    lib.orc_back(_ptr(xs), _ptr(xe), xs.shape[0], _ptr(o), _ptr(h), _ptr(d), _ptr(out), _ptr(y))
    return out


def fwd_tof_sino(xstart, xend, origin, voxsize, dim, tof, img):
    """TOF sinogram forward projection. Returns float64 [n, n_bins]."""
    lib = _load()
    xs, xe = _f32(xstart, 3), _f32(xend, 3)
    o, h, d = _geom(origin, voxsize, dim)
    ta = _tofargs(tof, xs.shape[0])
    x = np.ascontiguousarray(np.asarray(img, dtype=np.float64).reshape(tuple(d)))
    out = np.zeros((xs.shape[0], ta[4].value), dtype=np.float64)
    lib.orc_fwd_tof_sino(_ptr(xs), _ptr(xe), xs.shape[0], _ptr(o), _ptr(h), _ptr(d), *ta, _ptr(x), _ptr(out))
    return out


def back_tof_sino(xstart, xend, origin, voxsize, dim, tof, p):
    lib = _load()
    xs, xe = _f32(xstart, 3), _f32(xend, 3)
    o, h, d = _geom(origin, voxsize, dim)
    ta = _tofargs(tof, xs.shape[0])
    y = np.ascontiguousarray(np.asarray(p, dtype=np.float64).reshape(xs.shape[0], ta[4].value))
    out = np.zeros(tuple(d), dtype=np.float64)
    lib.orc_back_tof_sino(_ptr(xs), _ptr(xe), xs.shape[0], _ptr(o), _ptr(h), _ptr(d), *ta, _ptr(out), _ptr(y))
    return out


def _bins(b, n):
    b = np.ascontiguousarray(np.asarray(b, dtype=np.int16).reshape(n))
    return b


def fwd_tof_lm(xstart, xend, origin, voxsize, dim, tof, bins, img):
    """TOF listmode forward projection (only each event's bin). Returns float64 [n]."""
    lib = _load()
    xs, xe = _f32(xstart, 3), _f32(xend, 3)
    o, h, d = _geom(origin, voxsize, dim)
    ta = _tofargs(tof, xs.shape[0])
    b = _bins(bins, xs.shape[0])
    x = np.ascontiguousarray(np.asarray(img, dtype=np.float64).reshape(tuple(d)))
    out = np.zeros(xs.shape[0], dtype=np.float64)
    lib.orc_fwd_tof_lm(_ptr(xs), _ptr(xe), xs.shape[0], _ptr(o), _ptr(h), _ptr(d), *ta, _ptr(b), _ptr(x),
                       _ptr(out))
    return out


def back_tof_lm(xstart, xend, origin, voxsize, dim, tof, bins, p):
    lib = _load()
    xs, xe = _f32(xstart, 3), _f32(xend, 3)
    o, h, d = _geom(origin, voxsize, dim)
    ta = _tofargs(tof, xs.shape[0])
    b = _bins(bins, xs.shape[0])
    y = np.ascontiguousarray(np.asarray(p, dtype=np.float64).reshape(xs.shape[0]))
    out = np.zeros(tuple(d), dtype=np.float64)
    lib.orc_back_tof_lm(_ptr(xs), _ptr(xe), xs.shape[0], _ptr(o), _ptr(h), _ptr(d), *ta, _ptr(b), _ptr(out),
                        _ptr(y))
    return out


def count_samples(xstart, xend, origin, voxsize, dim, tof=None, bins=None, per_ray=False):
    """Plane samples whose stencil touches the grid (TOF listmode: with non-zero weight)."""
    lib = _load()
    xs, xe = _f32(xstart, 3), _f32(xend, 3)
    o, h, d = _geom(origin, voxsize, dim)
    ta = _tofargs(tof, xs.shape[0]) if tof is not None else _tofargs({"bin_width": 1.0, "sigma": 1.0, "n_sigmas": 1.0,
                                                          "n_bins": 1})
    b = _bins(bins, xs.shape[0]) if bins is not None else None
    pr = np.zeros(xs.shape[0], dtype=np.int64) if per_ray else None
    tot = lib.orc_count_samples(_ptr(xs), _ptr(xe), xs.shape[0], _ptr(o), _ptr(h), _ptr(d), *ta,
                                _ptr(b) if b is not None else None, _ptr(pr) if pr is not None else None)
    return (int(tot), pr) if per_ray else int(tot)


def tof_kernel(x, tof):
    """The TOF bin weight w(x) of one bin centred at 0 (Gaussian or table of `tof`), float64."""
    lib = _load()
    xx = np.ascontiguousarray(np.asarray(x, dtype=np.float64).ravel())
    ta = _tofargs(tof)
    out = np.empty_like(xx)
    lib.orc_tof_kernel(_ptr(xx), xx.size, ta[0], ta[1], ta[2], ta[5], ta[6], ta[7], ta[8], _ptr(out))
    return out


def _fwhm3(fwhm):
    f = np.ascontiguousarray(np.broadcast_to(np.asarray(fwhm, dtype=np.float64), (3,)))
    if not np.all(np.isfinite(f)) or np.any(f < 0):
        raise ValueError("fwhm must be finite and >= 0")
    return f


def gauss3d(img, voxsize, fwhm):
    """Resolution model: the image blurred by a 3D Gaussian of FWHM `fwhm` mm (scalar or per axis),
    sampled on the voxel grid, truncated at 4 sigma, zero outside the grid (float64 result)."""
    lib = _load()
    x = np.ascontiguousarray(np.asarray(img, dtype=np.float64))
    if x.ndim != 3:
        raise ValueError("img must be 3-D")
    h = np.ascontiguousarray(np.asarray(voxsize, dtype=np.float32).reshape(3))
    d = np.ascontiguousarray(np.asarray(x.shape, dtype=np.int32))
    f = _fwhm3(fwhm)
    out = np.empty_like(x)
    lib.orc_gauss3d(_ptr(x), _ptr(out), _ptr(d), _ptr(h), _ptr(f))
    return out


def lm_osem(xstart, xend, bins, origin, voxsize, dim, tof, sens, bg, n_iter, n_sub, x0, fwhm=None):
    """Listmode TOF OSEM; returns the float64 image after n_iter x n_sub updates.  With `fwhm`
    (mm, scalar or per axis) the system model includes the Gaussian resolution model."""
    lib = _load()
    xs, xe = _f32(xstart, 3), _f32(xend, 3)
    o, h, d = _geom(origin, voxsize, dim)
    ta = _tofargs(tof, xs.shape[0])
    b = _bins(bins, xs.shape[0])
    s = np.ascontiguousarray(np.asarray(sens, dtype=np.float64).reshape(tuple(d)))
    x = np.array(np.asarray(x0, dtype=np.float64).reshape(tuple(d)), copy=True, order="C")
    f = None if fwhm is None else _fwhm3(fwhm)
    lib.orc_lm_osem(_ptr(xs), _ptr(xe), _ptr(b), xs.shape[0], _ptr(o), _ptr(h), _ptr(d), *ta, _ptr(s),
                    ctypes.c_double(bg), ctypes.c_int32(n_iter), ctypes.c_int32(n_sub), _ptr(x),
                    None if f is None else _ptr(f))
    return x


def tof_sino_osem(xstart, xend, subset, n_sub, origin, voxsize, dim, tof, y, bg, n_iter, x0):
    """TOF sinogram OSEM (Gaussian kernel): LOR l in subset ``subset[l]``; per subset
    x <- x * A_j^T (y / (A_j x + bg)) / A_j^T 1 (0 where A_j^T 1 == 0).  y: [n, n_bins] counts.
    Returns the float64 image after n_iter passes over the n_sub subsets."""
    lib = _load()
    xs, xe = _f32(xstart, 3), _f32(xend, 3)
    n = xs.shape[0]
    o, h, d = _geom(origin, voxsize, dim)
    ta = _tofargs(tof)
    if ta[5] is not None:
        raise ValueError("tof_sino_osem: Gaussian kernel only")
    sb = np.ascontiguousarray(np.asarray(subset, dtype=np.int32).reshape(n))
    yy = np.ascontiguousarray(np.asarray(y, dtype=np.float64).reshape(n, ta[4].value))
    x = np.array(np.asarray(x0, dtype=np.float64).reshape(tuple(d)), copy=True, order="C")
    lib.orc_tof_sino_osem(_ptr(xs), _ptr(xe), n, _ptr(sb), int(n_sub), _ptr(o), _ptr(h), _ptr(d), *ta[:5], _ptr(yy),
                          ctypes.c_double(bg), int(n_iter), _ptr(x))
    return x
