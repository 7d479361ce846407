"""Python entry points with the names of the C ABI (include/ppmi.h).

``pp_*`` take caller-allocated GPU tensors exactly like the C functions and
launch on torch's current stream.  ``fwd``/``back``/... are conveniences that
allocate the output with torch and call the ``pp_*`` function.
"""
from __future__ import annotations

import ctypes

import torch

from ._lib import (TofParams, _bins, _crystal_events, _dev, _img, _order, _rays, as_geom, as_tof, check, load, ptr,
                   stream_of)


def pp_fwd(xstart, xend, geom, img, p, order=None):
    """Non-TOF forward projection into p[n] (overwritten). Sec. 2.1 of the paper.
    order: optional int32 processing order (pp_lm_presort); results stay indexed by ray."""
    g = as_geom(geom)
    _dev(xstart, xend, img, p, order)
    n = _rays(xstart, xend)
    _img(img, g)
    _order(order, n)
    if p.dtype != torch.float32 or p.numel() != n:
        raise ValueError("p must be float32 [n]")
    check(load().pp_fwd(ptr(xstart), ptr(xend), n, g.c(), ptr(img), ptr(p), ptr(order), stream_of(p)))
    return p


def pp_back(xstart, xend, geom, img, p, order=None):
    """Non-TOF back projection, img += A^T p (adjoint of pp_fwd)."""
    g = as_geom(geom)
    _dev(xstart, xend, img, p, order)
    n = _rays(xstart, xend)
    _img(img, g)
    _order(order, n)
    if p.dtype != torch.float32 or p.numel() != n:
        raise ValueError("p must be float32 [n]")
    check(load().pp_back(ptr(xstart), ptr(xend), n, g.c(), ptr(img), ptr(p), ptr(order), stream_of(img)))
    return img


def pp_fwd_tof_sino(xstart, xend, geom, tof, img, p):
    """TOF sinogram forward projection into p[n, n_bins] (overwritten)."""
    g, t = as_geom(geom), as_tof(tof)
    _dev(xstart, xend, img, p, t.sigma_per_ray, t.offset_per_ray)
    n = _rays(xstart, xend)
    _img(img, g)
    if p.dtype != torch.float32 or p.numel() != n * t.n_bins:
        raise ValueError("p must be float32 [n, n_bins]")
    check(load().pp_fwd_tof_sino(ptr(xstart), ptr(xend), n, g.c(), t.c(n), ptr(img), ptr(p), stream_of(p)))
    return p


def pp_back_tof_sino(xstart, xend, geom, tof, img, p):
    """TOF sinogram back projection, img += A^T p."""
    g, t = as_geom(geom), as_tof(tof)
    _dev(xstart, xend, img, p, t.sigma_per_ray, t.offset_per_ray)
    n = _rays(xstart, xend)
    _img(img, g)
    if p.dtype != torch.float32 or p.numel() != n * t.n_bins:
        raise ValueError("p must be float32 [n, n_bins]")
    check(load().pp_back_tof_sino(ptr(xstart), ptr(xend), n, g.c(), t.c(n), ptr(img), ptr(p), stream_of(img)))
    return img


def pp_fwd_tof_lm(xstart, xend, tof_bin, geom, tof, img, p, order=None):
    """TOF listmode forward projection (event's bin only) into p[n] (overwritten)."""
    g, t = as_geom(geom), as_tof(tof)
    _dev(xstart, xend, tof_bin, img, p, order, t.sigma_per_ray, t.offset_per_ray)
    n = _rays(xstart, xend)
    _bins(tof_bin, n)
    _img(img, g)
    _order(order, n)
    if p.dtype != torch.float32 or p.numel() != n:
        raise ValueError("p must be float32 [n]")
    check(load().pp_fwd_tof_lm(ptr(xstart), ptr(xend), ptr(tof_bin), n, g.c(), t.c(n), ptr(img), ptr(p),
                               ptr(order), stream_of(p)))
    return p


def pp_fwd_tof_lm_gather(xstart, xend, tof_bin, geom, tof, img, p, order, xstart_out, xend_out, tof_bin_out, p_out):
    """pp_fwd_tof_lm into p[n] that also writes the events and projections in processing order
    (xstart_out[i] = xstart[order[i]], ..., p_out[i] = p[order[i]])."""
    g, t = as_geom(geom), as_tof(tof)
    _dev(xstart, xend, tof_bin, img, p, order, xstart_out, xend_out, tof_bin_out, p_out)
    n = _rays(xstart, xend)
    _bins(tof_bin, n)
    _img(img, g)
    if order is None:
        raise ValueError("order is required")
    _order(order, n)
    if _rays(xstart_out, xend_out) != n:
        raise ValueError("xstart_out, xend_out must be float32 [n, 3]")
    _bins(tof_bin_out, n)
    for a in (p, p_out):
        if a.dtype != torch.float32 or a.numel() != n:
            raise ValueError("p and p_out must be float32 [n]")
    check(load().pp_fwd_tof_lm_gather(ptr(xstart), ptr(xend), ptr(tof_bin), n, g.c(), t.c(n), ptr(img), ptr(p),
                                      ptr(order), ptr(xstart_out), ptr(xend_out), ptr(tof_bin_out), ptr(p_out),
                                      stream_of(p)))
    return p


def pp_fwd_tof_lm_batch(xstart, xend, tof_bin, geom, tof, imgs, p, order=None):
    """pp_fwd_tof_lm through a batch of images: imgs [B, *dim] -> p [B, n] (overwritten)."""
    g, t = as_geom(geom), as_tof(tof)
    _dev(xstart, xend, tof_bin, imgs, p, order, t.sigma_per_ray, t.offset_per_ray)
    n = _rays(xstart, xend)
    _bins(tof_bin, n)
    _order(order, n)
    if imgs.dtype != torch.float32 or imgs.numel() % g.n_vox:
        raise ValueError(f"imgs must be float32 [B, {g.n_vox} voxels]")
    nb = imgs.numel() // g.n_vox
    if p.dtype != torch.float32 or p.numel() != nb * n:
        raise ValueError("p must be float32 [B, n]")
    check(load().pp_fwd_tof_lm_batch(ptr(xstart), ptr(xend), ptr(tof_bin), n, g.c(), t.c(n), ptr(imgs), nb, ptr(p),
                                     ptr(order), stream_of(p)))
    return p


def pp_back_tof_lm_batch(xstart, xend, tof_bin, geom, tof, imgs, p, order=None):
    """pp_back_tof_lm for a batch of value arrays: imgs [B, *dim] += A^T p[b] for p [B, n]."""
    g, t = as_geom(geom), as_tof(tof)
    _dev(xstart, xend, tof_bin, imgs, p, order, t.sigma_per_ray, t.offset_per_ray)
    n = _rays(xstart, xend)
    _bins(tof_bin, n)
    _order(order, n)
    if imgs.dtype != torch.float32 or imgs.numel() % g.n_vox:
        raise ValueError(f"imgs must be float32 [B, {g.n_vox} voxels]")
    nb = imgs.numel() // g.n_vox
    if p.dtype != torch.float32 or p.numel() != nb * n:
        raise ValueError("p must be float32 [B, n]")
    check(load().pp_back_tof_lm_batch(ptr(xstart), ptr(xend), ptr(tof_bin), n, g.c(), t.c(n), ptr(imgs), nb, ptr(p),
                                      ptr(order), stream_of(p)))
    return imgs


def pp_back_tof_lm(xstart, xend, tof_bin, geom, tof, img, p, order=None):
    """TOF listmode back projection, img += A^T p."""
    g, t = as_geom(geom), as_tof(tof)
    _dev(xstart, xend, tof_bin, img, p, order, t.sigma_per_ray, t.offset_per_ray)
    n = _rays(xstart, xend)
    _bins(tof_bin, n)
    _img(img, g)
    _order(order, n)
    if p.dtype != torch.float32 or p.numel() != n:
        raise ValueError("p must be float32 [n]")
    check(load().pp_back_tof_lm(ptr(xstart), ptr(xend), ptr(tof_bin), n, g.c(), t.c(n), ptr(img), ptr(p),
                                ptr(order), stream_of(img)))
    return img


def presort_workspace(n, device):
    """A byte tensor large enough for pp_lm_presort of n events."""
    nbytes = int(load().pp_lm_presort_workspace_bytes(int(n)))
    return torch.empty(max(nbytes, 1), dtype=torch.uint8, device=device)


def pp_lm_presort(xstart, xend, tof_bin, geom, tof, order, workspace, n_sub=1):
    """Processing order that groups events on neighbouring LORs (subset-major if n_sub > 1)."""
    g = as_geom(geom)
    _dev(xstart, xend, tof_bin, order, workspace)
    n = _rays(xstart, xend)
    _order(order, n)
    tc = None
    if tof_bin is not None:
        _bins(tof_bin, n)
        tc = as_tof(tof).c(n)
    check(load().pp_lm_presort(ptr(xstart), ptr(xend), ptr(tof_bin), n, g.c(), tc, int(n_sub), ptr(order),
                               ptr(workspace), workspace.numel() * workspace.element_size(), stream_of(order)))
    return order


def pp_lm_presort_noalloc(xstart, xend, tof_bin, geom, tof, order, n_sub=1):
    """pp_lm_presort with the library's own per-GPU workspace (no allocation; limited n)."""
    g = as_geom(geom)
    _dev(xstart, xend, tof_bin, order)
    n = _rays(xstart, xend)
    _order(order, n)
    tc = None
    if tof_bin is not None:
        _bins(tof_bin, n)
        tc = as_tof(tof).c(n)
    check(load().pp_lm_presort_noalloc(ptr(xstart), ptr(xend), ptr(tof_bin), n, g.c(), tc, int(n_sub), ptr(order),
                                       stream_of(order)))
    return order


def presort(xstart, xend, geom, tof_bin=None, tof=None, n_sub=1):
    order = torch.empty(xstart.shape[0], dtype=torch.int32, device=xstart.device)
    if xstart.shape[0] == 0:
        return order
    return pp_lm_presort(xstart, xend, tof_bin, geom, tof, order, presort_workspace(xstart.shape[0], xstart.device),
                         n_sub)


def pp_gather_events(xstart, xend, tof_bin, order, xstart_out, xend_out, tof_bin_out):
    """out[i] = in[order[i]] for the event arrays (library kernel)."""
    _dev(xstart, xend, tof_bin, order, xstart_out, xend_out, tof_bin_out)
    n = _rays(xstart, xend)
    _rays(xstart_out, xend_out)
    _order(order, n)
    if xstart_out.shape[0] != n or (tof_bin is not None and (tof_bin_out is None or tof_bin_out.numel() != n)):
        raise ValueError("output arrays must match the input event count")
    check(load().pp_gather_events(ptr(xstart), ptr(xend), ptr(tof_bin), ptr(order), n, ptr(xstart_out),
                                  ptr(xend_out), ptr(tof_bin_out), stream_of(order)))


def gather_events(xstart, xend, tof_bin, order):
    xs = torch.empty_like(xstart)
    xe = torch.empty_like(xend)
    tb = torch.empty_like(tof_bin) if tof_bin is not None else None
    if xstart.shape[0]:
        pp_gather_events(xstart, xend, tof_bin, order, xs, xe, tb)
    return xs, xe, tb


def pp_poisson_nll(p, bg, y, grad, partial):
    """Poisson loss of p + bg against y: grad[:] = 1 - y / (p + bg), partial[b] = the float64 partial
    sums of sum(ybar - y log ybar) (library kernel, one pass); returns partial."""
    _dev(p, y, grad, partial)
    n = p.numel()
    for a in (p, y, grad):
        if a.dtype != torch.float32 or a.numel() != n or not a.is_contiguous():
            raise ValueError("p, y, grad must be contiguous float32 of one size")
    if partial.dtype != torch.float64 or partial.dim() != 1 or not partial.is_contiguous():
        raise ValueError("partial must be a contiguous float64 vector")
    check(load().pp_poisson_nll(ptr(p), float(bg), ptr(y), n, ptr(grad), ptr(partial), partial.numel(),
                                stream_of(p)))
    return partial


def pp_fill(dst, value):
    """dst[:] = value with the library's fill kernel (graph-capture safe)."""
    _dev(dst)
    if dst.dtype != torch.float32:
        raise TypeError("float32 only")
    check(load().pp_fill(ptr(dst), dst.numel(), float(value), stream_of(dst)))
    return dst


def pp_tof_gaussian_table(tof, dx_max, lut=None):
    """(n, x0, dx) of the table of the Gaussian bin weight of `tof` at spacing <= dx_max mm;
    with `lut` (float32 CUDA tensor of >= n entries) the library also fills it."""
    t = as_tof(tof)
    base = TofParams(t.bin_width, t.sigma, t.n_sigmas, t.n_bins, t.center_offset)
    n, x0, step = ctypes.c_int32(), ctypes.c_float(), ctypes.c_float()
    if lut is not None:
        _dev(lut)
        if lut.dtype != torch.float32:
            raise ValueError("lut must be float32")
    check(load().pp_tof_gaussian_table(base.c(), float(dx_max), ptr(lut), 0 if lut is None else lut.numel(),
                                       ctypes.byref(n), ctypes.byref(x0), ctypes.byref(step),
                                       None if lut is None else stream_of(lut)))
    return n.value, x0.value, step.value


def gaussian_tof_table(tof, dx, device="cuda"):
    """TofParams whose kernel is the table of its own Gaussian bin weight
    w(x) = G(x + bw/2) - G(x - bw/2) over its support [-win, win], win = n_sigmas sigma + bw/2,
    at the largest spacing <= `dx` mm that puts the last entry on +win (pp_tof_gaussian_table:
    evaluated by the library on the device)."""
    t = as_tof(tof)
    n, _, _ = pp_tof_gaussian_table(t, dx)
    w = torch.empty(n, dtype=torch.float32, device=device)
    _, x0, step = pp_tof_gaussian_table(t, dx, w)
    return TofParams(t.bin_width, t.sigma, t.n_sigmas, t.n_bins, t.center_offset, w, x0, step)


def fwhm3(fwhm):
    """A resolution-model FWHM (mm, scalar or per axis) as the C float[3] the library takes."""
    if isinstance(fwhm, (int, float)):
        fwhm = (fwhm, fwhm, fwhm)
    f = [float(v) for v in fwhm]
    if len(f) != 3:
        raise ValueError("fwhm: a scalar or 3 values")
    return (ctypes.c_float * 3)(*f)


def pp_gauss3d(src, dst, tmp, geom, fwhm):
    """dst = G src, the Gaussian resolution model of FWHM `fwhm` mm; tmp is overwritten."""
    g = as_geom(geom)
    _dev(src, dst, tmp)
    for a in (src, dst, tmp):
        _img(a, g)
    check(load().pp_gauss3d(ptr(src), ptr(dst), ptr(tmp), g.c(), fwhm3(fwhm), stream_of(dst)))
    return dst


def gauss3d(img, geom, fwhm):
    """The image blurred by the resolution model (a new tensor)."""
    dst, tmp = torch.empty_like(img), torch.empty_like(img)
    return pp_gauss3d(img, dst, tmp, geom, fwhm)


def pp_count_samples(xstart, xend, tof_bin, geom, tof, counts):
    """Work counter: plane samples per ray that touch the grid (listmode: inside the TOF window)."""
    g = as_geom(geom)
    _dev(xstart, xend, tof_bin, counts)
    n = _rays(xstart, xend)
    if counts.dtype != torch.int32 or counts.numel() != n:
        raise ValueError("counts must be int32 [n]")
    tc = None
    if tof_bin is not None:
        _bins(tof_bin, n)
        t = as_tof(tof)
        _dev(xstart, t.sigma_per_ray, t.offset_per_ray)
        tc = t.c(n)
    check(load().pp_count_samples(ptr(xstart), ptr(xend), ptr(tof_bin), n, g.c(), tc, ptr(counts),
                                  stream_of(counts)))
    return counts


def count_samples(xstart, xend, geom, tof_bin=None, tof=None):
    counts = torch.empty(xstart.shape[0], dtype=torch.int32, device=xstart.device)
    return pp_count_samples(xstart, xend, tof_bin, geom, tof, counts)


# ------------------------------------------------------------- conveniences

def fwd(xstart, xend, geom, img, order=None):
    p = torch.empty(xstart.shape[0], dtype=torch.float32, device=xstart.device)
    return pp_fwd(xstart, xend, geom, img, p, order)


def back(xstart, xend, geom, p, img=None, order=None):
    g = as_geom(geom)
    if img is None:
        img = torch.zeros(g.dim, dtype=torch.float32, device=xstart.device)
    return pp_back(xstart, xend, g, img, p, order)


def fwd_tof_sino(xstart, xend, geom, tof, img):
    t = as_tof(tof)
    p = torch.empty((xstart.shape[0], t.n_bins), dtype=torch.float32, device=xstart.device)
    return pp_fwd_tof_sino(xstart, xend, geom, t, img, p)


def back_tof_sino(xstart, xend, geom, tof, p, img=None):
    g = as_geom(geom)
    if img is None:
        img = torch.zeros(g.dim, dtype=torch.float32, device=xstart.device)
    return pp_back_tof_sino(xstart, xend, g, tof, img, p)


def fwd_tof_lm(xstart, xend, tof_bin, geom, tof, img, order=None):
    p = torch.empty(xstart.shape[0], dtype=torch.float32, device=xstart.device)
    return pp_fwd_tof_lm(xstart, xend, tof_bin, geom, tof, img, p, order)


def back_tof_lm_batch(xstart, xend, tof_bin, geom, tof, p, order=None):
    """p [B, n] -> back projections [B, *dim] (new tensors)."""
    g = as_geom(geom)
    p = p.contiguous()
    nb = p.shape[0]
    imgs = torch.zeros((nb, *g.dim), dtype=torch.float32, device=p.device)
    return pp_back_tof_lm_batch(xstart, xend, tof_bin, geom, tof, imgs, p, order)


def fwd_tof_lm_gather(xstart, xend, tof_bin, geom, tof, img, order):
    """-> (p, xstart_sorted, xend_sorted, tof_bin_sorted, p_sorted): the projections indexed by event and
    the events with their projections in processing order (new tensors)."""
    n = xstart.shape[0]
    p, p_out = (torch.empty(n, dtype=torch.float32, device=xstart.device) for _ in range(2))
    xs_out, xe_out = torch.empty_like(xstart), torch.empty_like(xend)
    b_out = torch.empty_like(tof_bin)
    pp_fwd_tof_lm_gather(xstart, xend, tof_bin, geom, tof, img, p, order, xs_out, xe_out, b_out, p_out)
    return p, xs_out, xe_out, b_out, p_out


def fwd_tof_lm_batch(xstart, xend, tof_bin, geom, tof, imgs, order=None):
    """imgs [B, *dim] -> projections [B, n]."""
    g = as_geom(geom)
    imgs = imgs.contiguous()
    nb = imgs.numel() // g.n_vox if g.n_vox else 0
    p = torch.empty((nb, xstart.shape[0]), dtype=torch.float32, device=xstart.device)
    return pp_fwd_tof_lm_batch(xstart, xend, tof_bin, geom, tof, imgs, p, order)


def back_tof_lm(xstart, xend, tof_bin, geom, tof, p, img=None, order=None):
    g = as_geom(geom)
    if img is None:
        img = torch.zeros(g.dim, dtype=torch.float32, device=xstart.device)
    return pp_back_tof_lm(xstart, xend, tof_bin, g, tof, img, p, order)


# ----------------------------------------------------- crystal-index events
#
# Events given as (start crystal, end crystal) index pairs into a table of crystal positions;
# each entry point computes exactly what its coordinate counterpart computes for
# crystal_xyz[pair[:, 0]], crystal_xyz[pair[:, 1]].

def pp_fwd_crystals(crystal_xyz, pair, geom, img, p, order=None):
    g = as_geom(geom)
    _dev(crystal_xyz, pair, img, p, order)
    n, nc = _crystal_events(crystal_xyz, pair)
    _img(img, g)
    _order(order, n)
    if p.dtype != torch.float32 or p.numel() != n:
        raise ValueError("p must be float32 [n]")
    check(load().pp_fwd_crystals(ptr(crystal_xyz), nc, ptr(pair), n, g.c(), ptr(img), ptr(p), ptr(order),
                                 stream_of(p)))
    return p


def pp_back_crystals(crystal_xyz, pair, geom, img, p, order=None):
    g = as_geom(geom)
    _dev(crystal_xyz, pair, img, p, order)
    n, nc = _crystal_events(crystal_xyz, pair)
    _img(img, g)
    _order(order, n)
    if p.dtype != torch.float32 or p.numel() != n:
        raise ValueError("p must be float32 [n]")
    check(load().pp_back_crystals(ptr(crystal_xyz), nc, ptr(pair), n, g.c(), ptr(img), ptr(p), ptr(order),
                                  stream_of(img)))
    return img


def pp_fwd_tof_lm_crystals(crystal_xyz, pair, tof_bin, geom, tof, img, p, order=None):
    g, t = as_geom(geom), as_tof(tof)
    _dev(crystal_xyz, pair, tof_bin, img, p, order, t.sigma_per_ray, t.offset_per_ray)
    n, nc = _crystal_events(crystal_xyz, pair)
    _bins(tof_bin, n)
    _img(img, g)
    _order(order, n)
    if p.dtype != torch.float32 or p.numel() != n:
        raise ValueError("p must be float32 [n]")
    check(load().pp_fwd_tof_lm_crystals(ptr(crystal_xyz), nc, ptr(pair), ptr(tof_bin), n, g.c(), t.c(n), ptr(img),
                                        ptr(p), ptr(order), stream_of(p)))
    return p


def pp_back_tof_lm_crystals(crystal_xyz, pair, tof_bin, geom, tof, img, p, order=None):
    g, t = as_geom(geom), as_tof(tof)
    _dev(crystal_xyz, pair, tof_bin, img, p, order, t.sigma_per_ray, t.offset_per_ray)
    n, nc = _crystal_events(crystal_xyz, pair)
    _bins(tof_bin, n)
    _img(img, g)
    _order(order, n)
    if p.dtype != torch.float32 or p.numel() != n:
        raise ValueError("p must be float32 [n]")
    check(load().pp_back_tof_lm_crystals(ptr(crystal_xyz), nc, ptr(pair), ptr(tof_bin), n, g.c(), t.c(n), ptr(img),
                                         ptr(p), ptr(order), stream_of(img)))
    return img


def pp_lm_presort_crystals(crystal_xyz, pair, tof_bin, geom, tof, order, workspace, n_sub=1):
    """pp_lm_presort for crystal-index events (same key, same order)."""
    g = as_geom(geom)
    _dev(crystal_xyz, pair, tof_bin, order, workspace)
    n, nc = _crystal_events(crystal_xyz, pair)
    _order(order, n)
    tc = None
    if tof_bin is not None:
        _bins(tof_bin, n)
        tc = as_tof(tof).c(n)
    check(load().pp_lm_presort_crystals(ptr(crystal_xyz), nc, ptr(pair), ptr(tof_bin), n, g.c(), tc, int(n_sub),
                                        ptr(order), ptr(workspace), workspace.numel() * workspace.element_size(),
                                        stream_of(order)))
    return order


def presort_crystals(crystal_xyz, pair, geom, tof_bin=None, tof=None, n_sub=1):
    order = torch.empty(pair.shape[0], dtype=torch.int32, device=pair.device)
    if pair.shape[0] == 0:
        return order
    return pp_lm_presort_crystals(crystal_xyz, pair, tof_bin, geom, tof, order,
                                  presort_workspace(pair.shape[0], pair.device), n_sub)


def count_samples_crystals(crystal_xyz, pair, geom, tof_bin=None, tof=None):
    g = as_geom(geom)
    _dev(crystal_xyz, pair, tof_bin)
    n, nc = _crystal_events(crystal_xyz, pair)
    counts = torch.empty(n, dtype=torch.int32, device=pair.device)
    tc = None
    if tof_bin is not None:
        _bins(tof_bin, n)
        t = as_tof(tof)
        _dev(pair, t.sigma_per_ray, t.offset_per_ray)
        tc = t.c(n)
    check(load().pp_count_samples_crystals(ptr(crystal_xyz), nc, ptr(pair), ptr(tof_bin), n, g.c(), tc, ptr(counts),
                                           stream_of(counts)))
    return counts


def gather_crystal_events(pair, tof_bin, order):
    """(pair[order], tof_bin[order]) as new tensors (tof_bin may be None)."""
    _dev(pair, tof_bin, order)
    if pair.dtype != torch.int32 or pair.dim() != 2 or pair.shape[1] != 2:
        raise ValueError("pair must be int32 [n, 2]")
    n = pair.shape[0]
    _order(order, n)
    if tof_bin is not None:
        _bins(tof_bin, n)
    pair_out = torch.empty_like(pair)
    tb_out = None if tof_bin is None else torch.empty_like(tof_bin)
    check(load().pp_gather_crystal_events(ptr(pair), ptr(tof_bin), ptr(order), n, ptr(pair_out), ptr(tb_out),
                                          stream_of(pair_out)))
    return pair_out, tb_out


def fwd_crystals(crystal_xyz, pair, geom, img, order=None):
    p = torch.empty(pair.shape[0], dtype=torch.float32, device=pair.device)
    return pp_fwd_crystals(crystal_xyz, pair, geom, img, p, order)


def back_crystals(crystal_xyz, pair, geom, p, img=None, order=None):
    g = as_geom(geom)
    if img is None:
        img = torch.zeros(g.dim, dtype=torch.float32, device=pair.device)
    return pp_back_crystals(crystal_xyz, pair, g, img, p, order)


def fwd_tof_lm_crystals(crystal_xyz, pair, tof_bin, geom, tof, img, order=None):
    p = torch.empty(pair.shape[0], dtype=torch.float32, device=pair.device)
    return pp_fwd_tof_lm_crystals(crystal_xyz, pair, tof_bin, geom, tof, img, p, order)


def back_tof_lm_crystals(crystal_xyz, pair, tof_bin, geom, tof, p, img=None, order=None):
    g = as_geom(geom)
    if img is None:
        img = torch.zeros(g.dim, dtype=torch.float32, device=pair.device)
    return pp_back_tof_lm_crystals(crystal_xyz, pair, tof_bin, g, tof, img, p, order)
