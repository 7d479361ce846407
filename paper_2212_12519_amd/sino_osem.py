"""TOF sinogram OSEM on libppmi.so, in LOR chunks and optionally in shards.

Binding of pp_tof_sino_sensitivity / pp_tof_sino_osem_subset (argument
checks and marshalling) and the loop over iterations and subsets.  Each
subset update is one library call: forward TOF sinogram projection of a chunk
of LORs into a workspace, ratio y / (expectation + bg), back projection into
an accumulator image, chunk after chunk, then the multiplicative update
x <- x * A_j^T(ratio) / A_j^T 1 (the paper's Sec. 4 on the memory of TOF
sinogram reconstructions and chunk-wise processing).  With n_shards > 1 the
LORs of a subset are back projected into that many private images and summed
in the update pass -- the layout of a multi-GPU reconstruction on one device.
"""
from __future__ import annotations

import torch

from ._lib import _dev, _rays, as_geom, as_tof, check, load, ptr, stream_of


def _subset_args(xstart, xend, y, tof):
    n = _rays(xstart, xend)
    if y is not None and (y.dtype != torch.float32 or y.shape != (n, tof.n_bins)):
        raise ValueError("y must be float32 [n_lors, n_bins]")
    return n


def pp_tof_sino_sensitivity(xstart, xend, geom, tof, sens, work):
    """sens += A^T 1 over the LORs (chunks of work.shape[0] LORs through `work` [m, n_bins])."""
    g, t = as_geom(geom), as_tof(tof)
    _dev(xstart, xend, sens, work)
    n = _subset_args(xstart, xend, None, t)
    if sens.dtype != torch.float32 or sens.numel() != g.n_vox:
        raise ValueError("sens must be float32 with one entry per voxel")
    if work.dtype != torch.float32 or work.dim() != 2 or work.shape[1] != t.n_bins:
        raise ValueError("work must be float32 [m, n_bins]")
    check(load().pp_tof_sino_sensitivity(ptr(xstart), ptr(xend), n, g.c(), t.c(n), ptr(sens), ptr(work),
                                         work.shape[0], stream_of(sens)))
    return sens


def pp_tof_sino_osem_subset(xstart, xend, y, geom, tof, bg, x, acc, sens, work):
    """One subset update of x in place; acc: [n_shards, *dim] zero images (zero again afterwards)."""
    g, t = as_geom(geom), as_tof(tof)
    _dev(xstart, xend, y, x, acc, sens, work)
    n = _subset_args(xstart, xend, y, t)
    for name, a in (("x", x), ("sens", sens)):
        if a.dtype != torch.float32 or a.numel() != g.n_vox:
            raise ValueError(f"{name} must be float32 with one entry per voxel")
    if acc.dtype != torch.float32 or acc.numel() % g.n_vox or acc.numel() == 0:
        raise ValueError("acc must be float32 [n_shards, n_vox]")
    if work.dtype != torch.float32 or work.dim() != 2 or work.shape[1] != t.n_bins:
        raise ValueError("work must be float32 [m, n_bins]")
    check(load().pp_tof_sino_osem_subset(ptr(xstart), ptr(xend), ptr(y), n, g.c(), t.c(n), float(bg), ptr(x),
                                         ptr(acc), acc.numel() // g.n_vox, ptr(sens), ptr(work), work.shape[0],
                                         stream_of(x)))
    return x


def tof_sino_osem(subsets, geom, tof, x0, n_iter, bg=0.0, n_shards=1, work_lors=1 << 22, sens=None):
    """OSEM over `subsets`, a list of (xstart, xend, y) per subset (LORs of a subset contiguous,
    y [n, n_bins] counts), from x0, n_iter passes over the subsets in list order.  Returns
    (x, sens) with sens the list of subset sensitivities A_j^T 1 (computed unless given)."""
    g, t = as_geom(geom), as_tof(tof)
    dev = x0.device
    m = max(1, min(int(work_lors), max(s[0].shape[0] for s in subsets)))
    work = torch.empty((m, t.n_bins), dtype=torch.float32, device=dev)
    if sens is None:
        sens = []
        for xs, xe, _ in subsets:
            s = torch.zeros(g.dim, dtype=torch.float32, device=dev)
            if xs.shape[0]:
                pp_tof_sino_sensitivity(xs, xe, g, t, s, work)
            sens.append(s)
    x = x0.to(device=dev, dtype=torch.float32).reshape(g.dim).contiguous().clone()
    acc = torch.zeros((int(n_shards),) + tuple(g.dim), dtype=torch.float32, device=dev)
    for _ in range(int(n_iter)):
        for (xs, xe, y), s in zip(subsets, sens):
            pp_tof_sino_osem_subset(xs, xe, y, g, t, bg, x, acc, s, work)
    return x, sens
