"""Seeded TOF listmode events drawn from a voxel phantom.

Stand-in for the measured NEMA acquisition the paper uses (Sec. 2.6), which
is not available here.  Recipe, per proposed event:

1. emission voxel drawn with probability proportional to its value, then a
   uniform point inside that voxel;
2. an isotropic direction;
3. the line through the point is intersected with the detector cylinder;
4. each intersection is snapped to the nearest crystal (angle) and ring (z);
   the pair is oriented as in the span-1 sinogram (so an event's start/end
   and TOF sign agree with the sinogram LOR of the same crystal pair) and is
   rejected if its ring difference exceeds ``max_rd``, its radial bin falls
   outside the sinogram, or a ring falls outside the scanner;
5. TOF: the true signed distance of the emission point along the snapped LOR
   from its midpoint (positive towards the end point) plus N(0, sigma) is
   binned with width ``bin_width`` (bin t covers
   ``[(t - n_bins/2) w, (t - n_bins/2 + 1) w)``), events outside
   ``[0, n_bins)`` rejected;
6. accepted events keep their (random) generation order.
"""
from __future__ import annotations

import math

import torch

from .phantom import ImageGrid
from .scanner import CylinderScanner


def _rng(seed, device):
    g = torch.Generator(device=device)
    g.manual_seed(int(seed))
    return g


def generate_tof_lm_events(scanner: CylinderScanner, n_rad: int, max_rd: int, grid: ImageGrid,
                           image: torch.Tensor, n_events: int, seed: int, tof_bin_width: float,
                           tof_sigma: float, n_tof_bins: int, device="cpu", chunk=None,
                           return_points=False, return_crystals=False):
    """Returns (xstart float32 [n,3], xend float32 [n,3], tof_bin int16 [n]) on ``device``; with
    return_points also the emission points (float64 [n,3]), with return_crystals also the
    crystal indices of the end points (int32 [n,2], index ring * n_crystals + crystal into
    ``scanner.crystal_table()``, whose rows are bit-identical to xstart / xend)."""
    device = torch.device(device)
    g = _rng(seed, device)
    w = image.to(device=device, dtype=torch.float64).reshape(-1)
    cdf = torch.cumsum(w, 0)
    total = cdf[-1].item()
    if total <= 0:
        raise ValueError("phantom has no activity")
    n0, n1, n2 = grid.dim
    N = scanner.n_crystals
    two_pi = 2.0 * math.pi
    rad_lo, rad_hi = -(n_rad // 2), n_rad - n_rad // 2
    chunk = chunk or max(4096, min(1 << 23, 12 * n_events))
    outs, n_have = [], 0
    while n_have < n_events:
        u = torch.rand(chunk, generator=g, device=device, dtype=torch.float64)
        idx = torch.searchsorted(cdf, u * total).clamp_(max=w.numel() - 1)
        i2 = idx % n2
        i1 = (idx // n2) % n1
        i0 = idx // (n1 * n2)
        jit = torch.rand((chunk, 3), generator=g, device=device, dtype=torch.float64) - 0.5
        p = torch.stack([grid.origin[0] + (i0.to(torch.float64) + jit[:, 0]) * grid.voxsize[0],
                         grid.origin[1] + (i1.to(torch.float64) + jit[:, 1]) * grid.voxsize[1],
                         grid.origin[2] + (i2.to(torch.float64) + jit[:, 2]) * grid.voxsize[2]], dim=1)
        cth = 2.0 * torch.rand(chunk, generator=g, device=device, dtype=torch.float64) - 1.0
        phi = two_pi * torch.rand(chunk, generator=g, device=device, dtype=torch.float64)
        sth = torch.sqrt(torch.clamp(1.0 - cth * cth, min=0.0))
        d = torch.stack([sth * torch.cos(phi), sth * torch.sin(phi), cth], dim=1)
        # cylinder intersection |p_xy + t d_xy| = R
        a = d[:, 0] ** 2 + d[:, 1] ** 2
        b = 2.0 * (p[:, 0] * d[:, 0] + p[:, 1] * d[:, 1])
        c = p[:, 0] ** 2 + p[:, 1] ** 2 - scanner.radius**2
        ok = a > 1e-12
        a_s = torch.where(ok, a, torch.ones_like(a))
        disc = torch.sqrt(torch.clamp(b * b - 4.0 * a_s * c, min=0.0))
        t1 = (-b - disc) / (2.0 * a_s)
        t2 = (-b + disc) / (2.0 * a_s)
        e1 = p + t1[:, None] * d
        e2 = p + t2[:, None] * d
        ca = torch.remainder(torch.round(torch.atan2(e1[:, 1], e1[:, 0]) * (N / two_pi)).to(torch.int64), N)
        cb = torch.remainder(torch.round(torch.atan2(e2[:, 1], e2[:, 0]) * (N / two_pi)).to(torch.int64), N)
        ra = torch.round(e1[:, 2] / scanner.ring_pitch + 0.5 * (scanner.n_rings - 1)).to(torch.int64)
        rb = torch.round(e2[:, 2] / scanner.ring_pitch + 0.5 * (scanner.n_rings - 1)).to(torch.int64)
        ok &= (ra >= 0) & (ra < scanner.n_rings) & (rb >= 0) & (rb < scanner.n_rings) & (ca != cb)
        ok &= (ra - rb).abs() <= max_rd
        # sinogram orientation: (a, b) is the stored order iff its view lies in [0, N/2)
        m = torch.remainder(cb - ca, N) - N // 2  # wrap(b - a - N/2) into [-N/2, N/2)
        par = torch.remainder(m, 2)
        v = torch.remainder(ca - (par - m) // 2 + N // 4, N)
        swap = v >= N // 2
        ci = torch.where(swap, cb, ca)
        cj = torch.where(swap, ca, cb)
        ri = torch.where(swap, rb, ra)
        rj = torch.where(swap, ra, rb)
        m = torch.remainder(cj - ci, N) - N // 2
        ok &= (m >= rad_lo) & (m < rad_hi)
        xs = scanner.crystal_xyz(ri, ci)
        xe = scanner.crystal_xyz(rj, cj)
        dl = xe - xs
        length = torch.linalg.vector_norm(dl, dim=1)
        ok &= length > 0
        length = torch.where(length > 0, length, torch.ones_like(length))
        s_true = ((p - 0.5 * (xs + xe)) * dl).sum(1) / length
        s_meas = s_true + tof_sigma * torch.randn(chunk, generator=g, device=device, dtype=torch.float64)
        tb = torch.floor(s_meas / tof_bin_width + 0.5 * n_tof_bins).to(torch.int64)
        ok &= (tb >= 0) & (tb < n_tof_bins)
        sel = torch.nonzero(ok).squeeze(1)
        take = sel[: n_events - n_have]
        piece = [xs[take].to(torch.float32), xe[take].to(torch.float32), tb[take].to(torch.int16)]
        if return_points:
            piece.append(p[take])
        if return_crystals:
            piece.append(torch.stack([ri[take] * N + ci[take], rj[take] * N + cj[take]], 1).to(torch.int32))
        outs.append(piece)
        n_have += take.numel()
    res = [torch.cat([o[k] for o in outs]).contiguous() for k in range(len(outs[0]))]
    return tuple(res)


def tof_per_ray_params(n, sigma, seed, width_range=(0.8, 1.25), offset_sd=5.0, n_bad=0, device="cpu"):
    """Per-ray TOF parameters for `n` rays: sigma_l = sigma * U(width_range) (a timing resolution
    that varies with the crystal pair or the count rate) and a centre offset ~ N(0, offset_sd) mm
    (a per-LOR timing calibration).  With n_bad > 0 the first entries are made unusable in turn:
    sigma 0, sigma < 0, sigma NaN, offset +inf (such rays must contribute nothing).  Returns
    float32 (sigma_per_ray, offset_per_ray) tensors on `device`."""
    g = torch.Generator().manual_seed(int(seed))
    lo, hi = width_range
    sig = sigma * (lo + (hi - lo) * torch.rand(n, generator=g, dtype=torch.float64))
    off = offset_sd * torch.randn(n, generator=g, dtype=torch.float64)
    sig, off = sig.to(torch.float32), off.to(torch.float32)
    bad = [(sig, 0.0), (sig, -1.0), (sig, float("nan")), (off, float("inf"))]
    for i in range(min(n_bad, n)):
        arr, val = bad[i % 4]
        arr[i] = val
    return sig.to(device), off.to(device)
