"""Brute-force dense system matrix for tiny problems -- an independent check of the oracle.

Formulation (different mechanism from the oracle, same reading of the paper):
for every LOR l and every voxel v,

    A[l, v] = ell * [t(v_p) in [0, 1]] * hat(U(v_p) - v_u) * hat(W(v_p) - v_w) * w_tof(s(v_p))

where ``hat(x) = max(0, 1 - |x|)`` is the bilinear interpolation kernel
written as a tent function (no floor, no neighbour enumeration, zero padding
is automatic because only grid voxels exist), the plane parameter ``t`` is
computed in mm (not voxel-index) space, and the TOF weight is obtained by
Gauss-Legendre quadrature of the truncated Gaussian density over the TOF bin
(the convolution with the rect written out), not from an erf formula.  Per-ray
TOF parameters (``sigma_per_ray`` / ``offset_per_ray`` in the tof dict) replace
the scalar sigma / centre offset row by row; rows with an unusable entry stay 0.
"""
from __future__ import annotations

import math

import numpy as np

_GL_X, _GL_W = np.polynomial.legendre.leggauss(48)


def tof_weight_quadrature(s, centre, bin_width, sigma, n_sigmas):
    """int over the bin [centre - bw/2, centre + bw/2] of g(s - tau) d tau, with g the Gaussian
    density of std ``sigma`` set to zero beyond ``n_sigmas * sigma``."""
    trunc = n_sigmas * sigma
    lo = max(s - centre - 0.5 * bin_width, -trunc)  # integrate g(x) for x = s - tau
    hi = min(s - centre + 0.5 * bin_width, trunc)
    if hi <= lo:
        return 0.0
    x = 0.5 * (hi - lo) * _GL_X + 0.5 * (hi + lo)
    g = np.exp(-0.5 * (x / sigma) ** 2) / (sigma * np.sqrt(2.0 * np.pi))
    return float(0.5 * (hi - lo) * np.dot(_GL_W, g))


def system_matrix(xstart, xend, origin, voxsize, dim, tof=None, mode="nontof", bins=None):
    """Dense A: [n_lors, n_vox] (non-TOF / listmode) or [n_lors, n_bins, n_vox] (sinogram TOF)."""
    xs = np.asarray(xstart, dtype=np.float32)
    xe = np.asarray(xend, dtype=np.float32)
    o = np.asarray(origin, dtype=np.float32).astype(np.float64)
    h = np.asarray(voxsize, dtype=np.float32).astype(np.float64)
    dim = tuple(int(v) for v in dim)
    nv = dim[0] * dim[1] * dim[2]
    grid_idx = np.stack(np.meshgrid(*[np.arange(n) for n in dim], indexing="ij"), axis=-1).reshape(-1, 3)
    centres = o + grid_idx * h  # mm
    n = xs.shape[0]
    if mode == "sino":
        nb = int(tof["n_bins"])
        A = np.zeros((n, nb, nv))
    else:
        A = np.zeros((n, nv))
    for l in range(n):
        s32, e32 = xs[l], xe[l]
        if not (np.all(np.isfinite(s32)) and np.all(np.isfinite(e32))):
            continue
        d32 = (e32 - s32).astype(np.float32)
        p = int(np.argmax(np.abs(d32)))
        if d32[p] == 0:
            continue
        s = s32.astype(np.float64)
        d = e32.astype(np.float64) - s
        length = np.sqrt(np.sum(d * d))
        ell = h[p] * length / abs(d[p])
        inplane = [a for a in range(3) if a != p]
        if mode == "lm":
            b = int(bins[l])
            if b < 0 or b >= int(tof["n_bins"]):
                continue
        sig_l, off_l = (tof.get("sigma"), tof.get("center_offset", 0.0)) if tof is not None else (None, 0.0)
        if tof is not None and tof.get("sigma_per_ray") is not None:  # this ray's own kernel width
            sig_l = float(np.float32(tof["sigma_per_ray"][l]))
            if not (math.isfinite(sig_l) and sig_l > 0.0):
                continue
        if tof is not None and tof.get("offset_per_ray") is not None:  # this ray's own centre offset
            off_l = float(np.float32(tof["offset_per_ray"][l]))
            if not math.isfinite(off_l):
                continue
        for v in range(nv):
            c = centres[v]
            t = (c[p] - s[p]) / d[p]  # the plane through this voxel's centre
            if t < 0.0 or t > 1.0:
                continue
            x = s + t * d  # ray point on that plane (mm)
            wgt = 1.0
            for a in inplane:
                wgt *= max(0.0, 1.0 - abs((x[a] - c[a]) / h[a]))
            if wgt == 0.0:
                continue
            if mode == "nontof":
                A[l, v] = ell * wgt
                continue
            spos = (t - 0.5) * length
            wfn = tof.get("weight_fn")  # an explicit bin-weight function of x = s - c_b, if given

            def weight(cb):
                if wfn is not None:
                    return wfn(spos - cb)
                return tof_weight_quadrature(spos, cb, tof["bin_width"], sig_l, tof["n_sigmas"])

            if mode == "sino":
                for b in range(nb):
                    cb = (b - 0.5 * (nb - 1)) * tof["bin_width"] + off_l
                    A[l, b, v] = ell * wgt * weight(cb)
            else:
                cb = (b - 0.5 * (int(tof["n_bins"]) - 1)) * tof["bin_width"] + off_l
                A[l, v] = ell * wgt * weight(cb)
    return A


def gauss_matrix(dim, voxsize, fwhm):
    """Dense resolution-model matrix G[v, u] for a tiny grid, written without separability: the
    isotropic Gaussian exp(-|x_v - x_u|^2 / (2 sigma^2)) of the 3-D displacement in mm, kept
    where every axis offset is within that axis' truncation radius floor(4 sigma / h_a + 1/2)
    voxels, divided by its sum over that box (so that G 1 = 1 away from the edges).  Voxels
    outside the grid simply do not exist (zero padding)."""
    dim = tuple(int(d) for d in dim)
    h = np.asarray(voxsize, dtype=np.float32).astype(np.float64)
    f = np.broadcast_to(np.asarray(fwhm, dtype=np.float64), (3,))
    assert np.all(f == f[0]) and f[0] > 0, "isotropic kernel only"
    sigma = f[0] / math.sqrt(8.0 * math.log(2.0))
    r = np.floor(4.0 * sigma / h + 0.5).astype(int)
    # normalisation over the truncation box
    offs = np.stack(np.meshgrid(*[np.arange(-r[a], r[a] + 1) for a in range(3)], indexing="ij"), -1)
    norm = np.exp(-np.sum((offs * h) ** 2, axis=-1) / (2.0 * sigma**2)).sum()
    idx = np.stack(np.meshgrid(*[np.arange(d) for d in dim], indexing="ij"), -1).reshape(-1, 3)
    delta = idx[:, None, :] - idx[None, :, :]
    inside = np.all(np.abs(delta) <= r, axis=-1)
    g = np.exp(-np.sum((delta * h) ** 2, axis=-1) / (2.0 * sigma**2)) / norm
    return np.where(inside, g, 0.0)
