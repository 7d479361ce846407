"""Shared test helpers: random rays, error norms, seeded workloads."""
from __future__ import annotations

import numpy as np


def f32(x):
    return float(np.float32(x))


def tofd(bin_width, sigma, n_sigmas, n_bins, center_offset=0.0):
    return {"bin_width": f32(bin_width), "sigma": f32(sigma), "n_sigmas": f32(n_sigmas), "n_bins": int(n_bins),
            "center_offset": f32(center_offset)}


def random_rays(rng, n, origin, voxsize, dim, inside_frac=0.0, grid_step=None):
    """Rays whose endpoints lie on a sphere around the grid (a fraction optionally starting inside)."""
    o = np.asarray(origin, float)
    h = np.asarray(voxsize, float)
    c = o + 0.5 * (np.asarray(dim) - 1) * h
    r = 0.5 * np.linalg.norm(np.asarray(dim) * h) + 2.0
    u = rng.normal(size=(n, 3))
    u /= np.linalg.norm(u, axis=1, keepdims=True)
    v = rng.normal(size=(n, 3))
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    off = rng.uniform(-0.6, 0.6, size=(n, 3)) * (np.asarray(dim) * h)
    xs = c + off * 0.5 + r * u
    xe = c + off * 0.5 - r * u + 0.3 * r * v
    k = int(inside_frac * n)
    if k:
        xs[:k] = c + rng.uniform(-0.45, 0.45, size=(k, 3)) * (np.asarray(dim) * h)
    if grid_step:
        xs = np.round(xs / grid_step) * grid_step
        xe = np.round(xe / grid_step) * grid_step
    return xs.astype(np.float32), xe.astype(np.float32)


def rel_l2(got, ref):
    got = np.asarray(got, dtype=np.float64).ravel()
    ref = np.asarray(ref, dtype=np.float64).ravel()
    den = np.linalg.norm(ref)
    return float(np.linalg.norm(got - ref) / (den if den > 0 else 1.0))


def tof_of(spec):
    """TofSpec -> dict with float32-rounded values (what the library sees)."""
    return tofd(spec.bin_width, spec.sigma, spec.n_sigmas, spec.n_bins, spec.center_offset)


def geom_of(grid):
    return {"dim": tuple(grid.dim), "voxsize": tuple(grid.voxsize), "origin": tuple(grid.origin)}
