"""The TOF bin weight as the listmode kernels evaluate it, isolated.

A grid whose only non-zero voxel sits at the origin, and rays along axis 0 through that voxel's
centre: only the plane through the origin contributes, with bilinear weight 1, so the listmode
forward projection is p = ell * w(x), ell = the voxel size along axis 0, at the sample's distance
x from the bin centre.  The ray midpoint is the origin and bin 14 of 29 is centred there, so a
per-ray centre offset o puts the sample at x = -o exactly.  Sweeping o over the whole support
reads w(x) from the GPU (Sec. 2.1: Gaussian convolved with the bin rect, truncated at n_sigmas as
in Sec. 2.6) and compares it with the definition evaluated in float64:
  * the fitted polynomial (one sigma, per-ray offsets allowed): within 5e-7 of the peak weight;
  * the erf form (forced by a per-ray sigma equal to sigma): within the Hastings bound.
"""
import math

import numpy as np
import pytest
import torch
from scipy.special import erf

from synth import configs as C

SIG = float(np.float32(C.TOF_CLIN.sigma))
BW, NS, NB = 28.0, 3.0, 29


def exact_w(x):
    c = NS * SIG
    g = lambda y: 0.5 * erf(np.clip(y, -c, c) / (math.sqrt(2.0) * SIG))
    return g(x + BW / 2) - g(x - BW / 2)


def _project(gpu, sigma_per_ray):
    d = torch.device("cuda")
    G = gpu.ImageGeom((5, 3, 3), (2.0, 2.0, 2.0))  # voxel (2, 1, 1) at the origin
    img = torch.zeros((5, 3, 3), dtype=torch.float32)
    img[2, 1, 1] = 1.0
    win = NS * SIG + BW / 2
    off = torch.linspace(-1.05 * win, 1.05 * win, 20001, dtype=torch.float32)
    n = off.numel()
    xs = torch.tensor([[-300.0, 0.0, 0.0]]).repeat(n, 1)
    xe = torch.tensor([[300.0, 0.0, 0.0]]).repeat(n, 1)
    bins = torch.full((n,), NB // 2, dtype=torch.int16)
    sig = torch.full((n,), SIG, dtype=torch.float32).to(d) if sigma_per_ray else None
    T = gpu.TofParams(BW, SIG, NS, NB, offset_per_ray=off.to(d), sigma_per_ray=sig)
    p = gpu.fwd_tof_lm(xs.to(d), xe.to(d), bins.to(d), G, T, img.to(d))
    torch.cuda.synchronize()
    x = -off.double().numpy()
    return x, p.double().cpu().numpy() / 2.0  # ell = 2 mm


@pytest.mark.gpu
@pytest.mark.parametrize("form", ["poly", "erf"])
def test_bin_weight_against_definition(gpu, form):
    x, w = _project(gpu, sigma_per_ray=(form == "erf"))
    ref = exact_w(x)
    peak = exact_w(np.zeros(1))[0]
    err = np.max(np.abs(w - ref))
    bound = 5e-7 * peak if form == "poly" else 1.5e-6
    print(f"{form}: max |w - exact| = {err:.3e} (peak {peak:.4f})")
    assert err <= bound
    outside = np.abs(x) >= (NS * SIG + BW / 2) * (1 + 1e-5)
    assert np.all(w[outside] == 0.0)
