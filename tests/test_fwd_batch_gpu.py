"""pp_fwd_tof_lm_batch: a batch of images through one pass over the events.  Each image's projection
must be exactly pp_fwd_tof_lm of that image alone (same arithmetic, same order), for the three forms
of the TOF weight (fitted polynomial, erf with per-event sigma, table), with and without a presort
order, and for more images than one launch takes (11 = 8 + 3); one image is also checked against the
FP64 oracle.  Through the C ABI."""
import numpy as np
import pytest
import torch

import oracle
from helpers import geom_of, rel_l2, tof_of
from synth import configs as C
from synth import generate_tof_lm_events, tof_per_ray_params

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def batch_case(gpu):
    img = C.phantom_small()
    t = C.TOF_CLIN
    xs, xe, bins = generate_tof_lm_events(C.SCANNER_SMALL, C.SINO_SMALL.n_rad, C.SINO_SMALL.max_rd, C.GRID_SMALL,
                                          img, 150_001, seed=81, tof_bin_width=t.bin_width, tof_sigma=t.sigma,
                                          n_tof_bins=t.n_bins)
    d = torch.device("cuda")
    gen = torch.Generator().manual_seed(82)
    imgs = torch.rand((11,) + tuple(C.GRID_SMALL.dim), generator=gen) * img[None]
    g = geom_of(C.GRID_SMALL)
    return xs.to(d), xe.to(d), bins.to(d), imgs.to(d), gpu.ImageGeom(g["dim"], g["voxsize"], g["origin"]), img


def _forms(gpu, xs):
    t = tof_of(C.TOF_CLIN)
    T = gpu.TofParams(t["bin_width"], t["sigma"], t["n_sigmas"], t["n_bins"])
    sig, _ = tof_per_ray_params(xs.shape[0], T.sigma, seed=83, device=xs.device)
    TP = gpu.TofParams(t["bin_width"], t["sigma"], t["n_sigmas"], t["n_bins"], sigma_per_ray=sig)
    TL = gpu.gaussian_tof_table(T, 0.05, device=xs.device)
    return {"poly": T, "erf_per_ray": TP, "table": TL}


@pytest.mark.parametrize("form", ["poly", "erf_per_ray", "table"])
@pytest.mark.parametrize("sorted_", [False, True])
def test_batch_equals_single_images(gpu, batch_case, form, sorted_):
    xs, xe, bins, imgs, G, _ = batch_case
    T = _forms(gpu, xs)[form]
    order = gpu.presort(xs, xe, G, bins, T) if sorted_ else None
    p = gpu.fwd_tof_lm_batch(xs, xe, bins, G, T, imgs, order)
    torch.cuda.synchronize()
    assert p.shape == (imgs.shape[0], xs.shape[0])
    for b in range(imgs.shape[0]):
        one = gpu.fwd_tof_lm(xs, xe, bins, G, T, imgs[b].contiguous(), order)
        assert torch.equal(p[b], one), (form, b)


def test_batch_matches_oracle_and_edge_cases(gpu, batch_case):
    xs, xe, bins, imgs, G, img = batch_case
    T = _forms(gpu, xs)["poly"]
    two = torch.stack([img.to(imgs.device), imgs[3]])
    p = gpu.fwd_tof_lm_batch(xs, xe, bins, G, T, two)
    torch.cuda.synchronize()
    g, t = geom_of(C.GRID_SMALL), tof_of(C.TOF_CLIN)
    ref = oracle.fwd_tof_lm(xs.cpu().numpy(), xe.cpu().numpy(), g["origin"], g["voxsize"], g["dim"], t,
                            bins.cpu().numpy(), img.numpy())
    assert rel_l2(p[0].double().cpu().numpy(), ref) <= 1e-5
    # no images, no events: nothing to do
    assert gpu.fwd_tof_lm_batch(xs, xe, bins, G, T, imgs[:0]).shape == (0, xs.shape[0])
    e3 = xs[:0].contiguous()
    assert gpu.fwd_tof_lm_batch(e3, e3, bins[:0].contiguous(), G, T, imgs[:2]).shape == (2, 0)
