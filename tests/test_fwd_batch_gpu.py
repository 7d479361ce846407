"""pp_fwd_tof_lm_batch: a batch of images through one pass over the events.  Each image's projection
must be exactly pp_fwd_tof_lm of that image alone (same arithmetic, same order), for the three forms
of the TOF weight (fitted polynomial, erf with per-event sigma, table), with and without a presort
order, and for more images than one launch takes (11 = 8 + 3); one image is also checked against the
FP64 oracle.  pp_back_tof_lm_batch, its adjoint: each image against pp_back_tof_lm of its values alone
(19 = 16 + 3 value arrays, an all-zero one among them), one against the oracle, the adjoint identity of
the two batched calls, accumulation and empty batches.  Through the C ABI."""
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


# ------------------------------------------------------------------ batched back projection

@pytest.fixture(scope="module")
def back_case(gpu, batch_case):
    xs, xe, bins, _, G, img = batch_case
    gen = torch.Generator().manual_seed(84)
    ys = torch.rand((19, xs.shape[0]), generator=gen).to(xs.device)  # 16 + 3: two launches
    ys[5] = 0.0  # an all-zero value array
    ys[7, ::3] = 0.0
    return xs, xe, bins, G, ys


@pytest.mark.parametrize("form", ["poly", "erf_per_ray", "table"])
@pytest.mark.parametrize("sorted_", [False, True])
def test_back_batch_equals_single_images(gpu, back_case, form, sorted_):
    """Each image of pp_back_tof_lm_batch against pp_back_tof_lm of its values alone: equal up to the
    rounding of the sheets' fixed point and the order of float atomic adds (relative L2 <= 1e-5)."""
    xs, xe, bins, G, ys = back_case
    T = _forms(gpu, xs)[form]
    order = gpu.presort(xs, xe, G, bins, T) if sorted_ else None
    imgs = gpu.back_tof_lm_batch(xs, xe, bins, G, T, ys, order)
    torch.cuda.synchronize()
    assert imgs.shape == (ys.shape[0],) + tuple(G.dim)
    assert not torch.any(imgs[5])
    for b in range(ys.shape[0]):
        one = gpu.back_tof_lm(xs, xe, bins, G, T, ys[b].contiguous(), order=order)
        assert rel_l2(imgs[b].double().cpu().numpy(), one.double().cpu().numpy()) <= 1e-5, (form, b)


def test_back_batch_oracle_adjoint_and_edge_cases(gpu, back_case, batch_case):
    xs, xe, bins, G, ys = back_case
    imgs_in = batch_case[3]
    T = _forms(gpu, xs)["poly"]
    order = gpu.presort(xs, xe, G, bins, T)
    imgs = gpu.back_tof_lm_batch(xs, xe, bins, G, T, ys[:4].contiguous(), order)
    torch.cuda.synchronize()
    g, t = geom_of(C.GRID_SMALL), tof_of(C.TOF_CLIN)
    ref = oracle.back_tof_lm(xs.cpu().numpy(), xe.cpu().numpy(), g["origin"], g["voxsize"], g["dim"], t,
                             bins.cpu().numpy(), ys[2].double().cpu().numpy())
    assert rel_l2(imgs[2].double().cpu().numpy(), ref) <= 1e-4
    # adjoint pair of the two batched calls: <A x_b, y_b> = <x_b, A^T y_b> per image
    p = gpu.fwd_tof_lm_batch(xs, xe, bins, G, T, imgs_in[:4].contiguous(), order)
    torch.cuda.synchronize()
    for b in range(4):
        lhs = float((p[b].double() * ys[b].double()).sum())
        rhs = float((imgs_in[b].double() * imgs[b].double()).sum())
        assert abs(lhs - rhs) <= 1e-5 * abs(lhs), b
    # the call adds into the images it is given; no images or no events: nothing to do
    again = gpu.pp_back_tof_lm_batch(xs, xe, bins, G, T, imgs.clone(), ys[:4].contiguous(), order)
    torch.cuda.synchronize()
    assert rel_l2(again.double().cpu().numpy(), 2.0 * imgs.double().cpu().numpy()) <= 1e-5
    assert gpu.back_tof_lm_batch(xs, xe, bins, G, T, ys[:0].contiguous()).shape == (0,) + tuple(G.dim)
    e3 = xs[:0].contiguous()
    z = gpu.back_tof_lm_batch(e3, e3, bins[:0].contiguous(), G, T, ys[:2, :0].contiguous())
    assert z.shape == (2,) + tuple(G.dim) and not torch.any(z)
