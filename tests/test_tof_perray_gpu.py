"""Per-ray TOF parameters (each LOR / event with its own Gaussian width and bin-centre offset,
generalising the single kernel of Sec. 2.2) on the GPU against the FP64 oracle with the same
float32 arrays: listmode and sinogram TOF, forward and back (direct and presorted / sheet
paths), the work counter, the table kernel with per-ray offsets, and a clinical-size case.

Tolerances as for the scalar kernel: forward 1e-5, back 1e-4, adjoint 1e-5 relative L2.  Rays
with an unusable entry (sigma 0, < 0, NaN; offset infinite) must give exactly 0."""
import numpy as np
import pytest
import torch

import oracle
from helpers import geom_of, rel_l2, tof_of
from synth import configs as C
from synth import generate_tof_lm_events, tof_per_ray_params

pytestmark = pytest.mark.gpu
FWD_TOL, BACK_TOL, ADJ_TOL = 1e-5, 1e-4, 1e-5
N_BAD = 8


def np64(t):
    return t.detach().cpu().numpy().astype(np.float64)


def params(gpu, tof, sig, off, which, lut=None):
    """(TofParams for the library, tof dict for the oracle) with the per-ray arrays in `which`."""
    kw, ko = {}, {}
    if "sigma" in which:
        kw["sigma_per_ray"], ko["sigma_per_ray"] = sig.cuda(), sig.numpy()
    if "offset" in which:
        kw["offset_per_ray"], ko["offset_per_ray"] = off.cuda(), off.numpy()
    if lut is not None:
        tab, x0, dx = lut
        kw.update(lut=torch.from_numpy(tab).cuda(), lut_x0=x0, lut_dx=dx)
        ko.update(lut=tab, lut_x0=x0, lut_dx=dx)
    T = gpu.TofParams(tof["bin_width"], tof["sigma"], tof["n_sigmas"], tof["n_bins"], tof["center_offset"], **kw)
    return T, dict(tof, **ko)


@pytest.fixture(scope="module")
def small(gpu):
    img = C.phantom_small()
    t = C.TOF_CLIN
    xs, xe, bins = generate_tof_lm_events(C.SCANNER_SMALL, C.SINO_SMALL.n_rad, C.SINO_SMALL.max_rd, C.GRID_SMALL,
                                          img, 60_001, seed=91, tof_bin_width=t.bin_width, tof_sigma=t.sigma,
                                          n_tof_bins=t.n_bins)
    g = geom_of(C.GRID_SMALL)
    G = gpu.ImageGeom(g["dim"], g["voxsize"], g["origin"])
    return xs, xe, bins, img, g, G, tof_of(t)


@pytest.mark.parametrize("which", [("sigma",), ("offset",), ("sigma", "offset")])
def test_per_ray_listmode_matches_oracle(gpu, small, which):
    xs, xe, bins, img, g, G, tof = small
    n = xs.shape[0]
    sig, off = tof_per_ray_params(n, tof["sigma"], seed=92, n_bad=N_BAD)
    T, tof_o = params(gpu, tof, sig, off, which)
    d = torch.device("cuda")
    xs_d, xe_d, b_d, img_d = xs.to(d), xe.to(d), bins.to(d), img.to(d)
    p = gpu.fwd_tof_lm(xs_d, xe_d, b_d, G, T, img_d)
    p_ref = oracle.fwd_tof_lm(xs.numpy(), xe.numpy(), g["origin"], g["voxsize"], g["dim"], tof_o, bins.numpy(),
                              img.numpy().astype(np.float64))
    assert rel_l2(np64(p), p_ref) <= FWD_TOL
    bad = [i for i in range(N_BAD) if ("sigma" in which and i % 4 < 3) or ("offset" in which and i % 4 == 3)]
    assert not torch.any(p[bad]) and not np.any(p_ref[bad])
    y = torch.rand(n, generator=torch.Generator().manual_seed(93))
    bk = gpu.back_tof_lm(xs_d, xe_d, b_d, G, T, y.to(d))
    b_ref = oracle.back_tof_lm(xs.numpy(), xe.numpy(), g["origin"], g["voxsize"], g["dim"], tof_o, bins.numpy(),
                               y.numpy().astype(np.float64))
    assert rel_l2(np64(bk), b_ref) <= BACK_TOL
    lhs, rhs = float(np.dot(np64(p), y.numpy())), float(np.sum(np64(bk) * img.numpy()))
    assert abs(lhs - rhs) <= ADJ_TOL * abs(lhs)
    # presorted order: the sheet path of the back projection
    order = gpu.presort(xs_d, xe_d, G, b_d, T)
    p2 = gpu.fwd_tof_lm(xs_d, xe_d, b_d, G, T, img_d, order=order)
    assert rel_l2(np64(p2), p_ref) <= FWD_TOL
    bk2 = gpu.back_tof_lm(xs_d, xe_d, b_d, G, T, y.to(d), order=order)
    assert rel_l2(np64(bk2), b_ref) <= BACK_TOL
    # the per-ray parameters do change the result (not silently ignored)
    p0 = gpu.fwd_tof_lm(xs_d, xe_d, b_d, G, gpu.TofParams(tof["bin_width"], tof["sigma"], tof["n_sigmas"],
                                                          tof["n_bins"]), img_d)
    assert rel_l2(np64(p0), p_ref) > 1e-3


@pytest.mark.parametrize("which", [("sigma",), ("sigma", "offset")])
def test_per_ray_sinogram_matches_oracle(gpu, small, which):
    _, _, _, img, g, G, tof = small
    xs, xe = C.SINO_SMALL.lors()
    n = xs.shape[0]
    sig, off = tof_per_ray_params(n, tof["sigma"], seed=94, n_bad=N_BAD)
    T, tof_o = params(gpu, tof, sig, off, which)
    d = torch.device("cuda")
    pt = gpu.fwd_tof_sino(xs.to(d), xe.to(d), G, T, img.to(d))
    ref = oracle.fwd_tof_sino(xs.numpy(), xe.numpy(), g["origin"], g["voxsize"], g["dim"], tof_o,
                              img.numpy().astype(np.float64))
    assert rel_l2(np64(pt), ref) <= FWD_TOL
    y = torch.rand(tuple(pt.shape), generator=torch.Generator().manual_seed(95))
    bt = gpu.back_tof_sino(xs.to(d), xe.to(d), G, T, y.to(d))
    bref = oracle.back_tof_sino(xs.numpy(), xe.numpy(), g["origin"], g["voxsize"], g["dim"], tof_o,
                                y.numpy().astype(np.float64))
    assert rel_l2(np64(bt), bref) <= BACK_TOL
    lhs, rhs = float(np.sum(np64(pt) * y.numpy())), float(np.sum(np64(bt) * img.numpy()))
    assert abs(lhs - rhs) <= ADJ_TOL * abs(lhs)


def test_per_ray_work_counter_matches_oracle(gpu, small):
    xs, xe, bins, img, g, G, tof = small
    sig, off = tof_per_ray_params(xs.shape[0], tof["sigma"], seed=96, n_bad=N_BAD)
    T, tof_o = params(gpu, tof, sig, off, ("sigma", "offset"))
    cnt = gpu.count_samples(xs.cuda(), xe.cuda(), G, bins.cuda(), T)
    _, per = oracle.count_samples(xs.numpy(), xe.numpy(), g["origin"], g["voxsize"], g["dim"], tof_o, bins.numpy(),
                                  per_ray=True)
    assert np.array_equal(cnt.cpu().numpy().astype(np.int64), per)
    assert not np.any(per[:N_BAD])


def test_table_kernel_with_per_ray_offsets(gpu, small):
    """A tabulated (asymmetric, non-Gaussian) kernel moved by each ray's own offset."""
    xs, xe, bins, img, g, G, tof = small
    x = -70.3 + 0.5 * np.arange(221)
    tab = (np.where(x < 0, np.exp(-0.5 * (x / 25.0) ** 2), np.exp(-0.5 * (x / 12.0) ** 2)) * 0.4).astype(np.float32)
    tab[0] = tab[-1] = 0.0
    sig, off = tof_per_ray_params(xs.shape[0], tof["sigma"], seed=97, n_bad=0)
    T, tof_o = params(gpu, tof, sig, off, ("offset",), lut=(tab, float(x[0]), 0.5))
    d = torch.device("cuda")
    xs_d, xe_d, b_d = xs.to(d), xe.to(d), bins.to(d)
    p = gpu.fwd_tof_lm(xs_d, xe_d, b_d, G, T, img.to(d))
    p_ref = oracle.fwd_tof_lm(xs.numpy(), xe.numpy(), g["origin"], g["voxsize"], g["dim"], tof_o, bins.numpy(),
                              img.numpy().astype(np.float64))
    assert rel_l2(np64(p), p_ref) <= FWD_TOL
    order = gpu.presort(xs_d, xe_d, G, b_d, T)
    y = torch.rand(xs.shape[0], generator=torch.Generator().manual_seed(98))
    bk = gpu.back_tof_lm(xs_d, xe_d, b_d, G, T, y.to(d), order=order)
    b_ref = oracle.back_tof_lm(xs.numpy(), xe.numpy(), g["origin"], g["voxsize"], g["dim"], tof_o, bins.numpy(),
                               y.numpy().astype(np.float64))
    assert rel_l2(np64(bk), b_ref) <= BACK_TOL
    lxs, lxe = C.SINO_SMALL.lors()
    _, loff = tof_per_ray_params(lxs.shape[0], tof["sigma"], seed=99, n_bad=0)
    Ts, tof_s = params(gpu, tof, sig, loff, ("offset",), lut=(tab, float(x[0]), 0.5))
    pt = gpu.fwd_tof_sino(lxs.to(d), lxe.to(d), G, Ts, img.to(d))
    ref = oracle.fwd_tof_sino(lxs.numpy(), lxe.numpy(), g["origin"], g["voxsize"], g["dim"], tof_s,
                              img.numpy().astype(np.float64))
    assert rel_l2(np64(pt), ref) <= FWD_TOL


def test_per_ray_clinical_sampled(gpu):
    """4M clinical events with per-event sigma and offset, presorted: 5,000 sampled events of the
    forward projection against the oracle, the back projection through the adjoint identity."""
    d = torch.device("cuda")
    t = C.TOF_CLIN
    img = C.phantom_clin(device=d)
    n = 4_000_000
    xs, xe, bins = generate_tof_lm_events(C.SCANNER_CLIN, C.SINO_CLIN.n_rad, C.SINO_CLIN.max_rd, C.GRID_CLIN, img, n,
                                          seed=100, tof_bin_width=t.bin_width, tof_sigma=t.sigma,
                                          n_tof_bins=t.n_bins, device=d)
    sig, off = tof_per_ray_params(n, t.sigma, seed=101, n_bad=N_BAD)
    grid = C.GRID_CLIN
    G = gpu.ImageGeom(grid.dim, grid.voxsize, grid.origin)
    tof = tof_of(t)
    T, _ = params(gpu, tof, sig, off, ("sigma", "offset"))
    order = gpu.presort(xs, xe, G, bins, T)
    p = gpu.fwd_tof_lm(xs, xe, bins, G, T, img, order=order)
    idx = torch.randperm(n, generator=torch.Generator().manual_seed(102))[:5000].sort().values
    idx = torch.cat([torch.arange(N_BAD), idx])
    tof_o = dict(tof, sigma_per_ray=sig[idx].numpy(), offset_per_ray=off[idx].numpy())
    g = geom_of(grid)
    ref = oracle.fwd_tof_lm(xs[idx.to(d)].cpu().numpy(), xe[idx.to(d)].cpu().numpy(), g["origin"], g["voxsize"],
                            g["dim"], tof_o, bins[idx.to(d)].cpu().numpy(), img.cpu().numpy().astype(np.float64))
    got = np64(p[idx.to(d)])
    assert rel_l2(got, ref) <= FWD_TOL
    assert not np.any(got[:N_BAD])
    y = torch.rand(n, generator=torch.Generator().manual_seed(103)).to(d)
    bk = gpu.back_tof_lm(xs, xe, bins, G, T, y, order=order)
    lhs = float(torch.dot(p.double(), y.double()))
    rhs = float(torch.sum(bk.double() * img.double()))
    assert abs(lhs - rhs) <= ADJ_TOL * abs(lhs)
