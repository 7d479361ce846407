"""Tabulated TOF kernel (the lookup-table alternative of Sec. 4, which also admits non-Gaussian
kernels) on the GPU against the FP64 oracle with the same float32 table: listmode and sinogram
TOF, forward and back, the work counter and listmode OSEM; and a finely tabulated Gaussian
against the closed-form (erf) kernel.

Tolerances as for the Gaussian kernel (forward 1e-5, back 1e-4, adjoint 1e-5, OSEM 1e-4 relative
L2).  Tabulated vs closed-form Gaussian at 0.05 mm spacing: linear interpolation errs by at most
h^2/8 max|w''| <= 2.5e-7 of the largest weight (sigma 24.8 mm), plus the float32 evaluation of
both (~1e-6): relative L2 <= 5e-6."""
import numpy as np
import pytest
import torch

import oracle
from helpers import geom_of, rel_l2, tof_of
from synth import configs as C
from synth import generate_tof_lm_events

pytestmark = pytest.mark.gpu
FWD_TOL, BACK_TOL, ADJ_TOL, OSEM_TOL = 1e-5, 1e-4, 1e-5, 1e-4


def np64(t):
    return t.detach().cpu().numpy().astype(np.float64)


def skewed_table():
    """A non-Gaussian, asymmetric kernel: a skewed bump over [-70.3, +39.7] mm around the bin
    centre.  The ends are off the lattice of plane positions of the small scanner's axis-aligned
    LORs (multiples of 2 mm from the bin centres): a sample exactly on an end is inside or
    outside the open support depending on rounding, which would make the sample counts of the
    two implementations differ by one without any difference in the projections (the table is 0
    there)."""
    x = -70.3 + 0.5 * np.arange(221)  # 0.5 mm spacing
    w = np.where(x < 0, np.exp(-0.5 * (x / 25.0) ** 2), np.exp(-0.5 * (x / 12.0) ** 2)) * 0.4
    w[0] = w[-1] = 0.0
    return w.astype(np.float32), float(x[0]), 0.5


@pytest.fixture(scope="module")
def small(gpu):
    img = C.phantom_small()
    t = C.TOF_CLIN
    xs, xe, bins = generate_tof_lm_events(C.SCANNER_SMALL, C.SINO_SMALL.n_rad, C.SINO_SMALL.max_rd, C.GRID_SMALL,
                                          img, 60_001, seed=81, tof_bin_width=t.bin_width, tof_sigma=t.sigma,
                                          n_tof_bins=t.n_bins)
    lut, x0, dx = skewed_table()
    g = geom_of(C.GRID_SMALL)
    tof = tof_of(t)
    G = gpu.ImageGeom(g["dim"], g["voxsize"], g["origin"])
    T = gpu.TofParams(tof["bin_width"], tof["sigma"], tof["n_sigmas"], tof["n_bins"], 0.0,
                      torch.from_numpy(lut).cuda(), x0, dx)
    tof_o = dict(tof, lut=lut, lut_x0=x0, lut_dx=dx)
    return xs, xe, bins, img, g, G, T, tof_o


def test_lut_listmode_matches_oracle(gpu, small):
    xs, xe, bins, img, g, G, T, tof_o = small
    d = torch.device("cuda")
    xs_d, xe_d, b_d, img_d = xs.to(d), xe.to(d), bins.to(d), img.to(d)
    p = gpu.fwd_tof_lm(xs_d, xe_d, b_d, G, T, img_d)
    p_ref = oracle.fwd_tof_lm(xs.numpy(), xe.numpy(), g["origin"], g["voxsize"], g["dim"], tof_o, bins.numpy(),
                              img.numpy().astype(np.float64))
    assert rel_l2(np64(p), p_ref) <= FWD_TOL
    y = torch.rand(xs.shape[0], generator=torch.Generator().manual_seed(82))
    bk = gpu.back_tof_lm(xs_d, xe_d, b_d, G, T, y.to(d))
    b_ref = oracle.back_tof_lm(xs.numpy(), xe.numpy(), g["origin"], g["voxsize"], g["dim"], tof_o, bins.numpy(),
                               y.numpy().astype(np.float64))
    assert rel_l2(np64(bk), b_ref) <= BACK_TOL
    lhs, rhs = float(np.dot(np64(p), y.numpy())), float(np.sum(np64(bk) * img.numpy()))
    assert abs(lhs - rhs) <= ADJ_TOL * abs(lhs)
    # presorted order gives the same results
    order = gpu.presort(xs_d, xe_d, G, b_d, T)
    p2 = gpu.fwd_tof_lm(xs_d, xe_d, b_d, G, T, img_d, order=order)
    assert rel_l2(np64(p2), p_ref) <= FWD_TOL
    bk2 = gpu.back_tof_lm(xs_d, xe_d, b_d, G, T, y.to(d), order=order)
    assert rel_l2(np64(bk2), b_ref) <= BACK_TOL


def test_lut_sinogram_matches_oracle(gpu, small):
    xs_l, xe_l, bins, img, g, G, T, tof_o = small
    xs, xe = C.SINO_SMALL.lors()
    d = torch.device("cuda")
    pt = gpu.fwd_tof_sino(xs.to(d), xe.to(d), G, T, img.to(d))
    ref = oracle.fwd_tof_sino(xs.numpy(), xe.numpy(), g["origin"], g["voxsize"], g["dim"], tof_o,
                              img.numpy().astype(np.float64))
    assert rel_l2(np64(pt), ref) <= FWD_TOL
    y = torch.rand(tuple(pt.shape), generator=torch.Generator().manual_seed(83))
    bt = gpu.back_tof_sino(xs.to(d), xe.to(d), G, T, y.to(d))
    bref = oracle.back_tof_sino(xs.numpy(), xe.numpy(), g["origin"], g["voxsize"], g["dim"], tof_o,
                                y.numpy().astype(np.float64))
    assert rel_l2(np64(bt), bref) <= BACK_TOL


def test_lut_work_counter_matches_oracle(gpu, small):
    xs, xe, bins, img, g, G, T, tof_o = small
    d = torch.device("cuda")
    cnt = gpu.count_samples(xs.to(d), xe.to(d), G, bins.to(d), T)
    _, per = oracle.count_samples(xs.numpy(), xe.numpy(), g["origin"], g["voxsize"], g["dim"], tof_o,
                                  bins.numpy(), per_ray=True)
    assert np.array_equal(cnt.cpu().numpy().astype(np.int64), per)


def test_lut_osem_matches_oracle(gpu, small):
    from paper_2212_12519_amd import osem

    xs, xe, bins, img, g, G, T, tof_o = small
    d = torch.device("cuda")
    lxs, lxe = C.SINO_SMALL.lors()
    sens = osem.sensitivity(lxs.to(d), lxe.to(d), G)
    x = osem.lm_osem(xs.to(d), xe.to(d), bins.to(d), G, T, sens, n_iter=2, n_sub=4, bg=0.1)
    sens_ref = oracle.back(lxs.numpy(), lxe.numpy(), g["origin"], g["voxsize"], g["dim"], np.ones(lxs.shape[0]))
    x_ref = oracle.lm_osem(xs.numpy(), xe.numpy(), bins.numpy(), g["origin"], g["voxsize"], g["dim"], tof_o,
                           sens_ref, 0.1, 2, 4, (sens_ref > 0).astype(np.float64))
    assert rel_l2(np64(x), x_ref) <= OSEM_TOL


def test_tabulated_gaussian_matches_closed_form_clinical(gpu):
    """2M clinical events: the Gaussian tabulated at 0.05 mm against the erf kernel, forward and
    (presorted) back projection, on the full clinical grid."""
    d = torch.device("cuda")
    t = C.TOF_CLIN
    img = C.phantom_clin(device=d)
    xs, xe, bins = generate_tof_lm_events(C.SCANNER_CLIN, C.SINO_CLIN.n_rad, C.SINO_CLIN.max_rd, C.GRID_CLIN, img,
                                          2_000_000, seed=84, tof_bin_width=t.bin_width, tof_sigma=t.sigma,
                                          n_tof_bins=t.n_bins, device=d)
    G = gpu.ImageGeom(C.GRID_CLIN.dim, C.GRID_CLIN.voxsize, C.GRID_CLIN.origin)
    T = gpu.TofParams(t.bin_width, t.sigma, t.n_sigmas, t.n_bins)
    TL = gpu.gaussian_tof_table(T, 0.05)
    order = gpu.presort(xs, xe, G, bins, T)
    p = gpu.fwd_tof_lm(xs, xe, bins, G, T, img, order=order)
    pl = gpu.fwd_tof_lm(xs, xe, bins, G, TL, img, order=order)
    assert rel_l2(np64(pl), np64(p)) <= 5e-6
    b = gpu.back_tof_lm(xs, xe, bins, G, T, p, order=order)
    bl = gpu.back_tof_lm(xs, xe, bins, G, TL, p, order=order)
    assert rel_l2(np64(bl), np64(b)) <= 5e-6
    c = gpu.count_samples(xs, xe, G, bins, T)
    cl = gpu.count_samples(xs, xe, G, bins, TL)
    # the table spans the same support; samples on its exact edges may differ by rounding
    assert abs(int(cl.sum()) - int(c.sum())) <= 1e-6 * int(c.sum()) + 10
