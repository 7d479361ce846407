"""Parity of the HIP projectors (through the C ABI) with the FP64 oracle.

Tolerances (relative L2 over the compared vector): forward 1e-5, back
projection 1e-4 (float32 atomics in nondeterministic order), adjoint identity
1e-5.  Small workloads are compared element by element in full; the
clinical-size workloads run at full size in the launch configuration the
benchmark times, and are compared on seeded samples of outputs the oracle
computes one by one, plus the adjoint identity over the whole operator.
"""
import numpy as np
import pytest
import torch

import oracle
from helpers import geom_of, random_rays, rel_l2, tof_of, tofd
from synth import configs as C
from synth import generate_tof_lm_events

pytestmark = pytest.mark.gpu

FWD_TOL, BACK_TOL, ADJ_TOL = 1e-5, 1e-4, 1e-5


def np64(t):
    return t.detach().cpu().numpy().astype(np.float64)


def inner64(a, b):
    return float(torch.sum(a.double() * b.double()).item())


# ----------------------------------------------------------------- small, full

@pytest.fixture(scope="module")
def small(gpu):
    xs, xe = C.SINO_SMALL.lors()
    img = C.phantom_small()
    rng = np.random.default_rng(C.SEED_SMALL_Y)
    y = rng.uniform(0, 1, size=xs.shape[0]).astype(np.float32)
    return xs, xe, img, torch.from_numpy(y)


def test_small_nontof_full(gpu, small):
    xs, xe, img, y = small
    g = geom_of(C.GRID_SMALL)
    dev = torch.device("cuda")
    xs_d, xe_d, img_d, y_d = xs.to(dev), xe.to(dev), img.to(dev), y.to(dev)
    p = gpu.fwd(xs_d, xe_d, gpu.ImageGeom(**g), img_d)
    bk = gpu.back(xs_d, xe_d, gpu.ImageGeom(**g), y_d)
    torch.cuda.synchronize()
    p_ref = oracle.fwd(xs.numpy(), xe.numpy(), g["origin"], g["voxsize"], g["dim"], img.numpy())
    b_ref = oracle.back(xs.numpy(), xe.numpy(), g["origin"], g["voxsize"], g["dim"], y.numpy())
    assert rel_l2(np64(p), p_ref) <= FWD_TOL
    assert rel_l2(np64(bk), b_ref) <= BACK_TOL
    assert abs(inner64(p, y_d) - inner64(img_d, bk)) <= ADJ_TOL * abs(inner64(p, y_d))
    # ragged tail: a count that is not a multiple of the 256-thread workgroup
    m = xs.shape[0] - 37
    p2 = gpu.fwd(xs_d[:m].contiguous(), xe_d[:m].contiguous(), gpu.ImageGeom(**g), img_d)
    assert torch.equal(p2, p[:m])


def test_small_tof_sino_full(gpu, small):
    xs, xe, img, _ = small
    g = geom_of(C.GRID_SMALL)
    tof = tof_of(C.TOF_CLIN)
    dev = torch.device("cuda")
    xs_d, xe_d, img_d = xs.to(dev), xe.to(dev), img.to(dev)
    T = gpu.TofParams(**{k: tof[k] for k in ("bin_width", "sigma", "n_sigmas", "n_bins", "center_offset")})
    pt = gpu.fwd_tof_sino(xs_d, xe_d, gpu.ImageGeom(**g), T, img_d)
    rng = np.random.default_rng(C.SEED_TOF_Y)
    yt = torch.from_numpy(rng.uniform(0, 1, size=(xs.shape[0], tof["n_bins"])).astype(np.float32))
    bt = gpu.back_tof_sino(xs_d, xe_d, gpu.ImageGeom(**g), T, yt.to(dev))
    torch.cuda.synchronize()
    pt_ref = oracle.fwd_tof_sino(xs.numpy(), xe.numpy(), g["origin"], g["voxsize"], g["dim"], tof, img.numpy())
    bt_ref = oracle.back_tof_sino(xs.numpy(), xe.numpy(), g["origin"], g["voxsize"], g["dim"], tof, yt.numpy())
    assert rel_l2(np64(pt), pt_ref) <= FWD_TOL
    assert rel_l2(np64(bt), bt_ref) <= BACK_TOL
    lhs, rhs = inner64(pt, yt.to(dev)), inner64(img_d, bt)
    assert abs(lhs - rhs) <= ADJ_TOL * abs(lhs)
    # the TOF bins of a fully covered LOR sum to erf(3/sqrt 2) x the non-TOF projection
    pn = gpu.fwd(xs_d, xe_d, gpu.ImageGeom(**g), img_d)
    from scipy.special import erf

    np.testing.assert_allclose(np64(pt.sum(1)), erf(3 / np.sqrt(2)) * np64(pn), rtol=2e-5, atol=1e-4)


def test_small_tof_lm_full(gpu):
    img = C.phantom_small()
    g = geom_of(C.GRID_SMALL)
    tofs = C.TOF_CLIN
    xs, xe, bins = generate_tof_lm_events(C.SCANNER_SMALL, C.SINO_SMALL.n_rad, C.SINO_SMALL.max_rd, C.GRID_SMALL,
                                          img, 200_003, seed=31, tof_bin_width=tofs.bin_width, tof_sigma=tofs.sigma,
                                          n_tof_bins=tofs.n_bins)
    tof = tof_of(tofs)
    T = gpu.TofParams(tof["bin_width"], tof["sigma"], tof["n_sigmas"], tof["n_bins"])
    dev = torch.device("cuda")
    y = torch.from_numpy(np.random.default_rng(32).uniform(0, 1, size=xs.shape[0]).astype(np.float32))
    p = gpu.fwd_tof_lm(xs.to(dev), xe.to(dev), bins.to(dev), gpu.ImageGeom(**g), T, img.to(dev))
    b = gpu.back_tof_lm(xs.to(dev), xe.to(dev), bins.to(dev), gpu.ImageGeom(**g), T, y.to(dev))
    torch.cuda.synchronize()
    p_ref = oracle.fwd_tof_lm(xs.numpy(), xe.numpy(), g["origin"], g["voxsize"], g["dim"], tof, bins.numpy(),
                              img.numpy())
    b_ref = oracle.back_tof_lm(xs.numpy(), xe.numpy(), g["origin"], g["voxsize"], g["dim"], tof, bins.numpy(),
                               y.numpy())
    assert rel_l2(np64(p), p_ref) <= FWD_TOL
    assert rel_l2(np64(b), b_ref) <= BACK_TOL
    lhs, rhs = inner64(p, y.to(dev)), inner64(img.to(dev), b)
    assert abs(lhs - rhs) <= ADJ_TOL * abs(lhs)
    # listmode bin t equals sinogram column t
    pt = gpu.fwd_tof_sino(xs.to(dev), xe.to(dev), gpu.ImageGeom(**g), T, img.to(dev))
    sel = pt.gather(1, bins.to(dev).long()[:, None]).squeeze(1)
    assert rel_l2(np64(p), np64(sel)) <= 1e-6


# ------------------------------------------------------------- edge cases

EDGE_GRIDS = [
    ((5, 4, 3), (1.0, 1.5, 2.0), (-2.0, -2.25, -2.0)),
    ((17, 9, 33), (2.0, 1.0, 1.25), (0.5, -3.0, 1.0)),
    ((40, 41, 7), (1.65, 1.65, 2.0), (-32.0, -33.0, -6.0)),
    # one and two voxels along the contiguous axis: the gathers' four-load path, and row pairs that
    # are the whole row
    ((6, 5, 1), (1.0, 1.0, 3.0), (-2.5, -2.0, 0.0)),
    ((7, 3, 2), (1.0, 2.0, 1.5), (-3.0, -2.0, -0.75)),
]


@pytest.mark.parametrize("gi", range(len(EDGE_GRIDS)))
def test_random_rays_all_axes(gpu, gi):
    """All principal axes and directions, rays starting inside the grid, grazing and missing rays,
    non-isotropic voxels and off-centre origins -- every variant against the oracle."""
    dim, vs, origin = EDGE_GRIDS[gi]
    rng = np.random.default_rng(300 + gi)
    xs, xe = random_rays(rng, 5000, origin, vs, dim, inside_frac=0.2)
    x = rng.uniform(0, 2, size=dim).astype(np.float32)
    y = rng.uniform(0, 1, size=xs.shape[0]).astype(np.float32)
    tof = tofd(3.0, 2.5, 3.0, 13, center_offset=0.7)
    T = gpu.TofParams(tof["bin_width"], tof["sigma"], tof["n_sigmas"], tof["n_bins"], tof["center_offset"])
    G = gpu.ImageGeom(dim, vs, origin)
    dev = torch.device("cuda")
    xs_d, xe_d = torch.from_numpy(xs).to(dev), torch.from_numpy(xe).to(dev)
    x_d, y_d = torch.from_numpy(x).to(dev), torch.from_numpy(y).to(dev)
    bins = rng.integers(-2, 15, size=xs.shape[0]).astype(np.int16)  # includes out-of-range bins
    b_d = torch.from_numpy(bins).to(dev)
    yt = rng.uniform(0, 1, size=(xs.shape[0], 13)).astype(np.float32)
    got = {
        "fwd": gpu.fwd(xs_d, xe_d, G, x_d),
        "back": gpu.back(xs_d, xe_d, G, y_d),
        "fwd_lm": gpu.fwd_tof_lm(xs_d, xe_d, b_d, G, T, x_d),
        "back_lm": gpu.back_tof_lm(xs_d, xe_d, b_d, G, T, y_d),
        "fwd_sino": gpu.fwd_tof_sino(xs_d, xe_d, G, T, x_d),
        "back_sino": gpu.back_tof_sino(xs_d, xe_d, G, T, torch.from_numpy(yt).to(dev)),
    }
    torch.cuda.synchronize()
    ref = {
        "fwd": oracle.fwd(xs, xe, origin, vs, dim, x),
        "back": oracle.back(xs, xe, origin, vs, dim, y),
        "fwd_lm": oracle.fwd_tof_lm(xs, xe, origin, vs, dim, tof, bins, x),
        "back_lm": oracle.back_tof_lm(xs, xe, origin, vs, dim, tof, bins, y),
        "fwd_sino": oracle.fwd_tof_sino(xs, xe, origin, vs, dim, tof, x),
        "back_sino": oracle.back_tof_sino(xs, xe, origin, vs, dim, tof, yt),
    }
    for k in got:
        tol = FWD_TOL if k.startswith("fwd") else BACK_TOL
        assert rel_l2(np64(got[k]), ref[k]) <= tol, k
    # every ray on its own (the forwards): a wrong neighbour at a row's end changes its ray by about a
    # sample's share (>= 1e-2), far above these bounds, even where the norm over all rays hides it
    for k in ("fwd", "fwd_lm", "fwd_sino"):
        g, r = np64(got[k]), ref[k]
        scale = max(np.abs(r).max(), 1e-30)
        assert np.all(np.abs(g - r) <= 1e-4 * np.abs(r) + 1e-5 * scale), k
    oob = (bins < 0) | (bins >= 13)
    assert not np.any(np64(got["fwd_lm"])[oob])


def test_degenerate_inputs(gpu):
    """Zero-length, NaN and Inf rays and rays missing the grid give exactly 0; n = 0 is a no-op."""
    dim, vs, origin = (4, 4, 4), (1.0, 1.0, 1.0), (-1.5, -1.5, -1.5)
    G = gpu.ImageGeom(dim, vs, origin)
    dev = torch.device("cuda")
    xs = torch.tensor([[1, 1, 1], [float("nan"), 0, 0], [-50, 30, 0], [0, 0, float("inf")]], dtype=torch.float32,
                      device=dev)
    xe = torch.tensor([[1, 1, 1], [5, 0, 0], [50, 30, 0], [0, 0, 5]], dtype=torch.float32, device=dev)
    img = torch.ones(dim, device=dev)
    assert not torch.any(gpu.fwd(xs, xe, G, img))
    assert not torch.any(gpu.back(xs, xe, G, torch.ones(4, device=dev)))
    T = gpu.TofParams(2.0, 1.0, 3.0, 5)
    bins = torch.full((4,), 2, dtype=torch.int16, device=dev)
    assert not torch.any(gpu.fwd_tof_lm(xs, xe, bins, G, T, img))
    assert not torch.any(gpu.fwd_tof_sino(xs, xe, G, T, img))
    e = torch.empty((0, 3), dtype=torch.float32, device=dev)
    assert gpu.fwd(e, e, G, img).numel() == 0
    z = torch.zeros(dim, device=dev)
    gpu.back(e, e, G, torch.empty(0, device=dev), z)
    torch.cuda.synchronize()
    assert not torch.any(z)


def test_largest_grid_far_corner(gpu):
    """The largest grid the library takes (1023 x 1024 x 1024 voxels, just under 2^30; a 4.3 GB image):
    axis-aligned rays through voxel centres of the far corner's row, column and line in an image of
    ones give exactly n_p h_p (pin 1) -- the forward gathers there use byte offsets near 2^32 -- and
    the back projection of ones along the last line puts h_p into the very last voxel."""
    dim, vs, origin = (1023, 1024, 1024), (1.0, 1.0, 1.0), (0.0, 0.0, 0.0)
    G = gpu.ImageGeom(dim, vs, origin)
    dev = torch.device("cuda")
    img = torch.ones(dim, device=dev)
    a, b, c = (d - 1 for d in dim)
    xs = torch.tensor([[-5, b, c], [a, -5, c], [a, b, -5], [-5, 512, 511]], dtype=torch.float32, device=dev)
    xe = torch.tensor([[dim[0] + 5, b, c], [a, dim[1] + 5, c], [a, b, dim[2] + 5], [dim[0] + 5, 512, 511]],
                      dtype=torch.float32, device=dev)
    p = gpu.fwd(xs, xe, G, img)
    assert p.tolist() == [float(dim[0]), float(dim[1]), float(dim[2]), float(dim[0])]
    T = gpu.TofParams(2.0, 1000.0, 3.0, 1)  # one bin much wider than the rays: weights near erf(1/(2 sqrt 2 1000))
    pt = gpu.fwd_tof_sino(xs, xe, G, T, img)
    assert torch.all(pt[:, 0] > 0)
    del img
    bk = torch.zeros(dim, device=dev)
    gpu.back(xs[2:3].contiguous(), xe[2:3].contiguous(), G, torch.ones(1, device=dev), bk)
    torch.cuda.synchronize()
    assert float(bk[a, b, c]) == 1.0 and float(bk[a, b, 0]) == 1.0
    assert float(bk.sum(dtype=torch.float64)) == float(dim[2])


# -------------------------------------------------- clinical sizes, sampled

@pytest.fixture(scope="module")
def clin(gpu):
    dev = torch.device("cuda")
    xs, xe = C.SINO_CLIN.lors(device=dev, radial_chunk=25)
    img = C.phantom_clin(device=dev)
    return xs, xe, img


def _sample(n, k, seed):
    return np.sort(np.random.default_rng(seed).choice(n, size=k, replace=False))


def test_clinical_nontof_fwd_full_size(gpu, clin):
    """335,008,000 LORs, 215x215x71 image: full-size forward, 20,000 sampled LORs vs oracle;
    back projection over the full sinogram checked by the adjoint identity."""
    xs, xe, img = clin
    G = gpu.ImageGeom(C.GRID_CLIN.dim, C.GRID_CLIN.voxsize, C.GRID_CLIN.origin)
    g = geom_of(C.GRID_CLIN)
    p = gpu.fwd(xs, xe, G, img)
    idx = torch.from_numpy(_sample(xs.shape[0], 20_000, 41)).to(xs.device)
    ref = oracle.fwd(xs[idx].cpu().numpy(), xe[idx].cpu().numpy(), g["origin"], g["voxsize"], g["dim"],
                     img.cpu().numpy())
    assert rel_l2(np64(p[idx]), ref) <= FWD_TOL
    gen = torch.Generator(device=xs.device)
    gen.manual_seed(C.SEED_CLIN_Y)
    y = torch.rand(xs.shape[0], generator=gen, device=xs.device)
    bk = gpu.back(xs, xe, G, y)
    lhs, rhs = inner64(p, y), inner64(img, bk)
    assert abs(lhs - rhs) <= ADJ_TOL * abs(lhs)
    del bk, y, p


def test_clinical_nontof_back_subset(gpu, clin):
    """Element-wise back projection parity on two full views (1.76M LORs) of the clinical sinogram."""
    xs, xe, img = clin
    g = geom_of(C.GRID_CLIN)
    G = gpu.ImageGeom(g["dim"], g["voxsize"], g["origin"])
    n_rad, n_views, n_planes = C.SINO_CLIN.shape
    sel = []
    for r in range(n_rad):
        for v in (0, 190):
            base = (r * n_views + v) * n_planes
            sel.append(torch.arange(base, base + n_planes))
    idx = torch.cat(sel).to(xs.device)
    xs_s, xe_s = xs[idx].contiguous(), xe[idx].contiguous()
    y = torch.from_numpy(np.random.default_rng(42).uniform(0, 1, size=idx.numel()).astype(np.float32))
    bk = gpu.back(xs_s, xe_s, G, y.to(xs.device))
    ref = oracle.back(xs_s.cpu().numpy(), xe_s.cpu().numpy(), g["origin"], g["voxsize"], g["dim"], y.numpy())
    assert rel_l2(np64(bk), ref) <= BACK_TOL


def test_clinical_tof_sino_full_size(gpu, clin):
    """29-bin TOF sinogram at full size (335M x 29 outputs): 5,000 sampled LORs vs the oracle
    (forward); back projection element-wise on those LORs; adjoint identity over a 1/8 slab."""
    xs, xe, img = clin
    g = geom_of(C.GRID_CLIN)
    G = gpu.ImageGeom(g["dim"], g["voxsize"], g["origin"])
    tof = tof_of(C.TOF_CLIN)
    T = gpu.TofParams(tof["bin_width"], tof["sigma"], tof["n_sigmas"], tof["n_bins"])
    pt = gpu.fwd_tof_sino(xs, xe, G, T, img)
    idx = torch.from_numpy(_sample(xs.shape[0], 5_000, 43)).to(xs.device)
    xs_s, xe_s = xs[idx].cpu().numpy(), xe[idx].cpu().numpy()
    ref = oracle.fwd_tof_sino(xs_s, xe_s, g["origin"], g["voxsize"], g["dim"], tof, img.cpu().numpy())
    assert rel_l2(np64(pt[idx]), ref) <= FWD_TOL
    y = np.random.default_rng(44).uniform(0, 1, size=ref.shape).astype(np.float32)
    bk = gpu.back_tof_sino(xs[idx].contiguous(), xe[idx].contiguous(), G, T, torch.from_numpy(y).to(xs.device))
    bref = oracle.back_tof_sino(xs_s, xe_s, g["origin"], g["voxsize"], g["dim"], tof, y)
    assert rel_l2(np64(bk), bref) <= BACK_TOL
    m = xs.shape[0] // 8
    gen = torch.Generator(device=xs.device)
    gen.manual_seed(C.SEED_TOF_Y)
    yy = torch.rand((m, tof["n_bins"]), generator=gen, device=xs.device)
    bb = gpu.back_tof_sino(xs[:m], xe[:m], G, T, yy)
    lhs, rhs = inner64(pt[:m], yy), inner64(img, bb)
    assert abs(lhs - rhs) <= ADJ_TOL * abs(lhs)
    del pt, bb, yy


@pytest.fixture(scope="module")
def lm40(gpu):
    dev = torch.device("cuda")
    img = C.phantom_clin(device=dev)
    t = C.TOF_CLIN
    xs, xe, bins = generate_tof_lm_events(C.SCANNER_CLIN, C.SINO_CLIN.n_rad, C.SINO_CLIN.max_rd, C.GRID_CLIN, img,
                                          C.N_EVENTS_LM, seed=C.SEED_EVENTS, tof_bin_width=t.bin_width,
                                          tof_sigma=t.sigma, n_tof_bins=t.n_bins, device=dev)
    return xs, xe, bins, img


def test_tof_lm_40m_events(gpu, lm40):
    """40M TOF listmode events at full size: 20,000 sampled events vs oracle (forward), the adjoint
    identity over all events, and element-wise back projection of the first 1M events."""
    xs, xe, bins, img = lm40
    g = geom_of(C.GRID_CLIN)
    G = gpu.ImageGeom(g["dim"], g["voxsize"], g["origin"])
    tof = tof_of(C.TOF_CLIN)
    T = gpu.TofParams(tof["bin_width"], tof["sigma"], tof["n_sigmas"], tof["n_bins"])
    p = gpu.fwd_tof_lm(xs, xe, bins, G, T, img)
    idx = torch.from_numpy(_sample(xs.shape[0], 20_000, 45)).to(xs.device)
    ref = oracle.fwd_tof_lm(xs[idx].cpu().numpy(), xe[idx].cpu().numpy(), g["origin"], g["voxsize"], g["dim"], tof,
                            bins[idx].cpu().numpy(), img.cpu().numpy())
    assert rel_l2(np64(p[idx]), ref) <= FWD_TOL
    assert float(p.min()) >= 0.0 and float(p.mean()) > 0.0
    gen = torch.Generator(device=xs.device)
    gen.manual_seed(46)
    y = torch.rand(xs.shape[0], generator=gen, device=xs.device)
    bk = gpu.back_tof_lm(xs, xe, bins, G, T, y)
    lhs, rhs = inner64(p, y), inner64(img, bk)
    assert abs(lhs - rhs) <= ADJ_TOL * abs(lhs)
    m = 1_000_000
    b1 = gpu.back_tof_lm(xs[:m], xe[:m], bins[:m], G, T, y[:m].contiguous())
    bref = oracle.back_tof_lm(xs[:m].cpu().numpy(), xe[:m].cpu().numpy(), g["origin"], g["voxsize"], g["dim"], tof,
                              bins[:m].cpu().numpy(), y[:m].cpu().numpy())
    assert rel_l2(np64(b1), bref) <= BACK_TOL


def test_work_counter_matches_oracle(gpu, small):
    """The sample counter used for throughput accounting equals the oracle's count exactly."""
    xs, xe, img, _ = small
    g = geom_of(C.GRID_SMALL)
    G = gpu.ImageGeom(g["dim"], g["voxsize"], g["origin"])
    dev = torch.device("cuda")
    cnt = gpu.count_samples(xs.to(dev), xe.to(dev), G)
    tot, per = oracle.count_samples(xs.numpy(), xe.numpy(), g["origin"], g["voxsize"], g["dim"], per_ray=True)
    assert np.array_equal(cnt.cpu().numpy().astype(np.int64), per)
    t = C.TOF_CLIN
    exs, exe, bins = generate_tof_lm_events(C.SCANNER_SMALL, C.SINO_SMALL.n_rad, C.SINO_SMALL.max_rd, C.GRID_SMALL,
                                            img, 50_000, seed=33, tof_bin_width=t.bin_width, tof_sigma=t.sigma,
                                            n_tof_bins=t.n_bins)
    tof = tof_of(t)
    T = gpu.TofParams(tof["bin_width"], tof["sigma"], tof["n_sigmas"], tof["n_bins"])
    c2 = gpu.count_samples(exs.to(dev), exe.to(dev), G, bins.to(dev), T)
    tot2, per2 = oracle.count_samples(exs.numpy(), exe.numpy(), g["origin"], g["voxsize"], g["dim"], tof=tof,
                                      bins=bins.numpy(), per_ray=True)
    assert np.array_equal(c2.cpu().numpy().astype(np.int64), per2)


def test_presort_order(gpu, lm40):
    """pp_lm_presort returns a permutation; projecting in that order gives bit-identical forward
    projections (each ray's sum does not depend on the order) and the same back projection up to
    float summation order, on the full 40M-event workload."""
    xs, xe, bins, img = lm40
    g = geom_of(C.GRID_CLIN)
    G = gpu.ImageGeom(g["dim"], g["voxsize"], g["origin"])
    tof = tof_of(C.TOF_CLIN)
    T = gpu.TofParams(tof["bin_width"], tof["sigma"], tof["n_sigmas"], tof["n_bins"])
    order = gpu.presort(xs, xe, G, bins, T)
    srt, _ = torch.sort(order.long())
    assert torch.equal(srt, torch.arange(xs.shape[0], device=xs.device))
    p0 = gpu.fwd_tof_lm(xs, xe, bins, G, T, img)
    p1 = gpu.fwd_tof_lm(xs, xe, bins, G, T, img, order=order)
    assert torch.equal(p0, p1)
    b0 = gpu.back_tof_lm(xs, xe, bins, G, T, p0)
    b1 = gpu.back_tof_lm(xs, xe, bins, G, T, p0, order=order)
    assert rel_l2(np64(b1), np64(b0)) <= 1e-5
    # non-TOF projections of the same events, in presorted order
    o2 = gpu.presort(xs, xe, G)
    assert torch.equal(gpu.fwd(xs, xe, G, img, order=o2), gpu.fwd(xs, xe, G, img))
    m = 200_000
    y = torch.rand(m, device=xs.device)
    bm = gpu.back(xs[:m].contiguous(), xe[:m].contiguous(), G, y, order=gpu.presort(xs[:m].contiguous(),
                                                                                 xe[:m].contiguous(), G))
    ref = oracle.back(xs[:m].cpu().numpy(), xe[:m].cpu().numpy(), g["origin"], g["voxsize"], g["dim"],
                      y.cpu().numpy())
    assert rel_l2(np64(bm), ref) <= BACK_TOL


SHEET_GRIDS = [
    ((300, 40, 16), (1.0, 2.0, 2.0)),  # lines along axis 0 longer than 256 planes: direct path
    ((30, 20, 200), (2.0, 2.0, 0.5)),  # axis 2 longer than the LDS column: direct path only
    ((64, 48, 7), (1.5, 2.0, 2.0)),    # ordinary sheets, short lines
    ((256, 40, 128), (1.0, 2.0, 1.0)),  # the sheet at its limits: 256-plane lines, 128 z rows (151 KB of LDS)
]


@pytest.mark.parametrize("gi", range(len(SHEET_GRIDS)))
def test_run_sheet_paths_on_grid_shapes(gpu, gi):
    """Ray lists made of long runs on few transaxial lines (the sheet path's input) on grids that
    switch the sheet path off for some or all lines, or stretch its column stride to the clamp:
    back projections of every variant against the oracle, in list order and presorted."""
    dim, vs = SHEET_GRIDS[gi]
    G = gpu.ImageGeom(dim, vs)
    origin = G.origin
    rng = np.random.default_rng(320 + gi)
    ext = np.array(dim) * np.array(vs)
    R = 0.75 * float(np.hypot(ext[0], ext[1])) + 5.0
    xs_l, xe_l = [], []
    for _ in range(40):  # 40 lines x 96 rays with random axial endpoints
        phi = rng.uniform(0, np.pi)
        off = rng.uniform(-0.3, 0.3) * min(ext[0], ext[1])
        c, s_ = np.cos(phi), np.sin(phi)
        p0 = np.array([-R * c - off * s_, -R * s_ + off * c])
        p1 = np.array([R * c - off * s_, R * s_ + off * c])
        z = rng.uniform(-0.5 * ext[2], 0.5 * ext[2], size=(96, 2))
        xs_l.append(np.column_stack([np.full(96, p0[0]), np.full(96, p0[1]), z[:, 0]]))
        xe_l.append(np.column_stack([np.full(96, p1[0]), np.full(96, p1[1]), z[:, 1]]))
    xs = np.concatenate(xs_l).astype(np.float32)
    xe = np.concatenate(xe_l).astype(np.float32)
    n = xs.shape[0]
    tof = tofd(6.0, 5.0, 3.0, 11)
    T = gpu.TofParams(tof["bin_width"], tof["sigma"], tof["n_sigmas"], tof["n_bins"])
    bins = rng.integers(0, 11, size=n).astype(np.int16)
    y = rng.uniform(0, 1, size=n).astype(np.float32)
    yt = rng.uniform(0, 1, size=(n, 11)).astype(np.float32)
    d = torch.device("cuda")
    xs_d, xe_d, b_d = torch.from_numpy(xs).to(d), torch.from_numpy(xe).to(d), torch.from_numpy(bins).to(d)
    y_d, yt_d = torch.from_numpy(y).to(d), torch.from_numpy(yt).to(d)
    ref = {
        "back": oracle.back(xs, xe, origin, vs, dim, y),
        "back_lm": oracle.back_tof_lm(xs, xe, origin, vs, dim, tof, bins, y),
        "back_sino": oracle.back_tof_sino(xs, xe, origin, vs, dim, tof, yt),
    }
    order = gpu.presort(xs_d, xe_d, G, b_d, T)
    got = {
        "back": gpu.back(xs_d, xe_d, G, y_d),
        "back_lm": gpu.back_tof_lm(xs_d, xe_d, b_d, G, T, y_d),
        "back_sino": gpu.back_tof_sino(xs_d, xe_d, G, T, yt_d),
        "back_lm_sorted": gpu.back_tof_lm(xs_d, xe_d, b_d, G, T, y_d, order=order),
    }
    torch.cuda.synchronize()
    for k, v in got.items():
        assert rel_l2(np64(v), ref[k.replace("_sorted", "")]) <= BACK_TOL, k
    p = gpu.fwd_tof_lm(xs_d, xe_d, b_d, G, T, torch.ones(dim, device=d), order=order)
    p_ref = oracle.fwd_tof_lm(xs, xe, origin, vs, dim, tof, bins, np.ones(dim))
    assert rel_l2(np64(p), p_ref) <= FWD_TOL


def _cus():
    return torch.cuda.get_device_properties(0).multi_processor_count


def _timed_back_vs_oracle(gpu, xs, xe, bins, seed):
    """The benchmark's back-projection call -- pp_lm_presort, then pp_back_tof_lm in that order --
    on the given events, element by element against the oracle."""
    g = geom_of(C.GRID_CLIN)
    G = gpu.ImageGeom(g["dim"], g["voxsize"], g["origin"])
    tof = tof_of(C.TOF_CLIN)
    T = gpu.TofParams(tof["bin_width"], tof["sigma"], tof["n_sigmas"], tof["n_bins"])
    n = xs.shape[0]
    y = np.random.default_rng(seed).uniform(0.2, 1.0, size=n).astype(np.float32)
    order = gpu.presort(xs, xe, G, bins, T)
    img = torch.zeros(G.dim, dtype=torch.float32, device=xs.device)
    gpu.pp_back_tof_lm(xs, xe, bins, G, T, img, torch.from_numpy(y).to(xs.device), order)
    ref = oracle.back_tof_lm(xs.cpu().numpy(), xe.cpu().numpy(), g["origin"], g["voxsize"], g["dim"], tof,
                             bins.cpu().numpy(), y)
    assert rel_l2(np64(img), ref) <= BACK_TOL
    return ref


def test_timed_back_call_prefix(gpu, lm40):
    """The first 2^21 events of the 40M workload, presorted and back projected as the benchmark
    does: at this size the launch gives each workgroup 8 groups of 256 rays, so sheets persist
    across groups."""
    xs, xe, bins, _ = lm40
    m = 1 << 21
    assert m > 7 * 1024 * _cus()  # 8 groups per workgroup
    ref = _timed_back_vs_oracle(gpu, xs[:m].contiguous(), xe[:m].contiguous(), bins[:m].contiguous(), 47)
    assert ref.max() > 0


def test_timed_back_call_dense_lines(gpu, lm40):
    """The events of the 40M workload whose transaxial direction lies in [0, pi/18): presorted,
    their lines are as densely populated as in the full 40M list (runs of the length the timed
    40M call sees), so the sheet loop and flush work as in the benchmark; element by element
    against the oracle."""
    xs, xe, bins, _ = lm40
    d = xe[:, :2] - xs[:, :2]
    phi = torch.remainder(torch.atan2(d[:, 1], d[:, 0]), np.pi)
    sel = torch.nonzero(phi < np.pi / 18).squeeze(1)
    assert sel.numel() > 7 * 1024 * _cus()
    _timed_back_vs_oracle(gpu, xs[sel].contiguous(), xe[sel].contiguous(), bins[sel].contiguous(), 48)


def test_sheet_flush_writes_below_grid(gpu):
    """Runs of rays on one transaxial line whose axial coordinate leaves the grid through z = 0
    just after plane 63: in the wave of planes 64-127 the only sample is the conservative end
    plane, whose z pair lies entirely below the grid (its value goes to the sheet's spare row).
    The flush must not carry that row into the image.  Non-TOF and TOF listmode, against the
    oracle."""
    dim, vs = (100, 8, 8), (1.0, 1.0, 1.0)
    G = gpu.ImageGeom(dim, vs)
    o = G.origin
    xs_l, xe_l = [], []
    for line, y0 in enumerate((-1.7, 0.3, 2.2)):
        for r in range(6):
            # axial index 3.0 at plane 0 falling to -1 at plane 63.5 (+ a small shift per ray)
            w0 = 3.0 + 0.004 * r
            slope = -4.0 / 63.5
            x_a, x_b = o[0] - 10.5, o[0] + 110.5
            z_a = o[2] + (w0 + slope * (x_a - o[0])) * vs[2]
            z_b = o[2] + (w0 + slope * (x_b - o[0])) * vs[2]
            xs_l.append((x_a, y0, z_a))
            xe_l.append((x_b, y0, z_b))
    xs = np.array(xs_l, dtype=np.float32)
    xe = np.array(xe_l, dtype=np.float32)
    n = xs.shape[0]
    rng = np.random.default_rng(49)
    y = rng.uniform(0.5, 1.5, size=n).astype(np.float32)
    tof = tofd(30.0, 20.0, 3.0, 5)
    bins = np.full(n, 2, dtype=np.int16)
    dv = torch.device("cuda")
    xs_d, xe_d = torch.from_numpy(xs).to(dv), torch.from_numpy(xe).to(dv)
    T = gpu.TofParams(tof["bin_width"], tof["sigma"], tof["n_sigmas"], tof["n_bins"])
    b = gpu.back(xs_d, xe_d, G, torch.from_numpy(y).to(dv))
    bl = gpu.back_tof_lm(xs_d, xe_d, torch.from_numpy(bins).to(dv), G, T, torch.from_numpy(y).to(dv))
    torch.cuda.synchronize()
    ref = oracle.back(xs, xe, o, vs, dim, y)
    ref_l = oracle.back_tof_lm(xs, xe, o, vs, dim, tof, bins, y)
    assert ref.sum() > 0 and ref_l.sum() > 0
    assert rel_l2(np64(b), ref) <= BACK_TOL
    assert rel_l2(np64(bl), ref_l) <= BACK_TOL
    # plane 64 (the end plane, stencil entirely below the grid) and beyond receive nothing
    assert float(b[64:].abs().sum()) == 0.0 and float(bl[64:].abs().sum()) == 0.0
    assert float(b[63].abs().sum()) > 0.0


def test_tof_gaussian_table_matches_oracle(gpu):
    """pp_tof_gaussian_table: the library's table of the Gaussian bin weight equals the oracle's
    TOF kernel at the table's nodes (float32 rounding), for the clinical kernel and a narrow one."""
    for spec in (C.TOF_CLIN, C.TofSpec(4.0, 1.3, 2.5, 9)):
        tof = tof_of(spec)
        T = gpu.TofParams(tof["bin_width"], tof["sigma"], tof["n_sigmas"], tof["n_bins"])
        TL = gpu.gaussian_tof_table(T, 0.05)
        n = TL.lut.numel()
        x = TL.lut_x0 + TL.lut_dx * np.arange(n, dtype=np.float64)
        ref = oracle.tof_kernel(x, tof)
        got = TL.lut.cpu().numpy().astype(np.float64)
        assert np.max(np.abs(got - ref)) <= 2.0 ** -24 * max(ref.max(), 1e-30) + 1e-12
        assert TL.lut_x0 + (n - 1) * TL.lut_dx == pytest.approx(-TL.lut_x0, rel=1e-6) and TL.lut_dx <= 0.05
