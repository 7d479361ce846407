"""Autograd wrappers: the Poisson data-fidelity gradient through the TOF listmode projector
(batch of 8 images 128 x 128 x 64, 40M events, background 0.1) against the analytic
A^T (1 - y / (A x + s)), against central finite differences on 64 voxels, and against the
FP64 oracle on a reduced event set; adjoint pairing and double backward."""
import numpy as np
import pytest
import torch

import oracle
from helpers import geom_of, rel_l2, tof_of
from synth import configs as C
from synth import generate_tof_lm_events
from synth.phantom import ellipsoid_lesion_phantom

pytestmark = pytest.mark.gpu


def np64(t):
    return t.detach().cpu().numpy().astype(np.float64)


@pytest.fixture(scope="module")
def dl(gpu):
    from paper_2212_12519_amd.autograd import JosephOperator

    dev = torch.device("cuda")
    t = C.TOF_CLIN
    src = C.phantom_clin(device=dev)
    xs, xe, bins = generate_tof_lm_events(C.SCANNER_CLIN, C.SINO_CLIN.n_rad, C.SINO_CLIN.max_rd, C.GRID_CLIN, src,
                                          C.N_EVENTS_LM, seed=C.SEED_EVENTS, tof_bin_width=t.bin_width,
                                          tof_sigma=t.sigma, n_tof_bins=t.n_bins, device=dev)
    grid = C.GRID_DL
    G = gpu.ImageGeom(grid.dim, grid.voxsize, grid.origin)
    T = gpu.TofParams(t.bin_width, t.sigma, t.n_sigmas, t.n_bins)
    imgs = torch.stack([ellipsoid_lesion_phantom(grid, seed=s, device=dev) for s in C.SEEDS_DL_IMAGES])
    op = JosephOperator(xs, xe, G, kind="tof_lm", tof=T, tof_bin=bins, presort=True)
    return op, imgs, (xs, xe, bins), G, T


def test_poisson_gradient_analytic_and_fd(gpu, dl):
    from paper_2212_12519_amd.autograd import poisson_nll

    op, imgs, _, G, T = dl
    s = C.BG_DL
    x = imgs.clone().requires_grad_(True)
    ybar = op(x) + s
    y = torch.ones_like(ybar)
    loss = poisson_nll(ybar, y)
    loss.backward()
    g = x.grad
    assert g.shape == imgs.shape
    with torch.no_grad():
        yb = ybar.detach()
        analytic = op.adjoint_raw((1.0 - y / yb).float())
    assert rel_l2(np64(g), np64(analytic)) <= 1e-5
    # central finite differences (float64 per event) on 64 voxels with positive sensitivity
    sens = op.adjoint_raw(torch.ones((1, op.n), device=imgs.device))[0]
    cand = torch.nonzero(sens.reshape(-1) > 0).squeeze(1)
    rng = np.random.default_rng(C.SEED_FD_VOXELS)
    pick = cand[torch.from_numpy(rng.choice(cand.numel(), size=64, replace=False)).to(cand.device)]
    fd, gv, scale = [], [], []
    for k, v in enumerate(pick.tolist()):
        b = k % imgs.shape[0]
        unit = torch.zeros(G.dim, device=imgs.device)
        unit.view(-1)[v] = 1.0
        a = op.apply_raw(unit).double()
        xv = float(imgs[b].reshape(-1)[v])
        h = 1e-3 * (abs(xv) + 1.0)
        yb = ybar[b].detach().double()
        terms = 2 * h * a - (torch.log(yb + h * a) - torch.log(yb - h * a))
        fd.append(float(terms.sum()) / (2 * h))
        scale.append(float((a * (1.0 - 1.0 / yb)).abs().sum()))
        gv.append(float(g[b].reshape(-1)[v]))
    fd, gv, scale = np.array(fd), np.array(gv), np.array(scale)
    # each gradient entry is one float32 atomic accumulation of ~1e4 signed terms (error ~ sqrt(N) u
    # of the absolute sum, u = 6e-8), so it is held to the back-projection tolerance, 1e-4, of that sum
    assert np.all(np.abs(fd - gv) <= 1e-4 * scale + 1e-6), np.max(np.abs(fd - gv) / (scale + 1e-12))


def test_gradient_matches_oracle(gpu, dl):
    """Reduced event set (200k events, one image): autograd gradient vs the FP64 oracle's
    A^T (1 - y / (A x + s))."""
    from paper_2212_12519_amd.autograd import JosephOperator, poisson_nll

    _, imgs, (xs, xe, bins), G, T = dl
    m = 200_000
    op = JosephOperator(xs[:m], xe[:m], G, kind="tof_lm", tof=T, tof_bin=bins[:m])
    x = imgs[0].clone().requires_grad_(True)
    loss = poisson_nll(op(x) + C.BG_DL, torch.ones(m, device=x.device))
    loss.backward()
    g = geom_of(C.GRID_DL)
    tof = tof_of(C.TOF_CLIN)
    a, b_, c = xs[:m].cpu().numpy(), xe[:m].cpu().numpy(), bins[:m].cpu().numpy()
    ybar = oracle.fwd_tof_lm(a, b_, g["origin"], g["voxsize"], g["dim"], tof, c, np64(imgs[0])) + C.BG_DL
    ref = oracle.back_tof_lm(a, b_, g["origin"], g["voxsize"], g["dim"], tof, c, 1.0 - 1.0 / ybar)
    assert rel_l2(np64(x.grad), ref) <= 1e-4


def test_adjoint_pair_and_double_backward(gpu, dl):
    """d<Ax, y>/dx = A^T y, d<x, A^T y>/dy = A x, and the Hessian-vector product of
    f(x) = |A x|^2 / 2 (double backward) equals A^T A v."""
    from paper_2212_12519_amd.autograd import JosephOperator

    _, imgs, (xs, xe, bins), G, T = dl
    m = 300_000
    op = JosephOperator(xs[:m], xe[:m], G, kind="tof_lm", tof=T, tof_bin=bins[:m], presort=True)
    x = imgs[1].clone().requires_grad_(True)
    y = torch.rand(m, device=x.device).requires_grad_(True)
    (gx,) = torch.autograd.grad((op(x) * y.detach()).sum(), x)
    assert rel_l2(np64(gx), np64(op.adjoint_raw(y.detach()))) <= 1e-5
    (gy,) = torch.autograd.grad((x.detach() * op.T(y)).sum(), y)
    assert rel_l2(np64(gy), np64(op.apply_raw(x.detach()))) <= 1e-5
    v = imgs[2].clone()
    z = imgs[1].clone().requires_grad_(True)
    f = 0.5 * (op(z) ** 2).sum()
    (gz,) = torch.autograd.grad(f, z, create_graph=True)
    (hv,) = torch.autograd.grad((gz * v).sum(), z)
    assert rel_l2(np64(hv), np64(op.adjoint_raw(op.apply_raw(v)))) <= 1e-5


@pytest.mark.parametrize("kind", ["nontof", "tof_sino"])
def test_sinogram_least_squares_gradient(gpu, kind):
    """grad of |A x - y|^2 / 2 through the sinogram operators equals the oracle's A^T (A x - y)."""
    from paper_2212_12519_amd.autograd import JosephOperator

    xs, xe = C.SINO_SMALL.lors()
    img = C.phantom_small()
    g = geom_of(C.GRID_SMALL)
    G = gpu.ImageGeom(g["dim"], g["voxsize"], g["origin"])
    tof = tof_of(C.TOF_CLIN)
    T = gpu.TofParams(tof["bin_width"], tof["sigma"], tof["n_sigmas"], tof["n_bins"])
    dev = torch.device("cuda")
    op = JosephOperator(xs.to(dev), xe.to(dev), G, kind=kind, tof=T if kind == "tof_sino" else None)
    shape = op.proj_shape
    y = torch.from_numpy(np.random.default_rng(61).uniform(0, 1, size=shape).astype(np.float32))
    x = img.to(dev).requires_grad_(True)
    (0.5 * ((op(x) - y.to(dev)) ** 2).sum()).backward()
    if kind == "nontof":
        r = oracle.fwd(xs.numpy(), xe.numpy(), g["origin"], g["voxsize"], g["dim"], img.numpy()) - y.numpy()
        ref = oracle.back(xs.numpy(), xe.numpy(), g["origin"], g["voxsize"], g["dim"], r)
    else:
        r = oracle.fwd_tof_sino(xs.numpy(), xe.numpy(), g["origin"], g["voxsize"], g["dim"], tof,
                                img.numpy()) - y.numpy()
        ref = oracle.back_tof_sino(xs.numpy(), xe.numpy(), g["origin"], g["voxsize"], g["dim"], tof, r)
    assert rel_l2(np64(x.grad), ref) <= 1e-4


def test_poisson_loss_kernel(gpu):
    """pp_poisson_nll against the loss and gradient written out in float64 torch operations: a size that
    is no multiple of the workgroup, zero data, a background, non-positive expectations (the IEEE
    results of the formula), no elements; and the loss's Hessian-vector product through a
    differentiated backward (y / ybar^2 times v)."""
    from paper_2212_12519_amd.autograd import poisson_nll

    dev = torch.device("cuda")
    gen = torch.Generator().manual_seed(95)
    n = 1_000_003
    p = (torch.rand(n, generator=gen) * 3.0).to(dev)
    y = torch.poisson(torch.rand(n, generator=gen) * 2.0).to(dev)
    bg = 0.1
    grad = torch.empty_like(p)
    partial = torch.empty(1000, dtype=torch.float64, device=dev)
    gpu.pp_poisson_nll(p, bg, y, grad, partial)
    torch.cuda.synchronize()
    yb = (p + bg).double()
    ref = (yb - y.double() * torch.log(yb)).sum()
    assert abs(float(partial.sum()) - float(ref)) <= 1e-12 * abs(float(ref))
    assert torch.equal(grad, (1.0 - y.double() / yb).float())
    # through autograd: the loss and its gradient
    pr = p.clone().requires_grad_(True)
    loss = poisson_nll(pr, y, bg)
    loss.backward()
    assert abs(float(loss.detach()) - float(ref)) <= 1e-12 * abs(float(ref))
    assert torch.equal(pr.grad, grad)
    # Hessian-vector product of the loss: d2L/dp2 = y / ybar^2
    pr2 = p[:1000].clone().requires_grad_(True)
    v = torch.rand(1000, generator=gen).to(dev)
    (g1,) = torch.autograd.grad(poisson_nll(pr2, y[:1000], bg), pr2, create_graph=True)
    (hv,) = torch.autograd.grad((g1 * v).sum(), pr2)
    yb2 = (p[:1000] + bg).double()
    assert rel_l2(np64(hv), (y[:1000].double() / yb2 ** 2 * v.double()).cpu().numpy()) <= 1e-6
    # non-positive expectations: the formula's IEEE values
    q = torch.tensor([-0.1, 0.0, 1.0], device=dev) - bg
    yq = torch.tensor([1.0, 1.0, 0.0], device=dev)
    gq, pq = torch.empty(3, device=dev), torch.empty(1, dtype=torch.float64, device=dev)
    gpu.pp_poisson_nll(q, bg, yq, gq, pq)
    torch.cuda.synchronize()
    ybq = (q + bg).double()
    rq = 1.0 - yq.double() / ybq
    assert torch.equal(torch.isnan(gq), torch.isnan(rq.float())) and torch.equal(gq[2:], rq[2:].float())
    assert not torch.isfinite(pq[0])
    # no elements: zero partial sums
    e = torch.empty(0, device=dev)
    pz = torch.full((3,), 5.0, dtype=torch.float64, device=dev)
    gpu.pp_poisson_nll(e, bg, e, e, pz)
    torch.cuda.synchronize()
    assert not torch.any(pz)
