"""pp_fwd_tof_lm_gather: the listmode TOF forward projection that also writes the events and their
projections in processing order.  Its projections must be exactly pp_fwd_tof_lm's (same arithmetic,
same order), its event copies exactly pp_gather_events', its value copy p[order]; the back projection of
the copies without an order array must equal the back projection of the events with the order (the same
rays in the same order, up to the order of float atomic adds); one projection is checked against the
FP64 oracle.  Also: order entries outside [0, n) (event i, value 0 at position i) and the refusal of
per-event TOF arrays.  Through the C ABI."""
import pytest
import torch

import oracle
from helpers import geom_of, rel_l2, tof_of
from synth import configs as C
from synth import generate_tof_lm_events, tof_per_ray_params

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def case(gpu):
    img = C.phantom_small()
    t = C.TOF_CLIN
    xs, xe, bins = generate_tof_lm_events(C.SCANNER_SMALL, C.SINO_SMALL.n_rad, C.SINO_SMALL.max_rd, C.GRID_SMALL,
                                          img, 200_003, seed=91, tof_bin_width=t.bin_width, tof_sigma=t.sigma,
                                          n_tof_bins=t.n_bins)
    d = torch.device("cuda")
    g = geom_of(C.GRID_SMALL)
    G = gpu.ImageGeom(g["dim"], g["voxsize"], g["origin"])
    return xs.to(d), xe.to(d), bins.to(d), img.to(d), G


def _tofs(gpu, xs):
    t = tof_of(C.TOF_CLIN)
    T = gpu.TofParams(t["bin_width"], t["sigma"], t["n_sigmas"], t["n_bins"])
    return {"poly": T, "table": gpu.gaussian_tof_table(T, 0.05, device=xs.device)}


@pytest.mark.parametrize("form", ["poly", "table"])
def test_outputs_equal_the_separate_calls(gpu, case, form):
    xs, xe, bins, img, G = case
    T = _tofs(gpu, xs)[form]
    order = gpu.presort(xs, xe, G, bins, T)
    p, xs2, xe2, b2, p2 = gpu.fwd_tof_lm_gather(xs, xe, bins, G, T, img, order)
    ref = gpu.fwd_tof_lm(xs, xe, bins, G, T, img, order)
    gx, ge, gb = gpu.gather_events(xs, xe, bins, order)
    torch.cuda.synchronize()
    assert torch.equal(p, ref)
    assert torch.equal(xs2, gx) and torch.equal(xe2, ge) and torch.equal(b2, gb)
    assert torch.equal(p2, p[order.long()])
    # the copies walked without an order array: the same rays in the same order
    y = torch.rand(xs.shape[0], generator=torch.Generator().manual_seed(92)).to(xs.device)
    b_ord = gpu.back_tof_lm(xs, xe, bins, G, T, y, order=order)
    b_cpy = gpu.back_tof_lm(xs2, xe2, b2, G, T, y[order.long()].contiguous())
    torch.cuda.synchronize()
    assert rel_l2(b_cpy.double().cpu().numpy(), b_ord.double().cpu().numpy()) <= 1e-6


def test_oracle_invalid_order_entries_and_refusals(gpu, case):
    xs, xe, bins, img, G = case
    T = _tofs(gpu, xs)["poly"]
    order = gpu.presort(xs, xe, G, bins, T)
    p, *_ = gpu.fwd_tof_lm_gather(xs, xe, bins, G, T, img, order)
    g, t = geom_of(C.GRID_SMALL), tof_of(C.TOF_CLIN)
    ref = oracle.fwd_tof_lm(xs.cpu().numpy(), xe.cpu().numpy(), g["origin"], g["voxsize"], g["dim"], t,
                            bins.cpu().numpy(), img.double().cpu().numpy())
    assert rel_l2(p.double().cpu().numpy(), ref) <= 1e-5
    # order entries outside [0, n): position i gets event i and the value 0; the events they displaced
    # are not projected (their p entries keep what the caller put there)
    n = xs.shape[0]
    bad = order.clone()
    pos = torch.tensor([0, 3, 1000, n - 1], device=xs.device)
    bad[pos] = torch.tensor([-1, n, -7, n + 5], dtype=bad.dtype, device=xs.device)
    p_a = torch.full((n,), -7.0, device=xs.device)
    p_b = p_a.clone()
    xs2, xe2, p2 = torch.empty_like(xs), torch.empty_like(xe), torch.empty(n, device=xs.device)
    b2 = torch.empty_like(bins)
    gpu.pp_fwd_tof_lm_gather(xs, xe, bins, G, T, img, p_a, bad, xs2, xe2, b2, p2)
    gpu.pp_fwd_tof_lm(xs, xe, bins, G, T, img, p_b, bad)
    torch.cuda.synchronize()
    assert torch.equal(p_a, p_b)
    src = torch.where((bad >= 0) & (bad < n), bad, torch.arange(n, device=xs.device, dtype=bad.dtype)).long()
    assert torch.equal(xs2, xs[src]) and torch.equal(xe2, xe[src]) and torch.equal(b2, bins[src])
    assert torch.equal(p2[pos], torch.zeros(4, device=xs.device))
    ok = torch.ones(n, dtype=torch.bool, device=xs.device)
    ok[pos] = False
    assert torch.equal(p2[ok], p_a[src][ok])
    # per-event TOF arrays are not reordered: refused; no order: refused
    sig, _ = tof_per_ray_params(n, T.sigma, seed=93, device=xs.device)
    TP = gpu.TofParams(T.bin_width, T.sigma, T.n_sigmas, T.n_bins, sigma_per_ray=sig)
    with pytest.raises(Exception):
        gpu.fwd_tof_lm_gather(xs, xe, bins, G, TP, img, order)
    with pytest.raises(ValueError):
        gpu.fwd_tof_lm_gather(xs, xe, bins, G, T, img, None)
    # no events: nothing to do
    e3 = xs[:0].contiguous()
    out = gpu.fwd_tof_lm_gather(e3, e3, bins[:0].contiguous(), G, T, img, order[:0].contiguous())
    assert all(o.shape[0] == 0 for o in out)
