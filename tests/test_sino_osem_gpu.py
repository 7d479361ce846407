"""TOF sinogram OSEM in LOR chunks and shards (pp_tof_sino_sensitivity, pp_tof_sino_osem_subset)
against the FP64 oracle's TOF sinogram OSEM.

Subsets are views (view mod n_sub); the oracle takes the subset of every LOR, the GPU the LORs of
each subset stored contiguously in their original order.  Tolerances: OSEM images after 3
iterations relative L2 <= 1e-4, sensitivities (back projections) <= 1e-4.  The workspace is sized
so that every subset runs in several chunks with a ragged last one, and the shard counts do not
divide the subsets.  At the clinical size, in the chunk and shard configuration of the benchmark,
one subset update is checked by the EM count identity, which holds at any size: with bg = 0,
sum_v sens_v x_new,v = sum of the counts y over the (LOR, bin) pairs with positive expectation.
"""
import numpy as np
import pytest
import torch

import oracle
from helpers import geom_of, rel_l2, tof_of
from synth import configs as C

pytestmark = pytest.mark.gpu
OSEM_TOL = 1e-4
BACK_TOL = 1e-4


def np64(t):
    return t.detach().cpu().numpy().astype(np.float64)


def view_subsets(spec, n_sub, views=None):
    """Subset (view mod n_sub) of every LOR of spec's sinogram in RVP order (plane fastest)."""
    n_rad, n_views, n_planes = spec.shape
    vs = np.arange(n_views) if views is None else np.asarray(views)
    v = vs[(np.arange(n_rad * len(vs) * n_planes) // n_planes) % len(vs)]
    return (v % n_sub).astype(np.int32)


def split(xs, xe, y, sub, n_sub, dev):
    out = []
    for j in range(n_sub):
        idx = torch.from_numpy(np.flatnonzero(sub == j))
        out.append((xs[idx].contiguous().to(dev), xe[idx].contiguous().to(dev), y[idx].contiguous().to(dev)))
    return out


def run_case(gpu, spec, grid, xs, xe, sub, n_sub, seed, shards, work_lors, n_iter=3, bg=0.1):
    dev = torch.device("cuda")
    g, tof = geom_of(grid), tof_of(C.TOF_CLIN)
    G = gpu.ImageGeom(g["dim"], g["voxsize"], g["origin"])
    T = gpu.TofParams(tof["bin_width"], tof["sigma"], tof["n_sigmas"], tof["n_bins"])
    rng = np.random.default_rng(seed)
    y = torch.from_numpy(rng.poisson(0.4, size=(xs.shape[0], tof["n_bins"])).astype(np.float32))
    x0 = torch.ones(grid.dim, dtype=torch.float32)
    from paper_2212_12519_amd import sino_osem

    subsets = split(xs, xe, y, sub, n_sub, dev)
    x, sens = sino_osem.tof_sino_osem(subsets, G, T, x0.to(dev), n_iter, bg=bg, n_shards=shards,
                                      work_lors=work_lors)
    torch.cuda.synchronize()
    for j in range(n_sub):
        idx = np.flatnonzero(sub == j)
        s_ref = oracle.back_tof_sino(xs.numpy()[idx], xe.numpy()[idx], g["origin"], g["voxsize"], g["dim"], tof,
                                     np.ones((idx.size, tof["n_bins"])))
        assert rel_l2(np64(sens[j]), s_ref) <= BACK_TOL, j
    x_ref = oracle.tof_sino_osem(xs.numpy(), xe.numpy(), sub, n_sub, g["origin"], g["voxsize"], g["dim"], tof,
                                 y.numpy(), bg, n_iter, x0.numpy())
    err = rel_l2(np64(x), x_ref)
    print(f"TOF-sino OSEM {grid.dim}: {n_iter} it x {n_sub} subsets, {shards} shards, chunks of {work_lors}: "
          f"rel L2 {err:.2e}")
    assert err <= OSEM_TOL
    assert float(x.min()) >= 0.0


@pytest.mark.parametrize("shards", [1, 3])
def test_small_sinogram_osem_matches_oracle(gpu, shards):
    """The small scanner's 64,512 LORs with the clinical TOF kernel, 4 view subsets of 16,128 LORs
    in chunks of 5,000 (three full, one of 1,128)."""
    xs, xe = C.SINO_SMALL.lors()
    sub = view_subsets(C.SINO_SMALL, 4)
    run_case(gpu, C.SINO_SMALL, C.GRID_SMALL, xs, xe, sub, 4, seed=61, shards=shards, work_lors=5_000)


def test_clinical_view_subset_osem_matches_oracle(gpu):
    """Clinical geometry and grid, views 0 and 190 (every 8th radial bin, all 2,204 planes): two
    subsets of 110,200 LORs, 4 shards, chunks of 30,000."""
    views = [0, 190]
    xs, xe = C.SINO_CLIN.lors(views=views)
    n_rad, _, n_planes = C.SINO_CLIN.shape
    keep = ((np.arange(xs.shape[0]) // (len(views) * n_planes)) % 8) == 0
    sub = view_subsets(C.SINO_CLIN, 2, views=[0, 1])[keep]
    idx = torch.from_numpy(np.flatnonzero(keep))
    run_case(gpu, C.SINO_CLIN, C.GRID_CLIN, xs[idx].contiguous(), xe[idx].contiguous(), sub, 2, seed=62, shards=4,
             work_lors=30_000)


def test_empty_subset_and_errors(gpu):
    """An empty subset has zero sensitivity: the update sets x to 0 (the oracle's definition);
    argument errors are reported before any launch."""
    from paper_2212_12519_amd import sino_osem

    dev = torch.device("cuda")
    g, tof = geom_of(C.GRID_SMALL), tof_of(C.TOF_CLIN)
    G = gpu.ImageGeom(g["dim"], g["voxsize"], g["origin"])
    T = gpu.TofParams(tof["bin_width"], tof["sigma"], tof["n_sigmas"], tof["n_bins"])
    e3 = torch.zeros((0, 3), dtype=torch.float32, device=dev)
    ey = torch.zeros((0, tof["n_bins"]), dtype=torch.float32, device=dev)
    x, sens = sino_osem.tof_sino_osem([(e3, e3, ey)], G, T, torch.ones(g["dim"], device=dev), 1)
    assert not torch.any(x) and not torch.any(sens[0])
    work = torch.zeros((10, tof["n_bins"]), dtype=torch.float32, device=dev)
    acc = torch.zeros((2,) + tuple(g["dim"]), dtype=torch.float32, device=dev)
    with pytest.raises(gpu.PPError) as ei:  # x inside the accumulators
        sino_osem.pp_tof_sino_osem_subset(e3, e3, ey, G, T, 0.1, acc[1], acc, sens[0], work)
    assert ei.value.code == 1


@pytest.mark.parametrize("subset", [3])
def test_clinical_subset_count_identity(gpu, subset):
    """Full clinical size, one view subset (1/8 of the 335,008,000 LORs) in the benchmark's chunks
    (2^22 LORs) and shards (4): with bg = 0, sum_v sens_v x_new,v equals the sum of y over the
    (LOR, bin) pairs with a positive expectation A x (checked through a separate forward
    projection of x, chunk by chunk)."""
    from paper_2212_12519_amd import sino_osem

    dev = torch.device("cuda")
    g, tof = geom_of(C.GRID_CLIN), tof_of(C.TOF_CLIN)
    G = gpu.ImageGeom(g["dim"], g["voxsize"], g["origin"])
    T = gpu.TofParams(tof["bin_width"], tof["sigma"], tof["n_sigmas"], tof["n_bins"])
    views = list(range(subset, C.SINO_CLIN.shape[1], 8))
    xs, xe = C.SINO_CLIN.lors(views=views, device=dev, radial_chunk=50)
    gen = torch.Generator(device=dev)
    gen.manual_seed(63)
    y = torch.poisson(torch.full((xs.shape[0], tof["n_bins"]), 0.02, device=dev), generator=gen)
    x = C.phantom_clin(device=dev).contiguous() + 0.5
    work = torch.empty((1 << 22, tof["n_bins"]), dtype=torch.float32, device=dev)
    sens = torch.zeros(g["dim"], dtype=torch.float32, device=dev)
    sino_osem.pp_tof_sino_sensitivity(xs, xe, G, T, sens, work)
    # the counts that take part: y where the expectation of x is positive
    want = 0.0
    for a in range(0, xs.shape[0], work.shape[0]):
        b = min(xs.shape[0], a + work.shape[0])
        q = gpu.fwd_tof_sino(xs[a:b], xe[a:b], G, T, x)
        want += float(torch.where(q > 0, y[a:b], torch.zeros_like(q)).double().sum())
    acc = torch.zeros((4,) + tuple(g["dim"]), dtype=torch.float32, device=dev)
    sino_osem.pp_tof_sino_osem_subset(xs, xe, y, G, T, 0.0, x, acc, sens, work)
    got = float((sens.double() * x.double()).sum())
    print(f"count identity: {got:.6e} vs {want:.6e} ({xs.shape[0]} LORs)")
    assert abs(got - want) <= 1e-4 * want
    assert not torch.any(acc)
