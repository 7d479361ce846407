"""Fused, batched listmode OSEM on the GPU against the FP64 oracle, and the batching /
graph-replay properties the serving loop relies on.  Tolerance for OSEM images after
3 iterations x 8 subsets: relative L2 <= 1e-4."""
import numpy as np
import pytest
import torch

import oracle
from helpers import geom_of, rel_l2, tof_of
from synth import configs as C
from synth import generate_tof_lm_events

pytestmark = pytest.mark.gpu
OSEM_TOL = 1e-4


def np64(t):
    return t.detach().cpu().numpy().astype(np.float64)


@pytest.fixture(scope="module")
def small_osem(gpu):
    img = C.phantom_small()
    t = C.TOF_CLIN
    xs, xe, bins = generate_tof_lm_events(C.SCANNER_SMALL, C.SINO_SMALL.n_rad, C.SINO_SMALL.max_rd, C.GRID_SMALL,
                                          img, 100_003, seed=51, tof_bin_width=t.bin_width, tof_sigma=t.sigma,
                                          n_tof_bins=t.n_bins)
    lxs, lxe = C.SINO_SMALL.lors()
    return xs, xe, bins, lxs, lxe


def test_osem_matches_oracle(gpu, small_osem):
    from paper_2212_12519_amd import osem

    xs, xe, bins, lxs, lxe = small_osem
    g = geom_of(C.GRID_SMALL)
    tof = tof_of(C.TOF_CLIN)
    G = gpu.ImageGeom(g["dim"], g["voxsize"], g["origin"])
    T = gpu.TofParams(tof["bin_width"], tof["sigma"], tof["n_sigmas"], tof["n_bins"])
    dev = torch.device("cuda")
    sens = osem.sensitivity(lxs.to(dev), lxe.to(dev), G)
    x = osem.lm_osem(xs.to(dev), xe.to(dev), bins.to(dev), G, T, sens, n_iter=3, n_sub=8, bg=0.1)
    sens_ref = oracle.back(lxs.numpy(), lxe.numpy(), g["origin"], g["voxsize"], g["dim"], np.ones(lxs.shape[0]))
    assert rel_l2(np64(sens), sens_ref) <= 1e-5
    x_ref = oracle.lm_osem(xs.numpy(), xe.numpy(), bins.numpy(), g["origin"], g["voxsize"], g["dim"], tof, sens_ref,
                           0.1, 3, 8, (sens_ref > 0).astype(np.float64))
    assert rel_l2(np64(x), x_ref) <= OSEM_TOL
    assert float(x.min()) >= 0.0
    assert not torch.any(x[sens == 0])


@pytest.fixture(scope="module")
def clin_frames(gpu):
    """Three frames of different sizes from the clinical event model on the 128^2 x 64 grid."""
    from paper_2212_12519_amd import osem

    dev = torch.device("cuda")
    t = C.TOF_CLIN
    img = C.phantom_clin(device=dev)
    xs, xe, bins = generate_tof_lm_events(C.SCANNER_CLIN, C.SINO_CLIN.n_rad, C.SINO_CLIN.max_rd, C.GRID_CLIN, img,
                                          3_000_000, seed=52, tof_bin_width=t.bin_width, tof_sigma=t.sigma,
                                          n_tof_bins=t.n_bins, device=dev)
    grid = C.GRID_DL
    G = gpu.ImageGeom(grid.dim, grid.voxsize, grid.origin)
    T = gpu.TofParams(t.bin_width, t.sigma, t.n_sigmas, t.n_bins)
    views = torch.arange(0, 380, 4)
    lxs, lxe = C.SINO_CLIN.lors(views=views, device=dev, radial_chunk=50)
    sens = osem.sensitivity(lxs, lxe, G)
    cuts = [(0, 1_700_000), (1_700_000, 2_300_000), (2_300_000, 3_000_000)]
    frames = [(xs[a:b].contiguous(), xe[a:b].contiguous(), bins[a:b].contiguous()) for a, b in cuts]
    return frames, G, T, sens


def test_batch_equals_alone(gpu, clin_frames):
    """Each frame's image is the same alone and in a batch with others (continuous batching
    correctness), including a frame that joins the batch after the others have started."""
    from paper_2212_12519_amd import osem

    frames, G, T, sens = clin_frames
    alone = [osem.lm_osem(a, b, c, G, T, sens, 3, 8, bg=0.1) for a, b, c in frames]
    prepared = [osem.prepare_frame(a, b, c, G, T, 8) for a, b, c in frames]
    xs_img = [osem.init_image(sens) for _ in frames]
    accs = [torch.zeros_like(sens) for _ in frames]
    table = osem.SlotTable(5, sens.device)
    for i in (0, 1):
        table.set(i + 1, *prepared[i], xs_img[i], accs[i], sens, 8, 24, 0.1)
    table.upload()
    osem.osem_steps(table, G, T, 5)  # frame 2 joins after five steps of the others
    table.advance_host(5)
    table.set(4, *prepared[2], xs_img[2], accs[2], sens, 8, 24, 0.1)
    table.upload()
    osem.osem_steps(table, G, T, 24)
    torch.cuda.synchronize()
    for i in range(3):
        assert rel_l2(np64(xs_img[i]), np64(alone[i])) <= OSEM_TOL, i


def test_graph_replay_matches_eager(gpu, clin_frames):
    """A captured graph of 8 steps, replayed 3 times with eager work and synchronisation in
    between, reproduces the eager result after each replay."""
    from paper_2212_12519_amd import osem

    frames, G, T, sens = clin_frames
    prep = [osem.prepare_frame(a, b, c, G, T, 8) for a, b, c in frames[:2]]

    def setup():
        xs_img = [osem.init_image(sens) for _ in prep]
        accs = [torch.zeros_like(sens) for _ in prep]
        table = osem.SlotTable(2, sens.device)
        for i in range(2):
            table.set(i, *prep[i], xs_img[i], accs[i], sens, 8, 24, 0.1)
        table.upload()
        return table, xs_img, accs

    t_e, x_e, a_e = setup()
    t_g, x_g, a_g = setup()
    graph = osem.capture_steps(t_g, G, T, 8)
    for rep in range(3):
        osem.osem_steps(t_e, G, T, 8)
        graph.replay()
        torch.cuda.synchronize()
        for i in range(2):
            assert rel_l2(np64(x_g[i]), np64(x_e[i])) <= OSEM_TOL, (rep, i)
        _ = (x_e[0] * 2.0).sum().item()  # eager work between replays


@pytest.mark.parametrize("n_ev,n_sub", [(7, 8), (1000, 1), (257, 3)])
def test_osem_edge_sizes_match_oracle(gpu, small_osem, n_ev, n_sub):
    """Frames with fewer events than subsets (empty subsets), a single subset, and ragged
    subset sizes, in one slot table with an empty slot between live ones."""
    from paper_2212_12519_amd import osem

    xs, xe, bins, lxs, lxe = small_osem
    g = geom_of(C.GRID_SMALL)
    tof = tof_of(C.TOF_CLIN)
    G = gpu.ImageGeom(g["dim"], g["voxsize"], g["origin"])
    T = gpu.TofParams(tof["bin_width"], tof["sigma"], tof["n_sigmas"], tof["n_bins"])
    d = torch.device("cuda")
    sens = osem.sensitivity(lxs.to(d), lxe.to(d), G)
    sens_ref = oracle.back(lxs.numpy(), lxe.numpy(), g["origin"], g["voxsize"], g["dim"], np.ones(lxs.shape[0]))
    frames = [(xs[:n_ev], xe[:n_ev], bins[:n_ev]), (xs[5000:5000 + 2 * n_ev], xe[5000:5000 + 2 * n_ev],
                                                      bins[5000:5000 + 2 * n_ev])]
    table = osem.SlotTable(3, d)
    imgs, keep = [], []
    for slot, (a, b, c) in zip((0, 2), frames):
        prep = osem.prepare_frame(a.to(d).contiguous(), b.to(d).contiguous(), c.to(d).contiguous(), G, T, n_sub)
        x = osem.init_image(sens)
        acc = torch.zeros_like(sens)
        table.set(slot, *prep, x, acc, sens, n_sub, 2 * n_sub, 0.1)
        imgs.append(x)
        keep.append((prep, acc))
    table.upload()
    osem.osem_steps(table, G, T, 2 * n_sub)
    torch.cuda.synchronize()
    for x, (a, b, c) in zip(imgs, frames):
        x_ref = oracle.lm_osem(a.numpy(), b.numpy(), c.numpy(), g["origin"], g["voxsize"], g["dim"], tof, sens_ref,
                               0.1, 2, n_sub, (sens_ref > 0).astype(np.float64))
        assert rel_l2(np64(x), x_ref) <= OSEM_TOL


@pytest.fixture(scope="module")
def serving_grids_oracle(gpu):
    """Clinical-model TOF events and, per serving grid (128x128x64 @ 2.78 mm, 215x215x71 @
    1.65x1.65x2 mm), a sensitivity image computed by the oracle: the non-TOF back projection of
    ones over 5 of the scanner's 380 views (every voxel is crossed; any positive sensitivity is a
    valid OSEM input).  GPU and oracle take the same float32 sensitivity."""
    dev = torch.device("cuda")
    t = C.TOF_CLIN
    img = C.phantom_clin(device=dev)
    xs, xe, bins = generate_tof_lm_events(C.SCANNER_CLIN, C.SINO_CLIN.n_rad, C.SINO_CLIN.max_rd, C.GRID_CLIN, img,
                                          1_000_000, seed=57, tof_bin_width=t.bin_width, tof_sigma=t.sigma,
                                          n_tof_bins=t.n_bins, device=dev)
    lxs, lxe = C.SINO_CLIN.lors(views=torch.arange(0, 380, 76))
    sens = {}
    for name, grid in (("dl", C.GRID_DL), ("clin", C.GRID_CLIN)):
        s = oracle.back(lxs.numpy(), lxe.numpy(), grid.origin, grid.voxsize, grid.dim, np.ones(lxs.shape[0]))
        sens[name] = (grid, s)
    return (xs, xe, bins), sens


@pytest.mark.parametrize("res", [None, 4.5])
@pytest.mark.parametrize("grid_name,n_ev", [("dl", 1_000_000), ("clin", 500_000)])
def test_osem_serving_grids_match_oracle(gpu, serving_grids_oracle, grid_name, n_ev, res):
    """Listmode TOF OSEM, 3 iterations x 8 subsets, on the two image grids the server runs
    (1M events on 128x128x64, 0.5M on 215x215x71), with and without the 4.5 mm resolution model,
    against the oracle: relative L2 <= 1e-4."""
    from paper_2212_12519_amd import osem

    (xs, xe, bins), sens_all = serving_grids_oracle
    grid, s64 = sens_all[grid_name]
    if res is not None:
        s64 = oracle.gauss3d(s64, grid.voxsize, res)
    s32 = s64.astype(np.float32)
    tof = tof_of(C.TOF_CLIN)
    G = gpu.ImageGeom(grid.dim, grid.voxsize, grid.origin)
    T = gpu.TofParams(tof["bin_width"], tof["sigma"], tof["n_sigmas"], tof["n_bins"])
    d = torch.device("cuda")
    a, b, c = xs[:n_ev].contiguous(), xe[:n_ev].contiguous(), bins[:n_ev].contiguous()
    x = osem.lm_osem(a, b, c, G, T, torch.from_numpy(s32).to(d), 3, 8, bg=0.1, res_fwhm=res)
    s_ref = s32.astype(np.float64)
    x_ref = oracle.lm_osem(a.cpu().numpy(), b.cpu().numpy(), c.cpu().numpy(), grid.origin, grid.voxsize, grid.dim,
                           tof, s_ref, 0.1, 3, 8, (s_ref > 0).astype(np.float64), fwhm=res)
    assert rel_l2(np64(x), x_ref) <= OSEM_TOL
    assert float(x.min()) >= 0.0
