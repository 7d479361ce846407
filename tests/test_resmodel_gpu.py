"""Image-based resolution model (Gaussian blur, 4.5 mm FWHM in the paper's OSEM) on the GPU
against the FP64 oracle: the blur alone on small, ragged and full clinical grids, and listmode
OSEM with the model (single frame, batched with and without the model, graph replay, the
sequential plain-call baseline).

Tolerances: the blur is a sum of at most 3 x 63 float32 products per voxel, relative L2 error
<= 1e-6 (max abs <= 1e-6 of the image maximum); OSEM images after 3 iterations x 8 subsets:
relative L2 <= 1e-4 (as without the model)."""
import numpy as np
import pytest
import torch

import oracle
from helpers import geom_of, rel_l2, tof_of
from synth import configs as C
from synth import generate_tof_lm_events

pytestmark = pytest.mark.gpu
BLUR_TOL = 1e-6
OSEM_TOL = 1e-4
FWHM = 4.5


def np64(t):
    return t.detach().cpu().numpy().astype(np.float64)


def _blur_case(gpu, dim, vs, fwhm, img):
    G = gpu.ImageGeom(dim, vs)
    dev = torch.device("cuda")
    x = torch.as_tensor(img, dtype=torch.float32).to(dev).contiguous()
    y = gpu.gauss3d(x, G, fwhm)
    torch.cuda.synchronize()
    ref = oracle.gauss3d(img.astype(np.float32).astype(np.float64), vs, fwhm)
    return np64(y), ref


@pytest.mark.parametrize("dim,vs,fwhm", [
    ((64, 64, 8), (4.0, 4.0, 2.0), FWHM),            # small grid
    ((37, 29, 53), (1.65, 2.2, 2.0), FWHM),          # ragged dims, anisotropic voxels
    ((33, 41, 17), (1.0, 1.0, 1.0), (6.0, 0.0, 3.0)),  # per-axis FWHM, no blur along axis 1
    ((128, 128, 64), (2.78, 2.78, 2.78), FWHM),      # the deep-learning grid
    ((5, 1, 300), (0.5, 1.0, 0.25), FWHM),           # radius > extent along axis 0; r = 31 (the limit) on axis 2
])
def test_gauss3d_matches_oracle(gpu, dim, vs, fwhm):
    rng = np.random.default_rng(61)
    img = rng.uniform(0.0, 1.0, size=dim)
    got, ref = _blur_case(gpu, dim, vs, fwhm, img)
    assert rel_l2(got, ref) <= BLUR_TOL
    assert np.max(np.abs(got - ref)) <= BLUR_TOL * np.max(np.abs(ref))


def test_gauss3d_clinical_phantom_and_identity(gpu):
    """Full clinical grid (215 x 215 x 71 @ 1.65 x 1.65 x 2 mm) with the lesion phantom; FWHM 0 is
    a bit-exact copy; a point source sums to 1."""
    g = C.GRID_CLIN
    img = C.phantom_clin().numpy().astype(np.float64)
    got, ref = _blur_case(gpu, g.dim, g.voxsize, FWHM, img)
    assert rel_l2(got, ref) <= BLUR_TOL
    assert np.max(np.abs(got - ref)) <= BLUR_TOL * np.max(np.abs(ref))
    same, _ = _blur_case(gpu, g.dim, g.voxsize, 0.0, img)
    np.testing.assert_array_equal(same, img.astype(np.float32))
    delta = np.zeros(g.dim)
    delta[107, 107, 35] = 1.0
    d, dref = _blur_case(gpu, g.dim, g.voxsize, FWHM, delta)
    assert abs(d.sum() - 1.0) < 1e-6 and np.max(np.abs(d - dref)) <= 1e-7


@pytest.fixture(scope="module")
def small_osem(gpu):
    img = C.phantom_small()
    t = C.TOF_CLIN
    xs, xe, bins = generate_tof_lm_events(C.SCANNER_SMALL, C.SINO_SMALL.n_rad, C.SINO_SMALL.max_rd, C.GRID_SMALL,
                                          img, 100_003, seed=53, tof_bin_width=t.bin_width, tof_sigma=t.sigma,
                                          n_tof_bins=t.n_bins)
    lxs, lxe = C.SINO_SMALL.lors()
    return xs, xe, bins, lxs, lxe


def test_osem_resolution_model_matches_oracle(gpu, small_osem):
    from paper_2212_12519_amd import osem

    xs, xe, bins, lxs, lxe = small_osem
    g = geom_of(C.GRID_SMALL)
    tof = tof_of(C.TOF_CLIN)
    G = gpu.ImageGeom(g["dim"], g["voxsize"], g["origin"])
    T = gpu.TofParams(tof["bin_width"], tof["sigma"], tof["n_sigmas"], tof["n_bins"])
    dev = torch.device("cuda")
    sens = osem.sensitivity(lxs.to(dev), lxe.to(dev), G, res_fwhm=FWHM)
    x = osem.lm_osem(xs.to(dev), xe.to(dev), bins.to(dev), G, T, sens, n_iter=3, n_sub=8, bg=0.1, res_fwhm=FWHM)
    back1 = oracle.back(lxs.numpy(), lxe.numpy(), g["origin"], g["voxsize"], g["dim"], np.ones(lxs.shape[0]))
    sens_ref = oracle.gauss3d(back1, g["voxsize"], FWHM)
    assert rel_l2(np64(sens), sens_ref) <= 1e-5
    x0 = (sens_ref > 0).astype(np.float64)
    x_ref = oracle.lm_osem(xs.numpy(), xe.numpy(), bins.numpy(), g["origin"], g["voxsize"], g["dim"], tof, sens_ref,
                           0.1, 3, 8, x0, fwhm=FWHM)
    assert rel_l2(np64(x), x_ref) <= OSEM_TOL
    # the model changes the result well beyond the tolerance (the test can tell them apart)
    x_plain = oracle.lm_osem(xs.numpy(), xe.numpy(), bins.numpy(), g["origin"], g["voxsize"], g["dim"], tof,
                             sens_ref, 0.1, 3, 8, x0)
    assert rel_l2(x_plain, x_ref) > 100 * OSEM_TOL
    assert float(x.min()) >= 0.0


@pytest.fixture(scope="module")
def clin_frames(gpu):
    from paper_2212_12519_amd import osem

    dev = torch.device("cuda")
    t = C.TOF_CLIN
    img = C.phantom_clin(device=dev)
    xs, xe, bins = generate_tof_lm_events(C.SCANNER_CLIN, C.SINO_CLIN.n_rad, C.SINO_CLIN.max_rd, C.GRID_CLIN, img,
                                          2_000_000, seed=54, tof_bin_width=t.bin_width, tof_sigma=t.sigma,
                                          n_tof_bins=t.n_bins, device=dev)
    grid = C.GRID_DL
    G = gpu.ImageGeom(grid.dim, grid.voxsize, grid.origin)
    T = gpu.TofParams(t.bin_width, t.sigma, t.n_sigmas, t.n_bins)
    views = torch.arange(0, 380, 4)
    lxs, lxe = C.SINO_CLIN.lors(views=views, device=dev, radial_chunk=50)
    sens_res = osem.sensitivity(lxs, lxe, G, res_fwhm=FWHM)
    sens = osem.sensitivity(lxs, lxe, G)
    cuts = [(0, 1_100_000), (1_100_000, 1_500_000), (1_500_000, 2_000_000)]
    frames = [(xs[a:b].contiguous(), xe[a:b].contiguous(), bins[a:b].contiguous()) for a, b in cuts]
    return frames, G, T, sens, sens_res


def test_mixed_batch_equals_alone(gpu, clin_frames):
    """One slot table holding frames with and without the resolution model: each frame's image
    equals its single-frame reconstruction, including a frame joining after three steps."""
    from paper_2212_12519_amd import osem

    frames, G, T, sens, sens_res = clin_frames
    use_res = [True, False, True]
    alone = [osem.lm_osem(a, b, c, G, T, sens_res if r else sens, 3, 8, bg=0.1, res_fwhm=FWHM if r else None)
             for (a, b, c), r in zip(frames, use_res)]
    prepared = [osem.prepare_frame(a, b, c, G, T, 8) for a, b, c in frames]
    imgs, keep = [], []
    table = osem.SlotTable(4, sens.device)

    def put(slot, i):
        s = sens_res if use_res[i] else sens
        x = osem.init_image(s)
        acc = torch.zeros_like(s)
        xf = tmp = None
        if use_res[i]:
            xf, tmp = osem.res_buffers(x, G, FWHM)
        table.set(slot, *prepared[i], x, acc, s, 8, 24, 0.1, xf, tmp)
        imgs.append(x)
        keep.append((acc, xf, tmp))

    put(0, 0)
    put(2, 1)
    table.upload()
    osem.osem_steps(table, G, T, 3, res_fwhm=FWHM)
    table.advance_host(3)
    put(3, 2)
    table.upload()
    osem.osem_steps(table, G, T, 24, res_fwhm=FWHM)
    torch.cuda.synchronize()
    for i in range(3):
        assert rel_l2(np64(imgs[i]), np64(alone[i])) <= OSEM_TOL, i


def test_resolution_graph_replay_matches_eager(gpu, clin_frames):
    """Graph of 8 steps with the resolution model, replayed 3 times with eager work and syncs in
    between: every replay matches the eager result."""
    from paper_2212_12519_amd import osem

    frames, G, T, _, sens = clin_frames
    prep = [osem.prepare_frame(a, b, c, G, T, 8) for a, b, c in frames[:2]]

    def setup():
        xs_img, hold = [], []
        table = osem.SlotTable(2, sens.device)
        for i in range(2):
            x = osem.init_image(sens)
            acc = torch.zeros_like(sens)
            xf, tmp = osem.res_buffers(x, G, FWHM)
            table.set(i, *prep[i], x, acc, sens, 8, 24, 0.1, xf, tmp)
            xs_img.append(x)
            hold.append((acc, xf, tmp))
        table.upload()
        return table, xs_img, hold

    t_e, x_e, h_e = setup()
    t_g, x_g, h_g = setup()
    graph = osem.capture_steps(t_g, G, T, 8, res_fwhm=FWHM)
    for rep in range(3):
        osem.osem_steps(t_e, G, T, 8, res_fwhm=FWHM)
        graph.replay()
        torch.cuda.synchronize()
        for i in range(2):
            assert rel_l2(np64(x_g[i]), np64(x_e[i])) <= OSEM_TOL, (rep, i)
            assert rel_l2(np64(h_g[i][1]), np64(h_e[i][1])) <= OSEM_TOL, (rep, i)  # x_fwd = G x kept in step
        _ = (x_e[0] * 2.0).sum().item()


def test_server_and_sequential_with_resolution_model(gpu, clin_frames):
    """The batched server and the sequential plain-call baseline (pp_gauss3d around the
    projector calls) give the same images with the model on."""
    from paper_2212_12519_amd import serve

    frames, G, T, _, sens = clin_frames
    trace = [serve.OsemRequest(i, a, b, c, G, 0.0) for i, (a, b, c) in enumerate(frames)]
    srv = serve.OsemServer(T, [(G, sens)], max_slots=2, hbm_budget=8e9, res_fwhm=FWHM)
    got = {r.rid: r.image for r in srv.run(trace)}
    ref = {r.rid: r.image for r in serve.run_sequential(trace, T, [(G, sens)], res_fwhm=FWHM)}
    for i in range(3):
        assert rel_l2(np64(got[i]), np64(ref[i])) <= OSEM_TOL, i
