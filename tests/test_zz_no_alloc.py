"""pp_lm_presort_noalloc (library-held per-GPU workspace) against pp_lm_presort
(caller workspace): the same order, bit for bit, on two calls in a row -- the
second on fewer events than the first, so stale contents of the shared
workspace would show -- and the size limit.  Through the C ABI."""
import numpy as np
import pytest
import torch

from synth import configs as C
from synth import generate_tof_lm_events


def _events(n, seed, device):
    img = C.phantom_clin()
    t = C.TOF_CLIN
    xs, xe, bins = generate_tof_lm_events(C.SCANNER_CLIN, C.SINO_CLIN.n_rad, C.SINO_CLIN.max_rd, C.GRID_CLIN, img, n,
                                          seed=seed, tof_bin_width=t.bin_width, tof_sigma=t.sigma,
                                          n_tof_bins=t.n_bins, device=device)
    return xs.contiguous(), xe.contiguous(), bins.contiguous()


def _max_events(lib, cap=64 << 20):
    lo, hi = 1, 1 << 24
    while lo < hi:  # largest n whose workspace fits the library's buffer
        mid = (lo + hi + 1) // 2
        if lib.pp_lm_presort_workspace_bytes(mid) <= cap:
            lo = mid
        else:
            hi = mid - 1
    return lo


@pytest.mark.gpu
def test_noalloc_presort_matches_workspace_presort(gpu):
    pp = gpu
    lib = pp.load()
    dev = torch.device("cuda:0")
    G = pp.ImageGeom(C.GRID_CLIN.dim, C.GRID_CLIN.voxsize, C.GRID_CLIN.origin)
    t = C.TOF_CLIN
    T = pp.TofParams(t.bin_width, t.sigma, t.n_sigmas, t.n_bins)
    n_max = _max_events(lib)
    assert 1_000_000 < n_max < 4_000_000, n_max
    xs, xe, bins = _events(n_max, seed=71, device=dev)
    print(f"noalloc presort: up to {n_max} events", flush=True)
    # two calls in a row on one GPU, the second on fewer events (and another subset count)
    for n, n_sub, with_tof in ((n_max, 1, True), (300_001, 8, True), (123_457, 3, False)):
        a, b, k = xs[:n].contiguous(), xe[:n].contiguous(), bins[:n].contiguous()
        tb, tt = (k, T) if with_tof else (None, None)
        want = pp.presort(a, b, G, tof_bin=tb, tof=tt, n_sub=n_sub)
        got = torch.full((n,), -7, dtype=torch.int32, device=dev)
        pp.pp_lm_presort_noalloc(a, b, tb, G, tt, got, n_sub=n_sub)
        torch.cuda.synchronize()
        g, w = got.cpu().numpy(), want.cpu().numpy()
        assert np.array_equal(np.sort(g), np.arange(n, dtype=np.int32)), "not a permutation"
        assert np.array_equal(g, w), f"n={n}: orders differ at {np.flatnonzero(g != w)[:5]}"
    # n beyond the buffer: rejected on the host, nothing launched
    big = n_max + 1
    order = torch.empty(big, dtype=torch.int32, device=dev)
    xs2 = torch.zeros((big, 3), dtype=torch.float32, device=dev)
    with pytest.raises(pp.PPError) as ei:
        pp.pp_lm_presort_noalloc(xs2, xs2, None, G, None, order)
    assert ei.value.code == 4  # PP_EINVAL_N
