"""Host-side checks of libppmi.so (no GPU needed): it loads, exports every function that
include/ppmi.h declares, and rejects bad arguments with the documented codes before
touching the GPU."""
import ctypes
import math
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ppmi.h")


def declared_functions():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\*?\s*(pp_[a-z0-9_]+)\s*\(", txt, re.M)))


@pytest.fixture(scope="module")
def lib():
    import paper_2212_12519_amd as pp

    return pp.load()


def test_exports_every_declared_symbol(lib):
    names = declared_functions()
    assert len(names) >= 12, names
    for n in names:
        assert hasattr(lib, n), n
    assert lib.pp_abi_version() == 9
    # the entry points the boundary is specified with: the six projectors, the batched OSEM pair
    for n in ("pp_fwd", "pp_back", "pp_fwd_tof_sino", "pp_back_tof_sino", "pp_fwd_tof_lm", "pp_back_tof_lm",
              "pp_lm_osem_subset_batched", "pp_osem_update_batched", "pp_strerror", "pp_abi_version",
              "pp_tof_gaussian_table"):
        assert n in names, n


def _geom(dim=(4, 4, 4), vs=(1.0, 1.0, 1.0), origin=(0.0, 0.0, 0.0)):
    from paper_2212_12519_amd._lib import CImage

    return CImage((ctypes.c_float * 3)(*origin), (ctypes.c_float * 3)(*vs), (ctypes.c_int32 * 3)(*dim))


def _tof(bw=1.0, sig=1.0, ns=3.0, nb=5):
    from paper_2212_12519_amd._lib import CTof

    return CTof(bw, sig, ns, 0.0, nb)


DUMMY = ctypes.c_void_p(16)  # never dereferenced: validation fails before any launch
DUMMY2 = ctypes.c_void_p(1 << 20)
DUMMY3 = ctypes.c_void_p(1 << 21)


def test_error_codes(lib):
    from paper_2212_12519_amd._lib import (PP_EINVAL_GEOM, PP_EINVAL_N, PP_EINVAL_PTR, PP_EINVAL_RES, PP_EINVAL_TOF,
                                           PP_OK)

    g = _geom()
    assert lib.pp_fwd(None, None, 0, g, None, None, None, None) == PP_OK  # n == 0: no-op
    assert lib.pp_fwd(None, None, 5, g, None, None, None, None) == PP_EINVAL_PTR
    assert lib.pp_fwd(DUMMY, DUMMY, -1, g, DUMMY, DUMMY, None, None) == PP_EINVAL_N
    assert lib.pp_fwd(DUMMY, DUMMY, 5, None, DUMMY, DUMMY, None, None) == PP_EINVAL_PTR
    for bad in (_geom(dim=(0, 4, 4)), _geom(vs=(1.0, 0.0, 1.0)), _geom(vs=(1.0, -2.0, 1.0)),
                _geom(vs=(float("nan"), 1.0, 1.0)), _geom(origin=(float("inf"), 0.0, 0.0)),
                _geom(dim=(2048, 2048, 512)), _geom(dim=(1024, 1024, 1024))):
        assert lib.pp_fwd(DUMMY, DUMMY, 5, bad, DUMMY, DUMMY, None, None) == PP_EINVAL_GEOM
        assert lib.pp_back(DUMMY, DUMMY, 5, bad, DUMMY, DUMMY, None, None) == PP_EINVAL_GEOM
    from paper_2212_12519_amd._lib import CTof

    def lut(n=16, x0=-4.0, dx=0.5):
        return CTof(1.0, 0.0, 0.0, 0.0, 5, 16, n, x0, dx)  # sigma / n_sigmas unused with a table

    for bad in (_tof(nb=0), _tof(nb=257), _tof(bw=0.0), _tof(sig=-1.0), _tof(ns=0.0), _tof(sig=float("nan")),
                lut(n=1), lut(n=(1 << 24) + 1), lut(dx=0.0), lut(dx=-1.0), lut(x0=float("inf")),
                lut(dx=float("nan")), lut(x0=3e38, dx=3e38)):
        assert lib.pp_fwd_tof_sino(DUMMY, DUMMY, 5, g, bad, DUMMY, DUMMY, None) == PP_EINVAL_TOF
        assert lib.pp_back_tof_lm(DUMMY, DUMMY, DUMMY, 5, g, bad, DUMMY, DUMMY, None, None) == PP_EINVAL_TOF
    # per-ray TOF parameters: a table takes per-ray offsets but not per-ray sigmas; OSEM takes neither
    lut_sig = lut()
    lut_sig.sigma_per_ray = DUMMY2.value
    assert lib.pp_fwd_tof_sino(DUMMY, DUMMY, 5, g, lut_sig, DUMMY, DUMMY, None) == PP_EINVAL_TOF
    assert lib.pp_back_tof_lm(DUMMY, DUMMY, DUMMY, 5, g, lut_sig, DUMMY, DUMMY, None, None) == PP_EINVAL_TOF
    lut_off = lut()
    lut_off.offset_per_ray = DUMMY2.value
    assert lib.pp_fwd_tof_sino(DUMMY, DUMMY, 0, g, lut_off, DUMMY, DUMMY, None) == PP_OK  # valid (n == 0)
    for field in ("sigma_per_ray", "offset_per_ray"):
        t = _tof()
        setattr(t, field, DUMMY2.value)
        assert lib.pp_lm_osem_subset_batched(DUMMY, 3, g, t, None) == PP_EINVAL_TOF
        assert lib.pp_fwd_tof_lm(DUMMY, DUMMY, DUMMY, 0, g, t, DUMMY, DUMMY, None, None) == PP_OK
    assert lib.pp_fwd_tof_lm(DUMMY, DUMMY, None, 5, g, _tof(), DUMMY, DUMMY, None, None) == PP_EINVAL_PTR
    # batched listmode projections: image count range, pointers, empty batches
    for f in (lib.pp_fwd_tof_lm_batch, lib.pp_back_tof_lm_batch):
        assert f(DUMMY, DUMMY, DUMMY, 5, g, _tof(), DUMMY, -1, DUMMY, None, None) == PP_EINVAL_N
        assert f(DUMMY, DUMMY, DUMMY, 5, g, _tof(), DUMMY, (1 << 20) + 1, DUMMY, None, None) == PP_EINVAL_N
        assert f(DUMMY, DUMMY, DUMMY, 5, g, _tof(), None, 2, DUMMY, None, None) == PP_EINVAL_PTR
        assert f(DUMMY, DUMMY, DUMMY, 5, g, _tof(), DUMMY, 2, None, None, None) == PP_EINVAL_PTR
        assert f(DUMMY, DUMMY, DUMMY, 5, g, _tof(), DUMMY, 0, DUMMY, None, None) == PP_OK
        assert f(DUMMY, DUMMY, DUMMY, 0, g, _tof(), DUMMY, 2, DUMMY, None, None) == PP_OK
    # Poisson loss: sizes, background, pointers; no elements still writes the partial sums
    pl = lib.pp_poisson_nll
    assert pl(DUMMY, 0.1, DUMMY, -1, DUMMY, DUMMY2, 4, None) == PP_EINVAL_N
    assert pl(DUMMY, 0.1, DUMMY, 5, DUMMY, DUMMY2, 0, None) == PP_EINVAL_N
    assert pl(DUMMY, 0.1, DUMMY, 5, DUMMY, DUMMY2, 65537, None) == PP_EINVAL_N
    assert pl(DUMMY, float("inf"), DUMMY, 5, DUMMY, DUMMY2, 4, None) == PP_EINVAL_N
    assert pl(DUMMY, 0.1, DUMMY, 5, None, DUMMY2, 4, None) == PP_EINVAL_PTR
    assert pl(DUMMY, 0.1, DUMMY, 0, DUMMY, None, 4, None) == PP_EINVAL_PTR
    # forward projection with the events written in processing order: order and outputs required,
    # per-event TOF arrays refused
    gf = lib.pp_fwd_tof_lm_gather
    outs = (DUMMY2, DUMMY2, DUMMY2, DUMMY2)
    assert gf(DUMMY, DUMMY, DUMMY, 5, g, _tof(), DUMMY, DUMMY, None, *outs, None) == PP_EINVAL_PTR
    for k in range(4):
        o = list(outs)
        o[k] = None
        assert gf(DUMMY, DUMMY, DUMMY, 5, g, _tof(), DUMMY, DUMMY, DUMMY3, *o, None) == PP_EINVAL_PTR
    assert gf(DUMMY, DUMMY, DUMMY, 0, g, _tof(), DUMMY, DUMMY, None, None, None, None, None, None) == PP_OK
    assert gf(DUMMY, DUMMY, DUMMY, -1, g, _tof(), DUMMY, DUMMY, DUMMY3, *outs, None) == PP_EINVAL_N
    for field in ("sigma_per_ray", "offset_per_ray"):
        t = _tof()
        setattr(t, field, DUMMY2.value)
        assert gf(DUMMY, DUMMY, DUMMY, 5, g, t, DUMMY, DUMMY, DUMMY3, *outs, None) == PP_EINVAL_TOF
    # crystal-index events: table size, pointers, 8-byte alignment of the pairs
    assert lib.pp_fwd_crystals(DUMMY, 0, DUMMY, 5, g, DUMMY2, DUMMY3, None, None) == PP_EINVAL_N
    assert lib.pp_fwd_crystals(None, 10, DUMMY, 5, g, DUMMY2, DUMMY3, None, None) == PP_EINVAL_PTR
    assert lib.pp_back_crystals(DUMMY, 10, None, 5, g, DUMMY2, DUMMY3, None, None) == PP_EINVAL_PTR
    assert lib.pp_back_crystals(DUMMY, 10, ctypes.c_void_p(20), 5, g, DUMMY2, DUMMY3, None, None) == PP_EINVAL_PTR
    assert lib.pp_fwd_crystals(DUMMY, 10, DUMMY, 0, g, DUMMY2, DUMMY3, None, None) == PP_OK
    assert lib.pp_fwd_tof_lm_crystals(DUMMY, 10, DUMMY, None, 5, g, _tof(), DUMMY2, DUMMY3, None, None) == \
        PP_EINVAL_PTR
    assert lib.pp_back_tof_lm_crystals(DUMMY, 10, DUMMY, DUMMY, 5, g, _tof(nb=0), DUMMY2, DUMMY3, None, None) == \
        PP_EINVAL_TOF
    assert lib.pp_count_samples_crystals(DUMMY, -1, DUMMY, None, 5, g, None, DUMMY2, None) == PP_EINVAL_N
    assert lib.pp_lm_presort_crystals(DUMMY, 10, DUMMY, None, 1000, g, None, 1, DUMMY2, DUMMY3, 1, None) == \
        PP_EINVAL_N  # workspace too small
    assert lib.pp_gather_crystal_events(DUMMY, None, DUMMY2, 10, ctypes.c_void_p(36), None, None) == PP_EINVAL_PTR
    assert lib.pp_gather_crystal_events(DUMMY, DUMMY, DUMMY2, 10, DUMMY3, None, None) == PP_EINVAL_PTR
    assert lib.pp_fwd_tof_lm(DUMMY, DUMMY, DUMMY, 5, g, None, DUMMY, DUMMY, None, None) == PP_EINVAL_PTR
    assert lib.pp_lm_osem_subset_batched(DUMMY, -1, g, _tof(), None) == PP_EINVAL_N
    assert lib.pp_lm_osem_subset_batched(DUMMY, 0, g, _tof(), None) == PP_OK
    assert lib.pp_osem_update_batched(DUMMY, -1, g, None, None) == PP_EINVAL_N
    assert lib.pp_osem_update_batched(None, 3, g, None, None) == PP_EINVAL_PTR
    assert lib.pp_osem_update_batched(DUMMY, 3, None, None, None) == PP_EINVAL_PTR
    assert lib.pp_osem_update_batched(DUMMY, 3, _geom(dim=(0, 4, 4)), None, None) == PP_EINVAL_GEOM
    f3 = ctypes.c_float * 3
    for bad in (f3(-1.0, 4.5, 4.5), f3(float("nan"), 4.5, 4.5), f3(4.5, float("inf"), 4.5), f3(4.5, 4.5, 1e4)):
        assert lib.pp_osem_update_batched(DUMMY, 3, g, bad, None) == PP_EINVAL_RES
        assert lib.pp_gauss3d(DUMMY, DUMMY2, DUMMY3, g, bad, None) == PP_EINVAL_RES
    # resolution model: pointers, aliasing, widths at the radius limit (31 voxels)
    ok = f3(4.5, 4.5, 4.5)
    assert lib.pp_gauss3d(None, DUMMY2, DUMMY3, g, ok, None) == PP_EINVAL_PTR
    assert lib.pp_gauss3d(DUMMY, DUMMY2, DUMMY3, g, None, None) == PP_EINVAL_PTR
    assert lib.pp_gauss3d(DUMMY, DUMMY, DUMMY3, g, ok, None) == PP_EINVAL_PTR  # dst aliases src
    assert lib.pp_gauss3d(DUMMY, DUMMY2, ctypes.c_void_p((1 << 20) + 4), g, ok, None) == PP_EINVAL_PTR  # tmp overlaps dst
    sig_max = 31.49 / 4.0  # radius floor(4 s + 1/2) = 31 voxels at 1 mm
    assert lib.pp_gauss3d(DUMMY, DUMMY2, DUMMY3, _geom(dim=(0, 4, 4)), ok, None) == PP_EINVAL_GEOM
    assert lib.pp_osem_update_batched(DUMMY, 0, g, f3(*(3 * [sig_max * 2.3548])), None) == PP_OK
    assert lib.pp_osem_update_batched(DUMMY, 0, g, f3(*(3 * [32.0 / 4.0 * 2.3549])), None) == PP_EINVAL_RES
    assert lib.pp_fill(None, 10, ctypes.c_float(0.0), None) == PP_EINVAL_PTR
    assert lib.pp_fill(None, -1, ctypes.c_float(0.0), None) == PP_EINVAL_N
    ws = lib.pp_lm_presort_workspace_bytes(1000)
    assert ws >= 3 * 4000
    assert lib.pp_lm_presort_workspace_bytes(0) == 0
    assert lib.pp_lm_presort(DUMMY, DUMMY, None, 1000, g, None, 1, DUMMY, DUMMY, ws - 1, None) == PP_EINVAL_N
    assert lib.pp_lm_presort(DUMMY, DUMMY, None, 1000, g, None, 1, None, DUMMY, ws, None) == PP_EINVAL_PTR
    assert lib.pp_lm_presort(DUMMY, DUMMY, None, -3, g, None, 1, DUMMY, DUMMY, ws, None) == PP_EINVAL_N
    assert lib.pp_lm_presort(DUMMY, DUMMY, None, 1000, g, None, 0, DUMMY, DUMMY, ws, None) == PP_EINVAL_N
    assert lib.pp_gather_events(DUMMY, DUMMY, DUMMY, DUMMY, 10, DUMMY, DUMMY, None, None) == PP_EINVAL_PTR
    assert lib.pp_gather_events(None, None, None, None, 0, None, None, None, None) == PP_OK
    assert lib.pp_osem_init(None, None, 10, None) == PP_EINVAL_PTR
    for c in range(6):
        assert lib.pp_strerror(c)
    # TOF sinogram calls take fewer than 2^31 rays (larger sets go in chunks)
    big = 1 << 31
    assert lib.pp_fwd_tof_sino(DUMMY, DUMMY, big, g, _tof(), DUMMY2, DUMMY3, None) == PP_EINVAL_N
    assert lib.pp_back_tof_sino(DUMMY, DUMMY, big, g, _tof(), DUMMY2, DUMMY3, None) == PP_EINVAL_N
    assert lib.pp_back_tof_sino(DUMMY, DUMMY, big - 1, g, _tof(nb=0), DUMMY2, DUMMY3, None) == PP_EINVAL_TOF


def test_tof_gaussian_table_host(lib):
    """pp_tof_gaussian_table: size query (no device memory touched) and its error codes."""
    from paper_2212_12519_amd._lib import PP_EINVAL_N, PP_EINVAL_PTR, PP_EINVAL_TOF, PP_OK

    n, x0, dx = ctypes.c_int32(), ctypes.c_float(), ctypes.c_float()
    t = _tof(bw=28.0, sig=58.5 / 2.355, ns=3.0, nb=29)
    assert lib.pp_tof_gaussian_table(t, 0.05, None, 0, ctypes.byref(n), ctypes.byref(x0), ctypes.byref(dx),
                                     None) == PP_OK
    win = 3.0 * float(ctypes.c_float(58.5 / 2.355).value) + 14.0
    assert n.value == math.ceil(2 * win / float(ctypes.c_float(0.05).value)) + 1
    assert x0.value == pytest.approx(-win, rel=1e-7) and dx.value <= 0.05
    assert x0.value + (n.value - 1) * dx.value == pytest.approx(win, rel=1e-6)
    assert lib.pp_tof_gaussian_table(None, 0.05, None, 0, None, None, None, None) == PP_EINVAL_PTR
    for bad in (_tof(sig=0.0), _tof(ns=-1.0), _tof(bw=float("nan"))):
        assert lib.pp_tof_gaussian_table(bad, 0.05, None, 0, None, None, None, None) == PP_EINVAL_TOF
    for dxm in (0.0, -1.0, float("inf"), 1e-6):  # 1e-6 mm: more than 2^24 entries
        assert lib.pp_tof_gaussian_table(t, dxm, None, 0, None, None, None, None) == PP_EINVAL_N
    assert lib.pp_tof_gaussian_table(t, 0.05, DUMMY, n.value - 1, None, None, None, None) == PP_EINVAL_N


def test_osem_chunks(lib):
    assert lib.pp_osem_chunks(0, 8) == 0
    assert lib.pp_osem_chunks(1, 8) == 1
    assert lib.pp_osem_chunks(8 * 1024, 8) == 1
    assert lib.pp_osem_chunks(8 * 1024 + 1, 8) == 2
    assert lib.pp_osem_chunks(20_000_000, 8) == (2_500_000 + 1023) // 1024


def test_python_tof_params_per_ray_checks():
    """The binding rejects per-ray arrays that are not float32 CUDA tensors, and a call whose
    ray count differs from their length (no GPU needed: both checks come first)."""
    import paper_2212_12519_amd as pp

    with pytest.raises(ValueError):
        pp.TofParams(28.0, 24.8, 3.0, 29, sigma_per_ray=[1.0, 2.0])
    t = pp.TofParams(28.0, 24.8, 3.0, 29)
    assert not t.per_ray
    assert t.c(5).sigma_per_ray is None and t.c().offset_per_ray is None


def test_python_binding_rejects_cpu_tensors():
    import torch

    import paper_2212_12519_amd as pp

    x = torch.zeros((4, 3))
    with pytest.raises(TypeError):
        pp.fwd(x, x, pp.ImageGeom((2, 2, 2), (1, 1, 1)), torch.zeros(2, 2, 2))


def test_tof_weight_form(lib):
    """pp_tof_weight_form (host-only): the fitted polynomial for the clinical kernel and for a
    per-ray offset, the table when one is given, the erf for per-ray sigma and where no fit of the
    fixed degrees reaches the bound (truncation at 8 sigma: w spans too many decades)."""
    from paper_2212_12519_amd._lib import PP_EINVAL_PTR, PP_EINVAL_TOF, PP_OK, CTof

    form = ctypes.c_int32(-1)

    def f(t):
        form.value = -1
        assert lib.pp_tof_weight_form(t, ctypes.byref(form)) == PP_OK
        return form.value

    clin = (28.0, 58.5 / 2.355, 3.0, 29)
    assert f(_tof(*clin)) == 2
    assert f(_tof(28.0, 58.5 / 2.355, 8.0, 29)) == 0
    assert f(CTof(*clin[:3], 0.0, clin[3], None, 0, 0.0, 0.0, None, DUMMY)) == 2  # per-ray offset only
    assert f(CTof(*clin[:3], 0.0, clin[3], None, 0, 0.0, 0.0, DUMMY, None)) == 0  # per-ray sigma
    assert f(CTof(*clin[:3], 0.0, clin[3], DUMMY, 100, -50.0, 1.0, None, None)) == 1  # table
    assert lib.pp_tof_weight_form(_tof(sig=0.0), ctypes.byref(form)) == PP_EINVAL_TOF
    assert lib.pp_tof_weight_form(_tof(*clin), None) == PP_EINVAL_PTR


def test_tof_sino_osem_argument_errors(lib):
    """pp_tof_sino_sensitivity / pp_tof_sino_osem_subset reject bad counts, shards, workspaces,
    per-ray TOF parameters and overlapping images before any launch."""
    from paper_2212_12519_amd._lib import PP_EINVAL_N, PP_EINVAL_PTR, PP_EINVAL_TOF, CTof

    g = _geom()
    t = _tof()
    per = CTof(1.0, 1.0, 3.0, 0.0, 5, None, 0, 0.0, 0.0, DUMMY, None)
    f = lib.pp_tof_sino_osem_subset
    nvb = 4 * 4 * 4 * 4  # bytes of one image of _geom()
    X, A, S, W = ctypes.c_void_p(1 << 24), ctypes.c_void_p(1 << 25), ctypes.c_void_p(1 << 26), ctypes.c_void_p(1 << 27)
    assert f(DUMMY, DUMMY, DUMMY, 10, g, t, 0.1, X, A, 0, S, W, 100, None) == PP_EINVAL_N  # no shard
    assert f(DUMMY, DUMMY, DUMMY, 10, g, t, 0.1, X, A, 1025, S, W, 100, None) == PP_EINVAL_N
    assert f(DUMMY, DUMMY, DUMMY, 10, g, t, 0.1, X, A, 1, S, W, 0, None) == PP_EINVAL_N  # no workspace rows
    assert f(DUMMY, DUMMY, DUMMY, 10, g, t, float("nan"), X, A, 1, S, W, 100, None) == PP_EINVAL_N
    assert f(DUMMY, DUMMY, DUMMY, -1, g, t, 0.1, X, A, 1, S, W, 100, None) == PP_EINVAL_N
    assert f(DUMMY, DUMMY, DUMMY, 10, g, per, 0.1, X, A, 1, S, W, 100, None) == PP_EINVAL_TOF
    assert f(DUMMY, DUMMY, None, 10, g, t, 0.1, X, A, 1, S, W, 100, None) == PP_EINVAL_PTR
    # x inside the second shard image; workspace over sens
    A2 = ctypes.c_void_p((1 << 24) - nvb)
    assert f(DUMMY, DUMMY, DUMMY, 10, g, t, 0.1, X, A2, 2, S, W, 100, None) == PP_EINVAL_PTR
    assert f(DUMMY, DUMMY, DUMMY, 10, g, t, 0.1, X, A, 1, S, ctypes.c_void_p((1 << 26) - 8), 100,
             None) == PP_EINVAL_PTR
    s = lib.pp_tof_sino_sensitivity
    assert s(DUMMY, DUMMY, 10, g, t, S, W, 0, None) == PP_EINVAL_N
    assert s(DUMMY, DUMMY, 10, g, per, S, W, 10, None) == PP_EINVAL_TOF
    assert s(DUMMY, DUMMY, 10, g, t, None, W, 10, None) == PP_EINVAL_PTR
    assert s(DUMMY, DUMMY, 0, g, t, None, None, 10, None) == 0  # nothing to do
