"""The run/sheet back projection's fixed-point accumulation (presorted listmode TOF), on rays whose
values span many orders of magnitude in one sheet.  Three transaxial lines, each with three classes
of events at different TOF positions along the line: large values (about 1e6) at one end, values ten
times smaller in the middle (they keep about 19 bits in the sheet's fixed point) and signed values
1e9 times smaller at the other end (too small for the sheet: they take the float atomics of the
direct scatter).  Checked against the FP64 oracle in full and on the voxels that only the middle or
only the small class reaches, so that values far below a sheet's largest are neither lost nor
swamped by it.  Through the C ABI."""
import numpy as np
import pytest
import torch

import oracle
from helpers import rel_l2, tofd

pytestmark = pytest.mark.gpu

BACK_TOL = 1e-4
DIM, VS = (128, 128, 16), (4.0, 4.0, 4.0)
ORIGIN = tuple(-(n - 1) / 2 * h for n, h in zip(DIM, VS))
TOF = tofd(28.0, 58.5 / 2.355, 3.0, 29)
# (TOF bins, value scale, signed) per class: bin centres -252..-168 mm, -28..28 mm, 168..252 mm
CLASSES = {"large": ((5, 8), 1e6, False), "middle": ((13, 15), 1e5, False), "small": ((20, 23), 1e-3, True)}


def _events(seed):
    rng = np.random.default_rng(seed)
    xs, xe, bins, p, cls = [], [], [], [], []
    for a in rng.uniform(0.0, np.pi, size=3):
        d = np.array([np.cos(a), np.sin(a)])
        nrm = np.array([-d[1], d[0]])
        off = rng.uniform(-40.0, 40.0)
        e0, e1 = off * nrm - 300.0 * d, off * nrm + 300.0 * d  # the same transaxial line for all its events
        for ci, (name, ((b0, b1), scale, signed)) in enumerate(CLASSES.items()):
            n = {"large": 120, "middle": 80, "small": 56}[name]
            z = rng.uniform(-28.0, 28.0, size=(n, 2))
            xs.append(np.column_stack([np.full(n, e0[0]), np.full(n, e0[1]), z[:, 0]]))
            xe.append(np.column_stack([np.full(n, e1[0]), np.full(n, e1[1]), z[:, 1]]))
            bins.append(rng.integers(b0, b1 + 1, size=n))
            v = scale * rng.uniform(0.5, 1.5, size=n)
            if signed:
                v *= rng.choice([-1.0, 1.0], size=n)
            p.append(v)
            cls.append(np.full(n, ci))
    cat = np.concatenate
    return (cat(xs).astype(np.float32), cat(xe).astype(np.float32), cat(bins).astype(np.int16),
            cat(p).astype(np.float32), cat(cls))


def test_sheet_dynamic_range(gpu):
    xs, xe, bins, p, cls = _events(91)
    dev = torch.device("cuda")
    G = gpu.ImageGeom(DIM, VS, ORIGIN)
    T = gpu.TofParams(TOF["bin_width"], TOF["sigma"], TOF["n_sigmas"], TOF["n_bins"])
    xs_d, xe_d, b_d = torch.from_numpy(xs).to(dev), torch.from_numpy(xe).to(dev), torch.from_numpy(bins).to(dev)
    order = gpu.presort(xs_d, xe_d, G, b_d, T)
    got = gpu.back_tof_lm(xs_d, xe_d, b_d, G, T, torch.from_numpy(p).to(dev), order=order)
    torch.cuda.synchronize()
    got = got.cpu().numpy().astype(np.float64)

    def ref(mask):
        return oracle.back_tof_lm(xs, xe, ORIGIN, VS, DIM, TOF, bins, np.where(mask, p, 0.0))

    r_all = ref(np.ones_like(cls, dtype=bool))
    r_cls = [ref(cls == c) for c in range(3)]
    assert rel_l2(got, r_all) <= BACK_TOL
    for c, name in ((1, "middle"), (2, "small")):
        only = (r_cls[c] != 0) & np.all([r_cls[o] == 0 for o in range(3) if o != c], axis=0)
        assert only.sum() > 1000, (name, int(only.sum()))
        err = rel_l2(got[only], r_all[only])
        print(f"{name}: {int(only.sum())} voxels reached by that class only, rel L2 {err:.2e}")
        assert err <= BACK_TOL, name


def test_sheet_coarsening_keeps_sums(gpu):
    """Forty transaxial lines of 15,000 events each, values growing by six orders of magnitude with the
    TOF bin (the presort orders a line's events by bin, so the later groups of 256 rays of a line carry
    larger bounds than the first): the sheet's fixed point is coarsened in place as a line continues
    across groups, and values are rounded with carried remainders.  Checked against the FP64 oracle:
    relative L2 over the image and the image sum, which plain rounding of small values would bias."""
    rng = np.random.default_rng(92)
    n_line, per = 40, 15_000
    xs, xe, bins, p = [], [], [], []
    for a in rng.uniform(0.0, np.pi, size=n_line):
        d = np.array([np.cos(a), np.sin(a)])
        nrm = np.array([-d[1], d[0]])
        off = rng.uniform(-60.0, 60.0)
        e0, e1 = off * nrm - 300.0 * d, off * nrm + 300.0 * d
        z = rng.uniform(-28.0, 28.0, size=(per, 2))
        xs.append(np.column_stack([np.full(per, e0[0]), np.full(per, e0[1]), z[:, 0]]))
        xe.append(np.column_stack([np.full(per, e1[0]), np.full(per, e1[1]), z[:, 1]]))
        b = rng.integers(4, 25, size=per)
        bins.append(b)
        p.append(10.0 ** ((b - 4) * 0.3) * rng.uniform(0.5, 1.5, size=per))
    xs, xe = np.concatenate(xs).astype(np.float32), np.concatenate(xe).astype(np.float32)
    bins, p = np.concatenate(bins).astype(np.int16), np.concatenate(p).astype(np.float32)
    dev = torch.device("cuda")
    G = gpu.ImageGeom(DIM, VS, ORIGIN)
    T = gpu.TofParams(TOF["bin_width"], TOF["sigma"], TOF["n_sigmas"], TOF["n_bins"])
    xs_d, xe_d, b_d = torch.from_numpy(xs).to(dev), torch.from_numpy(xe).to(dev), torch.from_numpy(bins).to(dev)
    order = gpu.presort(xs_d, xe_d, G, b_d, T)
    got = gpu.back_tof_lm(xs_d, xe_d, b_d, G, T, torch.from_numpy(p).to(dev), order=order)
    torch.cuda.synchronize()
    got = got.cpu().numpy().astype(np.float64)
    ref = oracle.back_tof_lm(xs, xe, ORIGIN, VS, DIM, TOF, bins, p.astype(np.float64))
    err = rel_l2(got, ref)
    sum_err = abs(got.sum() - ref.sum()) / ref.sum()
    print(f"{xs.shape[0]} events: rel L2 {err:.2e}, image sum rel error {sum_err:.2e}")
    assert err <= BACK_TOL
    assert sum_err <= 1e-5
