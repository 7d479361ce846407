"""Host-side logic of the serving loop (no GPU): arrival traces, footprints, latency statistics,
and the OSEM slot-table bookkeeping that mirrors the device's per-step updates."""
import math

import numpy as np
import pytest
import torch


def test_make_trace_distribution():
    from paper_2212_12519_amd.serve import make_trace

    n_pool = 5_000_000
    pool = (torch.zeros((n_pool, 3)), torch.zeros((n_pool, 3)), torch.zeros(n_pool, dtype=torch.int16))
    grids = ["a", "b"]
    tr = make_trace(pool, grids, 2000, seed=1, events_range=(1000, 1_000_000), rate_hz=50.0)
    assert [r.rid for r in tr] == list(range(2000))
    arr = np.array([r.arrival for r in tr])
    assert np.all(np.diff(arr) > 0)
    gaps = np.diff(np.concatenate([[0.0], arr]))
    assert abs(gaps.mean() - 1 / 50.0) < 0.1 / 50.0  # exponential inter-arrival times
    sizes = np.array([r.xstart.shape[0] for r in tr])
    assert sizes.min() >= 1000 and sizes.max() <= 1_000_000
    logs = np.log(sizes)
    assert abs(logs.mean() - 0.5 * (math.log(1000) + math.log(1e6))) < 0.2  # log-uniform
    assert {r.grid for r in tr} == {"a", "b"}
    # deterministic for a seed
    tr2 = make_trace(pool, grids, 5, seed=1, events_range=(1000, 1_000_000), rate_hz=50.0)
    assert [r.arrival for r in tr2] == [r.arrival for r in tr[:5]]


def test_footprint_and_latency_stats():
    from paper_2212_12519_amd.serve import OsemResult, frame_footprint, latency_stats

    assert frame_footprint(1_000_000, 1000) == 26_000_000 + 8000
    res = [OsemResult(i, None, float(i), float(i), float(i) + 1.0 + 0.01 * i) for i in range(100)]
    st = latency_stats(res, 0.0)
    assert st["n"] == 100
    assert st["p50_s"] == pytest.approx(np.percentile(1.0 + 0.01 * np.arange(100), 50))
    assert st["p99_s"] == pytest.approx(np.percentile(1.0 + 0.01 * np.arange(100), 99))
    assert st["frames_per_s"] == pytest.approx(100 / (99 + 1.0 + 0.99))


def test_slot_table_host_mirror():
    """The host mirror applies the same per-step rule as the device kernel: live slots advance
    subset = (subset + 1) mod n_sub and lose one step; finished or inactive slots do not."""
    from paper_2212_12519_amd._lib import COsemSlot

    tbl = (COsemSlot * 3)()
    tbl[0].active, tbl[0].n_sub, tbl[0].steps_left = 1, 8, 24
    tbl[1].active, tbl[1].n_sub, tbl[1].steps_left, tbl[1].subset = 1, 4, 2, 3
    tbl[2].active, tbl[2].n_sub, tbl[2].steps_left = 0, 8, 5

    class T:  # minimal stand-in for SlotTable (no device buffers)
        host = tbl

    from paper_2212_12519_amd.osem import SlotTable

    SlotTable.advance_host(T, 5)
    assert (tbl[0].subset, tbl[0].steps_left) == (5, 19)
    assert (tbl[1].subset, tbl[1].steps_left) == (1, 0)  # 3 -> 0 -> 1, then finished
    assert (tbl[2].subset, tbl[2].steps_left) == (0, 5)


def test_admission_per_grid_fifo():
    """A request waiting for a slot of its own grid does not hold up requests of another grid;
    within a grid, requests are admitted in arrival order (no overtaking)."""
    from collections import deque

    from paper_2212_12519_amd import serve

    class Req:
        def __init__(self, rid, grid):
            self.rid, self.grid = rid, grid

    class Srv(serve.OsemServer):
        def __init__(self, free):
            self.free = dict(free)
            self.admitted = []

        def _admit(self, req, now):
            if self.free[req.grid] == 0:
                return False
            self.free[req.grid] -= 1
            self.admitted.append(req.rid)
            return True

    import paper_2212_12519_amd._lib as L

    ga = L.ImageGeom((4, 4, 4), (1, 1, 1))
    gb = L.ImageGeom((8, 8, 4), (1, 1, 1))
    srv = Srv({ga: 1, gb: 2})
    q = deque([Req(0, ga), Req(1, ga), Req(2, gb), Req(3, ga), Req(4, gb), Req(5, gb)])
    left = srv._admit_queue(q, 0.0)
    assert srv.admitted == [0, 2, 4]
    assert [r.rid for r in left] == [1, 3, 5]
