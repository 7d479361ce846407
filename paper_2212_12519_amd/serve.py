"""Continuous-batching server for short-frame listmode TOF OSEM reconstructions.

Motivation from the paper: data-driven motion correction reconstructs many very
short frames (Sec. 1), and OSEM should keep every operation on the GPU
(Sec. 2.6, Sec. 4).  Requests (a frame's events, an image grid, iterations x
subsets) arrive over time.  The server

* admits queued requests whenever a slot of their grid's table is free and
  the frame fits the HBM budget (events in subset-major presorted order,
  image, accumulator), first-come first-served within each grid: a request
  waiting for its grid's slots does not hold up requests of another grid;
* advances every admitted frame by one OSEM subset update per step, all
  frames of a grid in one fused launch pair -- frames at different
  iterations / subsets coexist, new frames join between steps, finished
  frames leave (continuous batching at subset granularity);
* replays a HIP graph captured once per grid (the slot table is read from
  device memory, so the same graph serves every mix);
* optionally includes the image-based Gaussian resolution model in the
  system model (the paper's OSEM does, Sec. 2.6): blur passes per step inside
  the same graph;
* records arrival, admission and completion times for p50 / p99 latency.

``run_sequential`` is the baseline: the same trace served one frame at a
time, FIFO, with plain projector calls (pp_fwd_tof_lm, a torch ratio,
pp_back_tof_lm, a torch image update; pp_gauss3d around them with the
resolution model) per subset.
"""
from __future__ import annotations

import math
import time
from collections import deque
from dataclasses import dataclass, field

import numpy as np
import torch

from ._lib import as_geom, as_tof, load
from . import osem as O
from .projectors import back_tof_lm, fwd_tof_lm, gauss3d


@dataclass
class OsemRequest:
    rid: int
    xstart: torch.Tensor
    xend: torch.Tensor
    tof_bin: torch.Tensor
    grid: object  # ImageGeom
    arrival: float  # seconds after the start of the trace
    n_iter: int = 3
    n_sub: int = 8
    bg: float = 0.1


@dataclass
class OsemResult:
    rid: int
    image: torch.Tensor
    arrival: float
    admitted: float
    finished: float

    @property
    def latency(self):
        return self.finished - self.arrival


def frame_footprint(n_events, n_vox, res=False):
    """HBM bytes a frame holds while admitted: presorted event copy (26 B/event), x and acc
    (plus x_fwd and the scratch image with the resolution model)."""
    return 26 * int(n_events) + (4 if res else 2) * 4 * int(n_vox)


@dataclass
class _Live:
    req: OsemRequest
    slot: int
    tensors: tuple
    x: torch.Tensor
    admitted: float
    nbytes: int


@dataclass
class _GridState:
    geom: object
    sens: torch.Tensor
    table: O.SlotTable
    free: list
    live: dict = field(default_factory=dict)
    graph: object = None
    dirty: bool = False


class OsemServer:
    def __init__(self, tof, sens_by_grid, max_slots=64, hbm_budget=32e9, steps_per_tick=1, use_graph=True,
                 device="cuda", res_fwhm=None):
        """sens_by_grid: [(geom, sensitivity image)], the sensitivity including the resolution
        model when res_fwhm (mm) is given."""
        self.tof = as_tof(tof)
        self.res_fwhm = res_fwhm
        self.device = torch.device(device)
        self.budget = float(hbm_budget)
        self.steps = int(steps_per_tick)
        self.use_graph = use_graph
        self.grids = {}
        for geom, sens in sens_by_grid:
            g = as_geom(geom)
            self.grids[g] = _GridState(g, sens, O.SlotTable(max_slots, self.device), list(range(max_slots)))
        self.in_use = 0
        self.rejected = []
        self.waited_budget, self.waited_slot = set(), set()  # requests admission deferred, by cause
        self.peak_bytes = 0
        self.peak_live = 0
        load()

    def _admit(self, req, now):
        st = self.grids[as_geom(req.grid)]
        nbytes = frame_footprint(req.xstart.shape[0], st.geom.n_vox, self.res_fwhm is not None)
        if nbytes > self.budget:
            self.rejected.append(req.rid)  # can never fit: refuse instead of blocking the queue
            return True
        if not st.free:
            self.waited_slot.add(req.rid)
            return False
        if self.in_use + nbytes > self.budget:
            self.waited_budget.add(req.rid)
            return False
        slot = st.free.pop(0)
        xs, xe, tb = O.prepare_frame(req.xstart, req.xend, req.tof_bin, st.geom, self.tof, req.n_sub)
        x = O.init_image(st.sens)
        acc = torch.zeros_like(st.sens)
        xf = tmp = None
        if self.res_fwhm is not None:
            xf, tmp = O.res_buffers(x, st.geom, self.res_fwhm)
        st.table.set(slot, xs, xe, tb, x, acc, st.sens, req.n_sub, req.n_iter * req.n_sub, req.bg, xf, tmp)
        st.live[slot] = _Live(req, slot, (xs, xe, tb, acc, xf, tmp), x, now, nbytes)
        st.dirty = True
        self.in_use += nbytes
        self.peak_bytes = max(self.peak_bytes, self.in_use)
        self.peak_live = max(self.peak_live, sum(len(g.live) for g in self.grids.values()))
        return True

    def _admit_queue(self, queue, now):
        """Admits what fits, in arrival order within each grid; returns the requests left waiting.
        Once a request of a grid has to wait, later requests of that grid wait behind it."""
        waiting, blocked = deque(), set()
        for req in queue:
            g = as_geom(req.grid)
            if g in blocked or not self._admit(req, now):
                blocked.add(g)
                waiting.append(req)
        return waiting

    def _step(self, st):
        if st.dirty:
            st.table.upload()
            st.dirty = False
        if self.use_graph:
            if st.graph is None:
                st.graph = O.capture_steps(st.table, st.geom, self.tof, self.steps, self.res_fwhm)
            st.graph.replay()
        else:
            O.osem_steps(st.table, st.geom, self.tof, self.steps, self.res_fwhm)
        st.table.advance_host(self.steps)

    def run(self, trace, clock=time.perf_counter):
        """Serve a trace of OsemRequests (arrival times relative to the start); returns OsemResults."""
        pending = deque(sorted(trace, key=lambda r: r.arrival))
        queue = deque()
        results = []
        t0 = clock()
        done_ev = torch.cuda.Event()
        while pending or queue or any(st.live for st in self.grids.values()):
            now = clock() - t0
            while pending and pending[0].arrival <= now:
                queue.append(pending.popleft())
            queue = self._admit_queue(queue, now)
            live = [st for st in self.grids.values() if st.live]
            if not live:
                if pending:
                    time.sleep(max(0.0, pending[0].arrival - (clock() - t0)))
                continue
            for st in live:
                self._step(st)
            done_ev.record()
            done_ev.synchronize()
            now = clock() - t0
            for st in live:
                for slot in [s for s, lv in st.live.items() if st.table.host[s].steps_left <= 0]:
                    lv = st.live.pop(slot)
                    st.table.clear(slot)
                    st.free.append(slot)
                    st.dirty = True
                    self.in_use -= lv.nbytes
                    results.append(OsemResult(lv.req.rid, lv.x, lv.req.arrival, lv.admitted, now))
        return results


def run_sequential(trace, tof, sens_by_grid, presorted=True, clock=time.perf_counter, res_fwhm=None):
    """Baseline: the same trace, one frame at a time (FIFO), plain projector calls per subset
    (pp_fwd_tof_lm, torch ratio, pp_back_tof_lm, torch image update; with res_fwhm a pp_gauss3d
    before the forward and after the back projection).  presorted=True first puts the frame's
    events in subset-major presorted order (pp_lm_presort + pp_gather_events); presorted=False
    uses the events as given, each subset copied out of the strided view."""
    tof = as_tof(tof)
    sens = {as_geom(g): s for g, s in sens_by_grid}
    results = []
    t0 = clock()
    for req in sorted(trace, key=lambda r: r.arrival):
        now = clock() - t0
        if req.arrival > now:
            time.sleep(req.arrival - now)
        start = clock() - t0
        g = as_geom(req.grid)
        sv = sens[g]
        ns = req.n_sub
        if presorted:
            xs, xe, tb = O.prepare_frame(req.xstart, req.xend, req.tof_bin, g, tof, ns)
            n = xs.shape[0]
            base, rem = n // ns, n % ns
            subsets = []
            for j in range(ns):
                a = j * base + min(j, rem)
                b = a + base + (1 if j < rem else 0)
                subsets.append((xs[a:b], xe[a:b], tb[a:b]))
        else:
            subsets = [(req.xstart[j::ns].contiguous(), req.xend[j::ns].contiguous(), req.tof_bin[j::ns].contiguous())
                       for j in range(ns)]
        x = O.init_image(sv)
        acc = torch.zeros_like(sv)
        pos = sv > 0
        for _ in range(req.n_iter):
            for sx, se, sb in subsets:
                xf = x if res_fwhm is None else gauss3d(x, g, res_fwhm)
                ybar = fwd_tof_lm(sx, se, sb, g, tof, xf) + req.bg
                ratio = torch.where(ybar > 0, 1.0 / ybar, torch.zeros_like(ybar))
                acc.zero_()
                back_tof_lm(sx, se, sb, g, tof, ratio, img=acc)
                ab = acc if res_fwhm is None else gauss3d(acc, g, res_fwhm)
                x = torch.where(pos, x * ab / (sv / ns), torch.zeros_like(x))
        torch.cuda.current_stream().synchronize()
        results.append(OsemResult(req.rid, x, req.arrival, start, clock() - t0))
    return results


def latency_stats(results, t_first=None):
    lat = np.array([r.latency for r in results])
    if not len(lat):
        return {}
    t_first = min(r.arrival for r in results) if t_first is None else t_first
    span = max(r.finished for r in results) - t_first
    return {"n": len(lat), "p50_s": float(np.percentile(lat, 50)), "p99_s": float(np.percentile(lat, 99)),
            "mean_s": float(lat.mean()), "frames_per_s": len(lat) / span if span > 0 else math.inf,
            "makespan_s": span}


def make_trace(pool, grids, n_requests, seed, events_range, rate_hz, n_iter=3, n_sub=8, bg=0.1):
    """Poisson arrivals; log-uniform event counts; each frame a random contiguous slice of the
    event pool; grids drawn uniformly from `grids`."""
    xs, xe, tb = pool
    rng = np.random.default_rng(seed)
    n_pool = xs.shape[0]
    t, out = 0.0, []
    lo, hi = math.log(events_range[0]), math.log(events_range[1])
    for rid in range(n_requests):
        t += rng.exponential(1.0 / rate_hz)
        n = int(min(n_pool, round(math.exp(rng.uniform(lo, hi)))))
        o = int(rng.integers(0, n_pool - n + 1))
        g = grids[int(rng.integers(0, len(grids)))]
        out.append(OsemRequest(rid, xs[o:o + n], xe[o:o + n], tb[o:o + n], g, t, n_iter, n_sub, bg))
    return out


# Slots per grid of the latency-oriented configuration: a step of a few average frames (5M events
# each, 8 subsets) already fills the GPU, so more slots only make admitted frames share the GPU
# longer (higher latency, the same throughput).  The budget-bound configuration of the benchmark
# gives each grid BUDGET_SLOTS slots, so that the HBM budget, not the table, limits admission.
SERVE_SLOTS = 6
BUDGET_SLOTS = 128


def bench_leg(args, log):
    """Serving measurement for bench.py: Poisson-arriving TOF LM-OSEM frames (3 it x 8 subsets,
    0.5M-20M events log-uniform, 128x128x64 or 215x215x71 grid), continuous batching vs sequential
    plain calls on the same traces.
      * overload: 256 requests at 3x the sequential service rate (frames/s = capacity), batched with
        SERVE_SLOTS slots per grid, with BUDGET_SLOTS slots per grid (the 32 GB HBM budget binds),
        sequential plain calls on presorted events and on the events as given (first 64);
      * load 1.25x and 0.5x of the sequential service rate, 128 requests each, batched and
        sequential (presorted): latency is service time plus queueing.
    Returns a dict for the benchmark's JSON line."""
    from synth import configs as C
    from synth import generate_tof_lm_events
    import paper_2212_12519_amd as pp

    dev = torch.device("cuda")
    t = C.TOF_CLIN
    T = pp.TofParams(t.bin_width, t.sigma, t.n_sigmas, t.n_bins)
    src = C.phantom_clin(device=dev)
    pool = generate_tof_lm_events(C.SCANNER_CLIN, C.SINO_CLIN.n_rad, C.SINO_CLIN.max_rd, C.GRID_CLIN, src,
                                  C.N_EVENTS_LM, seed=C.SEED_SERVE, tof_bin_width=t.bin_width, tof_sigma=t.sigma,
                                  n_tof_bins=t.n_bins, device=dev)
    lxs, lxe = C.SINO_CLIN.lors(device=dev, radial_chunk=25)
    grids = [pp.ImageGeom(g.dim, g.voxsize, g.origin) for g in C.SERVE_GRIDS]
    res = None if getattr(args, "no_res", False) else O.RES_FWHM_MM
    sens = [(g, O.sensitivity(lxs, lxe, g, res_fwhm=res)) for g in grids]
    del lxs, lxe
    torch.cuda.empty_cache()
    n_req = int(getattr(args, "serve_requests", None) or C.N_REQUESTS)
    budget = 32e9

    def server(slots):
        sv = OsemServer(T, sens, max_slots=slots, hbm_budget=budget, steps_per_tick=1, use_graph=True,
                        res_fwhm=res)
        sv.run(make_trace(pool, grids, 4, C.SEED_SERVE + 2, (500_000, 600_000), 1e9))  # warm-up and capture
        return sv

    def batched(sv, trace, label):
        sv.waited_budget, sv.waited_slot, sv.peak_bytes, sv.peak_live = set(), set(), 0, 0
        out = sv.run(trace)
        st = latency_stats(out, 0.0)
        st.update({"slots_per_grid": sv.grids[grids[0]].table.capacity, "peak_live_frames": sv.peak_live,
                   "peak_admitted_gb": sv.peak_bytes / 1e9, "waited_for_hbm_budget": len(sv.waited_budget),
                   "waited_for_slot": len(sv.waited_slot), "rejected": len(sv.rejected)})
        log(f"serving {label}: p50 {st['p50_s']:.3f} s p99 {st['p99_s']:.3f} s, {st['frames_per_s']:.2f} frames/s, "
            f"peak {sv.peak_live} frames / {sv.peak_bytes / 1e9:.1f} GB, waited budget {len(sv.waited_budget)} "
            f"slot {len(sv.waited_slot)}")
        return out, st

    def sequential(trace, label, presorted=True):
        out = run_sequential(trace, T, sens, presorted=presorted, res_fwhm=res)
        st = latency_stats(out, 0.0)
        log(f"serving {label}: p50 {st['p50_s']:.3f} s p99 {st['p99_s']:.3f} s, {st['frames_per_s']:.2f} frames/s")
        return out, st

    sv = server(SERVE_SLOTS)
    # calibrate the sequential (presorted) service time on a burst from the same distribution
    cal = make_trace(pool, grids, 16, C.SEED_SERVE + 1, C.SERVE_EVENTS_RANGE, 1e9)
    run_sequential(cal[:2], T, sens, res_fwhm=res)
    t0 = time.perf_counter()
    run_sequential(cal, T, sens, res_fwhm=res)
    service = (time.perf_counter() - t0) / len(cal)
    # overload: Poisson arrivals at 3x the sequential service rate, so frames/s measures capacity
    rate = 3.0 / service
    trace = make_trace(pool, grids, n_req, C.SEED_SERVE, C.SERVE_EVENTS_RANGE, rate)
    log(f"serving: {n_req} requests, sequential service ~{service * 1e3:.0f} ms/frame, arrival rate {rate:.2f}/s")
    res_b, sb = batched(sv, trace, f"batched ({SERVE_SLOTS} slots/grid)")
    res_s, ss = sequential(trace, "sequential presorted")
    n_u = min(n_req, 64)
    _, su = sequential(trace[:n_u], f"sequential as-given (first {n_u})", presorted=False)
    sb_u = latency_stats([r for r in res_b if r.rid < n_u], 0.0)
    by_id = {r.rid: r.image for r in res_s}
    diffs = [float(torch.linalg.vector_norm(r.image - by_id[r.rid]) / torch.linalg.vector_norm(by_id[r.rid]))
             for r in res_b[:16]]
    del res_b, res_s
    # the same overload trace with the HBM budget as the binding limit
    sv_big = server(BUDGET_SLOTS)
    _, sbb = batched(sv_big, trace, f"batched ({BUDGET_SLOTS} slots/grid, budget-bound)")
    del sv_big
    torch.cuda.empty_cache()
    # latency at loads below and just above the sequential service rate
    loads = {}
    n_load = max(8, n_req // 2)
    for load_x in (1.25, 0.5):
        tr = make_trace(pool, grids, n_load, C.SEED_SERVE + 3, C.SERVE_EVENTS_RANGE, load_x / service)
        _, b_st = batched(sv, tr, f"batched at {load_x}x load")
        _, s_st = sequential(tr, f"sequential presorted at {load_x}x load")
        loads[f"{load_x}x"] = {"requests": n_load, "arrival_rate_hz": load_x / service, "batched": b_st,
                               "sequential_plain_presorted": s_st}
    return {"requests": n_req, "arrival_rate_hz": rate, "offered_load_vs_sequential": 3.0, "iterations": 3,
            "subsets": 8, "resolution_model_fwhm_mm": res, "sequential_service_s": service, "batched": sb,
            "batched_budget_bound": sbb, "sequential_plain_presorted": ss,
            "sequential_plain_as_given": dict(su, note=f"first {n_u} requests of the same trace"),
            "batched_first_requests": sb_u,
            "speedup_frames_per_s_vs_plain_presorted": sb["frames_per_s"] / ss["frames_per_s"],
            "max_rel_l2_batched_vs_plain": max(diffs) if diffs else None,
            "hbm_budget_gb": budget / 1e9, "load_sweep": loads}
