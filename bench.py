"""Benchmark: TOF listmode forward + back projection throughput on one MI355X.

Workload (one step = one pass of the projector pair over one batch):
  40,000,000 seeded synthetic TOF listmode events drawn from the clinical
  ellipsoid/lesion phantom (scanner radius 410 mm, 64 rings x 760 crystals,
  ring difference <= 20, 400 radial bins), image 215 x 215 x 71 voxels of
  1.65 x 1.65 x 2.0 mm, 29 TOF bins of 28 mm, Gaussian FWHM 58.5 mm truncated
  at 3 sigma.  A step zeroes the back-projection image, presorts the unsorted
  events (pp_lm_presort), runs pp_fwd_tof_lm_gather over all events in that
  order (the projections, and the events with their projections written in
  processing order) and pp_back_tof_lm of the result on those copies (read
  contiguously, no order array).  Inputs are resident in HBM before timing
  starts.

Prints ONE JSON line (see the field list in the design notes): value =
events / s over the timed steps, a live roofline figure for the dominant
kernel (HIP events on the launch stream), the FP64 oracle timed on the host
cores on a bounded sample, and secondary legs (clinical non-TOF and TOF
sinogram projections, listmode-OSEM serving when available).
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


# the sources the listmode step's kernels and their launch configuration are built from
STEP_SOURCES = ("api.hip", "joseph.hpp", "launch.hpp", "presort.hip", "projectors.hip", "sheet.hpp")


# the sources of the clinical sinogram legs' kernels
SINO_SOURCES = ("api.hip", "joseph.hpp", "launch.hpp", "projectors.hip", "sheet.hpp")


def kernel_sources_sha(sources=STEP_SOURCES):
    """sha256 over the given kernel sources (default: the listmode step's)."""
    import hashlib

    d = os.path.join(ROOT, "paper_2212_12519_amd", "csrc")
    h = hashlib.sha256()
    for f in sources:
        h.update(f.encode())
        h.update(open(os.path.join(d, f), "rb").read())
    return h.hexdigest()


TRAFFIC_JSON = os.path.join(ROOT, "profiles", "tof_lm_40M_traffic.json")
SINO_TRAFFIC_JSON = os.path.join(ROOT, "profiles", "clinical_sino_traffic.json")
# the sinogram legs' device kernels
SINO_KERNELS = {"nontof_fwd": "ppmi::k_fwd", "nontof_back": "ppmi::k_back_runs<ppmi::ModeNonTof>",
                "tof_fwd": "ppmi::k_fwd_tof_sino<false>",
                "tof_back": "ppmi::k_back_runs<ppmi::ModeTofSino<false, false> >"}


def traffic_record(which):
    """(path, sources) of a traffic record: "lm" (the listmode step) or "sino" (the sinogram legs)."""
    return (TRAFFIC_JSON, STEP_SOURCES) if which == "lm" else (SINO_TRAFFIC_JSON, SINO_SOURCES)


def profiled_kernel_bytes(which, kernel):
    """HBM bytes per launch of `kernel` from the committed counter record `which`, or None when the
    record is missing or the kernel sources changed since the counters were taken."""
    path, sources = traffic_record(which)
    try:
        rec = json.load(open(path))
    except (OSError, ValueError):
        return None
    if kernel_sources_sha(sources) != rec.get("source_sha256"):
        return None
    k = rec.get("kernels", {}).get(kernel)
    return k["traffic_bytes"] if k else None
# the device kernel each timed entry point of the listmode step launches
KERNEL_OF = {"pp_lm_presort": "ppmi::k_lm_keys<unsigned int>", "pp_fwd_tof_lm_gather": "ppmi::k_fwd_tof_lm<2, false, true>",
             "pp_back_tof_lm": "ppmi::k_back_runs<ppmi::ModeTofLm<2, false, false> >"}


def profiled_traffic(entry):
    """HBM bytes per launch of the listmode-step kernel behind `entry` (see profiled_kernel_bytes)."""
    return profiled_kernel_bytes("lm", KERNEL_OF.get(entry, ""))


def kernel_short_name(name):
    """'void ns::k<T>(args...)' -> 'ns::k<T>'."""
    name = name.strip()
    if name.startswith("void "):
        name = name[5:]
    return name.split("(", 1)[0]


def write_traffic(fetch_csv, write_csv, which="lm", copy_bytes=1 << 30):
    """Turn two rocprofv3 counter-collection CSVs (FETCH_SIZE, WRITE_SIZE; KiB per dispatch) of
    `bench.py --only lm` (which="lm") or `--only sino` (which="sino") into the traffic record: per
    library kernel the mean KiB per launch, scaled to bytes by what the same counters read for the
    run's 1 GiB device copy."""
    import csv

    def per_kernel(path, counter):
        acc = {}
        for row in csv.DictReader(open(path)):
            if row["Counter_Name"] != counter:
                continue
            acc.setdefault(kernel_short_name(row["Kernel_Name"]), []).append(float(row["Counter_Value"]))
        return acc

    fe, wr = per_kernel(fetch_csv, "FETCH_SIZE"), per_kernel(write_csv, "WRITE_SIZE")
    copy = [k for k in fe if "copyBuffer" in k]
    if not copy:
        raise SystemExit("no device copy kernel in the counter file")
    cf, cw = max(max(fe[k]) for k in copy), max(max(wr[k]) for k in copy)
    fs, ws = copy_bytes / (cf * 1024.0), copy_bytes / (cw * 1024.0)
    kernels = {}
    for k in sorted(set(fe) & set(wr)):
        if k.startswith("ppmi::"):
            f, w = sum(fe[k]) / len(fe[k]), sum(wr[k]) / len(wr[k])
            kernels[k] = {"fetch_kib": f, "write_kib": w, "launches": len(fe[k]),
                          "traffic_bytes": 1024.0 * (f * fs + w * ws)}
    path, sources = traffic_record(which)
    rec = {"kernels": kernels, "copy_bytes": copy_bytes, "copy_fetch_kib": cf, "copy_write_kib": cw,
           "fetch_scale": fs, "write_scale": ws, "source_sha256": kernel_sources_sha(sources),
           "sources": ["paper_2212_12519_amd/csrc/" + f for f in sources]}
    with open(path, "w") as fh:
        json.dump(rec, fh, indent=1)
    print(json.dumps(rec, indent=1))


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--events", type=int, default=None, help="override the 40M-event workload (testing only)")
    ap.add_argument("--no-sino", action="store_true", help="skip the sinogram legs")
    ap.add_argument("--no-serve", action="store_true", help="skip the OSEM serving leg")
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    ap.add_argument("--cpu-seconds", type=float, default=25.0, help="calibrated oracle time for the CPU baseline")
    ap.add_argument("--only", default=None, help="profiling helper: lm | sino | sino_osem | res | serve | autograd")
    ap.add_argument("--serve-requests", type=int, default=None, help="requests in the serving leg (default 256)")
    ap.add_argument("--no-res", action="store_true", help="serving leg without the resolution model")
    ap.add_argument("--write-traffic", nargs="+", metavar="ARG", default=None,
                    help="no GPU work: FETCH_CSV WRITE_CSV [lm|sino] -- write the traffic record from two "
                         "rocprofv3 counter CSVs of --only lm (default) or --only sino")
    return ap.parse_args()


def timed_phases(phases, reset, steps, warmup):
    """Per step: reset(), then each phase in turn, each bracketed by HIP events on the
    current stream.  Returns (wall seconds over `steps`, [mean ms per phase])."""
    import torch

    for _ in range(warmup):
        reset()
        for f in phases:
            f()
    torch.cuda.synchronize()
    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(len(phases) + 1)] for _ in range(steps)]
    t0 = time.perf_counter()
    for e in evs:
        reset()
        e[0].record()
        for j, f in enumerate(phases):
            f()
            e[j + 1].record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = [sum(e[j].elapsed_time(e[j + 1]) for e in evs) / steps for j in range(len(phases))]
    return wall, ms


def timed_pairs(fn_a, fn_b, reset, steps, warmup):
    wall, (ta, tb) = timed_phases([fn_a, fn_b], reset, steps, warmup)
    return wall, ta, tb


def lm_leg(args, pp, C, dev):
    import torch

    from synth import generate_tof_lm_events

    n_ev = args.events or C.N_EVENTS_LM
    grid, tofs = C.GRID_CLIN, C.TOF_CLIN
    img = C.phantom_clin(device=dev)
    t0 = time.perf_counter()
    xs, xe, bins, pair = generate_tof_lm_events(C.SCANNER_CLIN, C.SINO_CLIN.n_rad, C.SINO_CLIN.max_rd, grid, img,
                                                n_ev, seed=C.SEED_EVENTS, tof_bin_width=tofs.bin_width,
                                                tof_sigma=tofs.sigma, n_tof_bins=tofs.n_bins, device=dev,
                                                return_crystals=True)
    torch.cuda.synchronize()
    log(f"generated {n_ev} events in {time.perf_counter() - t0:.1f} s")
    G = pp.ImageGeom(grid.dim, grid.voxsize, grid.origin)
    T = pp.TofParams(tofs.bin_width, tofs.sigma, tofs.n_sigmas, tofs.n_bins)
    n_samples = int(pp.count_samples(xs, xe, G, bins, T).sum(dtype=torch.int64).item())
    p = torch.empty(n_ev, dtype=torch.float32, device=dev)
    bimg = torch.empty(grid.dim, dtype=torch.float32, device=dev)
    order = torch.empty(n_ev, dtype=torch.int32, device=dev)
    sort_ws = pp.presort_workspace(n_ev, dev)

    # one step: presort the unsorted batch; forward project in that order, the projection also writing
    # the events and their values in that order (the gather fused into the forward, which reads every
    # event anyway); back project those copies, which the back projection then reads contiguously
    xs_s, xe_s, bins_s, p_s = torch.empty_like(xs), torch.empty_like(xe), torch.empty_like(bins), torch.empty_like(p)
    wall, (t_sort, t_fwd, t_back) = timed_phases(
        [lambda: pp.pp_lm_presort(xs, xe, bins, G, T, order, sort_ws),
         lambda: pp.pp_fwd_tof_lm_gather(xs, xe, bins, G, T, img, p, order, xs_s, xe_s, bins_s, p_s),
         lambda: pp.pp_back_tof_lm(xs_s, xe_s, bins_s, G, T, bimg, p_s)],
        lambda: pp.pp_fill(bimg, 0.0), args.steps, args.warmup)
    del xs_s, xe_s, bins_s, p_s
    # the same projector pair in the events' own (unsorted) order (skipped when profiling the step)
    t_fwd_u = t_back_u = float("nan")
    crys, per_ray, nontof, gathered = {}, {}, {}, {}
    if args.only is None:
        _, t_fwd_u, t_back_u = timed_pairs(lambda: pp.pp_fwd_tof_lm(xs, xe, bins, G, T, img, p),
                                           lambda: pp.pp_back_tof_lm(xs, xe, bins, G, T, bimg, p),
                                           lambda: pp.pp_fill(bimg, 0.0), 2, 1)
        # the same step on crystal-index events (8 instead of 24 bytes of geometry per event)
        table = C.SCANNER_CLIN.crystal_table(device=dev)
        wall_c, (cs, cf, cb) = timed_phases(
            [lambda: pp.pp_lm_presort_crystals(table, pair, bins, G, T, order, sort_ws),
             lambda: pp.pp_fwd_tof_lm_crystals(table, pair, bins, G, T, img, p, order),
             lambda: pp.pp_back_tof_lm_crystals(table, pair, bins, G, T, bimg, p, order)],
            lambda: pp.pp_fill(bimg, 0.0), 3, 1)
        crys = {"t_presort_ms": cs, "t_fwd_ms": cf, "t_back_ms": cb, "events_per_s": n_ev / (wall_c / 3)}
        log(f"TOF-LM crystal-index events: presort {cs:.2f} ms, fwd {cf:.2f} ms, back {cb:.2f} ms")
        # the same projector pair with a sigma and a centre offset per event (presorted order)
        from synth import tof_per_ray_params

        sig, off = tof_per_ray_params(n_ev, tofs.sigma, seed=C.SEED_EVENTS + 1000, device=dev)
        TP = pp.TofParams(tofs.bin_width, tofs.sigma, tofs.n_sigmas, tofs.n_bins, sigma_per_ray=sig,
                          offset_per_ray=off)
        pp.pp_lm_presort(xs, xe, bins, G, T, order, sort_ws)
        _, pf, pb = timed_pairs(lambda: pp.pp_fwd_tof_lm(xs, xe, bins, G, TP, img, p, order),
                                lambda: pp.pp_back_tof_lm(xs, xe, bins, G, TP, bimg, p, order),
                                lambda: pp.pp_fill(bimg, 0.0), 3, 1)
        per_ray = {"t_fwd_ms": pf, "t_back_ms": pb}
        log(f"TOF-LM per-event sigma and offset: fwd {pf:.2f} ms, back {pb:.2f} ms")
        del sig, off, TP
        # non-TOF listmode on the same events (the paper's slowest GPU case): presort without
        # TOF bins, forward and back projection of the whole chord
        n_samples_nt = int(pp.count_samples(xs, xe, G).sum(dtype=torch.int64).item())
        wall_n, (ns_, nf, nb_) = timed_phases(
            [lambda: pp.pp_lm_presort(xs, xe, None, G, None, order, sort_ws),
             lambda: pp.pp_fwd(xs, xe, G, img, p, order),
             lambda: pp.pp_back(xs, xe, G, bimg, p, order)],
            lambda: pp.pp_fill(bimg, 0.0), 5, 2)
        alg_nt = (24 + 4) * n_ev + 16 * n_samples_nt
        nontof = {"t_presort_ms": ns_, "t_fwd_ms": nf, "t_back_ms": nb_, "events_per_s": n_ev / (wall_n / 5),
                  "samples_per_event": n_samples_nt / n_ev, "fwd_alg_gbs": alg_nt / (nf * 1e-3) / 1e9,
                  "back_alg_gbs": alg_nt / (nb_ * 1e-3) / 1e9}
        log(f"non-TOF LM: presort {ns_:.2f} ms, fwd {nf:.2f} ms, back {nb_:.2f} ms, "
            f"{n_samples_nt / n_ev:.1f} samples/event")
        # the events stored in presorted order once (pp_gather_events), then the projector pair without
        # an order array: the regime of iterative reconstruction, where the order is reused
        pp.pp_lm_presort(xs, xe, bins, G, T, order, sort_ws)
        xs_g, xe_g, bins_g = pp.gather_events(xs, xe, bins, order)
        _, t_gather, _ = timed_pairs(lambda: pp.pp_gather_events(xs, xe, bins, order, xs_g, xe_g, bins_g),
                                     lambda: None, lambda: None, 3, 1)
        wall_g, gf, gb = timed_pairs(lambda: pp.pp_fwd_tof_lm(xs_g, xe_g, bins_g, G, T, img, p),
                                     lambda: pp.pp_back_tof_lm(xs_g, xe_g, bins_g, G, T, bimg, p),
                                     lambda: pp.pp_fill(bimg, 0.0), 5, 1)
        gathered = {"t_gather_ms": t_gather, "t_fwd_ms": gf, "t_back_ms": gb, "events_per_s_fwd_back": n_ev / (wall_g / 5)}
        log(f"TOF-LM on events stored in presorted order: gather {t_gather:.2f} ms (once), fwd {gf:.2f} ms, "
            f"back {gb:.2f} ms")
        del xs_g, xe_g, bins_g
    log(f"TOF-LM: presort {t_sort:.2f} ms, fwd {t_fwd:.2f} ms, back {t_back:.2f} ms, wall "
        f"{1e3 * wall / args.steps:.2f} ms/step; unsorted order: fwd {t_fwd_u:.2f} ms back {t_back_u:.2f} ms; "
        f"{n_samples / n_ev:.1f} samples/event")
    per_event = 24 + 2 + 4  # endpoints, bin, projection value
    alg_bytes = per_event * n_ev + 16 * n_samples
    dom_name, dom_ms = ("pp_back_tof_lm", t_back) if t_back >= t_fwd else ("pp_fwd_tof_lm_gather", t_fwd)
    achieved = alg_bytes / (dom_ms * 1e-3) / 1e9
    res = {
        "n_events": n_ev, "wall_s": wall, "t_presort_ms": t_sort, "t_fwd_ms": t_fwd, "t_back_ms": t_back,
        "unsorted_t_fwd_ms": t_fwd_u, "unsorted_t_back_ms": t_back_u,
        "samples_per_event": n_samples / n_ev, "alg_bytes_per_launch": alg_bytes,
        "dominant": dom_name, "achieved_gbs": achieved,
        "fwd_alg_gbs": alg_bytes / (t_fwd * 1e-3) / 1e9, "back_alg_gbs": alg_bytes / (t_back * 1e-3) / 1e9,
        "crystal_index_events": crys, "per_event_tof_params": per_ray, "nontof_listmode": nontof,
        "presorted_events_stored": gathered,
    }
    return res, (xs, xe, bins, img, G, T)


def resmodel_leg(args, pp, C, dev):
    """The resolution model's separable Gaussian (pp_gauss3d, 4.5 mm FWHM) on the clinical grid and
    the 128 x 128 x 64 serving grid.  Two byte counts: the three separable passes, each reading and
    writing the image (24 B per voxel), and the image read and written once (8 B per voxel, what
    any implementation must move)."""
    import torch

    from paper_2212_12519_amd.osem import RES_FWHM_MM

    out = {}
    for name, grid in (("clinical_215x215x71", C.GRID_CLIN), ("serving_128x128x64", C.GRID_DL)):
        G = pp.ImageGeom(grid.dim, grid.voxsize, grid.origin)
        src = torch.rand(grid.dim, generator=torch.Generator().manual_seed(5)).to(dev)
        dst, tmp = torch.empty_like(src), torch.empty_like(src)
        fwhm = (RES_FWHM_MM,) * 3
        _, t, _ = timed_pairs(lambda: pp.pp_gauss3d(src, dst, tmp, G, fwhm), lambda: None, lambda: None, 20, 3)
        alg = 3 * 8 * src.numel()
        once = 8 * src.numel()
        out[name] = {"t_ms": t, "alg_bytes": alg, "alg_gbs": alg / (t * 1e-3) / 1e9,
                     "alg_frac": alg / (t * 1e-3) / 1e9 / HBM_PEAK_GBS,
                     "compulsory_bytes": once, "compulsory_frac": once / (t * 1e-3) / 1e9 / HBM_PEAK_GBS}
        log(f"resolution model {name}: {t * 1e3:.1f} us, {alg / (t * 1e-3) / 1e9:.0f} GB/s (3 passes), "
            f"{once / (t * 1e-3) / 1e9:.0f} GB/s (image read + written once)")
    return out


def cpu_leg(args, lm_inputs, C):
    import numpy as np

    import oracle

    xs, xe, bins, img, G, T = lm_inputs
    tof = {"bin_width": T.bin_width, "sigma": T.sigma, "n_sigmas": T.n_sigmas, "n_bins": T.n_bins}
    img64 = img.cpu().numpy().astype(np.float64)
    g = C.GRID_CLIN

    def run(n):
        a, b, c = xs[:n].cpu().numpy(), xe[:n].cpu().numpy(), bins[:n].cpu().numpy()
        t0 = time.perf_counter()
        pv = oracle.fwd_tof_lm(a, b, g.origin, g.voxsize, g.dim, tof, c, img64)
        oracle.back_tof_lm(a, b, g.origin, g.voxsize, g.dim, tof, c, pv)
        return time.perf_counter() - t0

    n0 = 500_000
    t_cal = run(n0)
    n = int(min(xs.shape[0], max(n0, n0 * args.cpu_seconds / max(t_cal, 1e-6))))
    dt = run(n)
    log(f"oracle: {n} events fwd+back in {dt:.1f} s on {oracle.max_threads()} threads")
    return {"value": n / dt, "unit": "events/s", "cores": oracle.max_threads(), "kind": "oracle",
            "sample": f"first {n} of the {xs.shape[0]} events, TOF-LM fwd+back, FP64 C/OpenMP oracle"}


def sino_leg(args, pp, C, dev):
    import torch

    grid = C.GRID_CLIN
    G = pp.ImageGeom(grid.dim, grid.voxsize, grid.origin)
    t0 = time.perf_counter()
    xs, xe = C.SINO_CLIN.lors(device=dev, radial_chunk=25)
    img = C.phantom_clin(device=dev)
    n = xs.shape[0]
    torch.cuda.synchronize()
    log(f"generated {n} sinogram LORs in {time.perf_counter() - t0:.1f} s")
    n_samples = int(pp.count_samples(xs, xe, G).sum(dtype=torch.int64).item())
    out = {}
    p = torch.empty(n, dtype=torch.float32, device=dev)
    bimg = torch.empty(grid.dim, dtype=torch.float32, device=dev)
    reps = max(2, min(args.steps, 3))
    wall, tf, tb = timed_pairs(lambda: pp.pp_fwd(xs, xe, G, img, p), lambda: pp.pp_back(xs, xe, G, bimg, p),
                               lambda: pp.pp_fill(bimg, 0.0), reps, 1)
    alg = (24 + 4) * n + 16 * n_samples

    def measured(key, t_ms):
        b = profiled_kernel_bytes("sino", SINO_KERNELS[key])
        return (None, None) if b is None else (b / (t_ms * 1e-3) / 1e9, b / (t_ms * 1e-3) / 1e9 / HBM_PEAK_GBS)

    mf, mff = measured("nontof_fwd", tf)
    mb, mbf = measured("nontof_back", tb)
    out["nontof"] = {"n_lors": n, "t_fwd_ms": tf, "t_back_ms": tb, "lors_per_s_fwd_back": n / ((tf + tb) * 1e-3),
                     "samples_per_lor": n_samples / n, "fwd_alg_gbs": alg / (tf * 1e-3) / 1e9,
                     "fwd_alg_frac": alg / (tf * 1e-3) / 1e9 / HBM_PEAK_GBS,
                     "fwd_hbm_measured_gbs": mf, "fwd_hbm_measured_frac": mff,
                     "back_alg_gbs": alg / (tb * 1e-3) / 1e9, "back_hbm_measured_gbs": mb,
                     "back_hbm_measured_frac": mbf}
    log(f"sino non-TOF: fwd {tf:.1f} ms back {tb:.1f} ms")
    del p
    tofs = C.TOF_CLIN
    T = pp.TofParams(tofs.bin_width, tofs.sigma, tofs.n_sigmas, tofs.n_bins)
    pt = torch.empty((n, tofs.n_bins), dtype=torch.float32, device=dev)
    wall, tf, tb = timed_pairs(lambda: pp.pp_fwd_tof_sino(xs, xe, G, T, img, pt),
                               lambda: pp.pp_back_tof_sino(xs, xe, G, T, bimg, pt),
                               lambda: pp.pp_fill(bimg, 0.0), reps, 1)
    alg_t = (24 + 4 * tofs.n_bins) * n + 16 * n_samples
    mf, mff = measured("tof_fwd", tf)
    mb, mbf = measured("tof_back", tb)
    out["tof_sino"] = {"n_lors": n, "n_bins": tofs.n_bins, "t_fwd_ms": tf, "t_back_ms": tb,
                       "lors_per_s_fwd_back": n / ((tf + tb) * 1e-3), "fwd_alg_gbs": alg_t / (tf * 1e-3) / 1e9,
                       "fwd_alg_frac": alg_t / (tf * 1e-3) / 1e9 / HBM_PEAK_GBS,
                       "fwd_hbm_measured_gbs": mf, "fwd_hbm_measured_frac": mff,
                       "back_hbm_measured_gbs": mb, "back_hbm_measured_frac": mbf}
    log(f"sino TOF: fwd {tf:.1f} ms back {tb:.1f} ms")
    del pt, xs, xe
    torch.cuda.empty_cache()
    return out


def autograd_leg(args, pp, C, dev, lm_inputs):
    """Batch of 8 images 128 x 128 x 64 (2.78 mm) through the TOF listmode projector inside
    torch.autograd with the Poisson NLL (background 0.1, y = 1 per event): one step = forward
    projection of the batch, the loss, and its backward (the back projection of the batch).
    Events are presorted once when the operator is built."""
    import torch

    from paper_2212_12519_amd.autograd import JosephOperator, poisson_nll
    from synth.phantom import ellipsoid_lesion_phantom

    xs, xe, bins, _, _, T = lm_inputs
    grid = C.GRID_DL
    G = pp.ImageGeom(grid.dim, grid.voxsize, grid.origin)
    imgs = torch.stack([ellipsoid_lesion_phantom(grid, seed=s, device=dev) for s in C.SEEDS_DL_IMAGES])
    op = JosephOperator(xs, xe, G, kind="tof_lm", tof=T, tof_bin=bins, presort=True)
    y = torch.ones((imgs.shape[0], op.n), dtype=torch.float32, device=dev)
    state = {}

    def fwd():
        x = imgs.clone().requires_grad_(True)
        state["x"], state["loss"] = x, poisson_nll(op(x), y, C.BG_DL)

    def bwd():
        state["loss"].backward()

    steps = max(2, min(args.steps, 5))
    wall, (tf, tb) = timed_phases([fwd, bwd], lambda: None, steps, 1)
    n_img = imgs.shape[0]
    res = {"batch": n_img, "image": list(grid.dim), "n_events": op.n, "t_forward_ms": tf, "t_backward_ms": tb,
           "ms_per_step": 1e3 * wall / steps, "image_events_per_s": n_img * op.n / (wall / steps)}
    log(f"autograd batch of {n_img}: forward+loss {tf:.1f} ms, backward {tb:.1f} ms, "
        f"{n_img * op.n / (wall / steps) / 1e6:.0f} M image-events/s")
    del op, imgs, y, state
    torch.cuda.empty_cache()
    return res


def sino_osem_leg(args, pp, C, dev):
    """TOF sinogram OSEM on the full clinical sinogram (335,008,000 LORs x 29 bins): 8 view subsets
    (view mod 8), counts y = the TOF forward projection of the phantom (expected counts), one
    iteration = 8 subset updates, each in chunks of 2^22 LORs through a 0.49 GB workspace, with
    1 shard (the plain path) and 4 shards (four private accumulator images summed in the update
    pass).  Reports s per iteration and the peak device memory of the leg."""
    import torch

    from paper_2212_12519_amd import sino_osem

    grid, tofs = C.GRID_CLIN, C.TOF_CLIN
    G = pp.ImageGeom(grid.dim, grid.voxsize, grid.origin)
    T = pp.TofParams(tofs.bin_width, tofs.sigma, tofs.n_sigmas, tofs.n_bins)
    n_sub, work_lors = 8, 1 << 22
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    torch.cuda.reset_peak_memory_stats(dev)
    base = torch.cuda.memory_allocated(dev)
    img = C.phantom_clin(device=dev)
    work = torch.empty((work_lors, tofs.n_bins), dtype=torch.float32, device=dev)
    subsets = []
    for j in range(n_sub):
        xs, xe = C.SINO_CLIN.lors(views=list(range(j, C.SINO_CLIN.shape[1], n_sub)), device=dev, radial_chunk=50)
        y = torch.empty((xs.shape[0], tofs.n_bins), dtype=torch.float32, device=dev)
        for a in range(0, xs.shape[0], work_lors):
            b = min(xs.shape[0], a + work_lors)
            pp.pp_fwd_tof_sino(xs[a:b], xe[a:b], G, T, img, y[a:b])
        subsets.append((xs, xe, y))
    n = sum(s[0].shape[0] for s in subsets)
    t0 = time.perf_counter()
    _, sens = sino_osem.tof_sino_osem(subsets, G, T, torch.ones(grid.dim, device=dev), 0, work_lors=work_lors)
    torch.cuda.synchronize()
    t_sens = time.perf_counter() - t0
    out = {"n_lors": n, "n_bins": tofs.n_bins, "subsets": n_sub, "work_lors": work_lors, "t_sensitivity_s": t_sens}
    for shards in (1, 4):
        x = torch.ones(grid.dim, dtype=torch.float32, device=dev)
        acc = torch.zeros((shards,) + tuple(grid.dim), dtype=torch.float32, device=dev)

        def iteration():
            for (xs, xe, y), s in zip(subsets, sens):
                sino_osem.pp_tof_sino_osem_subset(xs, xe, y, G, T, 0.0, x, acc, s, work)

        reps = 2
        wall, (t_it,) = timed_phases([iteration], lambda: None, reps, 1)
        out[f"shards_{shards}"] = {"s_per_iteration": t_it * 1e-3, "lors_per_s": n / (t_it * 1e-3)}
        log(f"TOF-sino OSEM, {shards} shard(s): {t_it:.1f} ms per iteration (8 subsets)")
    out["peak_device_gb"] = (torch.cuda.max_memory_allocated(dev) - base) / 1e9
    out["resident_data_gb"] = sum(s[0].numel() * 8 + s[2].numel() * 4 for s in subsets) / 1e9
    log(f"TOF-sino OSEM peak device memory {out['peak_device_gb']:.1f} GB "
        f"(LORs + counts {out['resident_data_gb']:.1f} GB)")
    del subsets, sens, work, img
    torch.cuda.empty_cache()
    return out


def main():
    args = parse()
    if args.write_traffic:
        if len(args.write_traffic) not in (2, 3) or args.write_traffic[2:] not in ([], ["lm"], ["sino"]):
            raise SystemExit("--write-traffic FETCH_CSV WRITE_CSV [lm|sino]")
        write_traffic(*args.write_traffic)
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (got --gpus {args.gpus}); the library has no multi-GPU path.",
              file=sys.stderr)
        sys.exit(2)
    import torch

    import paper_2212_12519_amd as pp
    from synth import configs as C

    pp.load()
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    result = {"metric": "TOF listmode fwd+back events/s + OSEM frame p50/p99 latency vs plain"}
    extra = {}
    lm = lm_inputs = None
    if args.only in (None, "lm", "autograd"):
        lm, lm_inputs = lm_leg(args, pp, C, dev)
    if args.only is not None:
        # a plain device copy of known size (1 GiB read + 1 GiB written), so hardware byte
        # counters collected on a profiling run can be scaled to bytes
        src = torch.ones(1 << 28, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        extra["calibration_copy_bytes"] = src.numel() * 4
        del src, dst
    if args.only == "lm":
        print(json.dumps({"lm": lm, **extra}))
        return
    if args.only in (None, "sino") and not args.no_sino:
        extra["sinogram"] = sino_leg(args, pp, C, dev)
    if args.only in (None, "sino_osem") and not args.no_sino:
        extra["tof_sino_osem"] = sino_osem_leg(args, pp, C, dev)
    if args.only in ("sino", "sino_osem"):
        print(json.dumps(extra))
        return
    if args.only in (None, "autograd"):
        extra["autograd"] = autograd_leg(args, pp, C, dev, lm_inputs)
    if args.only == "autograd":
        print(json.dumps(extra))
        return
    if args.only in (None, "res"):
        extra["resolution_model"] = resmodel_leg(args, pp, C, dev)
    if args.only == "res":
        print(json.dumps(extra))
        return
    if args.only in (None, "serve") and not args.no_serve:
        from paper_2212_12519_amd import serve

        extra["osem_serving"] = serve.bench_leg(args, log)
    if args.only == "serve":
        print(json.dumps(extra))
        return
    cpu = None
    if not args.no_cpu and lm_inputs is not None:
        cpu = cpu_leg(args, lm_inputs, C)
    value = lm["n_events"] * args.steps / lm["wall_s"]
    ach = lm["achieved_gbs"]
    result.update({
        "value": value, "unit": "events/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": 1e3 * lm["wall_s"] / args.steps, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "TOF listmode fwd+back, 40M unsorted events (step = presort + fwd writing the events in "
                               "processing order + back of those), clinical "
                               "phantom 215x215x71 @ 1.65x1.65x2.0 mm, 29 TOF bins x 28 mm, FWHM 58.5 mm, 3 sigma",
                   "n_events": lm["n_events"], "image": list(C.GRID_CLIN.dim), "tof_bins": C.TOF_CLIN.n_bins},
        "roofline": {"bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": ach / HBM_PEAK_GBS, "traffic": profiled_traffic(lm["dominant"]), "entry": lm["dominant"],
                     "kernel": KERNEL_OF[lm["dominant"]],
                     "alg_bytes_per_launch": lm["alg_bytes_per_launch"]},
        "cpu_baseline": cpu,
        "lm": {k: lm[k] for k in ("t_presort_ms", "t_fwd_ms", "t_back_ms", "unsorted_t_fwd_ms", "unsorted_t_back_ms",
                                  "samples_per_event", "fwd_alg_gbs", "back_alg_gbs", "nontof_listmode")},
    })
    result.update(extra)
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
