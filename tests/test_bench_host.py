"""Host-side checks of bench.py (no GPU): the one-GPU contract and the traffic record that turns
hardware byte counters into bytes per launch."""
import csv
import importlib.util
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def load_bench():
    spec = importlib.util.spec_from_file_location("bench_under_test", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_bench_measures_one_gpu_only():
    """--gpus N > 1 exits with status 2 and says why, before touching a GPU."""
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], cwd=ROOT,
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def _counter_csv(path, counter, rows):
    with open(path, "w", newline="") as fh:
        w = csv.DictWriter(fh, fieldnames=["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"])
        w.writeheader()
        for i, (name, value) in enumerate(rows):
            w.writerow({"Dispatch_Id": i, "Kernel_Name": name, "Counter_Name": counter, "Counter_Value": value})


def test_traffic_record_scales_counters_by_the_copy(tmp_path, monkeypatch):
    """Counters in KiB per dispatch, scaled by what they read for a 1 GiB copy: the copy's fetch reads
    half its bytes (scale 2), its write all of them (scale 1); a kernel's traffic is the mean over its
    launches, fetch and write each scaled."""
    bench = load_bench()
    monkeypatch.setattr(bench, "TRAFFIC_JSON", str(tmp_path / "traffic.json"))
    back = "void " + bench.KERNEL_OF["pp_back_tof_lm"] + "(ppmi::ModeTofLm<false, false>, ...)"
    copy = "__amd_rocclr_copyBuffer(unsigned char*, ...)"
    fetch, write = tmp_path / "f.csv", tmp_path / "w.csv"
    _counter_csv(fetch, "FETCH_SIZE", [(copy, 524288.0), (back, 900.0), (back, 1100.0)])
    _counter_csv(write, "WRITE_SIZE", [(copy, 1048576.0), (back, 400.0), (back, 600.0)])
    bench.write_traffic(str(fetch), str(write))
    rec = json.load(open(tmp_path / "traffic.json"))
    assert rec["fetch_scale"] == 2.0 and rec["write_scale"] == 1.0
    k = rec["kernels"][bench.KERNEL_OF["pp_back_tof_lm"]]
    assert k["launches"] == 2
    assert k["traffic_bytes"] == 1024.0 * (1000.0 * 2.0 + 500.0 * 1.0)
    assert rec["source_sha256"] == bench.kernel_sources_sha()


def test_sino_traffic_record_and_lookup(tmp_path, monkeypatch):
    """The sinogram record keeps every library kernel of the counter files (not the copy), and a
    lookup returns its bytes while the sinogram kernels' sources are unchanged, None otherwise."""
    bench = load_bench()
    monkeypatch.setattr(bench, "SINO_TRAFFIC_JSON", str(tmp_path / "sino.json"))
    fwd = "void " + bench.SINO_KERNELS["tof_fwd"] + "(ppmi::RaySrc, ...)"
    copy = "__amd_rocclr_copyBuffer(unsigned char*, ...)"
    fetch, write = tmp_path / "f.csv", tmp_path / "w.csv"
    _counter_csv(fetch, "FETCH_SIZE", [(copy, 524288.0), (fwd, 300.0)])
    _counter_csv(write, "WRITE_SIZE", [(copy, 1048576.0), (fwd, 100.0)])
    bench.write_traffic(str(fetch), str(write), "sino")
    rec = json.load(open(tmp_path / "sino.json"))
    assert list(rec["kernels"]) == [bench.SINO_KERNELS["tof_fwd"]]
    assert bench.profiled_kernel_bytes("sino", bench.SINO_KERNELS["tof_fwd"]) == 1024.0 * (300.0 * 2.0 + 100.0)
    rec["source_sha256"] = "stale"
    json.dump(rec, open(tmp_path / "sino.json", "w"))
    assert bench.profiled_kernel_bytes("sino", bench.SINO_KERNELS["tof_fwd"]) is None
