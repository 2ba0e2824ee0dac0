"""Host logic of bench.py, on the CPU: kernel-name classification, the rocprofv3 summary built
from synthetic CSV files (durations per kind, the split last pass's alternating dispatches,
counter scaling by the copy calibration), and the source-hash gate on reported traffic."""
import csv
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402

NS = "fhtfbp::(anonymous namespace)::"


def _write_csv(path, rows):
    os.makedirs(os.path.dirname(path), exist_ok=True)
    with open(path, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=list(rows[0].keys()))
        w.writeheader()
        w.writerows(rows)


def test_kernel_kinds():
    assert bench._kind(f"void {NS}fht_first_kernel<32, 2, 16>({NS}PassArgs)") == "first"
    assert bench._kind(f"{NS}fht_image_tile_kernel(fhtfbp::PassArgs)") == "last"
    assert bench._kind(f"void {NS}fht_cols_kernel<2>(fhtfbp::PassArgs)") == "last_vh"
    assert bench._kind(f"void {NS}fht_cols_kernel<1>(fhtfbp::PassArgs)") == "middle"
    assert bench._kind("void at::native::elementwise_kernel<128, 4>(...)") is None


def test_pass_model_bytes_per_kind():
    n2 = 1024.0 * 1024
    assert bench.pass_model_bytes("first", 1024, [5, 5]) == 32 * n2
    assert bench.pass_model_bytes("last", 1024, [5, 5]) == 20 * n2
    assert bench.pass_model_bytes("last_v", 1024, [5, 4, 1]) == 12 * n2
    assert bench.pass_model_bytes("last_h", 1024, [5, 4, 1]) == 16 * n2


def _synthetic_run(d, last_names):
    """Two steps: first + last kernels, with known durations and counter values."""
    first = f"void {NS}fht_first_kernel<32, 2, 16>({NS}PassArgs)"
    seq = []
    t = 1000
    for step in range(2):
        for name, dur in [(first, 4000)] + [(nm, du) for nm, du in last_names]:
            seq.append({"Kernel_Name": name, "Start_Timestamp": t, "End_Timestamp": t + dur})
            t += dur + 10
    _write_csv(os.path.join(d, "trace", "x_kernel_trace.csv"), seq)
    _write_csv(os.path.join(d, "trace", "x_kernel_stats.csv"),
               [{"Name": first, "TotalDurationNs": 8000},
                {"Name": "elementwise", "TotalDurationNs": 8000}])
    # counters: KiB per dispatch; fetch reads half of the bytes (scale 2), write all (scale 1)
    for tag, cname, val in (("fetch", "FETCH_SIZE", 100.0), ("write", "WRITE_SIZE", 50.0)):
        rows, did = [], 0
        for _ in range(2):
            for name in [first] + [nm for nm, _ in last_names]:
                did += 1
                rows.append({"Kernel_Name": name, "Dispatch_Id": did, "Counter_Name": cname,
                             "Counter_Value": val})
        _write_csv(os.path.join(d, tag, "x_counter_collection.csv"), rows)
    gib_kib = float(1 << 20)
    _write_csv(os.path.join(d, "copyf", "x_counter_collection.csv"),
               [{"Kernel_Name": "copy_kernel", "Dispatch_Id": 1, "Counter_Name": "FETCH_SIZE",
                 "Counter_Value": gib_kib / 2}])
    _write_csv(os.path.join(d, "copyw", "x_counter_collection.csv"),
               [{"Kernel_Name": "copy_kernel", "Dispatch_Id": 1, "Counter_Name": "WRITE_SIZE",
                 "Counter_Value": gib_kib}])


def _summary_json(text):
    line = [ln for ln in text.splitlines() if ln.startswith("JSON ")][-1]
    return json.loads(line[5:])


def test_summary_fused_last_pass(tmp_path):
    last = f"{NS}fht_image_tile_kernel(fhtfbp::PassArgs)"
    _synthetic_run(str(tmp_path), [(last, 2000)])
    js = _summary_json(bench.rocprof_summary(str(tmp_path), 1024, 512, 2))
    k = js["kernels"]
    assert js["kernel_source_hash"] == bench.kernel_source_hash()
    assert k["first"]["dispatches"] == 2 and k["first"]["avg_us"] == 4.0
    assert k["last"]["dispatches"] == 2 and k["last"]["avg_us"] == 2.0
    assert js["copy_factor"] == {"fetch": 2.0, "write": 1.0}
    assert k["first"]["fetch_size_bytes"] == 100 * 1024 * 2
    assert k["first"]["write_size_bytes"] == 50 * 1024
    assert k["last"]["hbm_bytes"] == 100 * 1024 * 2 + 50 * 1024
    assert k["last"]["pass_model_bytes"] == 20 * 1024 * 1024 * 512


def test_summary_split_last_pass_alternates(tmp_path):
    vh = f"void {NS}fht_cols_kernel<2>(fhtfbp::PassArgs)"
    _synthetic_run(str(tmp_path), [(vh, 1000), (vh, 1500)])
    js = _summary_json(bench.rocprof_summary(str(tmp_path), 1024, 512, 2))
    k = js["kernels"]
    assert k["last_v"]["dispatches"] == 2 and k["last_v"]["avg_us"] == 1.0
    assert k["last_h"]["dispatches"] == 2 and k["last_h"]["avg_us"] == 1.5
    assert k["last_v"]["pass_model_bytes"] == 12 * 1024 * 1024 * 512
    assert k["last_h"]["pass_model_bytes"] == 16 * 1024 * 1024 * 512


def test_traffic_is_reported_only_for_the_current_sources(tmp_path):
    good = tmp_path / "good.txt"
    stale = tmp_path / "stale.txt"
    kern = {"first": {"hbm_bytes": 123}}
    good.write_text("header\nJSON " + json.dumps(
        {"kernel_source_hash": bench.kernel_source_hash(), "kernels": kern}) + "\n")
    stale.write_text("JSON " + json.dumps({"kernel_source_hash": "0" * 16, "kernels": kern}))
    assert bench.traffic_from_profile(str(good), "first")[0] == 123
    v, why = bench.traffic_from_profile(str(stale), "first")
    assert v is None and "changed" in why
    assert bench.traffic_from_profile(str(tmp_path / "missing.txt"), "first")[0] is None



def test_roofline_fraction_on_algorithmic_bytes():
    """The roofline's `achieved` divides the method's 20 N^2 bytes per slice (linogram read once,
    image written once) by the dominant kernel's launch time; the pass design's own byte model
    of that kernel is reported beside it, never as `achieved`."""
    n, batch, ms = 1024, 512, 3.883
    pm_gb = bench.pass_model_bytes("first", n, [5, 5]) * batch / 1e9
    r = bench.roofline_record("first", ms, n, batch, pm_gb, None, "none")
    alg = 20.0 * n * n * batch
    assert r["algorithmic_GB_per_launch"] == round(alg / 1e9, 3)
    assert abs(r["achieved"] - alg / (ms * 1e-3) / 1e9) < 0.1
    assert abs(r["frac"] - alg / (ms * 1e-3) / 1e9 / 8000.0) < 1e-4
    assert abs(r["frac"] - 0.3457) < 1e-3
    assert abs(r["pass_model_frac"] - 32.0 / 20.0 * r["frac"]) < 1e-3
    assert r["traffic"] is None and r["bound"] == "hbm"
