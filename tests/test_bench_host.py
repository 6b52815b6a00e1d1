"""Host-side measurement code (no GPU): the bench line's roofline object,
the gate on the committed counter summary, the counter scaling of
bench_traffic.py and the bench's FP64 oracle baseline."""
import csv
import json
import math
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402

PROFILE = os.path.join(ROOT, "profiles", "multistep_kernel_cyl_d160.md")


def _profile_bench_line():
    for line in open(PROFILE):
        if line.startswith('{"metric"'):
            return json.loads(line)
    raise AssertionError("no bench line in the profile")


def test_roofline_reproduces_the_committed_d160_profile():
    """The roofline fields of the profile's bench line follow from its stored
    counter summary and its live launch time (rounded to 0.01 us there)."""
    line = _profile_bench_line()
    stated = line["roofline"]
    counters = json.load(open(bench.TRAFFIC_FILE))
    assert counters["kernel_sha256_16"] in stated["counters"]
    nodes = line["config"]["nx"] * line["config"]["ny"]
    roof = bench.roofline(nodes, stated["steps_per_launch"], stated["launch_us"] * 1e-6, counters)
    assert roof["traffic"] == stated["traffic"] == counters["bytes_per_launch"]
    assert roof["floor_bytes_per_launch"] == stated["floor_bytes_per_launch"] == 72 * nodes
    for k in ("achieved", "frac", "frac_of_floor", "traffic_over_floor", "effective_GBs"):
        assert math.isclose(roof[k], stated[k], rel_tol=2e-4), k
    for k in ("fp32_TFLOPs", "frac"):
        assert math.isclose(roof["valu"][k], stated["valu"][k], rel_tol=2e-3), k
    # the fraction is of the physical traffic, so it cannot pass the peak
    assert roof["frac"] <= 1.0 and roof["frac_of_floor"] <= roof["frac"]
    # the per-update accounting passes it once steps share a pass
    assert roof["effective_GBs"] > bench.PEAK_HBM_GBS


def test_roofline_without_counters_reports_only_the_floor():
    roof = bench.roofline(1000, 4, 1e-6, None)
    assert roof["achieved"] is None and roof["frac"] is None and roof["traffic"] is None
    assert roof["floor_bytes_per_launch"] == 72000
    assert math.isclose(roof["frac_of_floor"], 72000 / 1e-6 / 1e9 / bench.PEAK_HBM_GBS, rel_tol=1e-3)
    assert math.isclose(roof["effective_GBs"], 4 * 72000 / 1e-6 / 1e9, rel_tol=1e-3)
    assert roof["kernel"] == "multistep_kernel" and "stale" in roof["counters"]
    assert bench.roofline(1000, 1, 1e-6, None)["kernel"] == "step_kernel"
    assert bench.roofline(1000, 2, 1e-6, None)["kernel"] == "step2_kernel"


def test_stored_counters_only_for_the_current_source_and_configuration(tmp_path, monkeypatch):
    good = {"kernel_sha256_16": bench.kernel_hash(), "workload": "cyl_d160", "collision": "bgk",
            "variant": "t4_h10u_s10", "bytes_per_launch": 123}
    path = tmp_path / "traffic.json"
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(path))
    assert bench.stored_counters("cyl_d160", "bgk", "t4_h10u_s10") is None  # no file
    path.write_text(json.dumps(good))
    assert bench.stored_counters("cyl_d160", "bgk", "t4_h10u_s10")["bytes_per_launch"] == 123
    for key, other in (("workload", "cyl_d80"), ("collision", "mrt"), ("variant", "t4_h8_s8")):
        args = {"workload": "cyl_d160", "collision": "bgk", "variant": "t4_h10u_s10", key: other}
        assert bench.stored_counters(args["workload"], args["collision"], args["variant"]) is None, key
    path.write_text(json.dumps(dict(good, kernel_sha256_16="0" * 16)))
    assert bench.stored_counters("cyl_d160", "bgk", "t4_h10u_s10") is None
    path.write_text("not json")
    assert bench.stored_counters("cyl_d160", "bgk", "t4_h10u_s10") is None


def _counter_csv(path, rows):
    with open(path, "w", newline="") as fh:
        w = csv.DictWriter(fh, fieldnames=["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"])
        w.writeheader()
        for i, (kernel, counter, value) in enumerate(rows):
            w.writerow({"Dispatch_Id": i, "Kernel_Name": kernel, "Counter_Name": counter, "Counter_Value": value})


def test_bench_traffic_scales_each_counter_by_the_copy_of_known_size(tmp_path):
    """Synthetic counter files: the copy probe reads and writes the nine FP32
    populations of every node of the lattice; FETCH_SIZE counts half its
    bytes and WRITE_SIZE all of them (KiB per dispatch), and the step kernel's
    counts are scaled by the same factors and averaged over its dispatches."""
    from lbm_inputs import WORKLOADS

    w = WORKLOADS["cyl_d10"]
    nodes = w["nx"] * w["ny"]
    copy_b = 9 * nodes * 4 - (9 * nodes * 4) % 16
    kname = "void lbm::multistep_kernel<false, 10, 10, 4, 0, 2>(lbm::StepArgs)"
    fetch, write = tmp_path / "fetch.csv", tmp_path / "write.csv"
    _counter_csv(fetch, [("copy_probe_kernel(...)", "FETCH_SIZE", 0.5 * copy_b / 1024)] * 3
                 + [(kname, "FETCH_SIZE", v) for v in (1000.0, 1100.0, 1200.0)]
                 + [("other_kernel", "FETCH_SIZE", 9e9)])
    _counter_csv(write, [("copy_probe_kernel(...)", "WRITE_SIZE", copy_b / 1024)] * 3
                 + [(kname, "WRITE_SIZE", v) for v in (2000.0, 2000.0, 2000.0)])
    out = tmp_path / "summary.json"
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench_traffic.py"), str(fetch), str(write),
                        "--workload", "cyl_d10", "--variant", "t4_h10u_s10", "--out", str(out)],
                       capture_output=True, text=True, cwd=ROOT)
    assert r.returncode == 0, r.stderr
    d = json.load(open(out))
    assert d["fetch_scale"] == pytest.approx(0.5) and d["write_scale"] == pytest.approx(1.0)
    assert d["read_bytes"] == round(1100.0 * 1024 / 0.5)
    assert d["write_bytes"] == round(2000.0 * 1024)
    assert d["bytes_per_launch"] == round(1100.0 * 1024 / 0.5 + 2000.0 * 1024)
    assert d["dispatches"] == [3, 3] and d["steps_per_launch"] == 4 and d["kernel"] == "multistep_kernel"
    assert d["state_bytes_per_launch"] == 72 * nodes and d["algorithmic_bytes_per_launch"] == 4 * 72 * nodes
    assert d["kernel_sha256_16"] == bench.kernel_hash()


def test_cpu_baseline_times_the_oracle_on_this_host(tmp_path, monkeypatch):
    """The bench's cpu_baseline leg on a small lattice with a short budget:
    the oracle built natively into a temporary library (removed afterwards),
    the head figure on every OpenMP thread, and the D = 10, 40, 80 samples on
    one thread and on all of them."""
    import tempfile

    from lbm_inputs import WORKLOADS

    monkeypatch.setattr(tempfile, "gettempdir", lambda: str(tmp_path))
    c = bench.cpu_baseline(dict(WORKLOADS["cyl_d10"]), budget_s=1.0)
    assert c["kind"] == "oracle" and c["unit"] == "MLUPS" and c["bytes_per_update"] == 144
    assert c["cores"] >= 1 and c["value"] > 0 and "410x210" in c["sample"]
    assert [(s["workload"], s["threads"]) for s in c["samples"]] == [
        (n, t) for n in ("cyl_d10", "cyl_d40", "cyl_d80") for t in (1, c["cores"])]
    assert all(s["steps"] >= 1 and s["mlups"] > 0 for s in c["samples"])
    assert c["build"].startswith("gcc ") and "-O3" in c["build"]
    assert not list(tmp_path.glob("liblbm_oracle_native_*"))
