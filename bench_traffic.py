"""Turns two rocprofv3 counter runs of bench.py (one with --pmc FETCH_SIZE,
one with --pmc WRITE_SIZE, both with the copy reference enabled) into the
HBM-traffic summary bench.py reports as roofline.traffic.

Each counter is scaled by what it reads for the library's streaming copy of
known size, run in the same process: FETCH_SIZE and WRITE_SIZE count in
units that differ from bytes by a fixed factor on this chip.

    python bench_traffic.py FETCH_CSV WRITE_CSV --variant t2_h4 [--workload cyl_d160] [--collision bgk]
                            [--valu VALU_CSV] [--out PATH]

The variant is the one bench.py reports in config.variant for the same run.
The summary goes to the file bench.py reads (profiles/traffic_step_kernel.json)
unless --out names another (for workloads other than the default one).
With --valu, a third run's counters (SQ_INSTS_VALU, SQ_INSTS_VALU_FMA_F32,
SQ_INSTS_VALU_ADD_F32, SQ_INSTS_VALU_MUL_F32, SQ_INSTS_VALU_TRANS_F32,
SQ_ACTIVE_INST_VALU, GRBM_GUI_ACTIVE) add the vector-ALU side: FP32
operations per launch (64 lanes per wave instruction, two per FMA) and the
VALU busy percentage, 100 SQ_ACTIVE_INST_VALU / CUs / (GRBM_GUI_ACTIVE /
XCDs), the GRBM count being the sum over the XCDs.
"""
import argparse
import csv
import json
import os
import sys

import bench
from lbm_inputs import WORKLOADS


def per_dispatch(path, counter, name_part):
    vals = [float(r["Counter_Value"]) for r in csv.DictReader(open(path))
            if r["Counter_Name"] == counter and name_part in r["Kernel_Name"]]
    if not vals:
        sys.exit(f"{path}: no {counter} rows for {name_part}")
    return sum(vals) / len(vals), len(vals)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("fetch_csv")
    ap.add_argument("write_csv")
    ap.add_argument("--workload", default="cyl_d160")
    ap.add_argument("--collision", default="bgk")
    ap.add_argument("--variant", required=True)
    ap.add_argument("--valu", help="counter_collection.csv of the VALU counter run")
    ap.add_argument("--out", default=bench.TRAFFIC_FILE, help="where to write the summary")
    a = ap.parse_args()
    steps = {"t2": 2, "t3": 3, "t4": 4}.get(a.variant[:2], 1)
    kname = {1: "step_kernel<", 2: "step2_kernel"}.get(steps, "multistep_kernel")
    w = WORKLOADS[a.workload]
    nodes = w["nx"] * w["ny"]
    copy_bytes = 9 * nodes * 4
    copy_bytes -= copy_bytes % 16
    f_step, n_f = per_dispatch(a.fetch_csv, "FETCH_SIZE", kname)
    w_step, n_w = per_dispatch(a.write_csv, "WRITE_SIZE", kname)
    f_copy, _ = per_dispatch(a.fetch_csv, "FETCH_SIZE", "copy_probe_kernel")
    w_copy, _ = per_dispatch(a.write_csv, "WRITE_SIZE", "copy_probe_kernel")
    fetch_scale = f_copy * 1024 / copy_bytes
    write_scale = w_copy * 1024 / copy_bytes
    read_b = f_step * 1024 / fetch_scale
    write_b = w_step * 1024 / write_scale
    alg = bench.BYTES_PER_NODE * nodes * steps
    state = bench.BYTES_PER_NODE * nodes
    out = {
        "workload": a.workload,
        "collision": a.collision,
        "variant": a.variant,
        "kernel": kname.rstrip("<"),
        "steps_per_launch": steps,
        "kernel_sha256_16": bench.kernel_hash(),
        "dispatches": [n_f, n_w],
        "bytes_per_launch": round(read_b + write_b),
        "read_bytes": round(read_b),
        "write_bytes": round(write_b),
        # 72 B per node update, times the updates of one launch
        "algorithmic_bytes_per_launch": alg,
        # one read and one write of the nine populations of every node
        "state_bytes_per_launch": state,
        "ratio_to_state": round((read_b + write_b) / state, 4),
        "ratio_to_algorithmic": round((read_b + write_b) / alg, 4),
        "fetch_size_kib": round(f_step, 1),
        "write_size_kib": round(w_step, 1),
        "copy_probe_bytes_each_way": copy_bytes,
        "copy_fetch_kib": round(f_copy, 1),
        "copy_write_kib": round(w_copy, 1),
        "fetch_scale": round(fetch_scale, 5),
        "write_scale": round(write_scale, 5),
    }
    if a.valu:
        c = {n: per_dispatch(a.valu, n, kname)[0] for n in (
            "SQ_INSTS_VALU", "SQ_INSTS_VALU_FMA_F32", "SQ_INSTS_VALU_ADD_F32", "SQ_INSTS_VALU_MUL_F32",
            "SQ_INSTS_VALU_TRANS_F32", "SQ_ACTIVE_INST_VALU", "GRBM_GUI_ACTIVE")}
        agent = [r for r in csv.DictReader(open(os.path.join(os.path.dirname(a.valu), "run_agent_info.csv")))
                 if r["Agent_Type"] == "GPU"][0]
        cus, xcc = int(agent["Cu_Count"]), int(agent["Num_Xcc"])
        flop = 64 * (2 * c["SQ_INSTS_VALU_FMA_F32"] + c["SQ_INSTS_VALU_ADD_F32"] + c["SQ_INSTS_VALU_MUL_F32"]
                     + c["SQ_INSTS_VALU_TRANS_F32"])
        out["valu"] = {
            "counters_per_launch": {k: round(v) for k, v in c.items()},
            "cus": cus, "xcc": xcc,
            "fp32_flop_per_launch": round(flop),
            "fp32_flop_per_update": round(flop / (nodes * steps), 1),
            "valu_insts_per_update": round(64 * c["SQ_INSTS_VALU"] / (nodes * steps), 1),
            "valu_busy_pct": round(100 * c["SQ_ACTIVE_INST_VALU"] / cus / (c["GRBM_GUI_ACTIVE"] / xcc), 1),
        }
    with open(a.out, "w") as fh:
        json.dump(out, fh, indent=1)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
