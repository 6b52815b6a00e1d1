"""Throughput benchmark of the D2Q9 solver on one MI355X.

One step = one pass of the whole hot path over the lattice: pull streaming,
half-way bounce-back on the cylinder, wall/outlet/inlet corrections, the
collision (BGK by default) and the FP64 momentum-exchange force (plus its
fixed-order history reduction every 64 steps).  The default workload is the
D = 160 cylinder channel (6560 x 3360 = 22.0 M nodes, Re = 100, U = 0.05,
free-slip walls), whose two population buffers (1.6 GB) are far larger than
the 256 MB Infinity Cache.  At this size the library's default kernel takes
two steps per launch with the intermediate populations in registers.

Prints one JSON line:
  value      MLUPS = nx * ny * steps / time / 1e6 (all nodes)
  roofline   algorithmic bytes (72 B per node update: 9 FP32 loads + 9 FP32
             stores) times the node updates of the timed region, over its
             duration, against the 8 TB/s HBM3E peak; `traffic` is the HBM
             bytes per launch from the committed rocprofv3 FETCH_SIZE /
             WRITE_SIZE summary when it was taken on the current kernel
             source and configuration (else null), and `hbm_GBs` the
             bandwidth that traffic implies at the measured launch rate
  cpu_baseline  the FP64 oracle timed on this host on a bounded sample
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

BYTES_PER_NODE = 72  # 9 FP32 loads + 9 FP32 stores per node update
PEAK_HBM_GBS = 8000.0
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_step_kernel.json")
KERNEL_SRC = os.path.join(ROOT, "paper_2605_02185_amd", "csrc", "lbm_kernels.hip")


def kernel_hash() -> str:
    return hashlib.sha256(open(KERNEL_SRC, "rb").read()).hexdigest()[:16]


def stored_counters(workload: str, collision: str, variant: str):
    """The committed counter summary (HBM bytes per launch, and the vector
    ALU figures when recorded), if it was taken on the current kernel source,
    workload, collision and variant; else None."""
    try:
        d = json.load(open(TRAFFIC_FILE))
    except (OSError, ValueError):
        return None
    if (d.get("kernel_sha256_16") != kernel_hash() or d.get("workload") != workload
            or d.get("collision", "bgk") != collision or d.get("variant") != variant):
        return None
    return d


def copy_ceiling(torch, lbm, nbytes: int, reps: int = 20) -> float:
    """GB/s of the library's plain streaming copy of nbytes (read + write
    counted): the bandwidth a kernel with perfect access patterns reaches."""
    nbytes -= nbytes % 16
    a = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    lbm.copy_probe(b, a, nbytes)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        lbm.copy_probe(b, a, nbytes)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del a, b
    return 2.0 * nbytes / (ms * 1e-3) / 1e9


def cpu_baseline(w: dict, budget_s: float) -> dict:
    """The FP64 oracle, as it stands, on this host: steps of the same lattice
    until about budget_s seconds of stepping have elapsed."""
    import oracle

    o = oracle.Oracle(oracle.OracleParams(**w))
    o.step(1)  # first touch of the buffers
    steps, t0 = 0, time.perf_counter()
    while True:
        o.step(1)
        steps += 1
        el = time.perf_counter() - t0
        if el >= budget_s or steps >= 200:
            break
    nodes = w["nx"] * w["ny"]
    o.close()
    return {
        "value": nodes * steps / el / 1e6,
        "unit": "MLUPS",
        "cores": oracle.threads(),
        "kind": "oracle",
        "sample": f"{steps} steps of the {w['nx']}x{w['ny']} lattice ({el:.1f} s, FP64, OpenMP)",
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=4000)
    ap.add_argument("--warmup", type=int, default=400)
    ap.add_argument("--workload", default="cyl_d160")
    ap.add_argument("--variant", type=int, default=0)
    ap.add_argument("--collision", choices=("bgk", "mrt"), default="bgk",
                    help="collision operator: BGK (Eq. 2) or MRT with the rates of Sec. 2.1 (Eq. 6)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-budget", type=float, default=15.0)
    ap.add_argument("--no-copy", action="store_true", help="skip the copy-ceiling reference")
    ap.add_argument("--no-graphs", action="store_true", help="plain launches instead of graph replay")
    ap.add_argument("--ensemble", action="store_true",
                    help="also time the 64-case ensemble (MRT, tau from Re) against 64 separate lattices")
    ap.add_argument("--closure", action="store_true",
                    help="also train and evaluate the learned boundary closure (about a minute)")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU only (got --gpus {args.gpus}); "
              "multi-GPU slab decomposition is design-only", file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_2605_02185_amd as lbm
    from lbm_inputs import PAPER_RATES, WORKLOADS

    torch.cuda.set_device(0)
    w = dict(WORKLOADS[args.workload])
    if args.collision == "mrt":
        w.update(collision=lbm.COLLISION_MRT, s_rates=PAPER_RATES)
    else:
        w = {k: v for k, v in w.items() if k not in ("collision", "s_rates")}
    p = lbm.make_params(**w)
    nodes = w["nx"] * w["ny"]
    stream = torch.cuda.current_stream()
    lat = lbm.Lattice(p, stream=stream.cuda_stream)
    if args.variant:
        lat.set_variant(args.variant)
    lat.set_graphs(not args.no_graphs)
    lat.step(args.warmup)
    lat.sync()

    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e0.record(stream)
    lat.step(args.steps)
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    lat.sync()  # raises if the run diverged
    gpu_ms = e0.elapsed_time(e1)
    ms_per_step = gpu_ms / args.steps
    mlups = nodes * args.steps / (gpu_ms * 1e-3) / 1e6
    fluid = nodes - lbm.geometry(p)[1]

    vname = lbm.variant_name(lat.variant)
    steps_per_launch = {"t2": 2, "t3": 3, "t4": 4}.get(vname[:2], 1)
    launch_ms = ms_per_step * steps_per_launch
    achieved = BYTES_PER_NODE * nodes * steps_per_launch / (launch_ms * 1e-3) / 1e9
    counters = stored_counters(args.workload, args.collision, vname)
    traffic = counters.get("bytes_per_launch") if counters else None
    valu = counters.get("valu") if counters else None
    roof = {
        "bound": "hbm",
        "achieved": round(achieved, 1),
        "peak": PEAK_HBM_GBS,
        "unit": "GB/s",
        "frac": round(achieved / PEAK_HBM_GBS, 4),
        "traffic": traffic,
        "kernel": {1: "step_kernel", 2: "step2_kernel"}.get(steps_per_launch, "multistep_kernel"),
        "steps_per_launch": steps_per_launch,
        "launch_us": round(launch_ms * 1e3, 2),
        "algorithmic_bytes_per_launch": BYTES_PER_NODE * nodes * steps_per_launch,
        "hbm_GBs": round(traffic / (launch_ms * 1e-3) / 1e9, 1) if traffic else None,
    }
    if valu:
        # the vector ALU side of the same kernel, from the stored counters
        roof["valu_busy_pct"] = valu["valu_busy_pct"]
        roof["fp32_TFLOPs"] = round(valu["fp32_flop_per_launch"] / (launch_ms * 1e-3) / 1e12, 2)
    out = {
        "metric": "D2Q9 MLUPS & % HBM roofline",
        "value": round(mlups, 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": args.workload,
            "nx": w["nx"], "ny": w["ny"], "diameter": w.get("diameter", 0), "u_in": w["u_in"],
            "re": w.get("re"), "tau": round(lbm.tau_of(p), 6), "wall": "free-slip",
            "outlet": "x-periodic" if w.get("x_periodic") else "copy-all", "collision": args.collision,
            "variant": vname,
            "graphs": not args.no_graphs,
        },
        "roofline": roof,
        "mlups_fluid": round(fluid * args.steps / (gpu_ms * 1e-3) / 1e6, 1),
        "wall_s": round(wall, 3),
    }
    if not args.no_copy:
        cc = copy_ceiling(torch, lbm, 9 * nodes * 4)
        out["copy_ceiling"] = {"GB/s": round(cc, 1), "frac_of_copy": round(achieved / cc, 4)}
    lat.close()
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(w, args.cpu_budget)
    if args.ensemble:
        out["ensemble"] = ensemble_result(torch, lbm)
    if args.closure:
        out["closure"] = closure_result()
    print(json.dumps(out), flush=True)


def ensemble_result(torch, lbm, steps: int = 1280) -> dict:
    """The 64 cylinder channels (D 8..32, Re 60..200, U = 0.05, tau from Re,
    MRT with the rates of Sec. 2.1): one Ensemble (its default variant)
    against the same cases as 64 separate lattices stepped one after the
    other, both after 128 warm-up steps; MLUPS over all nodes of all cases."""
    from lbm_inputs import ensemble

    cases = ensemble(mrt=True)
    nodes = sum(c["nx"] * c["ny"] for c in cases)
    ens = lbm.Ensemble([lbm.make_params(**c) for c in cases])
    vname = lbm.variant_name(ens.variant)
    ens.step(128)
    ens.sync()
    t0 = time.perf_counter()
    ens.step(steps)
    ens.sync()
    t_ens = time.perf_counter() - t0
    ens.close()
    lats = [lbm.Lattice(lbm.make_params(**c)) for c in cases]
    for lat in lats:
        lat.step(128)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for lat in lats:
        lat.step(steps)
    for lat in lats:
        lat.sync()
    t_sep = time.perf_counter() - t0
    for lat in lats:
        lat.close()
    return {"cases": len(cases), "nodes": nodes, "steps": steps, "variant": vname,
            "mlups": round(nodes * steps / t_ens / 1e6, 1),
            "separate_mlups": round(nodes * steps / t_sep / 1e6, 1),
            "speedup": round(t_sep / t_ens, 3)}


def closure_result() -> dict:
    """Learned closure at D = 40 with the bulk-damped MRT collision: train on
    full-domain samples (Re 80, 100, 120), then the full domain against the
    truncated window (plain and learned) from the same established state,
    statistics over the last 25k of 50k steps."""
    from paper_2605_02185_amd import closure as C

    log = lambda m: print(m, file=sys.stderr, flush=True)
    coll = C.damped_mrt()
    t0 = time.perf_counter()
    X, T = C.generate(collision=coll, log=log)
    t1 = time.perf_counter()
    net, norm, hist = C.fit(X, T, epochs=20, noise=C.NOISE, log=log)
    t2 = time.perf_counter()
    res = C.evaluate({"trunc_learned": (net, norm, C.MASK, 80, C.BETA, C.INTERVAL)}, collision=coll,
                     settle=C.SETTLE, log=log)
    res["samples"] = int(X.shape[0])
    res["data_s"] = round(t1 - t0, 2)
    res["train_s"] = round(t2 - t1, 2)
    res["val_loss"] = hist[-1]
    err = res["trunc_learned"].get("rel_err")
    res["cd_st_within_1pct"] = bool(err and err["mean_cd"] < 0.01 and err["st"] < 0.01)
    res["speedup_at_1pct"] = res["trunc_learned"]["speedup"] if res["cd_st_within_1pct"] else None
    return res


if __name__ == "__main__":
    main()
