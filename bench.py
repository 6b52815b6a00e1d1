"""Throughput benchmark of the D2Q9 solver on one MI355X.

One step = one pass of the whole hot path over the lattice: pull streaming,
half-way bounce-back on the cylinder, wall/outlet/inlet corrections, the
collision (BGK by default) and the FP64 momentum-exchange force (plus its
fixed-order history reduction every 96 steps).  The default workload is the
D = 160 cylinder channel (6560 x 3360 = 22.0 M nodes, Re = 100, U = 0.05,
free-slip walls), whose two population buffers (1.6 GB) are far larger than
the 256 MB Infinity Cache.  At this size the library's default kernel takes
four steps per launch with the intermediate populations in registers.

Prints one JSON line:
  value      MLUPS = nx * ny * steps / time / 1e6 (all nodes)
  roofline   for the dominant kernel, per launch (S steps):
             achieved  HBM bytes the rocprofv3 FETCH_SIZE / WRITE_SIZE
                       counters give per launch (`traffic`, scaled by what
                       they read for a copy of known size) over the live
                       launch time, against the 8 TB/s HBM3E peak (`frac`);
                       only while the committed counter summary was taken on
                       the current kernel source and configuration
             frac_of_floor  one read and one write of the state (72 B per
                       node: the least an S-step launch can move) over the
                       launch time, against the peak
             effective_GBs  72 B per node update times the updates (the
                       per-update accounting of the LBM literature; passes
                       the peak once several steps share one pass)
             valu      the vector-ALU side from the same counter summary
  cpu_baseline  the FP64 oracle, built with gcc -O3 -march=native on this
             host, timed on a bounded sample of the same lattice; samples of
             the other lattices at 1 and all threads
  ensemble   the 64-case ensemble against 64 separate lattices
  closure    the learned boundary closure against the full domain
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


def roofline(nodes: int, steps_per_launch: int, launch_s: float, counters) -> dict:
    """The bench line's roofline object for a launch of `steps_per_launch`
    steps over `nodes` nodes lasting `launch_s` seconds, with the stored
    counter summary `counters` (stored_counters) or None."""
    floor_bytes = BYTES_PER_NODE * nodes  # one read and one write of the state per launch
    effective = BYTES_PER_NODE * nodes * steps_per_launch / launch_s / 1e9
    floor_rate = floor_bytes / launch_s / 1e9
    traffic = counters.get("bytes_per_launch") if counters else None
    valu = counters.get("valu") if counters else None
    achieved = traffic / launch_s / 1e9 if traffic else None
    roof = {
        "bound": "hbm",
        "achieved": round(achieved, 1) if achieved else None,
        "peak": PEAK_HBM_GBS,
        "unit": "GB/s",
        "frac": round(achieved / PEAK_HBM_GBS, 4) if achieved else None,
        "traffic": traffic,
        "kernel": {1: "step_kernel", 2: "step2_kernel"}.get(steps_per_launch, "multistep_kernel"),
        "steps_per_launch": steps_per_launch,
        "launch_us": round(launch_s * 1e6, 2),
        "floor_bytes_per_launch": floor_bytes,
        "frac_of_floor": round(floor_rate / PEAK_HBM_GBS, 4),
        "traffic_over_floor": round(traffic / floor_bytes, 4) if traffic else None,
        "effective_GBs": round(effective, 1),
        "counters": ("profiles/traffic_step_kernel.json (kernel source " + counters["kernel_sha256_16"] + ")"
                     if counters else "stale: taken on another kernel source or configuration"),
    }
    if valu:
        # the vector ALU side of the same kernel, from the stored counters:
        # FP32 operations per launch over the live launch time, against the
        # 78.6 TFLOP/s of unpacked FP32 FMAs (256 CUs x 4 SIMDs x 16 lanes x
        # 2 x 2.4 GHz; the packed forms behind the 157.3 figure are not used)
        flops = valu["fp32_flop_per_launch"] / launch_s / 1e12
        roof["valu"] = {"busy_pct": valu["valu_busy_pct"], "fp32_TFLOPs": round(flops, 2),
                        "fp32_peak_TFLOPs": 78.6, "frac": round(flops / 78.6, 4),
                        "insts_per_update": valu["valu_insts_per_update"]}
    return roof


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


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform

    return platform.processor() or "unknown"


def _time_oracle(oracle, lib, w: dict, threads: int, max_steps: int, budget_s: float) -> dict:
    """Steps of one lattice on `threads` threads until max_steps or about
    budget_s seconds of stepping (set-up and the first step not timed)."""
    oracle.set_threads(threads, lib)
    o = oracle.Oracle(oracle.OracleParams(**w), lib_path=lib)
    o.step(1)  # first touch of the buffers
    steps, t0 = 0, time.perf_counter()
    while steps < max_steps:
        o.step(1)
        steps += 1
        el = time.perf_counter() - t0
        if el >= budget_s:
            break
    el = time.perf_counter() - t0
    o.close()
    nodes = w["nx"] * w["ny"]
    return {"lattice": f"{w['nx']}x{w['ny']}", "threads": threads, "steps": steps, "seconds": round(el, 2),
            "mlups": round(nodes * steps / el / 1e6, 2)}


def cpu_baseline(w: dict, budget_s: float) -> dict:
    """The FP64 oracle (its C source as it stands), compiled here with gcc
    -O3 -march=native and timed on this host: the benchmark's lattice on all
    the threads OpenMP is given (about 40 % of budget_s), then the D = 10,
    40 and 80 channels for up to 2000, 1000 and 200 steps on one thread and
    on all of them (the rest of the budget, split evenly)."""
    import tempfile

    import oracle
    from lbm_inputs import WORKLOADS

    lib = os.path.join(tempfile.gettempdir(), f"liblbm_oracle_native_{os.getpid()}.so")
    oracle.build_native(lib)
    try:
        nthreads = oracle.threads(lib)
        head = _time_oracle(oracle, lib, w, nthreads, 200, 0.4 * budget_s)
        samples = []
        per = 0.6 * budget_s / 6
        for name, steps in (("cyl_d10", 2000), ("cyl_d40", 1000), ("cyl_d80", 200)):
            for th in (1, nthreads):
                samples.append(dict(_time_oracle(oracle, lib, WORKLOADS[name], th, steps, per), workload=name))
        oracle.set_threads(nthreads, lib)
    finally:
        os.remove(lib)
    return {
        "value": head["mlups"],
        "unit": "MLUPS",
        "cores": nthreads,
        "kind": "oracle",
        "sample": f"{head['steps']} steps of the {head['lattice']} lattice ({head['seconds']} s, FP64, "
                  f"{nthreads} OpenMP threads)",
        "cpu_model": cpu_model(),
        "build": "gcc " + " ".join(oracle.NATIVE_FLAGS),
        "bytes_per_update": 144,
        "samples": samples,
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
    ap.add_argument("--cpu-budget", type=float, default=20.0)
    ap.add_argument("--no-copy", action="store_true", help="skip the copy-ceiling reference")
    ap.add_argument("--no-graphs", action="store_true", help="plain launches instead of graph replay")
    ap.add_argument("--no-ensemble", action="store_true",
                    help="skip the 64-case ensemble (MRT, tau from Re) against 64 separate lattices")
    ap.add_argument("--no-closure", action="store_true",
                    help="skip training and evaluating the learned boundary closure (about a minute)")
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
    launch_s = ms_per_step * steps_per_launch * 1e-3
    roof = roofline(nodes, steps_per_launch, launch_s, stored_counters(args.workload, args.collision, vname))
    achieved = roof["achieved"]
    walls = {lbm.WALL_FREE_SLIP: "free-slip", lbm.WALL_PERIODIC: "periodic", lbm.WALL_NEBB: "nebb",
             lbm.WALL_MOVING_BB: "moving-bb"}
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
            "re": w.get("re"), "tau": round(lbm.tau_of(p), 6), "wall": walls[p.wall],
            "outlet": ("x-periodic" if p.x_periodic else
                       "copy-all" if p.outlet_mode == lbm.OUTLET_COPY_ALL else "copy-unknown"),
            "collision": args.collision,
            "variant": vname,
            "graphs": not args.no_graphs,
        },
        "roofline": roof,
        "mlups_fluid": round(fluid * args.steps / (gpu_ms * 1e-3) / 1e6, 1),
        "wall_s": round(wall, 3),
    }
    if not args.no_copy:
        cc = copy_ceiling(torch, lbm, 9 * nodes * 4)
        out["copy_ceiling"] = {"GB/s": round(cc, 1),
                               "frac_of_copy": round(achieved / cc, 4) if achieved else None}
    lat.close()
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(w, args.cpu_budget)
    if not args.no_ensemble:
        out["ensemble"] = ensemble_result(torch, lbm)
    if not args.no_closure:
        out["closure"] = closure_result()
    print(json.dumps(out), flush=True)


def ensemble_result(torch, lbm, steps: int = 1920) -> dict:
    """The 64 cylinder channels (D 8..32, Re 60..200, U = 0.05, tau from Re,
    MRT with the rates of Sec. 2.1): one Ensemble (the variant its autotuner
    picks) against the same cases as 64 separate lattices (each on its own
    default), both after 192 warm-up steps, timed with HIP events on the
    stream they run on.  Per-case MLUPS: a case's node updates over the
    ensemble's time (all cases advance together), and over the case's own
    time when run alone."""
    from lbm_inputs import ensemble

    cases = ensemble(mrt=True)
    sizes = [c["nx"] * c["ny"] for c in cases]
    nodes = sum(sizes)
    stream = torch.cuda.current_stream()

    def timed(run):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record(stream)
        run()
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) * 1e-3

    t0 = time.perf_counter()
    ens = lbm.Ensemble([lbm.make_params(**c) for c in cases], stream=stream.cuda_stream)
    tune_s = time.perf_counter() - t0
    vname = lbm.variant_name(ens.variant)
    ens.step(192)
    ens.sync()
    t_ens = timed(lambda: ens.step(steps))
    ens.sync()
    ens.close()
    t_alone = []
    for c in cases:
        lat = lbm.Lattice(lbm.make_params(**c), stream=stream.cuda_stream)
        lat.step(192)
        t_alone.append(timed(lambda: lat.step(steps)))
        lat.sync()
        lat.close()
    t_sep = sum(t_alone)
    per_case = [round(n * steps / t_ens / 1e6, 1) for n in sizes]
    per_alone = [round(n * steps / t / 1e6, 1) for n, t in zip(sizes, t_alone)]
    return {"cases": len(cases), "nodes": nodes, "steps": steps, "variant": vname,
            "autotune_s": round(tune_s, 2),
            "mlups": round(nodes * steps / t_ens / 1e6, 1),
            "separate_mlups": round(nodes * steps / t_sep / 1e6, 1),
            "speedup": round(t_sep / t_ens, 3),
            "case_D": [c["diameter"] for c in cases],
            "per_case_mlups": per_case,
            "per_case_alone_mlups": per_alone}


def closure_result() -> dict:
    """Learned closure at D = 40 with the bulk-damped MRT collision: data
    from full-domain runs (Re 80, 100, 120; per-node mean residual and random
    samples), eight networks trained, the one closest to the full domain in
    the closed loop at the held-out Re = 120 kept; then at Re = 100 the full
    domain against the truncated window (plain, and learned top, bottom and
    guarded outlet), every run 300k steps from the initial state, statistics
    over the last 50k; speedup = the full domain's GPU time over the
    window's, spin-up included."""
    from paper_2605_02185_amd import closure as C

    log = lambda m: print(m, file=sys.stderr, flush=True)
    coll = C.damped_mrt()
    t0 = time.perf_counter()
    X, T, bias = C.generate(collision=coll, bias_snapshots=C.BIAS_SNAPSHOTS, log=log)
    t1 = time.perf_counter()
    net, norm, sel = C.fit_and_select(X, T, bias, collision=coll, log=log)
    t2 = time.perf_counter()
    nets = {"trunc_learned": dict(net=net, norm=norm, mask=7, taper=80, guard=C.OUTLET_GUARD, bias=bias)}
    res = C.evaluate(nets, collision=coll, start="cold", log=log)
    res["collision"] = "MRT, shear rates 1/tau, s_e = s_eps = 0.02"
    res["samples"] = int(X.shape[0])
    res["data_s"] = round(t1 - t0, 2)
    res["train_and_select_s"] = round(t2 - t1, 2)
    res["selection"] = sel
    err = res["trunc_learned"].get("rel_err")
    res["cd_st_within_1pct"] = bool(err and err["mean_cd"] < 0.01 and err["st"] < 0.01)
    res["cd_cl_st_within_1pct"] = bool(err and max(err.values()) < 0.01)
    return res


if __name__ == "__main__":
    main()
