"""Learned boundary closure for a truncated domain: data generation, training
and evaluation.  This module only sequences calls; every arithmetic step
(lattice steps, sampling, normalisation statistics, forward, backward, Adam)
runs in the kernels of liblbm.so.

Setting (all lattice units): the full domain is the 41 D x 21 D channel with
free-slip walls; the truncated window keeps the inlet and the cylinder and
cuts the domain 15.5 D behind the cylinder centre and 5.5 D to each side
(26 D x 11 D).  Its top, bottom and outlet are open boundaries, handled
either by the plain treatments (free-slip rows, extrapolated outlet) or by
the network, which adds a learned residual to them.
"""
from __future__ import annotations

import json
import time

import numpy as np

from . import Lattice, Mlp, column_moments, make_params, shedding_stats
from ._lib import COLLISION_MRT, OUTLET_COPY_UNKNOWN, WALL_FREE_SLIP

N_FEATURES = 36

# Collision of both the full and the truncated domain: MRT (Eq. 6) with the
# shear rates 1/tau and strongly damped energy modes (s_e = s_eps = 0.02, a
# bulk viscosity about 120 times that of the paper's 1.1).  The free-slip
# rows of the truncated window reflect sound; with weak bulk damping a
# transverse acoustic mode (period 2 H / c_s) stays trapped between them and
# dominates the lift signal, which no closure of the populations removes.
# The incompressible wake barely notices the bulk viscosity (full-domain
# mean Cd, lift amplitude and St move by < 0.5 %).
def damped_mrt(s_bulk=0.02):
    return dict(collision=COLLISION_MRT, s_rates=(1.0, s_bulk, s_bulk, 1.0, 1.1, 1.0, 1.1, 0.0, 0.0))


# Closed-loop settings measured at D = 40: training-input noise of 0.15
# standard deviations, rows plain within 2 D of the inlet and outlet, the
# network evaluated every 8 steps and its output low-passed with beta = 0.08
# per evaluation (a time constant of about 100 steps).  MASK = 3 closes the
# two rows; the outlet (bit 4) needs OUTLET_GUARD: an outlet residual changes
# the mass of the window, whose level no boundary fixes (a velocity inlet and
# an extrapolated outlet), and the learned outlet residuals drove the window
# to diverge within 0.5k-5k steps even when clamped to one standard
# deviation; shifting the three residuals of each outlet node to a zero sum
# (no mass, no x-momentum) makes it stable.  OUTLET_GUARD = (output clamp in
# standard deviations, outlet nodes kept plain next to each row, mass-free
# outlet residuals).
NOISE = 0.15
MASK = 3
BETA = 0.08
INTERVAL = 8
OUTLET_GUARD = (4.0, 40, True)
BIAS_SNAPSHOTS = 3000
# The closed loop is sensitive to the network's initialisation: over seeds
# 7-12, mean Cd and St of the window stay within 1 % of the full domain for
# most, the lift amplitude within 1.6-14 %.  fit_and_select trains one
# network per seed and keeps the one whose closed-loop window comes closest
# to the full domain at a held-out Reynolds number (VAL_RE, one of the
# training runs' but not the one reported).  Eight seeds: with four, often
# only one passed the lift bound below at the held-out Re, and the rule then
# had nothing to choose from.
SEEDS = tuple(range(7, 15))
VAL_RE = 120.0
# Seeds whose lift amplitude at the held-out Re is off by more than this are
# passed over: among the rest the one closest in mean Cd and St is kept (the
# closure's target is those two within 1 %).
CL_BOUND = 0.05


def scaled(d=40, interval=None):
    """The D = 40 settings carried to diameter d (U fixed): step counts scale
    with the flow time D/U, the rows' plain taper and the outlet guard's with
    D.  Above D = 40 the window is large enough for three-step launches, so
    the network is evaluated every 12 steps (a whole number of them), with
    the low-pass's time constant (interval / beta steps) scaled with D.  At
    d = 40 this is exactly the settings above.  An explicit `interval` keeps
    the same time constant (beta grows with it): fewer evaluations, a
    coarser-grained low-pass."""
    f = d / 40.0
    if interval is None:
        interval = INTERVAL if d <= 40 else 12
    if interval < 1:
        raise ValueError("interval must be at least one step")
    return dict(spin_up=int(round(175000 * f)), every=max(1, int(round(5 * f))),
                bias_every=max(1, int(round(25 * f))), total=int(round(300000 * f)),
                stats=int(round(50000 * f)), interval=interval, beta=min(1.0, BETA * interval / (INTERVAL * f)),
                guard=(OUTLET_GUARD[0], int(round(OUTLET_GUARD[1] * f)), OUTLET_GUARD[2]), taper=2 * d)


def full_domain(d=40, u=0.05, re=100.0, collision=None):
    """The 41 D x 21 D channel; `collision` (keyword arguments of make_params,
    e.g. MRT rates) applies to both the full and the truncated lattice."""
    return dict(nx=41 * d, ny=21 * d, diameter=d, cx2=21 * d, cy2=21 * d, u_in=u, re=re,
                wall=WALL_FREE_SLIP, **(collision or {}))


def window(d=40, u=0.05, re=100.0, collision=None):
    """The truncated lattice and its origin (ox, oy) inside the full domain."""
    kw = dict(nx=26 * d, ny=11 * d, diameter=d, cx2=21 * d, cy2=11 * d, u_in=u, re=re,
              wall=WALL_FREE_SLIP, outlet_mode=OUTLET_COPY_UNKNOWN, **(collision or {}))
    return kw, 0, 5 * d


def n_boundary(kw):
    return 2 * (kw["nx"] - 2) + (kw["ny"] - 2)


def generate(res=(80.0, 100.0, 120.0), d=40, u=0.05, spin_up=175000, snapshots=50000, every=5,
             per_snapshot=64, seed=2605, collision=None, bias_snapshots=0, bias_every=25, log=print):
    """Samples from full-domain runs at each Re: after spin_up steps, every
    `every` steps, `per_snapshot` random open-boundary nodes of the window.

    With bias_snapshots > 0 every boundary node is first sampled every
    bias_every steps after the spin-up (bias_snapshots snapshots, split over
    the Re); the per-node mean residual over them (bias, [nb][3]) is the
    fixed part of the closure, and the training targets are the residuals
    relative to it.  Returns device tensors X [N][36], T [N][3] (raw features
    and residuals) and the bias (host array, or None)."""
    import torch

    wkw, ox, oy = window(d, u, collision=collision)
    nb = n_boundary(wkw)
    n = snapshots * per_snapshot
    X = torch.empty((n, N_FEATURES), dtype=torch.float32, device="cuda")
    T = torch.empty((n, 3), dtype=torch.float32, device="cuda")
    rng = np.random.default_rng(seed)
    nodes = torch.from_numpy(rng.integers(0, nb, n).astype(np.int32)).cuda()
    split = lambda total: [total // len(res) + (1 if i < total % len(res) else 0) for i in range(len(res))]
    lats = []
    for re in res:
        lat = Lattice(make_params(**full_domain(d, u, re, collision), hist_capacity=4096))
        lat.step(spin_up)
        lats.append(lat)
    bias, bias_dev = None, None
    if bias_snapshots > 0:
        allnodes = torch.arange(nb, dtype=torch.int32, device="cuda")
        fscratch = torch.empty((nb, N_FEATURES), dtype=torch.float32, device="cuda")
        Tb = torch.empty((bias_snapshots, nb, 3), dtype=torch.float32, device="cuda")
        k = 0
        for lat, ns in zip(lats, split(bias_snapshots)):
            for _ in range(ns):
                lat.step(bias_every)
                lat.sample_boundary(ox, oy, wkw["nx"], wkw["ny"], allnodes, fscratch, Tb[k])
                k += 1
        mean, _ = column_moments(Tb.view(bias_snapshots, nb * 3))
        bias = mean.reshape(nb, 3).astype(np.float32)
        bias_dev = torch.from_numpy(bias).cuda()
        del Tb, fscratch
        log(f"closure data: per-node mean residual from {bias_snapshots} snapshots of all {nb} boundary nodes")
    off = 0
    for re, lat, ns in zip(res, lats, split(snapshots)):
        t0 = time.perf_counter()
        for _ in range(ns):
            lat.step(every)
            lat.sample_boundary(ox, oy, wkw["nx"], wkw["ny"], nodes[off:off + per_snapshot],
                                X[off:off + per_snapshot], T[off:off + per_snapshot], bias_dev)
            off += per_snapshot
        lat.sync()
        lat.close()
        log(f"closure data: Re {re:g}: {ns} snapshots ({time.perf_counter() - t0:.1f} s)")
    return X, T, bias


def fit(X, T, epochs=30, batch=4096, lr=1e-3, seed=7, val_frac=0.05, init=None, noise=0.0,
        features=None, log=print):
    """Trains a fresh network (last layer zero: starts as the plain treatment)
    on the raw samples, with optional input noise (z-scored units).
    `features` (36 booleans, default all) selects the inputs the network
    sees: a deselected feature gets a zero z-score scale, i.e. enters as 0.
    Returns (network, norm, validation-loss history)."""
    import torch

    n = X.shape[0]
    n_val = max(batch, int(n * val_frac))
    n_val = min(n_val, 65536, n // 2)
    n_tr = n - n_val
    mean, std = column_moments(X[:n_tr])
    _, tstd = column_moments(T[:n_tr])
    inv = 1.0 / np.maximum(std, 1e-12)
    if features is not None:
        inv = np.where(np.asarray(features, dtype=bool), inv, 0.0)
    norm = np.concatenate([mean, inv, np.maximum(tstd, 1e-12)]).astype(np.float32)
    rng = np.random.default_rng(seed)
    if init is None:
        init = _init_params(rng)
    net = Mlp(init)
    net.set_norm(norm)
    net.set_noise(noise, seed)
    Xv, Tv = X[n_tr:], T[n_tr:]
    hist = []
    steps = n_tr // batch
    for ep in range(epochs):
        perm = torch.from_numpy(rng.permutation(n_tr).astype(np.int32)).cuda()
        for s in range(steps):
            net.train_step(X, T, perm[s * batch:(s + 1) * batch], batch, lr)
        _, vloss = net.gradient(Xv, Tv)
        hist.append(vloss)
        if ep == 0 or (ep + 1) % 5 == 0 or ep == epochs - 1:
            log(f"closure fit: epoch {ep + 1}/{epochs} validation loss {vloss:.4e} (normalised)")
    return net, norm, hist


def fit_and_select(X, T, bias, seeds=SEEDS, val_re=VAL_RE, d=40, u=0.05, collision=None, epochs=20, noise=NOISE,
                   total=None, stats_steps=None, interval=None, log=print):
    """One network per seed (fit), each run in the closed loop (rows and
    guarded outlet, cold start, evaluated as scaled(d, interval) says) at
    Re = val_re against the full domain at that Re; returns (network, norm,
    table) for the seed whose larger relative error of mean Cd and St is
    smallest among those whose lift amplitude error is below CL_BOUND (all
    seeds when none is)."""
    sc = scaled(d, interval)
    total = sc["total"] if total is None else total
    stats_steps = sc["stats"] if stats_steps is None else stats_steps
    cands = {}
    for seed in seeds:
        net, norm, hist = fit(X, T, epochs=epochs, noise=noise, seed=seed, log=lambda m: None)
        cands[f"seed{seed}"] = dict(net=net, norm=norm, mask=7, taper=sc["taper"], guard=sc["guard"], bias=bias,
                                    interval=sc["interval"], beta=sc["beta"], val_loss=hist[-1])
    res = evaluate(cands, d=d, u=u, re=val_re, collision=collision, start="cold", total=total,
                   stats_steps=stats_steps, log=log)
    table = {name: {"val_loss": spec["val_loss"], "rel_err": res[name].get("rel_err"),
                    "diverged_step": res[name]["diverged_step"]} for name, spec in cands.items()}
    best, best_err = select(table)
    if best is None:
        raise RuntimeError("no candidate network ran stably in the closed loop")
    log(f"closure select: {best} (larger of the mean Cd and St errors {best_err:.4f} at Re {val_re:g})")
    return cands[best]["net"], cands[best]["norm"], {"chosen": best, "val_re": val_re, "candidates": table}


def select(table, cl_bound=None):
    """The selection rule of fit_and_select on its table ({name: {"rel_err":
    {"mean_cd", "cl_amp", "st"} or None, "diverged_step"}}): among the stable
    candidates whose lift amplitude error is below cl_bound (CL_BOUND by
    default; all stable ones when none is), the one whose larger error of
    mean Cd and St is smallest.  Adds "worst_cd_st" and "cl_ok" to each
    entry; returns (name, its larger error), or (None, inf) when none ran
    stably."""
    cl_bound = CL_BOUND if cl_bound is None else cl_bound
    for entry in table.values():
        err = entry.get("rel_err")
        ok = bool(err) and entry.get("diverged_step", 0) == 0
        entry["worst_cd_st"] = max(err["mean_cd"], err["st"]) if ok else float("inf")
        entry["cl_ok"] = ok and err["cl_amp"] < cl_bound
    pool = [n for n in table if table[n]["cl_ok"]] or list(table)
    best, best_err = None, float("inf")
    for name in pool:
        if table[name]["worst_cd_st"] < best_err:
            best, best_err = name, table[name]["worst_cd_st"]
    return best, best_err


def _init_params(rng):
    """He-uniform hidden layers, zero output layer."""
    p = np.zeros(6723, dtype=np.float32)
    lim1, lim2 = np.sqrt(6.0 / 36), np.sqrt(6.0 / 64)
    p[0:2304] = rng.uniform(-lim1, lim1, 2304)
    p[2368:6464] = rng.uniform(-lim2, lim2, 4096)
    return p


def _timed_steps(lat, n):
    import torch

    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    lat.step(n)
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) * 1e-3


def _stats(lat, first, n, kw, periods=8):
    bad = lat.diverged_step()
    if bad:
        return None, bad
    _, _, cd, cl = lat.forces(first, n)
    try:
        return shedding_stats(cd, cl, kw["diameter"], kw["u_in"], periods), 0
    except Exception:
        return None, 0


def _run_window(lat, spec):
    net = spec.get("net")
    if net is not None:
        lat.enable_closure(net, spec["norm"], spec.get("mask", MASK))
        lat.set_closure_filter(spec.get("beta", BETA), spec.get("taper", 80))
        lat.set_closure_interval(spec.get("interval", INTERVAL))
        lat.set_closure_guard(*spec.get("guard", (0.0, 0, False)))
        if spec.get("bias") is not None:
            lat.set_closure_bias(spec["bias"])


def evaluate(nets, d=40, u=0.05, re=100.0, start="cold", total=300000, stats_steps=50000, spin_up=175000,
             collision=None, variant=0, periods=8, log=print):
    """Full domain against truncated windows, statistics over the last
    `stats_steps` steps of every run (about 10 lift periods by default).

    start = "cold": every run starts from the initial state of the hot path
    (equilibrium of the inlet velocity with its small transverse
    perturbation) and runs `total` steps, the window with its closure from
    the first step; seconds are GPU time of all `total` steps, so the
    window's own spin-up to established shedding is included.
    start = "cut": the full domain runs `spin_up` steps and each window
    starts from the full state cut out there; seconds are GPU time of the
    `total - spin_up` steps after the cut.

    `nets` maps a label to a dict: net, norm, mask (1 top, 2 bottom, 4
    outlet), taper, beta, interval, guard (limit, outlet taper, mass-free
    outlet), bias (per-node fixed residual); the plain truncated run is
    always included.  `variant` (0: the
    library's default) selects the windows' kernel."""
    import torch

    full_kw = full_domain(d, u, re, collision)
    wkw, ox, oy = window(d, u, re, collision)
    full = Lattice(make_params(**full_kw, hist_capacity=stats_steps + 4096))
    cut = None
    if start == "cut":
        full.step(spin_up)
        S = torch.empty((9, full_kw["ny"], full_kw["nx"]), dtype=torch.float64, device="cuda")
        full.get_populations_device(S)
        cut = S[:, oy:oy + wkw["ny"], ox:ox + wkw["nx"]].contiguous()
        del S
    steps = total - (spin_up if start == "cut" else 0)
    secs = _timed_steps(full, steps)
    st, bad = _stats(full, full.t - stats_steps + 1, stats_steps, full_kw, periods)
    out = {"start": start, "total_steps": total, "stats_steps": stats_steps,
           "full": {"stats": st, "seconds": secs, "diverged_step": bad, "nodes": full_kw["nx"] * full_kw["ny"]}}
    full.close()
    log(f"closure eval: full {json.dumps(out['full'])}")
    runs = [("trunc_plain", {})] + list(nets.items())
    for name, spec in runs:
        lat = Lattice(make_params(**wkw, hist_capacity=stats_steps + 4096))
        if variant:
            lat.set_variant(variant)
        if cut is not None:
            lat.set_populations_device(cut)
        _run_window(lat, spec)
        secs = _timed_steps(lat, steps)
        st, bad = _stats(lat, lat.t - stats_steps + 1, stats_steps, wkw, periods)
        r = {"stats": st, "seconds": secs, "diverged_step": bad, "nodes": wkw["nx"] * wkw["ny"],
             "speedup": out["full"]["seconds"] / secs, "mask": spec.get("mask", 0)}
        ref = out["full"]["stats"]
        if ref and st:
            r["rel_err"] = {k: abs(st[k] / ref[k] - 1) for k in ("mean_cd", "cl_amp", "st")}
        out[name] = r
        lat.close()
        log(f"closure eval: {name} {json.dumps(r)}")
    return out


def main(argv=None):
    import argparse

    ap = argparse.ArgumentParser(description="train and evaluate the learned boundary closure")
    ap.add_argument("--d", type=int, default=40)
    ap.add_argument("--snapshots", type=int, default=50000)
    ap.add_argument("--epochs", type=int, default=20)
    ap.add_argument("--noise", type=float, default=NOISE)
    ap.add_argument("--start", choices=("cold", "cut"), default="cold")
    ap.add_argument("--total", type=int, default=None, help="steps per run (default: 300k at D = 40, scaled with D)")
    ap.add_argument("--stats", type=int, default=None, help="steps of statistics (default: 50k at D = 40, scaled)")
    ap.add_argument("--bgk", action="store_true", help="BGK instead of the bulk-damped MRT collision")
    ap.add_argument("--interval", type=int, default=None,
                    help="steps between network evaluations (default: 8 up to D = 40, 12 above)")
    ap.add_argument("--save", default=None, help="write the trained weights and norm (.npz)")
    args = ap.parse_args(argv)
    import torch

    torch.cuda.set_device(0)
    coll = None if args.bgk else damped_mrt()
    sc = scaled(args.d, args.interval)
    total = sc["total"] if args.total is None else args.total
    stats = sc["stats"] if args.stats is None else args.stats
    X, T, bias = generate(d=args.d, snapshots=args.snapshots, collision=coll, bias_snapshots=BIAS_SNAPSHOTS,
                          spin_up=sc["spin_up"], every=sc["every"], bias_every=sc["bias_every"])
    net, norm, sel = fit_and_select(X, T, bias, d=args.d, collision=coll, epochs=args.epochs, noise=args.noise,
                                    total=total, stats_steps=stats, interval=args.interval)
    if args.save:
        np.savez(args.save, params=net.get_params(), norm=norm, bias=bias)
    nets = {"trunc_rows_outlet": dict(net=net, norm=norm, mask=7, taper=sc["taper"], guard=sc["guard"], bias=bias,
                                      interval=sc["interval"], beta=sc["beta"])}
    res = evaluate(nets, d=args.d, start=args.start, total=total, stats_steps=stats, collision=coll,
                   spin_up=sc["spin_up"])
    res["settings"] = sc
    res["selection"] = sel
    print(json.dumps(res), flush=True)
    return res


if __name__ == "__main__":
    main()
