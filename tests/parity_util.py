"""Shared helpers of the GPU parity tests: run the library and the oracle
from the same seeded state and compare them."""
import sys

import numpy as np
import pytest

import oracle
import paper_2605_02185_amd as lbm
from lbm_inputs import perturbed_populations
from oracle import stats as ostats

# Table 1 weights, typed in from the paper (k = i - 1).
WT = [4 / 9, 1 / 9, 1 / 9, 1 / 9, 1 / 9, 1 / 36, 1 / 36, 1 / 36, 1 / 36]
TOL = 1e-5
ALL_WALLS = [lbm.WALL_FREE_SLIP, lbm.WALL_PERIODIC, lbm.WALL_NEBB, lbm.WALL_MOVING_BB]


def note(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _oracle_kwargs(kw):
    return {k: v for k, v in kw.items() if k != "hist_capacity"}


def run_both(kw, steps, seed=None, amp=0.05):
    """Run the GPU and the oracle from the same state; returns both objects
    after `steps` steps plus the two force histories."""
    note(f"parity case {kw} steps={steps} seed={seed}")
    lat = lbm.Lattice(lbm.make_params(**kw))
    o = oracle.Oracle(oracle.OracleParams(**_oracle_kwargs(kw)))
    if seed is not None:
        f0 = perturbed_populations(seed, kw["ny"], kw["nx"], WT, amp, dtype=np.float32)
        lat.set_populations(f0)
        o.set_fstar(f0.astype(np.float64))
    lat.step(steps)
    g = lat.forces() if steps else (np.zeros(0),) * 4
    ofx, ofy, bad = o.step(steps)
    assert bad == 0
    return lat, o, g, (ofx, ofy)


def compare_state(lat, o, solid=None, tol=TOL):
    rho, ux, uy = lat.fields()
    orho, oux, ouy = o.fields()
    f = lat.get_populations(np.float64)
    of = o.get_fstar()
    fluid = np.ones_like(orho, dtype=bool) if solid is None else solid == 0
    errs = {
        "rho": np.abs(rho - orho)[fluid].max(),
        "ux": np.abs(ux - oux)[fluid].max(),
        "uy": np.abs(uy - ouy)[fluid].max(),
        "f": np.abs(f - of)[:, fluid].max(),
    }
    note(f"  max errors {errs}")
    for k, v in errs.items():
        assert v <= tol, (k, v)
    return errs


def established(cl, n=3, tol=0.02):
    """The lift amplitude of each of the last n+1 periods, cut at successive
    upward crossings of the mean, stays within tol of the last one."""
    c = cl - cl.mean()
    ups = [i for i in range(len(c) - 1) if c[i] < 0.0 <= c[i + 1]]
    if len(ups) < n + 2:
        return False, []
    amps = [0.5 * np.ptp(cl[ups[-(i + 2)]:ups[-(i + 1)] + 1]) for i in range(n + 1)]
    return max(abs(a / amps[0] - 1) for a in amps[1:]) < tol, amps


def _next_upward_crossing(lat, look):
    """Step of the next upward crossing of the lift through its mean and the
    lift period, predicted from the last `look` steps of the history."""
    t = lat.t
    _, _, _, cl = lat.forces(t - look + 1, look)
    c = cl - cl.mean()
    ups = [i + (-c[i]) / (c[i + 1] - c[i]) for i in range(len(c) - 1) if c[i] < 0.0 <= c[i + 1]]
    assert len(ups) >= 2, "no lift period in the history"
    T = (ups[-1] - ups[0]) / (len(ups) - 1)
    return t - look + 1 + ups[-1] + T, T


def window_parity(kw, spin_up, window=None, periods=2, require_established=True, period_guess=None):
    """GPU statistics over a window against the oracle's, from the same state.

    With `period_guess` (steps) the window is placed by phase: after the
    spin-up the GPU steps on to an eighth of a period before the next upward
    crossing of the lift, so `periods` whole periods fit in (periods + 1/4)
    periods of steps, and `window` is derived."""
    note(f"shedding case {kw} spin-up {spin_up} window {window} periods {periods}")
    d, u = kw["diameter"], kw["u_in"]
    lat = lbm.Lattice(lbm.make_params(**kw))
    lat.step(spin_up)
    if period_guess:
        nxt, T = _next_upward_crossing(lat, int(2.5 * period_guess))
        start = int(nxt - T / 8)
        while start < lat.t:
            start += int(round(T))
        lat.step(start - lat.t)
        window = int(np.ceil((periods + 0.25) * T))
        note(f"  lift period {T:.1f} steps; window of {window} steps from step {lat.t}")
    t0 = lat.t
    state = lat.get_populations(np.float64)
    lat.step(window)
    assert lat.diverged_step() == 0
    _, _, cd, cl = lat.forces(t0 + 1, window)
    gpu = lbm.shedding_stats(cd, cl, d, u, periods)
    ok, amps = established(cl, n=min(3, periods - 1)) if periods >= 2 else (True, [])
    note(f"  GPU {gpu}, per-period amplitudes {np.round(amps, 5)}")

    o = oracle.Oracle(oracle.OracleParams(**_oracle_kwargs(kw)))
    o.set_fstar(state)
    fx, fy = [], []
    for first in range(0, window, 2000):
        a, b, bad = o.step(min(2000, window - first))
        assert bad == 0
        fx.append(a)
        fy.append(b)
        note(f"  oracle at window step {first + len(a)}")
    fx, fy = np.concatenate(fx), np.concatenate(fy)
    ocd, ocl = ostats.coefficients(fx, fy, u, d)
    ora = ostats.shedding(ocd, ocl, d, u, periods)
    note(f"  oracle {ora}")
    for k in ("mean_cd", "cl_amp", "st"):
        assert gpu[k] == pytest.approx(ora[k], rel=0.01), k
    if require_established:
        assert ok, "shedding not established at the start of the window"
    return gpu
