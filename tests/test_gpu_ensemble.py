"""Ensemble (batched) runs: every case of an Ensemble must evolve bit for
bit as it does in its own Lattice, including cases that stop at their step
budget while the others go on, and the autotuner must pick a valid variant."""
import os
import sys

import numpy as np
import pytest

import paper_2605_02185_amd as lbm
from lbm_inputs import channel, ensemble

pytestmark = pytest.mark.gpu


def note(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _alone(kw, steps, with_fields=False):
    lat = lbm.Lattice(lbm.make_params(**kw))
    lat.step(steps)
    out = (lat.get_populations(np.float64), lat.forces())
    return out + (lat.fields(),) if with_fields else out


def test_mixed_ensemble_matches_separate_runs_bitwise():
    # explicit tau: BGK at the Re-derived tau (about 0.51 at these D) diverges
    cases = [
        dict(channel(6, u=0.05, re=80), tau=0.62),
        dict(channel(9, u=0.05, re=150), tau=0.58, wall=lbm.WALL_PERIODIC),
        dict(channel(7, u=0.04, re=60), tau=0.7, wall=lbm.WALL_MOVING_BB, outlet_mode=lbm.OUTLET_COPY_UNKNOWN),
        dict(nx=300, ny=64, u_in=0.03, tau=0.7, wall=lbm.WALL_NEBB),
        dict(nx=130, ny=77, tau=0.6, u_in=0.0, x_periodic=True, wall=lbm.WALL_PERIODIC, perturb_amp=0.0),
    ]
    budgets = [300, 137, 300, 64, 200]
    note(f"ensemble of {len(cases)} cases, budgets {budgets}")
    ens = lbm.Ensemble([lbm.make_params(**kw) for kw in cases], budgets=budgets)
    ens.step(150)
    ens.step(1)
    ens.step(400)  # beyond every budget: each case stops at its own
    ens.sync()
    for i, (kw, b) in enumerate(zip(cases, budgets)):
        steps, bad = ens.info(i)
        assert (steps, bad) == (b, 0)
        f_alone, forces_alone, fields_alone = _alone(kw, b, with_fields=True)
        assert np.array_equal(ens.get_populations(i, np.float64), f_alone), i
        got = ens.forces(i)
        for a, c in zip(got, forces_alone):
            if a is not None:
                assert np.array_equal(a, c), i
        for a, c in zip(ens.fields(i), fields_alone):
            assert np.array_equal(a, c), i


MULTI = ["t3_h8_s2", "t3_h8_s4", "t4_h8_s2", "t4_h8_s4", "t4_h8_s8", "t4_h16u_s8", "t4_h10u_s10", "t3_h16u_s2"]


@pytest.mark.parametrize("name", MULTI)
def test_multistep_ensemble_matches_separate_runs_bitwise(name):
    """Three or four steps per launch over every active case: budgets that
    are not multiples of the step count (the rest runs one step per launch),
    a 96-step graph replay and calls of odd lengths still give every case
    the bits of its own run."""
    v = {lbm.variant_name(i): i for i in range(1, lbm.num_variants() + 1)}[name]
    cases = [
        dict(channel(6, u=0.05, re=80), tau=0.62),
        dict(channel(9, u=0.05, re=150), tau=0.58, wall=lbm.WALL_PERIODIC, collision=lbm.COLLISION_MRT,
             s_rates=(1, 1.1, 1.1, 1, 1.1, 1, 1.1, 0, 0)),
        dict(channel(7, u=0.04, re=60), tau=0.7, wall=lbm.WALL_MOVING_BB, outlet_mode=lbm.OUTLET_COPY_UNKNOWN,
             bounce=lbm.BOUNCE_FULLWAY),
        dict(nx=300, ny=64, u_in=0.03, tau=0.7, wall=lbm.WALL_NEBB),
        dict(nx=130, ny=77, tau=0.6, u_in=0.0, x_periodic=True, wall=lbm.WALL_PERIODIC, perturb_amp=0.0),
        dict(channel(8, u=0.05), tau=0.6, bounce=lbm.BOUNCE_INTERP),
    ]
    budgets = [300, 137, 251, 64, 200, 299]
    note(f"ensemble of {len(cases)} cases on {name}, budgets {budgets}")
    ens = lbm.Ensemble([lbm.make_params(**kw) for kw in cases], budgets=budgets)
    ens.set_variant(v)
    assert ens.variant == v
    ens.step(5)
    ens.step(150)
    ens.step(1)
    ens.step(400)  # beyond every budget
    ens.sync()
    for i, (kw, b) in enumerate(zip(cases, budgets)):
        steps, bad = ens.info(i)
        assert (steps, bad) == (b, 0)
        f_alone, forces_alone = _alone(kw, b)
        assert np.array_equal(ens.get_populations(i, np.float64), f_alone), i
        for a, c in zip(ens.forces(i), forces_alone):
            if a is not None:
                assert np.array_equal(a, c), i


def test_ensemble_rejects_variants_it_cannot_run():
    ens = lbm.Ensemble([lbm.make_params(**dict(channel(6), tau=0.6))])
    xcd = {lbm.variant_name(i): i for i in range(1, lbm.num_variants() + 1)}["v1_ty1_xcd_nt"]
    with pytest.raises(lbm.LbmError):
        ens.set_variant(xcd)
    with pytest.raises(lbm.LbmError):
        ens.set_variant(lbm.num_variants() + 1)


@pytest.mark.parametrize("mrt", [False, True])
def test_full_ensemble_of_64_channels_matches_separate_runs(mrt):
    """The 64-case ensemble (D in 8..32, Re in [60, 200], U = 0.05, tau from
    Re): 130 steps together, then every case checked against its own run."""
    cases = ensemble(mrt=mrt)
    ens = lbm.Ensemble([lbm.make_params(**kw) for kw in cases])
    ens.step(130)
    ens.sync()
    for i, kw in enumerate(cases):
        f_alone, forces_alone = _alone(kw, 130)
        assert np.array_equal(ens.get_populations(i, np.float64), f_alone), i
        assert np.array_equal(ens.forces(i)[0], forces_alone[0]), i


def test_ensemble_reports_only_the_diverging_case():
    cases = [dict(channel(8, u=0.05), tau=0.6), dict(nx=82, ny=42, diameter=2, u_in=0.2, tau=0.5001),
             dict(channel(8, u=0.05), tau=0.65)]
    ens = lbm.Ensemble([lbm.make_params(**kw) for kw in cases])
    ens.step(3000)
    with pytest.raises(lbm.DivergedError):
        ens.sync()
    assert ens.info(0)[1] == 0 and ens.info(2)[1] == 0
    assert ens.info(1)[1] > 0
    f_alone, _ = _alone(cases[2], 3000)
    assert np.array_equal(ens.get_populations(2, np.float64), f_alone)


def test_autotuner_picks_a_variant_and_caches_it(tmp_path):
    cache = str(tmp_path / "tune.txt")
    cases = [lbm.make_params(**channel(d, u=0.05)) for d in (8, 12, 16)]
    ens = lbm.Ensemble(cases, tune_cache=cache)
    v = ens.variant
    assert 1 <= v <= lbm.num_variants()
    text = open(cache).read().split()
    assert len(text) == 2 and int(text[1]) == v
    ens2 = lbm.Ensemble(cases, tune_cache=cache)  # cache hit
    assert ens2.variant == v
    lat = lbm.Lattice(lbm.make_params(**channel(10, u=0.05)))
    best = lat.autotune(10, cache)
    assert 1 <= best <= lbm.num_variants()
    assert len(open(cache).read().split()) == 4


def test_ensemble_at_the_reynolds_tau_needs_mrt():
    """tau = 3 U D / Re + 1/2 spans 0.507-0.56 over the 64 cases: with BGK
    most of them blow up within a few thousand steps, with the MRT rates of
    Sec. 2.1 none does (the paper's reason for MRT)."""
    out = {}
    for mrt in (False, True):
        cases = ensemble(mrt=mrt)
        ens = lbm.Ensemble([lbm.make_params(**kw) for kw in cases])
        ens.step(4000)
        out[mrt] = sum(1 for i in range(len(cases)) if ens.info(i)[1])
        ens.close()
    note(f"  diverged cases in 4000 steps: BGK {out[False]}, MRT {out[True]}")
    assert out[True] == 0
    assert out[False] >= 32


def test_smallest_and_largest_of_the_64_cases_match_the_oracle():
    """The 64-case MRT ensemble in one set of launches (the autotuned
    variant); its smallest (D = 8) and largest (D = 32) cases start from a
    seeded disturbed state and after 200 steps their populations, fields and
    per-step forces are compared with the FP64 oracle's at 1e-5."""
    import oracle
    from lbm_inputs import perturbed_populations
    from parity_util import WT, _oracle_kwargs, compare_state

    cases = ensemble(mrt=True)
    sizes = [c["nx"] * c["ny"] for c in cases]
    picks = [int(np.argmin(sizes)), int(np.argmax(sizes))]
    ens = lbm.Ensemble([lbm.make_params(**kw) for kw in cases])
    note(f"ensemble variant {lbm.variant_name(ens.variant)}; cases {picks}")
    f0 = {}
    for c in picks:
        kw = cases[c]
        f0[c] = perturbed_populations(2605 + c, kw["ny"], kw["nx"], WT, 0.03, dtype=np.float32)
        ens.set_populations(c, f0[c])
    ens.step(200)
    ens.sync()

    class _View:
        """The Lattice-like view compare_state reads."""

        def __init__(self, c):
            self.c = c

        def fields(self):
            return ens.fields(self.c)

        def get_populations(self, dtype):
            return ens.get_populations(self.c, dtype)

    for c in picks:
        kw = cases[c]
        note(f"  case {c}: D = {kw['diameter']}, {kw['nx']} x {kw['ny']}, Re = {kw['re']:.2f}")
        o = oracle.Oracle(oracle.OracleParams(**_oracle_kwargs(kw)))
        o.set_fstar(f0[c].astype(np.float64))
        ofx, ofy, bad = o.step(200)
        assert bad == 0
        solid = oracle.digitise(oracle.OracleParams(**_oracle_kwargs(kw)))
        compare_state(_View(c), o, solid)
        fx, fy, _, _ = ens.forces(c)
        note(f"  forces: max |dFx| {np.abs(fx - ofx).max():.2e}, max |dFy| {np.abs(fy - ofy).max():.2e}")
        assert np.abs(fx - ofx).max() < 1e-5 and np.abs(fy - ofy).max() < 1e-5


@pytest.mark.timeout(900)
def test_step_budgets_give_each_case_the_statistics_of_its_own_run():
    """C4 as the benchmark states it: the 64 MRT cases in one ensemble, each
    retiring after its own budget of 3000 D steps (150 convective units).
    Eight cases (D spread over 8..32) are also run alone; their force
    histories must equal the ensemble's bit for bit, and their shedding
    statistics over the last five periods (mean Cd, lift amplitude, St) are
    then the same.  Per-case MLUPS of the ensemble (a case's node updates over
    the ensemble's wall time) are printed next to those of the separate
    runs."""
    import time

    cases = ensemble(mrt=True)
    budgets = [3000 * c["diameter"] for c in cases]
    ens = lbm.Ensemble([lbm.make_params(**kw) for kw in cases], budgets=budgets)
    note(f"ensemble variant {lbm.variant_name(ens.variant)}; budgets {min(budgets)}..{max(budgets)} steps")
    t0 = time.perf_counter()
    ens.step(max(budgets))
    ens.sync()
    t_ens = time.perf_counter() - t0
    order = np.argsort([c["diameter"] for c in cases])
    picks = [int(order[i]) for i in np.linspace(0, len(cases) - 1, 8).round().astype(int)]
    shedding = 0
    for c in picks:
        kw, b = cases[c], budgets[c]
        steps, bad = ens.info(c)
        assert (steps, bad) == (b, 0), c
        lat = lbm.Lattice(lbm.make_params(**kw))
        t0 = time.perf_counter()
        lat.step(b)
        lat.sync()
        t_alone = time.perf_counter() - t0
        a = lat.forces()
        e = ens.forces(c)
        for x, y in zip(e, a):
            assert np.array_equal(x, y), c
        nodes = kw["nx"] * kw["ny"]
        msg = (f"  case {c}: D {kw['diameter']} Re {kw['re']:.1f}, {b} steps; ensemble {nodes * b / t_ens / 1e6:.0f}"
               f" MLUPS of its own, alone {nodes * b / t_alone / 1e6:.0f} MLUPS")
        lat.close()
        try:
            se = lbm.shedding_stats(e[2], e[3], kw["diameter"], kw["u_in"], 5)
            sa = lbm.shedding_stats(a[2], a[3], kw["diameter"], kw["u_in"], 5)
        except lbm.RangeError:
            note(msg + "; fewer than five lift periods")
            continue
        assert se == sa
        shedding += 1
        note(msg + f"; mean Cd {se['mean_cd']:.4f} Cl amp {se['cl_amp']:.4f} St {se['st']:.4f}")
    assert shedding >= 6


@pytest.mark.parametrize("graphs", [True, False])
def test_short_force_history_keeps_the_newest_steps(graphs):
    """A history ring smaller than the 96 steps the device folds at once:
    the newest hist_capacity steps must be the forces a long history holds
    for the same steps (two steps of a fold never share a slot)."""
    kw = dict(channel(8, u=0.05), tau=0.6)
    full = lbm.Lattice(lbm.make_params(**kw))
    full.step(250)
    ref = full.forces()
    for cap in (10, 95):
        lat = lbm.Lattice(lbm.make_params(**kw, hist_capacity=cap))
        lat.set_graphs(graphs)
        lat.step(250)
        got = lat.forces(251 - cap, cap)
        for a, b in zip(got, ref):
            assert np.array_equal(a, b[-cap:]), cap
        with pytest.raises(lbm.RangeError):
            lat.forces(250 - cap, 1)
    ens = lbm.Ensemble([lbm.make_params(**kw, hist_capacity=10), lbm.make_params(**kw)])
    ens.step(250)
    got = ens.forces(0, 241, 10)
    for a, b in zip(got, ref):
        assert np.array_equal(a, b[-10:])
