"""GPU parity: liblbm.so (gfx950 kernels, through the C ABI) against the FP64
oracle on identical seeded inputs.

Tolerance: |d rho|, |d u| and |d f*| <= 1e-5 after the stated number of steps
(FP32 storage and arithmetic against FP64); force coefficients within 1e-3.
Integer outputs (geometry, step counters, divergence step) must match exactly;
repeated runs and kernel variants must match bit for bit.
"""
import re

import numpy as np
import pytest

import oracle
import paper_2605_02185_amd as lbm
from lbm_inputs import WORKLOADS, channel, perturbed_populations
from parity_util import ALL_WALLS, TOL, WT, _oracle_kwargs, compare_state, note, run_both

pytestmark = pytest.mark.gpu


# ------------------------------------------------------------------ boxes
@pytest.mark.parametrize("nx,ny", [(3, 3), (64, 64), (517, 133)])
def test_periodic_box_random_state(nx, ny):
    kw = dict(nx=nx, ny=ny, tau=0.62, u_in=0.0, x_periodic=True, wall=lbm.WALL_PERIODIC)
    lat, o, _, _ = run_both(kw, 40, seed=nx * 1000 + ny)
    compare_state(lat, o)
    f = lat.get_populations(np.float64)
    m0 = perturbed_populations(nx * 1000 + ny, ny, nx, WT, 0.05, dtype=np.float32).astype(np.float64).sum()
    assert abs(f.sum() - m0) / m0 < 1e-6  # mass, to FP32 accumulation


@pytest.mark.parametrize("wall", [lbm.WALL_NEBB, lbm.WALL_MOVING_BB, lbm.WALL_FREE_SLIP])
def test_x_periodic_channel_with_walls(wall):
    kw = dict(nx=300, ny=37, tau=0.7, u_in=0.04, x_periodic=True, wall=wall, u_wall_bottom=0.0)
    lat, o, _, _ = run_both(kw, 50, seed=7 + wall)
    compare_state(lat, o)


# --------------------------------------------------- cylinder channels
@pytest.mark.parametrize("wall", ALL_WALLS)
@pytest.mark.parametrize("outlet", [lbm.OUTLET_COPY_ALL, lbm.OUTLET_COPY_UNKNOWN])
def test_channel_every_boundary_random_state(wall, outlet):
    """D = 6 channel (246 x 126: one full and one ragged tile per row), every
    wall mode and outlet mode, from a disturbed state."""
    kw = dict(channel(6, u=0.06), tau=0.6, wall=wall, outlet_mode=outlet)
    lat, o, (fx, fy, _, _), (ofx, ofy) = run_both(kw, 60, seed=100 + 10 * wall + outlet)
    solid = oracle.digitise(oracle.OracleParams(**_oracle_kwargs(kw)))
    compare_state(lat, o, solid)
    assert np.abs(fx - ofx).max() < 1e-5 and np.abs(fy - ofy).max() < 1e-5


@pytest.mark.parametrize("nx", [65, 128, 129, 40])
@pytest.mark.parametrize("wall,outlet", [(lbm.WALL_MOVING_BB, lbm.OUTLET_COPY_ALL),
                                         (lbm.WALL_FREE_SLIP, lbm.OUTLET_COPY_UNKNOWN)])
def test_outlet_at_every_wave_lane_position(nx, wall, outlet):
    """Channels whose outlet column falls on lane 0 of a wave (nx = 65, 129:
    the one-step kernel's boundary waves then take the node-by-node path, as
    the left neighbour the outlet copies is in the previous wave), on lane 63
    (nx = 128) or in the inlet's wave (nx = 40), with a small cylinder, from a
    disturbed state: against the oracle, then bit for bit across one-step
    variants with one, two and four nodes per lane and two fused ones."""
    kw = dict(nx=nx, ny=37, diameter=4, cx2=28, cy2=36, u_in=0.05, tau=0.62, wall=wall, outlet_mode=outlet)
    seed = 300 + nx + wall
    lat, o, (fx, fy, _, _), (ofx, ofy) = run_both(kw, 30, seed=seed)
    solid = oracle.digitise(oracle.OracleParams(**_oracle_kwargs(kw)))
    compare_state(lat, o, solid)
    assert np.abs(fx - ofx).max() < 1e-5 and np.abs(fy - ofy).max() < 1e-5
    by_name = {lbm.variant_name(v): v for v in range(1, lbm.num_variants() + 1)}
    ref_f, ref_forces = _run_gpu(kw, 37, by_name["v1_ty1_nt"], seed)
    for name in ("v1_ty1_xcd", "v2_ty1_nt", "v4_ty1_nt", "t2_h4", "t3_h8_s2"):
        f, forces = _run_gpu(kw, 37, by_name[name], seed)
        note(f"  variant {name}")
        assert np.array_equal(f, ref_f), name
        for a, b in zip(forces, ref_forces):
            if a is not None:
                assert np.array_equal(a, b), name


@pytest.mark.parametrize("wall", ALL_WALLS)
def test_uniform_flow_fixed_point(wall):
    kw = dict(nx=300, ny=70, u_in=0.08, tau=0.7, wall=wall, perturb_amp=0.0)
    lat, o, _, _ = run_both(kw, 20)
    compare_state(lat, o, tol=1e-6)


def test_minimal_channel():
    kw = dict(nx=3, ny=3, u_in=0.05, tau=0.8, wall=lbm.WALL_NEBB)
    lat, o, _, _ = run_both(kw, 10, seed=3)
    compare_state(lat, o)


def test_c1_fields_after_200_steps():
    """410 x 210, D = 10, U = 0.1, tau = 0.53, free-slip: fields within 1e-5."""
    kw = dict(WORKLOADS["cyl_d10"])
    lat, o, (fx, fy, cd, cl), (ofx, ofy) = run_both(kw, 200)
    solid = oracle.digitise(oracle.OracleParams(**_oracle_kwargs(kw)))
    compare_state(lat, o, solid)
    q = 0.5 * kw["u_in"] ** 2 * kw["diameter"]
    assert np.abs(cd - ofx / q).max() < 1e-3
    assert np.abs(cl - ofy / q).max() < 1e-3


def test_c1_force_trace_2000_steps():
    kw = dict(WORKLOADS["cyl_d10"])
    lat, o, (fx, fy, cd, cl), (ofx, ofy) = run_both(kw, 2000)
    q = 0.5 * kw["u_in"] ** 2 * kw["diameter"]
    dcd = np.abs(cd - ofx / q).max()
    dcl = np.abs(cl - ofy / q).max()
    note(f"  max |dCd| {dcd:.2e} max |dCl| {dcl:.2e}")
    assert dcd < 1e-3 and dcl < 1e-3


@pytest.mark.parametrize("name", ["cyl_d80", "cyl_d160", "slab_d160_of8"])
def test_full_size_multi_step_all_nodes(name):
    """The benchmark's lattices in the benchmark's launch configuration:
    four steps from a disturbed state (one launch of the four-step kernel
    by default at D = 80 and D = 160, a three-step and a one-step launch on
    the slab), every node against the oracle."""
    kw = dict(WORKLOADS[name])
    lat, o, (fx, fy, _, _), (ofx, ofy) = run_both(kw, 4, seed=160, amp=0.02)
    f = lat.get_populations(np.float64)
    of = o.get_fstar()
    solid = oracle.digitise(oracle.OracleParams(**_oracle_kwargs(kw)))
    err = np.abs(f - of)[:, solid == 0].max()
    note(f"  {name}: max |df*| {err:.2e}, forces {fx} vs {ofx}")
    assert err <= TOL
    assert np.abs(fx - ofx).max() < 1e-5 and np.abs(fy - ofy).max() < 1e-5


# ----------------------------------------------- determinism and variants
def _run_gpu(kw, steps, variant=0, seed=None):
    lat = lbm.Lattice(lbm.make_params(**kw))
    if variant:
        lat.set_variant(variant)
    if seed is not None:
        lat.set_populations(perturbed_populations(seed, kw["ny"], kw["nx"], WT, 0.05, dtype=np.float32))
    lat.step(steps)
    return lat.get_populations(), lat.forces()


@pytest.mark.parametrize("kw", [dict(WORKLOADS["cyl_d10"]),
                                dict(nx=517, ny=133, tau=0.6, u_in=0.0, x_periodic=True, wall=lbm.WALL_PERIODIC)])
def test_variants_and_repeats_are_bitwise_identical(kw):
    seed = None if "diameter" in kw else 9
    ref_f, ref_forces = _run_gpu(kw, 37, 0, seed)
    for v in range(1, lbm.num_variants() + 1):
        f, forces = _run_gpu(kw, 37, v, seed)
        note(f"  variant {lbm.variant_name(v)}")
        assert np.array_equal(f, ref_f), v
        for a, b in zip(forces, ref_forces):
            if a is not None:
                assert np.array_equal(a, b), v


def test_checkpoint_round_trip_is_bitwise():
    """A float64 checkpoint holds the stored FP32 deviations exactly."""
    kw = dict(WORKLOADS["cyl_d10"])
    a = lbm.Lattice(lbm.make_params(**kw))
    a.step(150)
    mid = a.get_populations(np.float64)
    a.step(70)
    end = a.get_populations(np.float64)
    fa = a.forces(151, 70)
    b = lbm.Lattice(lbm.make_params(**kw))
    b.set_populations(mid)
    b.step(70)
    assert np.array_equal(b.get_populations(np.float64), end)
    assert np.array_equal(b.forces(1, 70)[0], fa[0])


def test_force_ring_wraps_and_reports_range():
    kw = dict(WORKLOADS["cyl_d10"], hist_capacity=100)
    a = lbm.Lattice(lbm.make_params(**kw))
    a.step(250)
    fx, fy, _, _ = a.forces(151, 100)
    b = lbm.Lattice(lbm.make_params(**dict(WORKLOADS["cyl_d10"])))
    b.step(250)
    gx, gy, _, _ = b.forces(151, 100)
    assert np.array_equal(fx, gx) and np.array_equal(fy, gy)
    with pytest.raises(lbm.RangeError):
        a.forces(150, 1)
    with pytest.raises(lbm.RangeError):
        a.forces(250, 2)
    assert a.forces(251, 0)[0].size == 0
    a.step(0)
    assert a.t == 250


# --------------------------------------------------------- failure paths
def test_divergence_is_reported():
    kw = dict(nx=82, ny=42, diameter=2, u_in=0.2, tau=0.5001)
    lat = lbm.Lattice(lbm.make_params(**kw))
    lat.step(3000)
    with pytest.raises(lbm.DivergedError):
        lat.sync()
    s = lat.diverged_step()
    o = oracle.Oracle(oracle.OracleParams(**kw))
    _, _, obad = o.step(3000)
    note(f"  diverged at GPU step {s}, oracle step {obad}")
    assert s > 0 and obad > 0


def test_nan_state_is_reported_at_step_one():
    kw = dict(WORKLOADS["cyl_d10"])
    lat = lbm.Lattice(lbm.make_params(**kw))
    f = lat.get_populations()
    f[3, 100, 200] = np.nan
    lat.set_populations(f)
    lat.step(5)
    assert lat.diverged_step() == 1
    with pytest.raises(lbm.DivergedError):
        lat.forces(1, 5)


def test_device_buffers_round_trip():
    import torch

    kw = dict(WORKLOADS["cyl_d10"])
    lat = lbm.Lattice(lbm.make_params(**kw))
    lat.step(10)
    t = torch.empty((9, kw["ny"], kw["nx"]), dtype=torch.float64, device="cuda")
    lat.get_populations_device(t)
    host = lat.get_populations(np.float64)
    assert np.array_equal(t.cpu().numpy(), host)
    rho = torch.empty((kw["ny"], kw["nx"]), dtype=torch.float32, device="cuda")
    lat.fields_device(rho, None, None)
    assert np.array_equal(rho.cpu().numpy(), lat.fields()[0])
    t32 = t.float()
    lat.set_populations_device(t32)
    assert np.array_equal(lat.get_populations(), t32.cpu().numpy())


def test_graph_replay_matches_plain_launches():
    """lbm_step replays captured 96-step graphs; several replays with eager
    work in between must match plain launches bit for bit."""
    kw = dict(channel(6, u=0.06), tau=0.6, wall=lbm.WALL_NEBB)
    a = lbm.Lattice(lbm.make_params(**kw))
    b = lbm.Lattice(lbm.make_params(**kw))
    b.set_graphs(False)
    for n in (5, 64, 130, 1, 200, 63, 64):
        a.step(n)
        b.step(n)
        fa = a.get_populations(np.float64)  # eager work between replays
        assert np.array_equal(fa, b.get_populations(np.float64)), n
        assert np.array_equal(a.fields()[1], b.fields()[1])
    for x, y in zip(a.forces(), b.forces()):
        assert np.array_equal(x, y)
    assert a.t == b.t == 527


# ------------------------------------------- two steps per launch
TWO_STEP = [v for v in range(1, lbm.num_variants() + 1) if lbm.variant_name(v)[:3] in ("t2_", "t3_", "t4_")]


def _two_step_cases():
    cases = []
    for wall in ALL_WALLS:
        for outlet in (lbm.OUTLET_COPY_ALL, lbm.OUTLET_COPY_UNKNOWN):
            cases.append(dict(channel(6, u=0.06), tau=0.6, wall=wall, outlet_mode=outlet))
    cases += [
        dict(nx=3, ny=3, tau=0.62, u_in=0.0, x_periodic=True, wall=lbm.WALL_PERIODIC),
        dict(nx=64, ny=5, tau=0.62, u_in=0.0, x_periodic=True, wall=lbm.WALL_PERIODIC),
        dict(nx=125, ny=70, tau=0.7, u_in=0.04, x_periodic=True, wall=lbm.WALL_NEBB, u_wall_bottom=0.0),
        dict(nx=300, ny=37, tau=0.7, u_in=0.04, x_periodic=True, wall=lbm.WALL_MOVING_BB, u_wall_bottom=0.0),
        dict(nx=63, ny=9, tau=0.6, u_in=0.05, wall=lbm.WALL_FREE_SLIP),  # outlet at lane 62 of one strip
        dict(nx=3, ny=3, tau=0.8, u_in=0.05, wall=lbm.WALL_NEBB),
        dict(channel(6, u=0.06), tau=0.52, collision=lbm.COLLISION_MRT,
             s_rates=(1, 1.1, 1.1, 1, 1.1, 1, 1.1, 0, 0)),
        dict(channel(9, u=0.05, re=150), tau=0.58, wall=lbm.WALL_PERIODIC, collision=lbm.COLLISION_MRT,
             s_rates=(1, 1.1, 1.1, 1, 1.1, 1, 1.1, 0, 0)),
    ]
    return cases


@pytest.mark.parametrize("case", range(len(_two_step_cases())))
def test_two_step_variants_match_one_step_bitwise(case):
    """The two- and three-step kernels (f*(t+1), f*(t+2) kept in registers)
    give the one-step kernel's populations and force history bit for bit, for
    every wall and outlet treatment, periodic boxes down to 3 x 3, step
    counts that leave single steps (which then run alone) and graph replay."""
    kw = _two_step_cases()[case]
    steps = 131  # a 96-step graph, then plain launches of every size
    seed = 500 + case
    ref = _run_gpu(kw, steps, 0, seed)
    for v in TWO_STEP:
        note(f"  {kw} variant {lbm.variant_name(v)}")
        f, forces = _run_gpu(kw, steps, v, seed)
        assert np.array_equal(f, ref[0]), v
        for a, b in zip(forces, ref[1]):
            if a is not None:
                assert np.array_equal(a, b), v


@pytest.mark.parametrize("name", ["cyl_d40", "cyl_d80"])
def test_tall_segment_variants_match_one_step_bitwise(name):
    """Four steps per launch with tall segments (16 to 48 rows, each output
    row stored as it is made) on lattices large enough that most segments
    take that interior path: populations and forces after 101 steps (a
    96-step graph, then plain launches) equal the one-step kernel's bit for
    bit."""
    kw = dict(WORKLOADS[name])
    by_name = {lbm.variant_name(v): v for v in range(1, lbm.num_variants() + 1)}
    ref = _run_gpu(kw, 101, by_name["v1_ty1_nt"], 77)
    tall = [n for n in by_name if n.startswith("t4_h") and (int(re.match(r"t4_h(\d+)", n).group(1)) > 12
                                                         or re.match(r"t4_h\d+u", n))]
    assert tall
    for vn in ["t4_h8_s8"] + tall:
        note(f"  {name} variant {vn}")
        f, forces = _run_gpu(kw, 101, by_name[vn], 77)
        assert np.array_equal(f, ref[0]), vn
        for a, b in zip(forces, ref[1]):
            if a is not None:
                assert np.array_equal(a, b), vn


def test_default_variant_follows_the_lattice_size():
    """One step per launch below 2^18 nodes (cached stores, XCD bands), two
    from 2^18 (8-row segments, one-row boundary pieces loading all their
    rows first), three
    from 2^20 (2-row pieces), four from 2^21 (10-row interior segments
    storing rows as they are made, 10-row boundary pieces); variant 0
    restores the default."""
    small = lbm.Lattice(lbm.make_params(**WORKLOADS["cyl_d10"]))
    big = lbm.Lattice(lbm.make_params(**WORKLOADS["cyl_d40"]))
    assert lbm.variant_name(small.variant) == "v1_ty1_xcd"
    assert lbm.variant_name(big.variant) == "t3_h16u_s2"
    for name, want in (("cyl_d20_mrt", "t2_h8_u1"), ("slab_d160_of8", "t4_h10u_s10"), ("cyl_d80", "t4_h10u_s10"),
                       ("cyl_d160", "t4_h10u_s10")):
        lat = lbm.Lattice(lbm.make_params(**WORKLOADS[name]))
        assert lbm.variant_name(lat.variant) == want, name
        lat.close()
    big.set_variant(1)
    assert big.variant == 1
    big.set_variant(0)
    assert lbm.variant_name(big.variant) == "t3_h16u_s2"
