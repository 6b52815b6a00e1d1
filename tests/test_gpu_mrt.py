"""GPU parity of the multiple-relaxation-time collision (Eq. 6 with the
rates of Sec. 2.1) against the FP64 oracle, through the C ABI.

Same bar as the BGK path: |d rho|, |d u|, |d f*| <= 1e-5 after the stated
steps; force coefficients within 1e-3; kernel variants bit for bit.
"""
import numpy as np
import pytest

import oracle
import paper_2605_02185_amd as lbm
from lbm_inputs import PAPER_RATES, WORKLOADS, channel, perturbed_populations
from parity_util import ALL_WALLS, WT, _oracle_kwargs, compare_state, note, run_both

pytestmark = pytest.mark.gpu

MRT = dict(collision=lbm.COLLISION_MRT, s_rates=PAPER_RATES)


@pytest.mark.parametrize("nx,ny,tau", [(3, 3, 0.7), (64, 64, 0.52), (517, 133, 0.506)])
def test_periodic_box_random_state(nx, ny, tau):
    kw = dict(nx=nx, ny=ny, tau=tau, u_in=0.0, x_periodic=True, wall=lbm.WALL_PERIODIC, **MRT)
    lat, o, _, _ = run_both(kw, 40, seed=nx * 1000 + ny + 1)
    compare_state(lat, o)


def test_rates_of_every_moment_reach_the_kernel():
    """Distinct rates on each non-conserved moment, so a rate applied to the
    wrong moment shows."""
    kw = dict(nx=97, ny=41, tau=0.6, u_in=0.0, x_periodic=True, wall=lbm.WALL_PERIODIC,
              collision=lbm.COLLISION_MRT, s_rates=(1, 1.3, 0.7, 1, 1.5, 1, 0.9, 1.7, 1.2))
    lat, o, _, _ = run_both(kw, 30, seed=41, amp=0.1)
    compare_state(lat, o)


@pytest.mark.parametrize("wall", ALL_WALLS)
@pytest.mark.parametrize("outlet", [lbm.OUTLET_COPY_ALL, lbm.OUTLET_COPY_UNKNOWN])
def test_channel_every_boundary_random_state(wall, outlet):
    kw = dict(channel(6, u=0.06), tau=0.52, wall=wall, outlet_mode=outlet, **MRT)
    lat, o, (fx, fy, _, _), (ofx, ofy) = run_both(kw, 60, seed=200 + 10 * wall + outlet)
    solid = oracle.digitise(oracle.OracleParams(**_oracle_kwargs(kw)))
    compare_state(lat, o, solid)
    assert np.abs(fx - ofx).max() < 1e-5 and np.abs(fy - ofy).max() < 1e-5


def test_uniform_rates_agree_with_bgk():
    """All rates 1/tau: Eq. 6 is Eq. 2; the two GPU paths agree to FP32
    rounding."""
    tau = 0.6
    kw = dict(channel(6, u=0.06), tau=tau)
    out = []
    for extra in ({}, dict(collision=lbm.COLLISION_MRT, s_rates=(1 / tau,) * 9)):
        lat = lbm.Lattice(lbm.make_params(**kw, **extra))
        lat.set_populations(perturbed_populations(5, kw["ny"], kw["nx"], WT, 0.05, dtype=np.float32))
        lat.step(100)
        out.append(lat.get_populations(np.float64))
    err = np.abs(out[0] - out[1]).max()
    note(f"  MRT(1/tau) vs BGK max |df| {err:.2e}")
    assert err < 2e-6


@pytest.mark.parametrize("wall", ALL_WALLS)
def test_paper_lattice_fields_and_forces(wall):
    """800 x 400, D = 20, U = 0.02, Re = 100 (tau = 0.512), MRT, every wall
    treatment: 1500 steps from the initial state, every node and the force
    trace against the oracle."""
    kw = dict(WORKLOADS["cyl_d20_mrt"], wall=wall)
    lat, o, (fx, fy, cd, cl), (ofx, ofy) = run_both(kw, 1500)
    solid = oracle.digitise(oracle.OracleParams(**_oracle_kwargs(kw)))
    compare_state(lat, o, solid)
    q = 0.5 * kw["u_in"] ** 2 * kw["diameter"]
    dcd, dcl = np.abs(cd - ofx / q).max(), np.abs(cl - ofy / q).max()
    note(f"  max |dCd| {dcd:.2e} max |dCl| {dcl:.2e}")
    assert dcd < 1e-3 and dcl < 1e-3


def test_paper_lattice_two_steps_all_nodes_disturbed():
    """1600 x 800 (D = 40, the paper's grid-independence lattice) from a
    disturbed state: every population after two steps."""
    kw = dict(WORKLOADS["cyl_d40_mrt"])
    lat, o, (fx, fy, _, _), (ofx, ofy) = run_both(kw, 2, seed=40, amp=0.02)
    f = lat.get_populations(np.float64)
    of = o.get_fstar()
    solid = oracle.digitise(oracle.OracleParams(**_oracle_kwargs(kw)))
    err = np.abs(f - of)[:, solid == 0].max()
    note(f"  max |df*| {err:.2e}")
    assert err <= 1e-5
    assert np.abs(fx - ofx).max() < 1e-5 and np.abs(fy - ofy).max() < 1e-5


def test_variants_are_bitwise_identical():
    kw = dict(WORKLOADS["cyl_d20_mrt"])
    ref = None
    for v in range(1, lbm.num_variants() + 1):
        lat = lbm.Lattice(lbm.make_params(**kw))
        lat.set_variant(v)
        lat.set_populations(perturbed_populations(3, kw["ny"], kw["nx"], WT, 0.05, dtype=np.float32))
        lat.step(23)
        f, forces = lat.get_populations(), lat.forces()
        lat.close()
        note(f"  variant {lbm.variant_name(v)}")
        if ref is None:
            ref = (f, forces)
            continue
        assert np.array_equal(f, ref[0]), v
        for a, b in zip(forces, ref[1]):
            if a is not None:
                assert np.array_equal(a, b), v
