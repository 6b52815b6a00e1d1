"""GPU parity of the interpolated (Bouzidi) bounce-back on the cylinder
(Sec. 2.4) against the FP64 oracle, through the C ABI, and bit-for-bit
agreement of every kernel variant.  Same bar as the half-way path:
|d rho|, |d u|, |d f*| <= 1e-5 after the stated steps, forces to 1e-5
(lattice units) or Cd/Cl to 1e-3."""
import numpy as np
import pytest

import oracle
import paper_2605_02185_amd as lbm
from lbm_inputs import PAPER_RATES, WORKLOADS, channel, perturbed_populations
from parity_util import WT, _oracle_kwargs, compare_state, note, run_both

pytestmark = pytest.mark.gpu

INTERP = dict(bounce=lbm.BOUNCE_INTERP)
MRT = dict(collision=lbm.COLLISION_MRT, s_rates=PAPER_RATES)


@pytest.mark.parametrize("extra", [
    dict(wall=lbm.WALL_FREE_SLIP),
    dict(wall=lbm.WALL_MOVING_BB, outlet_mode=lbm.OUTLET_COPY_UNKNOWN),
    dict(wall=lbm.WALL_PERIODIC, **MRT),
    dict(wall=lbm.WALL_NEBB, tau=0.7, cx2=127, cy2=125),  # off-centre disk: other fractions
])
def test_channel_random_state(extra):
    kw = dict(channel(6, u=0.06), tau=0.6, **INTERP)
    kw.update(extra)
    lat, o, (fx, fy, _, _), (ofx, ofy) = run_both(kw, 60, seed=300 + len(str(extra)))
    solid = oracle.digitise(oracle.OracleParams(**_oracle_kwargs(kw)))
    compare_state(lat, o, solid)
    assert np.abs(fx - ofx).max() < 1e-5 and np.abs(fy - ofy).max() < 1e-5


def test_paper_lattice_fields_and_forces():
    """800 x 400, D = 20, U = 0.02, Re = 100, MRT: 1500 steps from the initial
    state, every node and the force trace against the oracle."""
    kw = dict(WORKLOADS["cyl_d20_mrt"], **INTERP)
    lat, o, (fx, fy, cd, cl), (ofx, ofy) = run_both(kw, 1500)
    solid = oracle.digitise(oracle.OracleParams(**_oracle_kwargs(kw)))
    compare_state(lat, o, solid)
    q = 0.5 * kw["u_in"] ** 2 * kw["diameter"]
    dcd, dcl = np.abs(cd - ofx / q).max(), np.abs(cl - ofy / q).max()
    note(f"  max |dCd| {dcd:.2e} max |dCl| {dcl:.2e}")
    assert dcd < 1e-3 and dcl < 1e-3


def test_full_size_multi_step_all_nodes():
    """3280 x 1680 (D = 80, the four-step kernel by default) from a
    disturbed state: every population after one launch."""
    kw = dict(WORKLOADS["cyl_d80"], **INTERP)
    lat, o, (fx, fy, _, _), (ofx, ofy) = run_both(kw, 4, seed=80, amp=0.02)
    f = lat.get_populations(np.float64)
    of = o.get_fstar()
    solid = oracle.digitise(oracle.OracleParams(**_oracle_kwargs(kw)))
    err = np.abs(f - of)[:, solid == 0].max()
    note(f"  variant {lbm.variant_name(lat.variant)} max |df*| {err:.2e}")
    assert err <= 1e-5
    assert np.abs(fx - ofx).max() < 1e-5 and np.abs(fy - ofy).max() < 1e-5


@pytest.mark.parametrize("kw", [dict(channel(10, u=0.05), tau=0.6, **INTERP),
                                dict(WORKLOADS["cyl_d20_mrt"], **INTERP)])
def test_variants_are_bitwise_identical(kw):
    ref = None
    for v in range(1, lbm.num_variants() + 1):
        lat = lbm.Lattice(lbm.make_params(**kw))
        lat.set_variant(v)
        lat.set_populations(perturbed_populations(4, kw["ny"], kw["nx"], WT, 0.03, dtype=np.float32))
        lat.step(131)
        f, forces = lat.get_populations(), lat.forces()
        lat.close()
        if ref is None:
            ref = (f, forces)
            continue
        note(f"  variant {lbm.variant_name(v)}")
        assert np.array_equal(f, ref[0]), v
        for a, b in zip(forces, ref[1]):
            if a is not None:
                assert np.array_equal(a, b), v
