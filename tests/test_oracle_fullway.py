"""Pins of the oracle's full-way bounce-back on the cylinder (Sec. 3.1): solid
nodes take part in the streaming and their collision reverses what arrived,
so a population sent towards the wall comes back to its fluid node one step
later than with half-way bounce-back.

Checked here against that definition on a random state (where each value
goes, step by step), against the invariants it implies (the mass of fluid
and solid nodes together is conserved; at rest a solid node stays at rest),
and against the known fact that full and half-way bounce-back share their
steady states, with the wall force of a body-force channel balancing the
body force exactly.
"""
import numpy as np
import pytest

from oracle import BB_FULLWAY, BB_HALFWAY, WALL_PERIODIC, Oracle, OracleParams, digitise

CX = np.array([0, 1, 0, -1, 0, 1, -1, -1, 1])
CY = np.array([0, 0, 1, 0, -1, 1, 1, -1, -1])
OPP = np.array([0, 3, 4, 1, 2, 7, 8, 5, 6])
WT = np.array([4 / 9, 1 / 9, 1 / 9, 1 / 9, 1 / 9, 1 / 36, 1 / 36, 1 / 36, 1 / 36])

BOX = dict(nx=40, ny=33, diameter=11, cx2=41, cy2=33, u_in=0.05, tau=0.7, x_periodic=True,
           wall=WALL_PERIODIC)


def _random_state(p, seed, amp=0.05):
    rng = np.random.default_rng(seed)
    return WT[:, None, None] * (1.0 + amp * rng.uniform(-1, 1, (9, p.ny, p.nx)))


def _wall_links(solid):
    """(k, sx, sy, x, y): fluid node (x, y) whose neighbour (sx, sy) = x + c_k
    is solid; everything periodic."""
    ny, nx = solid.shape
    out = []
    for y in range(ny):
        for x in range(nx):
            if solid[y, x]:
                continue
            for k in range(1, 9):
                sx, sy = (x + CX[k]) % nx, (y + CY[k]) % ny
                if solid[sy, sx]:
                    out.append((k, sx, sy, x, y))
    return out


def test_population_comes_back_one_step_later():
    """f*_k(x) sent towards the solid node x + c_k sits there in slot k after
    one step, leaves reversed, and is f_opp(k)(x) after the second step; with
    half-way bounce-back it is f_opp(k)(x) after the first.  What the solid
    node held in the given (post-collision) state is what reaches x first."""
    p = OracleParams(**BOX, bounce=BB_FULLWAY)
    solid = digitise(p)
    links = _wall_links(solid)
    assert len(links) > 40
    f0 = _random_state(p, 5)
    o = Oracle(p)
    o.set_fstar(f0)
    o.step(1)
    f1, fs1 = o.get_f(), o.get_fstar()
    o.step(1)
    f2 = o.get_f()
    for k, sx, sy, x, y in links:
        assert f1[k, sy, sx] == f0[k, y, x]
        # the given state is post-collision at the solid nodes too: it
        # streams out unchanged in the first step
        assert f1[OPP[k], y, x] == f0[OPP[k], sy, sx]
        assert fs1[OPP[k], sy, sx] == f1[k, sy, sx]
        assert f2[OPP[k], y, x] == f0[k, y, x]

    h = Oracle(OracleParams(**BOX, bounce=BB_HALFWAY))
    h.set_fstar(f0)
    h.step(1)
    g1 = h.get_f()
    for k, sx, sy, x, y in links:
        assert g1[OPP[k], y, x] == f0[k, y, x]


def test_mass_of_fluid_and_solid_is_conserved():
    """Periodic box: streaming moves every value of every node and both the
    collision and the reversal keep each node's mass, so the sum over all
    nodes stays put while the fluid alone exchanges mass with the wall."""
    p = OracleParams(**BOX, bounce=BB_FULLWAY)
    solid = digitise(p).astype(bool)
    o = Oracle(p)
    f0 = _random_state(p, 9)
    o.set_fstar(f0)
    m0 = f0.sum()
    fluid = []
    for _ in range(20):
        o.step(10)
        f = o.get_f()
        assert abs(f.sum() - m0) < 1e-11 * m0
        fluid.append(f[:, ~solid].sum())
    assert np.ptp(fluid) > 1e-6  # the solid really holds mass in transit


def test_solid_nodes_start_and_stay_at_rest_without_traffic():
    """From the initial state the solid nodes are at rest (f = w); the
    interior ones, which no fluid population reaches, stay there."""
    p = OracleParams(**BOX, bounce=BB_FULLWAY)
    solid = digitise(p).astype(bool)
    o = Oracle(p)
    f = o.get_f()
    assert np.array_equal(f[:, solid], np.broadcast_to(WT[:, None], (9, solid.sum())))
    o.step(50)
    f = o.get_f()
    ny, nx = solid.shape
    deep = np.zeros_like(solid)
    for y in range(ny):
        for x in range(nx):
            deep[y, x] = all(solid[(y + CY[k]) % ny, (x + CX[k]) % nx] for k in range(9))
    assert deep.sum() > 20
    assert np.abs(f[:, deep] - WT[:, None]).max() < 1e-15


def _channel(ny, bounce, tau=0.8, g=1e-6):
    nx = 3
    solid = np.zeros((ny, nx), np.uint8)
    solid[0, :] = solid[-1, :] = 1
    p = OracleParams(nx=nx, ny=ny, tau=tau, x_periodic=True, wall=WALL_PERIODIC, gx=g, u_in=0.0,
                     bounce=bounce)
    o = Oracle(p, solid)
    o.set_f(np.broadcast_to(WT[:, None, None], (9, ny, nx)).copy())
    nu = (tau - 0.5) / 3
    fx, _, _ = o.step(int(8 * ny * ny / nu))
    rho, ux, _ = o.fields()
    return rho[1:-1], ux[1:-1, 1], fx[-1]


@pytest.mark.parametrize("tau", [0.6, 0.8, 1.2])
def test_steady_channel_matches_half_way(tau):
    """Body-force channel between two solid rows: the steady states of the
    two schemes agree, and in both the force on the walls balances the
    body force on the fluid, sum(rho) g per step."""
    g = 1e-6
    rf, uf, ff = _channel(14, BB_FULLWAY, tau, g)
    rh, uh, fh = _channel(14, BB_HALFWAY, tau, g)
    assert np.abs(uf - uh).max() < 1e-6 * uh.max()
    assert ff == pytest.approx(g * rf.sum(), rel=1e-6)
    assert fh == pytest.approx(g * rh.sum(), rel=1e-6)
