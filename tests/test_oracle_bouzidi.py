"""Pins of the oracle's interpolated (link-wise) bounce-back, Sec. 2.4: the
linear scheme of Bouzidi, Firdaouss & Lallemand (2001) with the wall
fraction q of each link.

The wall fractions are checked against a bisection of the circle equation,
the scheme against half-way bounce-back at q = 1/2, and its accuracy on a
body-force channel whose walls sit at fractional positions, where the exact
parabola is known.
"""
import math

import numpy as np
import pytest

from oracle import BB_HALFWAY, BB_INTERP, WALL_PERIODIC, Oracle, OracleParams

CX = np.array([0, 1, 0, -1, 0, 1, -1, -1, 1])
CY = np.array([0, 0, 1, 0, -1, 1, 1, -1, -1])
WT = np.array([4 / 9, 1 / 9, 1 / 9, 1 / 9, 1 / 9, 1 / 36, 1 / 36, 1 / 36, 1 / 36])


@pytest.mark.parametrize("D,cx2,cy2", [(8, 61, 60), (10, 60, 60), (13, 70, 65)])
def test_wall_fractions_bisect_the_circle(D, cx2, cy2):
    """q is where the link leaves the disk's circle (centre (cx2, cy2)/2,
    radius D/2), found here by bisection of the distance to the centre."""
    p = OracleParams(nx=80, ny=70, diameter=D, cx2=cx2, cy2=cy2, u_in=0.05, tau=0.6, bounce=BB_INTERP)
    node, k, q = Oracle(p).links()
    cx, cy, R = cx2 / 2, cy2 / 2, D / 2
    assert len(q) > 0 and np.all(q > 0) and np.all(q <= 1)
    for n, kk, qq in zip(node, k, q):
        x, y = n % p.nx, n // p.nx
        lo, hi = 0.0, 1.0  # outside at 0 (fluid node), inside or on at 1 (solid node)
        r = lambda t: math.hypot(x + t * CX[kk] - cx, y + t * CY[kk] - cy)
        assert r(0.0) > R and r(1.0) <= R + 1e-12
        for _ in range(60):
            mid = 0.5 * (lo + hi)
            if r(mid) > R:
                lo = mid
            else:
                hi = mid
        # the cut point lies on the circle, and no earlier point of the link
        # is inside it; where the link grazes the circle the bisection's
        # root is ill-conditioned, so the two agree to 1e-7 there
        assert abs(r(qq) - R) < 1e-10
        assert qq < 1e-6 or r(qq - 1e-6) > R
        assert abs(qq - 0.5 * (lo + hi)) < 1e-7


def test_half_fraction_is_half_way_bounce_back():
    """At q = 1/2 both branches of the scheme return f*_k(x): the run and the
    force history equal half-way bounce-back to round-off."""
    base = dict(nx=123, ny=63, diameter=9, cx2=61, cy2=63, u_in=0.06, tau=0.62, perturb_amp=0.05)
    a = Oracle(OracleParams(**base, bounce=BB_HALFWAY))
    b = Oracle(OracleParams(**base, bounce=BB_INTERP, q_fixed=0.5))
    fa, ya, _ = a.step(300)
    fb, yb, _ = b.step(300)
    assert np.max(np.abs(a.get_f() - b.get_f())) < 1e-14
    assert np.max(np.abs(fa - fb)) < 1e-13 and np.max(np.abs(ya - yb)) < 1e-13


def _poiseuille(ny, q, bounce, tau=0.8, g=1e-6, steps=None):
    nx = 3
    solid = np.zeros((ny, nx), np.uint8)
    solid[0, :] = solid[-1, :] = 1
    p = OracleParams(nx=nx, ny=ny, tau=tau, x_periodic=True, wall=WALL_PERIODIC, gx=g, u_in=0.0,
                     bounce=bounce, q_fixed=q)
    o = Oracle(p, solid)
    o.set_f(np.broadcast_to(WT[:, None, None], (9, ny, nx)).copy())
    nu = (tau - 0.5) / 3
    o.step(steps or int(6 * ny * ny / nu))
    _, ux, _ = o.fields()
    y = np.arange(1, ny - 1)
    lo, hi = 1 - q, ny - 2 + q  # walls a fraction q beyond the first and last fluid rows
    exact = g / (2 * nu) * (y - lo) * (hi - y)
    return np.max(np.abs(ux[1:-1, 1] - exact)) / exact.max()


@pytest.mark.parametrize("q", [0.25, 0.7])
def test_channel_with_walls_between_nodes(q):
    """Body-force channel, walls at distance q beyond the first and last
    fluid rows: the interpolated scheme follows the parabola through the
    true walls to second order; half-way bounce-back, which puts the walls
    half a node away, misses it by O(|q - 1/2| / H)."""
    e1 = _poiseuille(12, q, BB_INTERP)
    e2 = _poiseuille(22, q, BB_INTERP)
    hw = _poiseuille(12, q, BB_HALFWAY)
    assert e1 < 0.01
    assert e1 / e2 > 3.0  # second order: (20/10)^2 = 4 nominally
    assert hw > 5 * e1
