"""Pins of the oracle's multiple-relaxation-time collision (Eq. 6, Sec. 2.1).

The transformation matrix and the equilibrium moments are checked against
their definitions as velocity polynomials and as moments of the Eq. 3
equilibrium, both written here from Table 1; the collision is checked
against what it must do in moment space (conserve rho and j, relax every
other moment by its own rate), against BGK when all rates are 1/tau, and
against the shear viscosity of Eq. 5 and a Couette profile.
"""
import numpy as np
import pytest

from oracle import (
    BGK,
    MRT,
    PAPER_S,
    WALL_MOVING_BB,
    WALL_PERIODIC,
    Oracle,
    OracleParams,
    mrt_matrix,
    mrt_meq,
)

# Table 1 (k = i - 1), typed in from the table.
CX = np.array([0, 1, 0, -1, 0, 1, -1, -1, 1], float)
CY = np.array([0, 0, 1, 0, -1, 1, 1, -1, -1], float)
WT = np.array([4 / 9, 1 / 9, 1 / 9, 1 / 9, 1 / 9, 1 / 36, 1 / 36, 1 / 36, 1 / 36])


def basis():
    """The nine moment polynomials of the Lallemand-Luo basis evaluated on
    the Table 1 velocities: 1, e, epsilon, j_x, q_x, j_y, q_y, p_xx, p_xy."""
    c2 = CX * CX + CY * CY
    return np.array([
        np.ones(9),
        -4 + 3 * c2,
        4 - 10.5 * c2 + 4.5 * c2 * c2,
        CX,
        (-5 + 3 * c2) * CX,
        CY,
        (-5 + 3 * c2) * CY,
        CX * CX - CY * CY,
        CX * CY,
    ])


def feq(rho, ux, uy):
    cu = CX * ux + CY * uy
    return WT * rho * (1 + 3 * cu + 4.5 * cu * cu - 1.5 * (ux * ux + uy * uy))


def test_transformation_matrix_is_the_moment_basis():
    """The printed M of Sec. 2.1 equals the basis polynomials on Table 1's
    velocities; its rows are orthogonal with the known norms."""
    M = mrt_matrix()
    assert np.array_equal(M, basis())
    G = M @ M.T
    assert np.array_equal(G, np.diag([9, 36, 36, 6, 12, 6, 12, 4, 4]).astype(float))


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_equilibrium_moments_are_the_moments_of_eq3(seed):
    """m_eq(rho, u) of Sec. 2.1 with the factor rho (the printed list is for
    rho = 1) equals M f_eq with f_eq from Eq. 3."""
    rng = np.random.default_rng(seed)
    for _ in range(20):
        rho = rng.uniform(0.8, 1.3)
        ux, uy = rng.uniform(-0.15, 0.15, 2)
        assert np.allclose(mrt_meq(rho, ux, uy), basis() @ feq(rho, ux, uy), atol=1e-15, rtol=0)
    # the printed values at rho = 1
    u, v = 0.07, -0.03
    q = u * u + v * v
    assert np.allclose(mrt_meq(1.0, u, v), [1, -2 + 3 * q, 1 - 3 * q, u, -u, v, -v, u * u - v * v, u * v],
                       atol=1e-16)


def _rand_state(rng, ny, nx, amp):
    return WT[:, None, None] * (1.0 + amp * rng.uniform(-1, 1, size=(9, ny, nx)))


def test_collision_relaxes_each_moment_at_its_own_rate():
    """Eq. 6 in moment space: m* - m_eq = (I - S)(m - m_eq); rho and j are
    conserved whatever their rates."""
    rng = np.random.default_rng(5)
    tau = 0.62
    rates = (0.3, 1.1, 1.25, 0.7, 1.4, 1.9, 1.05, 0.0, 0.0)
    p = OracleParams(nx=7, ny=5, tau=tau, x_periodic=True, wall=WALL_PERIODIC, collision=MRT,
                     s_rates=rates)
    o = Oracle(p)
    f = _rand_state(rng, 5, 7, 0.2)
    o.set_f(f)
    fs = o.get_fstar()
    B = basis()
    s = np.array(rates)
    s[7] = s[8] = 1 / tau
    for y in range(5):
        for x in range(7):
            fn, fsn = f[:, y, x], fs[:, y, x]
            m, ms = B @ fn, B @ fsn
            rho = m[0]
            meq = B @ feq(rho, m[3] / rho, m[5] / rho)
            for i in (0, 3, 5):
                assert ms[i] == pytest.approx(m[i], abs=1e-15)
            for i in (1, 2, 4, 6, 7, 8):
                assert ms[i] - meq[i] == pytest.approx((1 - s[i]) * (m[i] - meq[i]), abs=1e-14)


def test_uniform_rates_reduce_to_bgk():
    """With every rate 1/tau, M^{-1} S M = I/tau and Eq. 6 is Eq. 2."""
    rng = np.random.default_rng(6)
    tau = 0.71
    f0 = _rand_state(rng, 9, 11, 0.1)
    out = []
    for coll in (BGK, MRT):
        p = OracleParams(nx=11, ny=9, tau=tau, x_periodic=True, wall=WALL_PERIODIC, collision=coll,
                         s_rates=(1 / tau,) * 9)
        o = Oracle(p)
        o.set_f(f0)
        o.step(25)
        out.append(o.get_f())
    assert np.max(np.abs(out[0] - out[1])) < 1e-14


def test_periodic_box_conserves_mass_and_momentum():
    rng = np.random.default_rng(7)
    p = OracleParams(nx=16, ny=13, tau=0.52, x_periodic=True, wall=WALL_PERIODIC, collision=MRT)
    o = Oracle(p)
    f = _rand_state(rng, 13, 16, 0.05)
    o.set_f(f)
    o.step(200)
    g = o.get_f()
    for row in (np.ones(9), CX, CY):
        assert abs(np.tensordot(row, g, 1).sum() - np.tensordot(row, f, 1).sum()) < 1e-11


def _taylor_green_nu(L, tau, steps, rates):
    U0 = 0.01
    k = 2 * np.pi / L
    o = Oracle(OracleParams(nx=L, ny=L, tau=tau, x_periodic=True, wall=WALL_PERIODIC, collision=MRT,
                            s_rates=rates))
    x = np.arange(L)[None, :]
    y = np.arange(L)[:, None]
    ux = -U0 * np.cos(k * x) * np.sin(k * y)
    uy = U0 * np.sin(k * x) * np.cos(k * y)
    rho = 1 - 0.75 * U0 * U0 * (np.cos(2 * k * x) + np.cos(2 * k * y))
    f = np.stack([WT[q] * rho * (1 + 3 * (CX[q] * ux + CY[q] * uy) + 4.5 * (CX[q] * ux + CY[q] * uy) ** 2
                                 - 1.5 * (ux * ux + uy * uy)) for q in range(9)])
    o.set_f(f)
    o.step(20)
    _, a, b = o.fields()
    e1 = (a * a + b * b).sum()
    o.step(steps)
    _, a, b = o.fields()
    e2 = (a * a + b * b).sum()
    return -np.log(e2 / e1) / (4 * k * k * steps)


@pytest.mark.parametrize("bulk", [1.1, 1.6])
def test_shear_viscosity_set_by_the_stress_rates(bulk):
    """Eq. 5 with tau = 1/s_nu, the rate of p_xx and p_xy: the decay of a
    Taylor-Green vortex gives nu = (1/s_nu - 1/2)/3 whatever the other rates."""
    tau = 0.8
    rates = (1.0, bulk, bulk, 1.0, bulk, 1.0, bulk, 0.0, 0.0)
    nu = _taylor_green_nu(48, tau, int(0.05 * 48 * 48), rates)
    assert nu == pytest.approx((tau - 0.5) / 3, rel=0.01)


def test_couette_profile_error_is_second_order_in_the_wall_speed():
    """Moving-wall bounce-back (Eq. 11) with the paper's rates at tau = 0.512.
    Unlike BGK, unequal rates leave an O(U^2) density layer at the moving
    wall, so u = U (y + 1/2)/ny holds to a relative error that falls as U^2
    (and exactly once the rates are equal, where Eq. 6 is Eq. 2)."""
    ny, nx = 8, 3
    err = []
    for U in (0.02, 0.01):
        p = OracleParams(nx=nx, ny=ny, tau=0.512, x_periodic=True, wall=WALL_MOVING_BB, u_in=U,
                         u_wall_top=U, u_wall_bottom=0.0, collision=MRT, s_rates=PAPER_S)
        o = Oracle(p)
        o.set_f(np.broadcast_to(WT[:, None, None], (9, ny, nx)).copy())
        _, _, bad = o.step(60000)
        assert bad == 0
        _, ux, uy = o.fields()
        y = np.arange(ny)
        err.append(np.max(np.abs(ux[:, 1] - U * (y + 0.5) / ny)) / U)
        assert np.max(np.abs(uy)) < 1e-13
    assert err[0] < 2e-5
    assert 3.5 < err[0] / err[1] < 4.5


def test_forcing_with_mrt_is_rejected():
    with pytest.raises(Exception):
        Oracle(OracleParams(nx=4, ny=4, tau=0.8, x_periodic=True, wall=WALL_PERIODIC, collision=MRT, gx=1e-6))
