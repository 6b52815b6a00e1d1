"""Pins of the FP64 oracle against facts fixed by the paper and by mathematics.

Each test names what pins it; none of them re-types the oracle's formulas.
A plausible mistake in the oracle (a dropped term, a wrong sign, a swapped
direction, a wrong opposite) breaks at least one of these.
"""
import math

import numpy as np
import pytest

from oracle import (
    OUTLET_COPY_ALL,
    OUTLET_COPY_UNKNOWN,
    WALL_FREE_SLIP,
    WALL_MOVING_BB,
    WALL_NEBB,
    WALL_PERIODIC,
    Oracle,
    OracleParams,
    digitise,
    tau_of,
)

# Table 1 of the paper, typed in here from the table itself (k = i - 1).
CX = np.array([0, 1, 0, -1, 0, 1, -1, -1, 1])
CY = np.array([0, 0, 1, 0, -1, 1, 1, -1, -1])
WT = np.array([4 / 9, 1 / 9, 1 / 9, 1 / 9, 1 / 9, 1 / 36, 1 / 36, 1 / 36, 1 / 36])
ALL_WALLS = [WALL_FREE_SLIP, WALL_PERIODIC, WALL_NEBB, WALL_MOVING_BB]


def mom(f):
    """Moments of planar populations f[9, ...]: rho, jx, jy, Pxx, Pxy, Pyy."""
    rho = f.sum(0)
    jx = np.tensordot(CX, f, 1)
    jy = np.tensordot(CY, f, 1)
    pxx = np.tensordot(CX * CX, f, 1)
    pxy = np.tensordot(CX * CY, f, 1)
    pyy = np.tensordot(CY * CY, f, 1)
    return rho, jx, jy, pxx, pxy, pyy


def rand_state(rng, ny, nx, amp=0.05):
    """Populations near rest: w_k (1 + amp * uniform(-1, 1))."""
    return WT[:, None, None] * (1.0 + amp * rng.uniform(-1, 1, size=(9, ny, nx)))


# --------------------------------------------------------------- Eqs. 2-5
def test_equilibrium_moments_via_initial_state():
    """Eq. 3: the initial state is f_eq(1, (U, v(y))); its moments must be
    rho = 1, j = u, P = I/3 + u u (second-order Hermite equilibrium)."""
    p = OracleParams(nx=8, ny=13, u_in=0.08, perturb_amp=0.3, x_periodic=True, wall=WALL_PERIODIC)
    o = Oracle(p)
    f = o.get_f()
    rho, jx, jy, pxx, pxy, pyy = mom(f)
    y = np.arange(p.ny)[:, None] * np.ones((1, p.nx))
    v = 0.3 * 0.08 * np.sin(2 * np.pi * y / (p.ny - 1))
    u = 0.08
    assert np.allclose(rho, 1.0, atol=1e-15)
    assert np.allclose(jx, u, atol=1e-15)
    assert np.allclose(jy, v, atol=1e-15)
    assert np.allclose(pxx, 1 / 3 + u * u, atol=1e-15)
    assert np.allclose(pxy, u * v, atol=1e-15)
    assert np.allclose(pyy, 1 / 3 + v * v, atol=1e-15)


def test_collision_conserves_mass_and_momentum_and_relaxes_stress():
    """Eq. 2 with Eq. 3: f* keeps rho and rho u; the non-equilibrium stress
    P - rho(I/3 + uu) is multiplied by (1 - 1/tau)."""
    rng = np.random.default_rng(1)
    tau = 0.7
    p = OracleParams(nx=7, ny=5, tau=tau, x_periodic=True, wall=WALL_PERIODIC)
    o = Oracle(p)
    f = rand_state(rng, 5, 7, 0.2)
    o.set_f(f)
    fs = o.get_fstar()
    r0, jx0, jy0, pxx0, pxy0, pyy0 = mom(f)
    r1, jx1, jy1, pxx1, pxy1, pyy1 = mom(fs)
    assert np.allclose(r1, r0, atol=1e-15, rtol=0)
    assert np.allclose(jx1, jx0, atol=1e-15, rtol=0)
    assert np.allclose(jy1, jy0, atol=1e-15, rtol=0)
    ux, uy = jx0 / r0, jy0 / r0
    for P0, P1, eq in ((pxx0, pxx1, r0 * (1 / 3 + ux * ux)), (pxy0, pxy1, r0 * ux * uy),
                       (pyy0, pyy1, r0 * (1 / 3 + uy * uy))):
        assert np.allclose(P1 - eq, (1 - 1 / tau) * (P0 - eq), atol=1e-14)


def test_tau_one_gives_equilibrium_fixed_point():
    """tau = 1 makes f* = f_eq; then f_eq is a fixed point of the collision."""
    rng = np.random.default_rng(2)
    p = OracleParams(nx=6, ny=4, tau=1.0, x_periodic=True, wall=WALL_PERIODIC)
    o = Oracle(p)
    o.set_f(rand_state(rng, 4, 6, 0.3))
    fs = o.get_fstar()
    o.set_f(fs)
    assert np.allclose(o.get_fstar(), fs, atol=1e-16)


def test_tau_from_reynolds_eqs_16_17():
    """Eqs. 16-17: nu = U D / Re, tau = 3 nu + 1/2.  The paper's run (D = 20,
    U = 0.02, Re = 100) gives tau = 0.512."""
    assert tau_of(OracleParams(nx=800, ny=400, diameter=20, u_in=0.02, re=100)) == pytest.approx(0.512)
    assert tau_of(OracleParams(nx=410, ny=210, diameter=10, u_in=0.1, re=100)) == pytest.approx(0.53)
    assert tau_of(OracleParams(nx=9, ny=9, tau=0.9)) == 0.9


# ---------------------------------------------------- streaming + bounce-back
def test_periodic_box_conserves_mass_and_momentum():
    rng = np.random.default_rng(3)
    p = OracleParams(nx=24, ny=17, tau=0.6, x_periodic=True, wall=WALL_PERIODIC)
    o = Oracle(p)
    o.set_f(rand_state(rng, 17, 24))
    r0, jx0, jy0, *_ = mom(o.get_f())
    _, _, bad = o.step(50)
    assert bad == 0
    r1, jx1, jy1, *_ = mom(o.get_f())
    assert abs(r1.sum() - r0.sum()) < 1e-11
    assert abs(jx1.sum() - jx0.sum()) < 1e-12
    assert abs(jy1.sum() - jy0.sum()) < 1e-12


def test_closed_box_with_bounce_back_conserves_mass():
    """Half-way bounce-back on a solid frame plus an interior block: every
    population that hits a solid node returns to its own node, so total mass
    is conserved (momentum is not: the walls take it)."""
    rng = np.random.default_rng(4)
    nx, ny = 20, 16
    solid = np.zeros((ny, nx), np.uint8)
    solid[0, :] = solid[-1, :] = solid[:, 0] = solid[:, -1] = 1
    solid[6:9, 8:12] = 1
    p = OracleParams(nx=nx, ny=ny, tau=0.8, x_periodic=True, wall=WALL_PERIODIC)
    o = Oracle(p, solid)
    f = rand_state(rng, ny, nx)
    o.set_f(f)
    fluid = solid == 0
    m0 = f.sum(0)[fluid].sum()
    _, _, bad = o.step(100)
    assert bad == 0
    m1 = o.get_f().sum(0)[fluid].sum()
    assert abs(m1 - m0) < 1e-11


def _taylor_green_nu(L, tau, steps):
    U0 = 0.01
    k = 2 * np.pi / L
    p = OracleParams(nx=L, ny=L, tau=tau, x_periodic=True, wall=WALL_PERIODIC)
    o = Oracle(p)
    x = np.arange(L)[None, :]
    y = np.arange(L)[:, None]
    ux = -U0 * np.cos(k * x) * np.sin(k * y)
    uy = U0 * np.sin(k * x) * np.cos(k * y)
    rho = 1 - 0.75 * U0 * U0 * (np.cos(2 * k * x) + np.cos(2 * k * y))
    # equilibrium from the table and the Hermite form, written independently here
    f = np.empty((9, L, L))
    for q in range(9):
        cu = CX[q] * ux + CY[q] * uy
        f[q] = WT[q] * rho * (1 + 3 * cu + 4.5 * cu * cu - 1.5 * (ux * ux + uy * uy))
    o.set_f(f)
    o.step(20)
    _, ux1, uy1 = o.fields()
    e1 = (ux1 ** 2 + uy1 ** 2).sum()
    o.step(steps)
    _, ux2, uy2 = o.fields()
    e2 = (ux2 ** 2 + uy2 ** 2).sum()
    # kinetic energy decays as exp(-4 nu k^2 t)
    return -np.log(e2 / e1) / (4 * k * k * steps)


def test_taylor_green_decay_matches_eq5_viscosity():
    """Eq. 5: nu = (tau - 1/2)/3.  Fitted nu within 1 % at L = 64, and the
    error falls at second order with resolution."""
    tau = 0.8
    nu = (tau - 0.5) / 3
    err = []
    for L in (16, 32, 64):
        nu_fit = _taylor_green_nu(L, tau, steps=int(0.05 * L * L))
        err.append(abs(nu_fit / nu - 1))
    assert err[-1] < 0.01
    assert err[0] / err[1] > 3.0 and err[1] / err[2] > 3.0


def _channel_profile(p, solid=None, steps=4000, rho0=1.0):
    o = Oracle(p, solid)
    o.set_f(rho0 * np.broadcast_to(WT[:, None, None], (9, p.ny, p.nx)).copy())
    _, _, bad = o.step(steps)
    assert bad == 0
    _, ux, uy = o.fields()
    return ux[:, p.nx // 2], uy


def test_poiseuille_exact_at_magic_tau():
    """Body-force-driven channel between half-way bounce-back walls (solid rows
    y = 0 and y = ny-1, walls at y = 1/2 and ny - 3/2).  Steady state:
    u(y) = g/(2 nu) (y - 1/2)(ny - 3/2 - y).  With BGK the wall sits exactly
    half-way when (tau - 1/2)^2 = 3/16 (He et al. 1997), so the profile is
    exact to round-off there and second-order accurate otherwise."""
    ny, nx = 12, 4
    solid = np.zeros((ny, nx), np.uint8)
    solid[0, :] = solid[-1, :] = 1
    g = 1e-6
    tau = 0.5 + math.sqrt(3.0) / 4.0
    nu = (tau - 0.5) / 3
    p = OracleParams(nx=nx, ny=ny, tau=tau, x_periodic=True, wall=WALL_PERIODIC, gx=g, u_in=0)
    u, uy = _channel_profile(p, solid, steps=6000)
    y = np.arange(1, ny - 1)
    exact = g / (2 * nu) * (y - 0.5) * (ny - 1.5 - y)
    assert np.max(np.abs(u[1:-1] - exact)) < 1e-9 * exact.max() + 1e-15
    assert np.max(np.abs(uy[1:-1])) < 1e-15
    # away from the magic value the error is O(1/ny^2) but nonzero
    p.tau = 0.7
    nu = (0.7 - 0.5) / 3
    u, _ = _channel_profile(p, solid, steps=6000)
    exact = g / (2 * nu) * (y - 0.5) * (ny - 1.5 - y)
    rel = np.max(np.abs(u[1:-1] - exact)) / exact.max()
    assert 1e-6 < rel < 2.0 / (ny - 2) ** 2


def test_couette_moving_wall_bounce_back_eq11():
    """Eq. 11: top row moving bounce-back with u_w = (U, 0), bottom with
    u_w = 0; the walls sit half a link outside the first and last rows, so the
    steady profile is u(y) = U (y + 1/2)/ny, exactly, for any tau."""
    ny, nx, U = 10, 3, 0.02
    for tau, rho0 in ((0.6, 1.0), (1.3, 1.0), (0.8, 1.3)):
        # rho0 != 1 pins the density in the momentum term of Eq. 11
        p = OracleParams(nx=nx, ny=ny, tau=tau, x_periodic=True, wall=WALL_MOVING_BB,
                         u_in=U, u_wall_top=U, u_wall_bottom=0.0)
        u, uy = _channel_profile(p, steps=12000, rho0=rho0)
        y = np.arange(ny)
        assert np.max(np.abs(u - U * (y + 0.5) / ny)) < 1e-10
        assert np.max(np.abs(uy)) < 1e-12


def test_couette_nebb_wet_node_eqs_9_10():
    """Eqs. 9-10: wet-node walls on the first and last rows with u = (U, 0) on
    top and 0 at the bottom: u(y) = U y/(ny-1) exactly at steady state."""
    ny, nx, U = 10, 3, 0.02
    p = OracleParams(nx=nx, ny=ny, tau=0.8, x_periodic=True, wall=WALL_NEBB,
                     u_in=U, u_wall_top=U, u_wall_bottom=0.0)
    u, uy = _channel_profile(p, steps=12000)
    y = np.arange(ny)
    assert np.max(np.abs(u - U * y / (ny - 1))) < 1e-10
    assert np.max(np.abs(uy)) < 1e-12


@pytest.mark.parametrize("wall", ALL_WALLS)
@pytest.mark.parametrize("outlet", [OUTLET_COPY_ALL, OUTLET_COPY_UNKNOWN])
def test_uniform_flow_is_a_fixed_point_of_every_boundary(wall, outlet):
    """f_eq(1, (U, 0)) everywhere (no cylinder) must be left unchanged by the
    inlet, the outlet and every wall treatment (walls moving at U).  This pins
    every sign in Eqs. 7, 9-11, 13 and the inlet formulas."""
    U = 0.07
    p = OracleParams(nx=12, ny=9, u_in=U, tau=0.7, wall=wall, outlet_mode=outlet, perturb_amp=0.0)
    o = Oracle(p)
    f0 = o.get_f()
    _, _, bad = o.step(5)
    assert bad == 0
    assert np.max(np.abs(o.get_f() - f0)) < 1e-15


@pytest.mark.parametrize("wall", ALL_WALLS)
@pytest.mark.parametrize("outlet", [OUTLET_COPY_ALL, OUTLET_COPY_UNKNOWN])
def test_boundary_nodes_get_the_prescribed_moments(wall, outlet):
    """After a step from a disturbed state: inlet nodes carry u = (U, 0)
    (Zou-He); NEBB rows carry u = (U, 0); free-slip rows carry v = 0 and
    moving-BB rows a v = 0 only at steady state (not checked)."""
    rng = np.random.default_rng(7)
    U = 0.05
    p = OracleParams(nx=14, ny=11, u_in=U, tau=0.65, wall=wall, outlet_mode=outlet)
    o = Oracle(p)
    o.set_f(rand_state(rng, 11, 14, 0.05))
    o.step(1)
    rho, ux, uy = o.fields()
    rows = slice(None) if wall == WALL_PERIODIC else slice(1, -1)
    assert np.allclose(ux[rows, 0], U, atol=1e-15)
    assert np.allclose(uy[rows, 0], 0.0, atol=1e-15)
    if wall != WALL_PERIODIC:  # inlet corners are equilibrium nodes at rho = 1
        assert np.allclose(rho[[0, -1], 0], 1.0, atol=1e-15)
        assert np.allclose(ux[[0, -1], 0], U, atol=1e-15)
    inner = slice(1, -1)
    if wall == WALL_NEBB:
        assert np.allclose(ux[[0, -1], inner], U, atol=1e-15)
        assert np.allclose(uy[[0, -1], inner], 0.0, atol=1e-15)
    if wall == WALL_FREE_SLIP:
        assert np.allclose(uy[[0, -1], inner], 0.0, atol=1e-15)
    f = o.get_f()
    if outlet == OUTLET_COPY_ALL:  # the last column equals the one before it
        assert np.array_equal(f[:, :, -1], f[:, :, -2])
    else:  # the three populations entering from x = nx
        west = CX < 0
        assert np.array_equal(f[west][:, rows, -1], f[west][:, rows, -2])


@pytest.mark.parametrize("wall", ALL_WALLS)
@pytest.mark.parametrize("outlet", [OUTLET_COPY_ALL, OUTLET_COPY_UNKNOWN])
def test_mirror_symmetry_in_y(wall, outlet):
    """A state that is mirror-symmetric about the channel mid-height stays
    so under every wall and outlet treatment; this ties the top formulas to
    the bottom ones (a sign or direction slip on one side, or an outlet that
    copies a different set of directions at the top than at the bottom,
    breaks it)."""
    rng = np.random.default_rng(8)
    nx, ny = 16, 11
    p = OracleParams(nx=nx, ny=ny, u_in=0.05, tau=0.7, wall=wall, perturb_amp=0.0, outlet_mode=outlet)
    o = Oracle(p)
    f = rand_state(rng, ny, nx)
    mirror = [0, 1, 4, 3, 2, 8, 7, 6, 5]  # N<->S, NE<->SE, NW<->SW
    f = 0.5 * (f + f[mirror][:, ::-1, :])
    o.set_f(f)
    o.step(30)
    g = o.get_f()
    assert np.max(np.abs(g - g[mirror][:, ::-1, :])) < 1e-14


@pytest.mark.parametrize("wall", ALL_WALLS)
def test_copy_unknown_outlet_replaces_exactly_the_populations_with_no_source(wall):
    """The copy-unknown outlet (Eq. 13 applied to the missing populations,
    Fig. 2): at an outlet node a population k is unknown after streaming iff
    its source x - c_k lies outside the lattice: c_kx = +1 brings nothing in
    from x = nx, and at the two corners nothing comes from beyond the wall
    row either (with periodic walls the rows wrap and no corner exists).
    Derived here from Table 1 and the lattice size alone, on every outlet
    node, corners included: the known populations must be the
    post-collision values pulled along c_k (streaming, Eq. 2), untouched by
    the outlet, and each unknown one must equal its value at x = nx - 2 after
    the same step."""
    rng = np.random.default_rng(21)
    nx, ny = 13, 9
    p = OracleParams(nx=nx, ny=ny, u_in=0.04, tau=0.7, wall=wall, outlet_mode=OUTLET_COPY_UNKNOWN,
                     perturb_amp=0.0)
    o = Oracle(p)
    o.set_f(rand_state(rng, ny, nx, 0.05))
    fs = o.get_fstar()
    o.step(1)
    g = o.get_f()
    x = nx - 1
    for y in range(ny):
        src = [(x - CX[k], (y - CY[k]) % ny if wall == WALL_PERIODIC else y - CY[k]) for k in range(9)]
        unknown = [k for k in range(9) if not (0 <= src[k][0] < nx and 0 <= src[k][1] < ny)]
        if 0 < y < ny - 1 or wall == WALL_PERIODIC:
            assert sorted(unknown) == [3, 6, 7]  # W, NW, SW of Table 1
        for k in range(9):
            if k in unknown:
                assert g[k, y, x] == g[k, y, x - 1], (y, k)
            else:
                sx, sy = src[k]
                assert g[k, y, x] == fs[k, sy, sx], (y, k)


def test_inlet_corners_are_equilibrium_nodes_of_the_inlet_state():
    """The inlet corners (the paper is silent; read as Dirichlet nodes of
    rho = 1, u = (U, 0)): after a step from a disturbed state all nine
    independent moments of a corner must be those of Eq. 3 at that state,
    which fixes its nine populations.  The moment values follow from Eq. 3
    and Table 1: 1, U, 0, 1/3 + U^2, 0, 1/3, 0, U/3 and 1/9 + U^2/3 for
    1, cx, cy, cx^2, cx cy, cy^2, cx^2 cy, cx cy^2, cx^2 cy^2."""
    rng = np.random.default_rng(22)
    U = 0.06
    for wall in (WALL_FREE_SLIP, WALL_NEBB, WALL_MOVING_BB):
        p = OracleParams(nx=10, ny=8, u_in=U, tau=0.7, wall=wall)
        o = Oracle(p)
        o.set_f(rand_state(rng, 8, 10, 0.05))
        o.step(1)
        f = o.get_f()
        basis = [np.ones(9), CX, CY, CX * CX, CX * CY, CY * CY, CX * CX * CY, CX * CY * CY, CX * CX * CY * CY]
        want = [1.0, U, 0.0, 1 / 3 + U * U, 0.0, 1 / 3, 0.0, U / 3, 1 / 9 + U * U / 3]
        for y in (0, 7):
            got = [float(b @ f[:, y, 0]) for b in basis]
            assert np.allclose(got, want, atol=1e-15), (wall, y)


def test_reference_density_one_is_the_inlet_density_within_a_percent():
    """Eq. 15 divides by the inlet density; the reading takes rho_ref = 1 (a
    velocity inlet with an extrapolated outlet fixes no pressure level).  On
    the D = 10 channel (the benchmark's first configuration) the density the
    Zou-He inlet carries, averaged over its column and over steps 1000-2000,
    stays within 1 % of 1, so the reading moves Cd and Cl by less than the
    1 % the statistics are compared at."""
    p = OracleParams(nx=410, ny=210, diameter=10, u_in=0.1, tau=0.53)
    o = Oracle(p)
    o.step(1000)
    dens = []
    for _ in range(10):
        o.step(100)
        rho, _, _ = o.fields()
        dens.append(rho[1:-1, 0].mean())
    assert abs(np.mean(dens) - 1.0) < 0.01, dens


# -------------------------------------------------------------- geometry
def _brute_counts(D):
    """Pure-Python count of solid nodes, boundary nodes and fluid->solid links
    for the doubled-coordinate disk test of radius D/2 centred at (10.5D, 10.5D)."""
    nx, ny = 41 * D, 21 * D
    c = 21 * D

    def solid(x, y):
        return (2 * x - c) ** 2 + (2 * y - c) ** 2 <= D * D

    lo, hi = 10 * D - 2, 11 * D + 3
    ns = nb = nl = 0
    for y in range(lo, hi):
        for x in range(lo, hi):
            if solid(x, y):
                ns += 1
                continue
            links = sum(1 for q in range(1, 9) if solid(x + CX[q], y + CY[q]))
            nl += links
            nb += links > 0
    return ns, nb, nl


@pytest.mark.parametrize("D", [10, 20, 40])
def test_geometry_counts(D):
    p = OracleParams(nx=41 * D, ny=21 * D, diameter=D)
    s = digitise(p)
    ns, nb, nl = _brute_counts(D)
    assert int(s.sum()) == ns
    if D == 10:
        assert (ns, nb, nl) == (81, 48, 104)
    if D == 40:
        assert (ns, nb, nl) == (1257, 168, 392)
    # point symmetry about the centre: (x, y) -> (21D - x, 21D - y)
    ys, xs = np.nonzero(s)
    assert set(zip((21 * D - xs).tolist(), (21 * D - ys).tolist())) == set(zip(xs.tolist(), ys.tolist()))


# ------------------------------------------------------------------ Eq. 14
@pytest.mark.parametrize("D", [10, 13])
def test_force_at_rest_is_zero_on_the_digitised_disk(D):
    """rho = 1, u = 0: the disk is point-symmetric, so Eq. 14 sums to zero."""
    p = OracleParams(nx=41 * D, ny=21 * D, diameter=D, u_in=0.0, tau=0.8, x_periodic=True,
                     wall=WALL_PERIODIC, perturb_amp=0.0)
    o = Oracle(p)
    fx, fy, _ = o.step(1)
    assert abs(fx[0]) < 1e-13 and abs(fy[0]) < 1e-13


def test_force_equals_fluid_momentum_loss():
    """Newton's third law on a periodic box holding the disk: the collision
    conserves momentum, so one step changes the fluid's total momentum by
    exactly minus the force Eq. 14 puts on the body."""
    rng = np.random.default_rng(11)
    D = 6
    p = OracleParams(nx=41 * D, ny=21 * D, diameter=D, tau=0.7, x_periodic=True, wall=WALL_PERIODIC)
    o = Oracle(p)
    f = rand_state(rng, p.ny, p.nx, 0.01)
    f[1] += 0.004  # a net stream along +x and -y
    f[4] += 0.003
    o.set_f(f)
    fluid = digitise(p) == 0
    _, jx0, jy0, *_ = mom(o.get_f())
    fx, fy, _ = o.step(1)
    _, jx1, jy1, *_ = mom(o.get_f())
    assert abs(fx[0]) > 1e-3 and abs(fy[0]) > 1e-3
    assert jx1[fluid].sum() - jx0[fluid].sum() == pytest.approx(-fx[0], abs=1e-12)
    assert jy1[fluid].sum() - jy0[fluid].sum() == pytest.approx(-fy[0], abs=1e-12)


def test_flat_wall_at_rest_feels_the_pressure():
    """A solid bottom row under fluid at rest: each wall link pair carries
    2 (1/9 + 2/36) rho = rho/3 = p (c_s^2 = 1/3), pushing the wall down."""
    nx, ny = 9, 6
    solid = np.zeros((ny, nx), np.uint8)
    solid[0, :] = 1
    p = OracleParams(nx=nx, ny=ny, tau=0.9, x_periodic=True, wall=WALL_FREE_SLIP, u_in=0.0,
                     u_wall_top=0.0, u_wall_bottom=0.0, perturb_amp=0.0)
    o = Oracle(p, solid)
    fx, fy, _ = o.step(1)
    assert abs(fx[0]) < 1e-15
    assert fy[0] == pytest.approx(-nx / 3.0, abs=1e-13)


# ----------------------------------------------------------- failure paths
def test_divergence_is_reported():
    """tau -> 1/2 with a fast inlet is unstable (Sec. 2.1 and Sec. 3.1)."""
    p = OracleParams(nx=82, ny=42, diameter=2, u_in=0.2, tau=0.5001)
    o = Oracle(p)
    _, _, bad = o.step(3000)
    assert bad > 0


def test_nan_state_is_reported_at_the_first_step():
    p = OracleParams(nx=10, ny=8, u_in=0.05, tau=0.7)
    o = Oracle(p)
    f = o.get_f()
    f[3, 4, 5] = np.nan
    o.set_f(f)
    _, _, bad = o.step(10)
    assert bad == 1
