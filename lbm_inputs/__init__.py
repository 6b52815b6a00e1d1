"""Seeded synthetic inputs shared by the tests, the smoke check and the benchmark.

Holds workload sizes and random-number generators only: none of the solver's
arithmetic lives here, and neither the GPU package nor the oracle imports it.

Workloads (all lattice units; the cylinder centre sits at (10.5 D, 10.5 D) in a
41 D x 21 D channel, i.e. 10 D of fluid upstream, 30 D downstream and 10 D to
each wall measured from the cylinder surface; Sec. 3.1 of the paper):
  cyl_d10   410 x 210,  D = 10,  U = 0.1,  Re = 100, tau = 0.53, free-slip walls
  cyl_d40  1640 x 840,  D = 40,  U = 0.05, Re = 100
  cyl_d80  3280 x 1680, D = 80,  U = 0.05, Re = 100
  cyl_d160 6560 x 3360, D = 160, U = 0.05, Re = 100
The paper's own runs (Sec. 3.1), a 40 D x 20 D lattice with the centre 10 D
from the inlet and (up to half a node) from both walls, MRT collision:
  cyl_d20_mrt  800 x 400,  D = 20, U = 0.02, Re = 100, tau = 0.512
  cyl_d40_mrt 1600 x 800,  D = 40, U = 0.02, Re = 100, tau = 0.524
  ensemble 64 cases, D uniform in 8..32, Re uniform in [60, 200], U = 0.05
  trunc_d40 1040 x 440 truncated window around a D = 40 cylinder
"""
from __future__ import annotations

import numpy as np

MASK64 = (1 << 64) - 1


def splitmix64(seed: int):
    """SplitMix64 (Steele, Lea & Flood 2014): yields 64-bit integers."""
    state = seed & MASK64
    while True:
        state = (state + 0x9E3779B97F4A7C15) & MASK64
        z = state
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK64
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK64
        yield z ^ (z >> 31)


# diag(S) of Sec. 2.1; 0 in the two shear entries stands for 1/tau
PAPER_RATES = (1.0, 1.1, 1.1, 1.0, 1.1, 1.0, 1.1, 0.0, 0.0)
MRT = 1


def channel(d: int, u: float = 0.05, re: float = 100.0) -> dict:
    """The 41 D x 21 D cylinder channel as keyword arguments."""
    return dict(nx=41 * d, ny=21 * d, diameter=d, cx2=21 * d, cy2=21 * d, u_in=u, re=re)


def paper_channel(d: int = 20, u: float = 0.02, re: float = 100.0) -> dict:
    """The 40 D x 20 D lattice of Sec. 3.1 with the MRT collision."""
    return dict(nx=40 * d, ny=20 * d, diameter=d, cx2=20 * d, cy2=20 * d, u_in=u, re=re,
                collision=MRT, s_rates=PAPER_RATES)


WORKLOADS = {
    "cyl_d10": dict(channel(10, u=0.1), tau=0.53),
    "cyl_d40": channel(40),
    "cyl_d80": channel(80),
    "cyl_d160": channel(160),
    "cyl_d20_mrt": paper_channel(20),
    "cyl_d40_mrt": paper_channel(40),
    # one GPU's share of the D = 160 channel cut into eight slabs along x:
    # 820 of its 6560 columns, no cylinder; the x-periodic wrap stands in for
    # the ghost columns the neighbouring slabs would fill
    "slab_d160_of8": dict(nx=820, ny=3360, diameter=0, u_in=0.05, re=100.0, tau=0.74, x_periodic=True),
}


def truncated_window(d: int = 40, u: float = 0.05, re: float = 100.0) -> dict:
    """26 D x 11 D window: 10 D upstream of the centre, 15 D downstream and
    5 D to each side (lattice 1040 x 440 at D = 40)."""
    return dict(nx=26 * d, ny=11 * d, diameter=d, cx2=21 * d, cy2=11 * d, u_in=u, re=re)


def ensemble(n: int = 64, seed: int = 2605, u: float = 0.05, mrt: bool = False) -> list[dict]:
    """n cylinder channels with D = 8 + (r mod 25) and Re = 60 + 140 v, where r
    and v (uniform in [0, 1)) come from SplitMix64; tau from Re by Eqs. 16-17
    (0.507 to 0.560 for the 64 cases of seed 2605; 0.506 to 0.58 over the
    whole range of D and Re).  `mrt` selects the collision of Sec. 2.1 with
    its rates."""
    g = splitmix64(seed)
    cases = []
    for _ in range(n):
        d = 8 + next(g) % 25
        re = 60.0 + 140.0 * ((next(g) >> 11) * (1.0 / (1 << 53)))
        kw = channel(int(d), u=u, re=re)
        if mrt:
            kw.update(collision=MRT, s_rates=PAPER_RATES)
        cases.append(kw)
    return cases


def perturbed_populations(seed: int, ny: int, nx: int, base, amp: float = 0.05,
                          dtype=np.float64) -> np.ndarray:
    """[9][ny][nx] array base[k] * (1 + amp * uniform(-1, 1)); `base` is
    supplied by the caller (e.g. the lattice weights)."""
    rng = np.random.default_rng(seed)
    base = np.asarray(base, dtype=np.float64).reshape(9, 1, 1)
    out = base * (1.0 + amp * rng.uniform(-1.0, 1.0, size=(9, ny, nx)))
    return out.astype(dtype)
