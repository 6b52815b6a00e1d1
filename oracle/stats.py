"""Oracle post-processing of a force history (test infrastructure only).

* Force coefficients, Eq. 15: C = F / (1/2 rho_ref U^2 D), rho_ref = 1.
* Lattice-to-physical time step, Eq. 18: dt = dx * u_lattice / u_physical with
  dx = 1/D (Sec. 2.2); St = f D / U_phys = 1/(T dt) for a lift period of T steps.
* Shedding statistics (the paper reports mean Cd, the lift amplitude and St in
  Table 2 without defining how they were extracted; this module reads them as):
  - periods from upward crossings of Cl through its mean, located by linear
    interpolation between samples;
  - St = D / (T U) with T the mean crossing spacing over the last n periods;
  - Cl amplitude = (max - min)/2 and mean Cd, both over those same n periods.
"""
from __future__ import annotations

import numpy as np


def coefficients(fx, fy, u, d, rho_ref=1.0):
    q = 0.5 * rho_ref * u * u * d
    return np.asarray(fx) / q, np.asarray(fy) / q


def lattice_time_step(dx, u_lattice, u_physical):
    """Eq. 18."""
    return dx * u_lattice / u_physical


def _up_crossings(x):
    """Fractional indices where x goes from negative to non-negative."""
    out = []
    for i in range(len(x) - 1):
        if x[i] < 0.0 <= x[i + 1]:
            out.append(i + (-x[i]) / (x[i + 1] - x[i]))
    return out


def shedding(cd, cl, d, u, periods=5):
    """Returns dict(mean_cd, cl_amp, st, period) over the last `periods` lift periods."""
    cd = np.asarray(cd, dtype=np.float64)
    cl = np.asarray(cl, dtype=np.float64)
    xs = _up_crossings(cl - cl.mean())
    if len(xs) < periods + 1:
        raise ValueError("not enough lift periods in the history")
    xs = xs[-(periods + 1):]
    T = (xs[-1] - xs[0]) / periods
    i0, i1 = int(np.ceil(xs[0])), int(np.floor(xs[-1]))
    # re-centre on the window's own mean once, then take the crossings again
    window_mean = cl[i0:i1 + 1].mean()
    xs2 = _up_crossings(cl - window_mean)
    xs2 = [v for v in xs2 if xs[0] - 0.5 * T <= v]
    if len(xs2) >= periods + 1:
        xs2 = xs2[-(periods + 1):]
        T = (xs2[-1] - xs2[0]) / periods
        i0, i1 = int(np.ceil(xs2[0])), int(np.floor(xs2[-1]))
    seg_l = cl[i0:i1 + 1]
    seg_d = cd[i0:i1 + 1]
    return {
        "mean_cd": float(seg_d.mean()),
        "cl_amp": float(0.5 * (seg_l.max() - seg_l.min())),
        "st": float(d / (T * u)),
        "period": float(T),
    }
