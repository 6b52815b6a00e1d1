"""Pins of the oracle's post-processing: Eq. 15, Eq. 18 and the shedding statistics."""
import numpy as np
import pytest

from oracle import stats


def test_eq18_worked_example():
    """Sec. 3.1: dx = 1/20, u* = 0.02, u_phys = 1 gives dt = 1e-3."""
    assert stats.lattice_time_step(1 / 20, 0.02, 1.0) == pytest.approx(1e-3, rel=1e-15)


def test_strouhal_two_ways_agree():
    """St = 1/(T dt) in physical units equals D/(T U) in lattice units."""
    D, U, T = 20, 0.02, 2975.0
    dt = stats.lattice_time_step(1 / D, U, 1.0)
    assert 1.0 / (T * dt) == pytest.approx(D / (T * U), rel=1e-14)


def test_coefficients_eq15():
    cd, cl = stats.coefficients([0.5], [-0.25], u=0.1, d=10)
    assert cd[0] == pytest.approx(0.5 / (0.5 * 0.01 * 10))
    assert cl[0] == pytest.approx(-0.25 / (0.5 * 0.01 * 10))


@pytest.mark.parametrize("period", [97.3, 606.06, 4848.5])
def test_shedding_stats_recover_a_synthetic_sinusoid(period):
    """Lift = A sin(2 pi t/T + phi) and drag = mean + a sin(4 pi t/T):
    the extractor returns T, A and the mean (to sampling accuracy)."""
    D, U = 40, 0.05
    n = int(12 * period) + 7
    t = np.arange(n)
    A, mean_cd = 0.33, 1.37
    cl = A * np.sin(2 * np.pi * t / period + 0.4) + 0.01
    cd = mean_cd + 0.05 * np.sin(4 * np.pi * t / period + 1.0)
    s = stats.shedding(cd, cl, D, U, periods=5)
    assert s["period"] == pytest.approx(period, rel=1e-4)
    assert s["st"] == pytest.approx(D / (period * U), rel=1e-4)
    assert s["cl_amp"] == pytest.approx(A, rel=2e-3)
    assert s["mean_cd"] == pytest.approx(mean_cd, rel=2e-3)


def test_shedding_stats_reject_a_steady_history():
    with pytest.raises(ValueError):
        stats.shedding(np.ones(1000), np.zeros(1000), 10, 0.1)
