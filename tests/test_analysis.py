"""Trajectory analysis (host side) against closed forms and constructed cases."""
import math

import numpy as np
import pytest

from paper_2608_18541_amd import analysis as A


def test_collapse_time_recovers_a_single_exponential():
    pytest.importorskip("scipy")
    t = np.linspace(0.0, 3.0, 301)
    m = 0.8 * (0.25 + 0.75 * np.exp(-t / 0.54))          # collapse to a quarter, tau 0.54
    tau, y_inf = A.collapse_time(t, m)
    assert abs(tau - 0.54) < 1e-6 and abs(y_inf - 0.25) < 1e-6
    # the onset and a noisy record: the fit window starts at t_on
    rng = np.random.default_rng(4)
    t2 = np.linspace(0.0, 4.0, 401)
    m2 = np.where(t2 < 0.5, 1.0, 0.1 + 0.9 * np.exp(-(t2 - 0.5) / 1.29))
    m2 = m2 + rng.normal(0.0, 0.005, t2.size)
    tau2, y2 = A.collapse_time(t2, m2, t_on=0.5)
    assert abs(tau2 - 1.29) / 1.29 < 0.05 and abs(y2 - 0.1) < 0.05


def test_collapse_window_stops_before_a_reversal():
    """A projection that falls through zero (a reversal) is fitted only over
    its collapse: the part after y = 0.1 (here a linear run to -1) must not
    bias tau."""
    pytest.importorskip("scipy")
    t = np.linspace(0.0, 5.0, 1001)
    y = np.exp(-t / 0.4)
    tc = 0.4 * math.log(10.0)                             # y reaches 0.1 here
    y = np.where(t <= tc, y, 0.1 - (t - tc))
    tau, _ = A.collapse_time(t, y)
    assert abs(tau - 0.4) < 2e-3


def test_same_sign_intervals_on_straight_segments():
    """Straight-line histories: the crossings, hence the interval ends, are
    exact under linear interpolation."""
    t = np.linspace(0.0, 2.0, 21)                         # step 0.1
    a = 1.0 - t / 0.55                                    # crosses zero at 0.55
    b = -1.0 + t / 1.23                                   # crosses zero at 1.23
    iv = A.same_sign_intervals(t, a, b)
    assert len(iv) == 1
    assert abs(iv[0][0] - 0.55) < 1e-12 and abs(iv[0][1] - 1.23) < 1e-12
    s, e, d = A.transient_ferromagnetic_state(t, a, b)
    assert abs(d - 0.68) < 1e-12 and (s, e) == iv[0]


def test_transient_state_needs_the_slow_reversal():
    t = np.linspace(0.0, 3.0, 31)
    # the fast sublattice crosses and comes back; the slow one never reverses
    a = np.cos(np.pi * t / 1.5)                           # zeros at 0.75, 2.25
    b = -0.5 * np.ones_like(t)
    iv = A.same_sign_intervals(t, a, b)
    assert len(iv) == 1 and iv[0][1] is not None          # closed by the fast one
    assert A.transient_ferromagnetic_state(t, a, b) is None
    # parallel at the start: not the antiparallel initial state
    assert A.transient_ferromagnetic_state(t, np.ones_like(t), np.ones_like(t)) is None
    # a same-sign interval still open at the end
    iv2 = A.same_sign_intervals(t, 1.0 - t, -1.0 + 0.0 * t)
    assert iv2[-1][1] is None


def test_equilibration_time_of_an_exponential_approach():
    tau = 0.7
    t = np.linspace(0.0, 30 * tau, 30001)
    Tl = 900.0 - 600.0 * np.exp(-t / tau)                 # 300 K -> 900 K
    assert abs(A.equilibration_time(t, Tl, 0.9) - tau * math.log(10.0)) < 1e-3
    # cooling instead of heating
    Te = 900.0 + 600.0 * np.exp(-t / tau)
    assert abs(A.equilibration_time(t, Te, 0.9) - tau * math.log(10.0)) < 1e-3


def test_convergence_time_of_three_relaxing_temperatures():
    """Te = T + A e^{-t/tau}, Tl = T - B e^{-t/tau}, Ts between them: the
    largest difference is (A + B) e^{-t/tau}, below tol from
    tau ln((A + B) / tol) on."""
    tau, A_, B_ = 0.8, 1200.0, 500.0
    t = np.linspace(0.0, 10.0, 100001)
    Te = 850.0 + A_ * np.exp(-t / tau)
    Tl = 850.0 - B_ * np.exp(-t / tau)
    Ts = 850.0 + 0.3 * A_ * np.exp(-t / tau)
    tc = A.convergence_time(t, [Te, Tl, Ts], tol=20.0)
    assert abs(tc - tau * math.log((A_ + B_) / 20.0)) < 2e-4
    assert A.convergence_time(t, [Te, Tl], tol=1e-9) is None
    assert A.convergence_time(t, [Tl, Tl], tol=1.0) == 0.0


def test_critical_cooling_duration():
    ds = [1, 2, 3, 4, 5, 6, 7, 8]
    # the paper's kind of rows: switching from d = 5 on; from d = 7 on; never
    assert A.critical_cooling_duration(ds, [0, 0, 0, 0.1, 0.85, 1.0, 0.95, 1.0]) == 5.0
    assert A.critical_cooling_duration(ds, [0, 0, 0.6, 0.2, 0.4, 0.45, 1.0, 0.9]) == 7.0
    assert A.critical_cooling_duration(ds, [0, 0, 0, 0, 0, 0, 0.1, 0.3]) is None
    # a dip below the level after a first rise moves d_c past the dip
    assert A.critical_cooling_duration(ds, [0, 0.7, 0.8, 0.3, 0.6, 0.7, 0.8, 0.9]) == 5.0
    assert A.critical_cooling_duration(ds, [1.0] * 8) == 1.0
    assert A.critical_cooling_duration(ds, [0.5] * 8, level=0.5) == 1.0
    with pytest.raises(ValueError):
        A.critical_cooling_duration([2, 1], [0, 1])
