"""Trajectory analysis of the observable histories (host side).

The quantities the paper reads off its trajectories (Results, sublattice
dynamics and the three-temperature benchmark):

* the time constant of a sublattice's initial collapse, from a
  single-exponential fit;
* the transient ferromagnetic-like state: an interval in which two
  sublattices that are antiparallel at the start carry the same sign of
  m_z, before the slower one completes its reversal;
* the lattice's equilibration time (when it has covered 90% of its range)
  and the time at which the electron, lattice and spin temperatures come
  together;
* the critical cooling-duration multiplier of each peak temperature in a
  T_e^0 x d phase diagram.

Readings where the paper gives no procedure (fit window, interpolation of
crossings, the equilibrium level and the convergence tolerance) are stated
with each function.
"""
from __future__ import annotations

from typing import List, Optional, Sequence, Tuple

import numpy as np


def collapse_time(t: Sequence[float], m: Sequence[float], t_on: Optional[float] = None,
                  stop: float = 0.1) -> Tuple[float, float]:
    """Time constant tau of the initial collapse of a sublattice magnetisation
    m(t) (its z projection), from a least-squares fit of
    y(t) = y_inf + (1 - y_inf) exp(-(t - t_on) / tau) to y = m / m(t_on).

    Reading: the fit covers the samples from t_on (default the first sample)
    up to the first one where y has fallen to `stop` (or to its minimum when
    it never does), i.e. the collapse before any reversal or recovery.
    Returns (tau, y_inf)."""
    from scipy.optimize import curve_fit

    t = np.asarray(t, dtype=np.float64)
    m = np.asarray(m, dtype=np.float64)
    i0 = 0 if t_on is None else int(np.searchsorted(t, t_on))
    t0 = t[i0]
    y = m[i0:] / m[i0]
    tt = t[i0:] - t0
    below = np.nonzero(y <= stop)[0]
    i1 = int(below[0]) if below.size else int(np.argmin(y))
    i1 = max(i1, 2)
    tt, y = tt[: i1 + 1], y[: i1 + 1]
    # initial guess: the time the drop first reaches 1 - 1/e of its extent
    drop = 1.0 - y.min()
    k = int(np.argmax(1.0 - y >= (1.0 - np.exp(-1.0)) * drop))
    tau0 = max(tt[k], tt[1])

    def model(x, y_inf, tau):
        return y_inf + (1.0 - y_inf) * np.exp(-x / tau)

    (y_inf, tau), _ = curve_fit(model, tt, y, p0=(y.min(), tau0), maxfev=20000)
    return float(tau), float(y_inf)


def _crossing(t0: float, t1: float, a0: float, a1: float) -> float:
    """Time of the zero of the straight line through (t0, a0), (t1, a1)."""
    return t0 + (t1 - t0) * a0 / (a0 - a1)


def same_sign_intervals(t: Sequence[float], a: Sequence[float],
                        b: Sequence[float]) -> List[Tuple[float, Optional[float]]]:
    """Intervals in which a(t) and b(t) have the same sign.  Reading: the
    series are taken as straight between samples, so an interval opens and
    closes at the interpolated zero of the component that changed sign; one
    still open at the last sample ends with None."""
    t = np.asarray(t, dtype=np.float64)
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    same = np.sign(a) * np.sign(b) > 0
    out: List[Tuple[float, Optional[float]]] = []
    start = t[0] if same[0] else None
    for k in range(1, len(t)):
        if same[k] == same[k - 1]:
            continue
        # the component whose sign changed between k-1 and k fixes the time
        x = a if np.sign(a[k]) != np.sign(a[k - 1]) else b
        tc = _crossing(t[k - 1], t[k], x[k - 1], x[k])
        if same[k]:
            start = tc
        else:
            out.append((float(start), float(tc)))
            start = None
    if start is not None:
        out.append((float(start), None))
    return out


def transient_ferromagnetic_state(t: Sequence[float], mz_fast: Sequence[float],
                                  mz_slow: Sequence[float]) -> Optional[Tuple[float, float, float]]:
    """The transient ferromagnetic-like state of two sublattices that are
    antiparallel at the first sample: the first interval of same-sign m_z
    that closes by the slow sublattice's own reversal (its sign at the end of
    the interval differs from its initial sign).  Returns (start, end,
    duration), or None when there is no such interval."""
    t = np.asarray(t, dtype=np.float64)
    a = np.asarray(mz_fast, dtype=np.float64)
    b = np.asarray(mz_slow, dtype=np.float64)
    if not np.sign(a[0]) * np.sign(b[0]) < 0:
        return None
    for start, end in same_sign_intervals(t, a, b):
        if end is None:
            continue
        k = int(np.searchsorted(t, end))
        k = min(k, len(t) - 1)
        if np.sign(b[k]) != np.sign(b[0]):
            return start, end, end - start
    return None


def equilibration_time(t: Sequence[float], T: Sequence[float], frac: float = 0.9,
                       tail: float = 0.1) -> float:
    """First time at which T has covered `frac` of its range from T(0) to the
    equilibrium level.  Reading: the equilibrium level is the mean over the
    last `tail` of the record; the crossing is interpolated linearly."""
    t = np.asarray(t, dtype=np.float64)
    T = np.asarray(T, dtype=np.float64)
    n_tail = max(1, int(round(tail * len(T))))
    T_eq = T[-n_tail:].mean()
    goal = T[0] + frac * (T_eq - T[0])
    s = np.sign(T_eq - T[0])
    k = int(np.argmax(s * (T - goal) >= 0.0))
    if k == 0:
        return float(t[0])
    return float(_crossing(t[k - 1], t[k], T[k - 1] - goal, T[k] - goal))


def convergence_time(t: Sequence[float], temps: Sequence[Sequence[float]], tol: float) -> Optional[float]:
    """First sample time after which every pair of the given temperature
    histories stays within `tol` (kelvin) for the rest of the record, or
    None when they never do."""
    t = np.asarray(t, dtype=np.float64)
    X = np.asarray(temps, dtype=np.float64)
    spread = X.max(axis=0) - X.min(axis=0)
    bad = np.nonzero(spread > tol)[0]
    if bad.size == 0:
        return float(t[0])
    k = int(bad[-1]) + 1
    return float(t[k]) if k < len(t) else None


def critical_cooling_duration(ds: Sequence[float], P: Sequence[float],
                              level: float = 0.5) -> Optional[float]:
    """Critical cooling-duration multiplier d_c of one peak temperature, read
    from switching probabilities P at increasing multipliers ds.  Reading:
    the smallest d from which P stays at or above `level` for every larger
    d of the grid; None when the largest d is below it (no d_c in range)."""
    ds = np.asarray(ds, dtype=np.float64)
    P = np.asarray(P, dtype=np.float64)
    if ds.shape != P.shape or ds.size == 0 or np.any(np.diff(ds) <= 0):
        raise ValueError("ds must increase and match P")
    ok = P >= level
    if not ok[-1]:
        return None
    k = len(ok) - 1
    while k > 0 and ok[k - 1]:
        k -= 1
    return float(ds[k])


def strain_zz_profile(ncell, lattice: int, a: float, x) -> np.ndarray:
    """eps_zz(z) of the acoustic strain pulse (Results A): per z layer of unit
    cells, the mean displacement along z of the layer's atoms from their ideal
    sites (canonical site order, sites offset by a/4), differentiated along z
    by the periodic central difference."""
    Lx, Ly, Lz = (int(v) for v in ncell)
    nb = 2 if lattice == 1 else 1
    x = np.asarray(x, dtype=np.float64)
    idx = np.arange(x.shape[0])
    b = idx % nb
    z = (idx // nb) // (Lx * Ly)
    ideal = (z + 0.25 + 0.5 * b) * a
    box = Lz * a
    d = x[:, 2] - ideal
    d -= box * np.round(d / box)
    uz = np.bincount(z, weights=d, minlength=Lz) / np.bincount(z, minlength=Lz)
    return (np.roll(uz, -1) - np.roll(uz, 1)) / (2.0 * a)

