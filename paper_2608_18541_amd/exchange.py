"""The three-parameter radial exchange function and its re-derivation for a
lattice's nearest-neighbour distance (Methods, re-derivation of the radial
exchange function).

J(r) = 4 J1 x (1 - J2 x) e^{-x},  x = (r / J3)^2.

Published (J2, J3) sets are fitted to bcc metals; on another lattice the
function's maximum is not at the nearest-neighbour distance r1, and J(r1)
is not J1. The re-derivation puts the extremum at r1 (dJ/dx = 0 there) and
makes J(r1) = J1 exactly. Both conditions together fix x1 = (r1 / J3)^2
independently of r1: with J2 = (x1 - 1) / (x1 (x1 - 2)) from the first,
1 - J2 x1 = 1 / (2 - x1), and the second becomes 4 x1 e^{-x1} = 2 - x1,
whose only root in (0, 2) is x1 = 0.6458...  J3 = r1 / sqrt(x1) then scales
with the lattice.

Host-side set-up only; the kernels take per-pair exchange constants.
"""
from __future__ import annotations

import math
from typing import Tuple

import numpy as np


def radial_exchange(r, J1: float, J2: float, J3: float):
    """J(r) = 4 J1 x (1 - J2 x) e^{-x} with x = (r / J3)^2, in the units of J1."""
    x = (np.asarray(r, dtype=np.float64) / J3) ** 2
    return 4.0 * J1 * x * (1.0 - J2 * x) * np.exp(-x)


def radial_exchange_dr(r, J1: float, J2: float, J3: float):
    """dJ/dr = dJ/dx * 2 r / J3^2, with
    dJ/dx = 4 J1 e^{-x} (1 - x - J2 x (2 - x))."""
    r = np.asarray(r, dtype=np.float64)
    x = (r / J3) ** 2
    dJdx = 4.0 * J1 * np.exp(-x) * (1.0 - x - J2 * x * (2.0 - x))
    return dJdx * 2.0 * r / (J3 * J3)


def _x1_root() -> float:
    """Root of 4 x e^{-x} - (2 - x) in (0, 2) by bisection.  The function is
    -2 at 0, 8 e^{-2} > 0 at 2 and increasing in between (its derivative
    4 (1 - x) e^{-x} + 1 is at least 1 - 4 e^{-2} > 0), so the root is
    unique and bisection reaches the nearest doubles."""
    lo, hi = 0.0, 2.0
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if mid in (lo, hi):
            break
        if 4.0 * mid * math.exp(-mid) - (2.0 - mid) < 0.0:
            lo = mid
        else:
            hi = mid
    return 0.5 * (lo + hi)


def rederive_radial_exchange(r1: float) -> Tuple[float, float, float]:
    """(x1, J2, J3) that put the maximum of J(r) at the nearest-neighbour
    distance r1 (angstrom) with J(r1) = J1, for any J1 > 0.  J3 is in the
    units of r1."""
    if not r1 > 0.0:
        raise ValueError("r1 must be positive")
    x1 = _x1_root()
    J2 = (x1 - 1.0) / (x1 * (x1 - 2.0))
    J3 = r1 / math.sqrt(x1)
    return x1, J2, J3


def nearest_neighbour_distance(lattice: str, a: float) -> float:
    """r1 of a cubic lattice with constant a: sc a, bcc a sqrt(3)/2, fcc a / sqrt(2)."""
    f = {"sc": 1.0, "bcc": math.sqrt(3.0) / 2.0, "fcc": 1.0 / math.sqrt(2.0)}
    if lattice not in f:
        raise ValueError("lattice must be sc, bcc or fcc")
    return a * f[lattice]


def shell_distances(lattice: str, a: float) -> Tuple[float, float]:
    """Distances of the first two neighbour shells: sc a, a sqrt(2); bcc
    a sqrt(3)/2, a; fcc a / sqrt(2), a."""
    r1 = nearest_neighbour_distance(lattice, a)
    r2 = {"sc": a * math.sqrt(2.0), "bcc": a, "fcc": a}[lattice]
    return r1, r2


def shell_exchange_table(lattice: str, a: float, J1_pairs, J2: float, J3: float,
                         cutoff: float, n_shells: int):
    """Per-shell, per-species-pair exchange constants (eV) of J(r) on an
    ideal lattice, in the layout of the system description: n_shells 4 x 4
    tables, shell k holding J(r_k) for every pair (zero beyond the cutoff).
    On a frozen lattice every pair of a shell keeps its ideal distance, so
    these constants reproduce J(r) exactly.  J1_pairs is a 4 x 4 table of
    amplitudes (eV); J2 and J3 are shared by all pairs."""
    J1_pairs = np.asarray(J1_pairs, dtype=np.float64)
    if J1_pairs.shape != (4, 4) or not np.array_equal(J1_pairs, J1_pairs.T):
        raise ValueError("J1_pairs must be a symmetric 4 x 4 table")
    if not 1 <= n_shells <= 2:
        raise ValueError("one or two shells")
    out = []
    for r in shell_distances(lattice, a)[:n_shells]:
        f = float(radial_exchange(r, 1.0, J2, J3)) if r < cutoff else 0.0
        out.append(tuple(tuple(float(f * v) for v in row) for row in J1_pairs))
    return tuple(out)
