"""Switching statistics of ensembles of independent realizations.

Methods G (statistical procedure): a run has switched when the z component of the Gd sublattice
magnetisation has reversed sign and stays reversed to the end of the run;
probabilities over n realizations carry Wilson 95% score intervals.
"""
from __future__ import annotations

import math
from typing import Sequence, Tuple

import numpy as np

Z95 = 1.959963984540054


def wilson_ci(k: int, n: int, z: float = Z95) -> Tuple[float, float]:
    """Wilson score interval for k successes out of n trials."""
    if n <= 0:
        return (0.0, 1.0)
    p = k / n
    den = 1.0 + z * z / n
    centre = (p + z * z / (2 * n)) / den
    half = z * math.sqrt(p * (1.0 - p) / n + z * z / (4.0 * n * n)) / den
    return (max(0.0, centre - half), min(1.0, centre + half))


def switched(mz_gd: Sequence[float], tail_fraction: float = 0.1) -> bool:
    """True when every sample in the last ``tail_fraction`` of a run has the
    opposite sign to the first sample (a sustained reversal)."""
    m = np.asarray(mz_gd, dtype=np.float64)
    if m.size < 2 or m[0] == 0.0:
        return False
    k = max(1, int(math.ceil(tail_fraction * (m.size - 1))))
    tail = m[-k:]
    return bool(np.all(tail * m[0] < 0.0))


def homogeneity_chi2(k_a: Sequence[int], k_b: Sequence[int], n: int) -> Tuple[float, int, float]:
    """Whether two sets of switching counts (k_a[c], k_b[c] successes out of
    n each, per cell c) share their probabilities: the sum over cells with
    a pooled probability strictly between 0 and 1 of the squared
    two-proportion z statistic, its degrees of freedom (those cells) and the
    upper-tail p value of chi^2 with that many degrees of freedom by the
    Wilson-Hilferty cube-root normal approximation (about 1e-3 absolute at
    dof >= 10)."""
    chi2, dof = 0.0, 0
    for a, c in zip(np.ravel(k_a), np.ravel(k_b)):
        pp = (a + c) / (2.0 * n)
        if 0.0 < pp < 1.0:
            chi2 += (a - c) ** 2 / (2.0 * n * pp * (1.0 - pp))
            dof += 1
    if dof == 0:
        return 0.0, 0, 1.0
    wz = ((chi2 / dof) ** (1.0 / 3.0) - (1.0 - 2.0 / (9.0 * dof))) / math.sqrt(2.0 / (9.0 * dof))
    return chi2, dof, 0.5 * math.erfc(wz / math.sqrt(2.0))
