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
