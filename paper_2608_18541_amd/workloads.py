"""Ensemble and request-stream workloads built from the seeded presets.

* ``phase_diagram``: independent realizations of the laser-heated
  Gd25(FeCo)75 alloy over a grid of damping values x peak electron
  temperatures x seeds (Methods F: replicas share nothing; Methods G: n
  realizations per condition with an independent alloy and noise seed
  each).
* ``production_diagram``: the production runs (Results, phase diagram):
  frozen alloy lattice, literature anisotropy, zero field, and the
  three-stage stepped electron temperature, over a grid of peak
  temperatures x cooling-duration multipliers d x seeds.
* ``field_runs``: production runs at one condition under zero field, a
  0.5 T bias and a 10 T field opposing the reversal (Results, field
  (in)dependence of thermal switching).
* ``request_trace``: a Poisson stream of alloy simulations of mixed size,
  composition, peak temperature and length.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, replace
from typing import List, Optional

import numpy as np

from . import inputs as I


@dataclass
class RunSpec:
    """A run to perform; its seeded initial state is drawn on demand."""
    spec: I.SystemSpec
    n_steps: int
    tag: tuple = ()
    kind: str = "afm"
    p_gd: float = 0.25
    exact_count: bool = False

    @property
    def state(self) -> I.InitialState:
        return I.initial_state(self.spec, self.kind, p_gd=self.p_gd, exact_count=self.exact_count)


def alloy_run(L: int, alpha: float, T_peak: float, seed: int, run_id: int, n_steps: int,
              p_gd: float = 0.25, fwhm: float = 0.05, t0: float = 0.1,
              lattice_mode: int = 1) -> RunSpec:
    """One realization: sc alloy L^3 with the electron grid at 14.08 A cells
    (L/4 cells per side), laser calibrated to T_peak."""
    tn = max(1, L // 4)
    S0 = I.laser_S0_metal(T_peak, fwhm, t0)
    spec = I.gdfeco_sc_spec(L=L, tn=tn, alpha=alpha, S0=S0, fwhm=fwhm, t0=t0, seed=seed,
                            run_id=run_id, lattice_mode=lattice_mode)
    return RunSpec(spec, n_steps, (alpha, T_peak), "afm", p_gd)


def phase_diagram(L: int = 16, n_alpha: int = 8, n_temp: int = 8, n_seeds: int = 20,
                  n_steps: int = 20000, seed: int = 2026, alpha_range=(0.005, 0.04),
                  temp_range=(800.0, 2400.0), lattice_mode: int = 1) -> List[RunSpec]:
    """alpha log-spaced x T_peak linearly spaced x seeds; run_id enumerates
    the runs so every realization has its own alloy and noise stream."""
    a0, a1 = alpha_range
    alphas = [a0 * (a1 / a0) ** (k / max(1, n_alpha - 1)) for k in range(n_alpha)]
    t0, t1 = temp_range
    temps = [t0 + k * (t1 - t0) / max(1, n_temp - 1) for k in range(n_temp)]
    I.laser_S0_many(temps, 0.05, 0.1)        # calibrate every peak at once
    out = []
    rid = 0
    for a in alphas:
        for T in temps:
            for s in range(n_seeds):
                out.append(alloy_run(L, a, T, seed, rid, n_steps, lattice_mode=lattice_mode))
                rid += 1
    return out



def production_run(L: int, T0: float, d: float, seed: int, run_id: int, n_steps: int,
                   alpha: float = 0.01, base_ends=(0.1, 0.5), p_gd: float = 0.25,
                   lattice: str = "sc") -> RunSpec:
    """One production realization: an alloy with exactly round(p_gd N) Gd
    sites on a frozen lattice, the literature anisotropy on both species,
    B = 0, electrons held at T0 until d * base_ends[0] ps, at T0 / 2 until
    d * base_ends[1] ps, then at 300 K.  lattice "fcc": the paper's model
    (L^3 fcc cells, a = 3.6 A, the literature exchange, one electron cell);
    "sc": the 32^3 workload's alloy on L^3 simple-cubic cells.  The paper
    scales the stage durations by d but does not give the base durations;
    base_ends is this workload's choice."""
    if lattice == "fcc":
        spec = I.gdfeco_fcc_spec(L=L, alpha=alpha, seed=seed, run_id=run_id)
    else:
        spec = I.gdfeco_sc_spec(L=L, tn=max(1, L // 4), alpha=alpha, lattice_mode=0,
                                K=(I.GDFECO_K, I.GDFECO_K, 0.0, 0.0), seed=seed, run_id=run_id)
    spec = replace(spec, ttm_mode=2, step_T=(T0, 0.5 * T0, 300.0),
                   step_end=(d * base_ends[0], d * base_ends[1]))
    return RunSpec(spec, n_steps, (T0, d), "afm", p_gd, exact_count=True)


def production_diagram(L: int = 16, n_temp: int = 8, n_d: int = 8, n_seeds: int = 20,
                       n_steps: int = 50000, seed: int = 2027, temp_range=(800.0, 2900.0),
                       d_range=(1.0, 8.0), base_ends=(0.1, 0.5),
                       lattice: str = "sc") -> List[RunSpec]:
    """Peak T_e linearly spaced x d linearly spaced x seeds (the paper's
    8 x 8 x 20 grid: 800-2900 K, d = 1-8); run_id enumerates the runs."""
    t0, t1 = temp_range
    temps = [t0 + k * (t1 - t0) / max(1, n_temp - 1) for k in range(n_temp)]
    d0, d1 = d_range
    ds = [d0 + k * (d1 - d0) / max(1, n_d - 1) for k in range(n_d)]
    out = []
    rid = 0
    for T in temps:
        for d in ds:
            for s in range(n_seeds):
                out.append(production_run(L, T, d, seed, rid, n_steps, base_ends=base_ends,
                                          lattice=lattice))
                rid += 1
    return out


def field_runs(T0: float, d: float, n_seeds: int, L: int = 16, n_steps: int = 50000,
               seed: int = 2028, fields=(0.0, 0.5, 10.0), lattice: str = "sc") -> List[RunSpec]:
    """Production runs at (T0, d) under each field magnitude, seeds
    innermost.  The field points along +z: the Gd sublattice and the net
    moment start along +z and reverse to -z, so +z opposes the reversal
    (the paper's 10 T check); the 0.5 T bias is given the same direction."""
    out = []
    rid = 0
    for B in fields:
        for s in range(n_seeds):
            r = production_run(L, T0, d, seed, rid, n_steps, lattice=lattice)
            r.spec = replace(r.spec, B=(0.0, 0.0, float(B)))
            r.tag = (T0, d, B)
            out.append(r)
            rid += 1
    return out

@dataclass
class Request:
    rid: int
    arrival: float           # seconds after the start of the trace
    run: RunSpec


def request_trace(n: int = 600, rate: float = 50.0, seed: int = 7,
                  sizes=(8, 16, 24, 32, 48), x_range=(0.18, 0.32),
                  temp_range=(1000.0, 2200.0), steps_range=(5000, 30000),
                  steps_scale: float = 1.0, lattice_mode: int = 1) -> List[Request]:
    """Poisson arrivals (mean `rate` per second) of alloy simulations with a
    uniformly drawn cubic size, Gd fraction, peak T_e and step count
    (step counts multiplied by steps_scale)."""
    rng = np.random.default_rng(seed)
    draws = []
    t = 0.0
    for k in range(n):
        t += rng.exponential(1.0 / rate)
        draws.append((t, int(rng.choice(sizes)), float(rng.uniform(*x_range)),
                      float(rng.uniform(*temp_range)),
                      int(rng.integers(steps_range[0], steps_range[1] + 1))))
    I.laser_S0_many([d[3] for d in draws], 0.05, 0.1)
    out = []
    for k in range(n):
        t, L, x, T, steps = draws[k]
        steps = max(1, int(round(steps * steps_scale)))
        run = alloy_run(L, 0.01, T, seed, k, steps, p_gd=x, lattice_mode=lattice_mode)
        out.append(Request(k, t, run))
    return out
