"""Autotuner of the kernels' launch shape.

The knobs are the colour-pass block size and sites per thread, the lattice
kernels' block size, the number of steps captured per HIP graph replay and
the block size of the persistent per-run kernel (0 keeps every run on the
multi-kernel step), the order of the work tables over the XCDs, where
neighbours are binned and how many lanes share an atom's neighbour list.
Every setting performs the same arithmetic for every site, atom and cell,
so the tuner times real steps of the run being tuned: a coordinate search
(one knob at a time, the others held) keeps the fastest setting, and the
run's trajectory is bitwise what it would have been untuned.
"""
from __future__ import annotations

import json
import os
import time
from typing import Dict, List, Optional

KNOBS = {
    "persist_block": (0, 256, 512, 1024),
    "graph_steps": (8, 16, 32, 64),
    "spin_spt": (1, 2, 4),
    "spin_block": (0, 64, 128, 256),
    "atom_block": (64, 128, 256),
    "atom_lanes": (0, 1, 2, 4),
    "xcd_order": (0, 1),
    "bin_mode": (0, 1, 2),
    "merge_sweeps": (1, 0),
    "spin_access": (0, 1),
    "fuse_force": (1, 0),
}

_CACHE_FILE = os.path.join(os.path.expanduser("~"), ".cache", "paper_2608_18541_amd",
                           "tuning.json")


def _load_cache() -> dict:
    try:
        with open(_CACHE_FILE) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _save_cache(c: dict) -> None:
    try:
        os.makedirs(os.path.dirname(_CACHE_FILE), exist_ok=True)
        with open(_CACHE_FILE, "w") as f:
            json.dump(c, f, indent=1)
    except OSError:
        pass


def _time_steps(target, steps: int) -> float:
    target.advance(steps)
    target.synchronize()
    t0 = time.perf_counter()
    target.advance(steps)
    target.synchronize()
    return (time.perf_counter() - t0) / steps


def valid(t: dict) -> bool:
    """Whether a setting is accepted by the library (a block of the force
    kernel covers at least 64 atoms)."""
    lanes = t.get("atom_lanes", 0)
    return lanes == 0 or t.get("atom_block", 256) // lanes >= 64


def _steps_for(t: dict, steps: int) -> int:
    g = t["graph_steps"]
    return (max(steps, g) + g - 1) // g * g


def autotune(target, key: Optional[str] = None, steps: int = 64, rounds: int = 2,
             use_cache: bool = True, log: Optional[List] = None) -> Dict[str, int]:
    """Tunes a ``native.System`` or ``native.Batch`` in place and returns the
    chosen setting.  Each candidate is timed against the current best in
    interleaved rounds (best, candidate, best, candidate, ...), so a
    workload that speeds up or slows down as it evolves does not bias the
    comparison; a candidate replaces the best when its fastest round is at
    least 3% lower.  ``key`` names the workload for the cache (the search is
    skipped when a setting is cached)."""
    cache = _load_cache() if use_cache and key else {}
    if key and key in cache:
        target.set_tuning(**cache[key])
        return target.tuning()
    best = dict(target.tuning())
    for knob, values in KNOBS.items():
        for v in values:
            if v == best[knob]:
                continue
            trial = dict(best)
            trial[knob] = v
            if knob == "atom_lanes" and not valid(trial):
                trial["atom_block"] = 64 * v
            if not valid(trial):
                continue
            tb, tt = [], []
            for _ in range(rounds):
                for cfg, acc in ((best, tb), (trial, tt)):
                    target.set_tuning(**cfg)
                    acc.append(_time_steps(target, _steps_for(cfg, steps)))
            mb, mt = min(tb), min(tt)
            if log is not None:
                log.append((dict(trial), mt, mb))
            if mt < 0.97 * mb:
                best = trial
    target.set_tuning(**best)
    if key:
        cache = _load_cache()
        cache[key] = best
        _save_cache(cache)
    return best
