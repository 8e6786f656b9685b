"""Benchmark of the spin-lattice step on one MI355X.

Workload: the Gd25(FeCo)75 ferrimagnet on a 32^3 simple-cubic lattice
(32768 sites, a = 3.52 A, Bernoulli Gd p = 0.25, moments 7.63 / 1.92 mu_B,
nearest-neighbour TM-TM / Gd-Gd / TM-Gd exchange, alpha = 0.01, B = 0),
live Morse lattice at 300 K, 8^3 two-temperature grid with the 50 fs
laser, dt = 0.1 fs, one FP64 run on the plain one-run-per-launch path.
A step is one full timestep (spin colour sweep, velocity Verlet, electron-
phonon step, electron grid).  Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import numpy as np

HBM_PEAK_GBS = 8000.0
KERNELS = ["spin_pass", "atom_final", "kick_drift", "end_step"]


def bytes_per_unit(kernel: str, fp: int, n_species: int, z_list: float) -> float:
    """Algorithmic bytes per processed unit of each kernel:
    spin_pass per updated site, atom_final / kick_drift per atom."""
    t = 8 if fp == 0 else 4
    sp = 1 if n_species > 1 else 0
    if kernel == "spin_pass":
        return 6 * t + sp + 2                  # own spin read + write, species, cell id
    if kernel == "atom_final":
        return 3 * t + 6 * t + 3 * t + 4 * z_list + 4 + sp + 2
    if kernel == "kick_drift":
        return 3 * t + 6 * t + 6 * t + 3 * t + sp + 2
    return 0.0


def units_per_launch(kernel: str, n_sites: int, colours: int) -> float:
    if kernel == "spin_pass":
        return n_sites / colours
    if kernel in ("atom_final", "kick_drift"):
        return float(n_sites)
    return 0.0


def cpu_baseline(spec, st, budget_s: float = 20.0) -> dict:
    """The FP64 oracle on the host (one thread), a bounded number of full
    steps of the same workload."""
    from oracle import oracle as O
    orc = O.Oracle(spec, st.species, st.spins, st.vel)
    steps = 0
    t0 = time.perf_counter()
    while True:
        orc.step(1)
        steps += 1
        el = time.perf_counter() - t0
        if el > budget_s * 0.5 or steps >= 50:
            break
    return {"value": spec.n_sites * steps / el, "unit": "atom-steps/s", "cores": 1,
            "kind": "oracle",
            "sample": "%d full steps of the 32^3 alloy (all-pairs Morse, FP64, one thread), "
                      "%.1f s" % (steps, el)}


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3000)
    ap.add_argument("--warmup", type=int, default=200)
    ap.add_argument("--profile-steps", type=int, default=100)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py: this build measures one GPU; --gpus %d is not supported "
              "(runs are independent replicas, see DESIGN.md for the sharding plan)" % args.gpus,
              file=sys.stderr)
        return 2

    import torch
    from paper_2608_18541_amd import inputs as I
    from paper_2608_18541_amd import native as N

    torch.cuda.set_device(0)
    spec = I.gdfeco_sc_spec(L=32, tn=8, S0=I.cfg1_S0(), alpha=0.01)
    st = I.initial_state(spec, "afm")
    sys_ = N.System(spec, st, precision=N.SL_FP64, obs_every=100)
    print("bench: workload built, warmup %d steps" % args.warmup, file=sys.stderr, flush=True)
    sys_.step(args.warmup)
    sys_.synchronize()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sys_.step(args.steps)
    sys_.synchronize()
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    value = spec.n_sites * args.steps / el
    print("bench: timed %d steps in %.3f s" % (args.steps, el), file=sys.stderr, flush=True)

    # per-kernel device time of the same path, HIP events on the run's stream
    avg, cnt = sys_.step_profiled(args.profile_steps)
    per_step = {k: avg[i] * cnt[i] / args.profile_steps for i, k in enumerate(KERNELS)}
    dom = max(per_step, key=per_step.get)
    di = KERNELS.index(dom)
    # mean neighbour-list length of the Morse list at this density
    z_list = 18.0
    bpu = bytes_per_unit(dom, 0, spec.n_species, z_list)
    units = units_per_launch(dom, spec.n_sites, 2)
    alg_bytes = bpu * units
    achieved = alg_bytes / (avg[di] * 1e-3) / 1e9 if avg[di] > 0 else 0.0
    roof = {"bound": "hbm", "kernel": dom, "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 5), "traffic": None,
            "avg_launch_us": round(avg[di] * 1e3, 3), "bytes_per_launch": int(alg_bytes),
            "per_step_us": {k: round(v * 1e3, 3) for k, v in per_step.items()}}
    sys_.close()

    out = {
        "metric": "atom-steps/s per run; batched runs/s + p50/p99 latency vs plain path",
        "value": round(value, 1), "unit": "atom-steps/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(el / args.steps * 1e3, 5),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "Gd25(FeCo)75 sc 32^3 (32768 sites), live Morse lattice, "
                               "8^3 two-temperature grid + 50 fs laser, dt 0.1 fs, "
                               "plain FP64 single run",
                   "n_sites": spec.n_sites, "seq_len": None, "global_batch": 1,
                   "parallelism": "single run"},
        "roofline": roof,
    }
    if not args.no_cpu_baseline:
        print("bench: timing the CPU oracle", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(spec, st)
    print(json.dumps(out))
    return 0


if __name__ == "__main__":
    sys.exit(main())
