"""Continuous-batching server for streams of spin-lattice simulations.

Requests arrive over time.  A request is admitted into the device batch as
soon as a slot is free and its HBM footprint fits the memory budget
(first come, first served).  Every admitted run then advances inside the
same launches as the runs already in flight, its state staying resident on
the device until it completes.  Finished runs are collected and their slots
and memory released between chunks of steps.  Each run's arithmetic is
independent of what else is in the batch, so a result is bitwise the same
as that run alone.

The executor is anything with ``try_add(spec, state, n_steps, obs_every=,
obs_capacity=)``, ``advance(n)``, ``synchronize()``, ``runs()``,
``get(slot, state=)`` (the run's samples, and its state when asked) and
``remove(slot)`` (``native.Batch`` on the GPU; the tests
also drive it with a host-side stand-in).
"""
from __future__ import annotations

import collections
import time
from dataclasses import dataclass, field
from typing import Callable, Dict, List, Optional

import numpy as np

from .stats import switched


@dataclass
class Result:
    rid: int
    arrival: float
    admitted: float
    finished: float
    n_steps: int
    n_sites: int
    switched: Optional[bool] = None
    mz_gd: Optional[np.ndarray] = None
    state: Optional[dict] = None
    error: Optional[str] = None

    @property
    def latency(self) -> float:
        return self.finished - self.arrival


@dataclass
class ServeStats:
    n: int
    makespan: float
    throughput: float            # requests per second
    atom_steps_per_s: float
    p50: float
    p99: float
    mean: float


def percentile(xs, q: float) -> float:
    return float(np.percentile(np.asarray(xs, dtype=np.float64), q)) if len(xs) else 0.0


def summarize(results: List[Result], makespan: float) -> ServeStats:
    lat = [r.latency for r in results]
    work = sum(r.n_sites * r.n_steps for r in results)
    return ServeStats(n=len(results), makespan=makespan,
                      throughput=len(results) / makespan if makespan > 0 else 0.0,
                      atom_steps_per_s=work / makespan if makespan > 0 else 0.0,
                      p50=percentile(lat, 50), p99=percentile(lat, 99),
                      mean=float(np.mean(lat)) if lat else 0.0)


class Server:
    def __init__(self, executor, chunk: int = 500, obs_every: int = 100,
                 keep_state: bool = False, clock: Callable[[], float] = time.perf_counter,
                 sleep: Callable[[float], None] = time.sleep,
                 progress: Optional[Callable[[str], None]] = None, progress_every: float = 20.0):
        self.ex = executor
        self.progress = progress
        self.progress_every = progress_every
        self.chunk = chunk
        self.obs_every = obs_every
        self.keep_state = keep_state
        self.clock = clock
        self.sleep = sleep
        self.log: List[tuple] = []
        # wall time by activity: advancing the batch (device work and its
        # wait), admitting requests, collecting finished runs, idle waiting
        # for arrivals
        self.time_in = {"advance": 0.0, "admit": 0.0, "collect": 0.0, "idle": 0.0}

    def run(self, requests) -> List[Result]:
        pending = collections.deque(sorted(requests, key=lambda r: r.arrival))
        waiting: collections.deque = collections.deque()
        active: Dict[int, tuple] = {}
        done: List[Result] = []
        t0 = self.clock()
        next_report = self.progress_every
        while pending or waiting or active:
            now = self.clock() - t0
            if self.progress is not None and now >= next_report:
                self.progress("served %d, active %d, waiting %d, pending %d at %.0f s"
                              % (len(done), len(active), len(waiting), len(pending), now))
                next_report = now + self.progress_every
            while pending and pending[0].arrival <= now:
                waiting.append(pending.popleft())
            # admission: first come first served, by slot and HBM footprint
            ta = self.clock()
            while waiting:
                req = waiting[0]
                spec = req.run.spec
                cap = req.run.n_steps // self.obs_every + 2
                slot = self.ex.try_add(spec, req.run.state, req.run.n_steps,
                                       obs_every=self.obs_every, obs_capacity=cap)
                if slot is None:
                    if not active:
                        raise RuntimeError("request %d does not fit an empty server" % req.rid)
                    break
                waiting.popleft()
                active[slot] = (req, self.clock() - t0)
            tb = self.clock()
            self.time_in["admit"] += tb - ta
            if not active:
                if pending:
                    self.sleep(max(0.0, pending[0].arrival - (self.clock() - t0)))
                self.time_in["idle"] += self.clock() - tb
                continue
            self.ex.advance(self.chunk)
            try:
                self.ex.synchronize()
            except RuntimeError:
                pass                             # reported per run when collected
            tc = self.clock()
            self.time_in["advance"] += tc - tb
            self.log.append((tc - t0, len(active), len(waiting)))
            for info in self.ex.runs():
                s = info["slot"]
                if s not in active or info["steps_done"] < info["steps_target"]:
                    continue
                req, t_adm = active.pop(s)
                err = None
                try:
                    out = self.ex.get(s, state=self.keep_state)
                except RuntimeError as e:       # the run stopped on a numerical error
                    out, err = {}, str(e)
                fin = self.clock() - t0
                mz = np.array([o["M"][1][2] for o in out.get("obs", [])])
                res = Result(rid=req.rid, arrival=req.arrival, admitted=t_adm, finished=fin,
                             n_steps=req.run.n_steps, n_sites=req.run.spec.n_sites,
                             switched=switched(mz) if mz.size > 1 else None, mz_gd=mz,
                             state=out if self.keep_state else None, error=err)
                done.append(res)
                self.ex.remove(s)
            self.time_in["collect"] += self.clock() - tc
        self.makespan = self.clock() - t0
        return sorted(done, key=lambda r: r.rid)


def fifo_baseline(requests, service_time: Callable[[object], float]) -> List[Result]:
    """One request at a time in arrival order: start = max(arrival, previous
    finish), finish = start + service time (the plain single-run path's
    measured time for that request)."""
    out = []
    busy_until = 0.0
    for r in sorted(requests, key=lambda q: q.arrival):
        start = max(r.arrival, busy_until)
        fin = start + service_time(r)
        busy_until = fin
        out.append(Result(rid=r.rid, arrival=r.arrival, admitted=start, finished=fin,
                          n_steps=r.run.n_steps, n_sites=r.run.spec.n_sites))
    return out
