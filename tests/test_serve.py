"""Continuous-batching server: host scheduling logic on the CPU (a stand-in
executor with a simulated clock) and, on the GPU, that every served result
equals the same run alone."""
from dataclasses import dataclass, replace

import numpy as np
import pytest

from paper_2608_18541_amd import inputs as I
from paper_2608_18541_amd import serve as S
from paper_2608_18541_amd import workloads as W


class FakeClock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t

    def sleep(self, dt):
        self.t += dt


class FakeExecutor:
    """Host stand-in for a batch: fixed slots and memory budget, time per
    step proportional to the sites in flight (plus a launch floor)."""

    def __init__(self, clock, slots=4, budget=10_000, per_site=1e-8, floor=1e-5):
        self.clock, self.slots, self.budget = clock, slots, budget
        self.per_site, self.floor = per_site, floor
        self.runs_ = {}
        self.peak_mem = 0
        self.admissions = []

    def used(self):
        return sum(r["spec"].n_sites for r in self.runs_.values())

    def try_add(self, spec, state, n_steps, obs_every=0, obs_capacity=1):
        if len(self.runs_) >= self.slots or self.used() + spec.n_sites > self.budget:
            return None
        slot = min(set(range(self.slots)) - set(self.runs_))
        self.runs_[slot] = {"spec": spec, "target": n_steps, "done": 0, "every": obs_every}
        self.peak_mem = max(self.peak_mem, self.used())
        self.admissions.append((self.clock(), slot))
        return slot

    def advance(self, n):
        if not self.runs_:
            return
        steps = min(n, max(r["target"] - r["done"] for r in self.runs_.values()))
        sites = sum(r["spec"].n_sites for r in self.runs_.values() if r["done"] < r["target"])
        self.clock.t += n * (self.floor + self.per_site * sites)
        for r in self.runs_.values():
            r["done"] = min(r["target"], r["done"] + n)
        del steps

    def synchronize(self):
        pass

    def runs(self):
        return [{"slot": s, "steps_done": r["done"], "steps_target": r["target"]}
                for s, r in self.runs_.items()]

    def get(self, slot, state=True):
        r = self.runs_[slot]
        k = r["done"] // r["every"] + 1
        return {"obs": [{"M": np.array([[0, 0, -1.0]] * 2 + [[0, 0, 0]] * 2) if q else
                         np.array([[0, 0, 1.0]] * 4)} for q in range(k)]}

    def remove(self, slot):
        del self.runs_[slot]


@dataclass
class _Spec:
    n_sites: int


@dataclass
class _Run:
    spec: _Spec
    n_steps: int
    state: object = None


def _trace(n=40, rate=20.0, seed=3):
    rng = np.random.default_rng(seed)
    t, out = 0.0, []
    for k in range(n):
        t += rng.exponential(1.0 / rate)
        out.append(W.Request(k, t, _Run(_Spec(int(rng.choice([500, 1000, 4000]))),
                                          int(rng.integers(100, 3000)))))
    return out


def test_server_completes_and_respects_budget():
    clock = FakeClock()
    ex = FakeExecutor(clock, slots=4, budget=6000)
    srv = S.Server(ex, chunk=100, obs_every=100, clock=clock, sleep=clock.sleep)
    trace = _trace()
    res = srv.run(trace)
    assert [r.rid for r in res] == [q.rid for q in trace]
    assert ex.peak_mem <= 6000
    for r, q in zip(res, trace):
        assert r.admitted >= q.arrival - 1e-12
        assert r.finished > r.admitted
        assert r.switched is True
    # first come, first served
    adm = [r.admitted for r in res]
    assert all(a <= b + 1e-12 for a, b in zip(adm, adm[1:]))
    st = S.summarize(res, srv.makespan)
    assert st.p99 >= st.p50 > 0 and st.throughput > 0


def test_continuous_admission_overlaps_work():
    """A request arriving while others run joins at the next chunk boundary,
    not after the running ones finish."""
    clock = FakeClock()
    ex = FakeExecutor(clock, slots=4, budget=100_000)
    long = W.Request(0, 0.0, _Run(_Spec(1000), 10_000))
    late = W.Request(1, 0.001, _Run(_Spec(1000), 200))
    srv = S.Server(ex, chunk=100, obs_every=100, clock=clock, sleep=clock.sleep)
    res = srv.run([long, late])
    assert res[1].admitted < res[0].finished
    assert res[1].finished < res[0].finished


def test_fifo_baseline_queue():
    reqs = [W.Request(k, a, _Run(_Spec(1), 1)) for k, a in enumerate([0.0, 0.5, 0.6, 10.0])]
    out = S.fifo_baseline(reqs, lambda r: 1.0)
    assert [r.finished for r in out] == [1.0, 2.0, 3.0, 11.0]
    assert [round(r.latency, 9) for r in out] == [1.0, 1.5, 2.4, 1.0]


@pytest.mark.gpu
def test_served_results_equal_alone():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2608_18541_amd import native as N
    trace = W.request_trace(n=8, rate=200.0, seed=11, sizes=(6, 8, 10), steps_range=(60, 400))
    batch = N.Batch(precision=N.SL_FP32, max_runs=3)
    srv = S.Server(batch, chunk=64, obs_every=20, keep_state=True)
    res = srv.run(trace)
    assert len(res) == len(trace)
    for r, q in zip(res, trace):
        alone = N.System(q.run.spec, q.run.state, precision=N.SL_FP32, obs_every=20,
                         obs_capacity=q.run.n_steps // 20 + 2)
        alone.step(q.run.n_steps)
        a = alone.state()
        for k in ("s", "x", "v", "Te"):
            assert np.array_equal(a[k], r.state[k]), (q.rid, k)
        mz = np.array([o["M"][1][2] for o in alone.observables()])
        assert np.array_equal(mz, r.mz_gd)
        alone.close()
