"""The allocation-free entry point sl_step_noalloc against sl_step.

Two calls in a row through the C ABI, the second on a smaller system: each
steps a system with sl_step_noalloc and an identical system with sl_step,
and the two end bitwise equal (state and observable samples).  The caller's
allocator sees no allocation during the allocation-free calls.  The first
system is the plain FP64 alloy of the benchmark (merged, folded chunks with
unaligned head and tail steps); the second a 6^3 bcc Fe block in FP32 with
XCD-ordered tables.  A later allocation-free call continues a trajectory
that sl_step started.
"""
import sys

import numpy as np
import pytest

from paper_2608_18541_amd import inputs as I

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def N():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2608_18541_amd import native
    native.lib()
    return native


def _log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _same(N, a, b):
    sa, sb = a.state(), b.state()
    for k in ("s", "x", "v", "Te"):
        assert np.array_equal(sa[k], sb[k]), k
    oa, ob = a.observables(), b.observables()
    assert len(oa) == len(ob)
    for p, q in zip(oa, ob):
        assert np.array_equal(p["M"], q["M"]) and p["E_ex"] == q["E_ex"] and p["KE"] == q["KE"]


def _pair(N, spec, st, prec, obs_every, **tuning):
    a = N.System(spec, st, precision=prec, obs_every=obs_every)
    b = N.System(spec, st, precision=prec, obs_every=obs_every)
    if tuning:
        a.set_tuning(**tuning)
        b.set_tuning(**tuning)
    return a, b


def test_noalloc_equals_step_two_calls(N):
    # first call: the 32^3 alloy, FP64, live lattice and laser
    spec = I.gdfeco_sc_spec(L=32, tn=8, S0=0.3, t0=0.01, fwhm=0.005)
    st = I.initial_state(spec, "afm")
    _log("noalloc: 32^3 alloy FP64, 230 steps")
    a, b = _pair(N, spec, st, N.SL_FP64, 100)
    n0 = a._alloc.n_allocs
    a.step_noalloc(230)
    a.synchronize()
    assert a._alloc.n_allocs == n0
    b.step(230)
    _same(N, a, b)
    # second call: a smaller system, FP32, XCD-ordered tables
    spec2 = I.fe_bcc_spec(L=6, seed=21, run_id=3)
    st2 = I.initial_state(spec2, "tilt")
    _log("noalloc: 6^3 bcc FP32, 77 steps")
    c, d = _pair(N, spec2, st2, N.SL_FP32, 10, xcd_order=1)
    n1 = c._alloc.n_allocs
    c.step_noalloc(77)
    c.synchronize()
    assert c._alloc.n_allocs == n1
    d.step(77)
    _same(N, c, d)
    # sl_step first, then the allocation-free call continues the trajectory
    _log("noalloc: continue after sl_step")
    b.step(60)
    a.step_noalloc(60)
    _same(N, a, b)
    for s in (a, b, c, d):
        s.close()


def test_noalloc_with_staged_rows_requested(N):
    # a bcc run whose tuning asks for LDS-staged colour passes: sl_step takes
    # them, the allocation-free call (which builds no tile table) the
    # per-site gathers; the same bits, and the staged passes still run after
    spec = I.fe_bcc_spec(L=8, lattice_mode=0, seed=22, run_id=4)
    st = I.initial_state(spec, "tilt")
    _log("noalloc: 8^3 bcc FP32 with spin_access 1")
    a, b = _pair(N, spec, st, N.SL_FP32, 10, spin_access=1, merge_sweeps=0)
    n0 = a._alloc.n_allocs
    a.step_noalloc(33)
    a.synchronize()
    assert a._alloc.n_allocs == n0
    b.step(33)
    _same(N, a, b)
    a.step(20)
    b.step(20)
    _same(N, a, b)
    a.close()
    b.close()
