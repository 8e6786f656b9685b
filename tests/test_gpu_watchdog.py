"""The numeric watchdog on the GPU.

A NaN is written into one run's spin array between two advances of a batch
of three runs (a host write into the device memory the library took from
the caller's allocator; the spin x components are the first array of a
run's allocation).  That run stops with SL_ENUMERIC and its watchdog bit;
the other two complete their steps and stay bitwise equal to the same runs
alone.  Once on the multi-kernel step (FP64) and once in the persistent
per-run kernel (FP32).
"""
import sys

import numpy as np
import pytest

from paper_2608_18541_amd import inputs as I

pytestmark = pytest.mark.gpu

ERR_NUMERIC = 16


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


def _poke_nan(alloc, block, fp32):
    """Writes a NaN into the first element of the spin-x array of the run
    whose allocation starts at `block` (a host-to-device copy on the
    library's stream, torch's current one)."""
    import torch
    t = alloc._live[block]
    off = block - t.data_ptr()
    b = np.array([np.nan], dtype=np.float32 if fp32 else np.float64).view(np.uint8).copy()
    t[off:off + b.size] = torch.from_numpy(b).to(t.device)
    torch.cuda.synchronize()


@pytest.mark.parametrize("prec,persist", [(0, 0), (1, 1024)])
def test_nan_spin_freezes_only_its_run(N, prec, persist):
    runs = []
    for k in range(3):
        spec = I.gdfeco_sc_spec(L=8, tn=2, alpha=0.02, S0=0.3, t0=0.004, fwhm=0.003,
                                seed=300 + k, run_id=k)
        runs.append((spec, I.initial_state(spec, "afm")))
    _log("watchdog: prec=%d persist_block=%d" % (prec, persist))
    b = N.Batch(precision=prec, max_runs=3)
    b.set_tuning(persist_block=persist)
    slots, blocks = [], []
    for sp, st in runs:
        h0 = len(b._alloc.history)
        slots.append(b.add(sp, st, 120, obs_every=10))
        blocks.append(b._alloc.history[h0][0])     # the run's main allocation
    b.advance(40)
    b.synchronize()
    _poke_nan(b._alloc, blocks[1], prec == 1)
    b.advance(80)
    with pytest.raises(N.SLError) as e:
        b.synchronize()
    assert e.value.code == N.SL_ENUMERIC and "non-finite" in str(e.value), str(e.value)
    bad = b.stats(slots[1])
    assert bad["error"] & ERR_NUMERIC and bad["steps"] < 120, bad
    with pytest.raises(N.SLError) as e2:
        b.get(slots[1])
    assert e2.value.code == N.SL_ENUMERIC
    for k in (0, 2):
        g = b.get(slots[k])
        st = b.stats(slots[k])
        assert st["error"] == 0 and st["steps"] == 120, st
        sp, st0 = runs[k]
        alone = N.System(sp, st0, precision=prec, obs_every=10)
        alone.step(120)
        a = alone.state()
        for key in ("s", "x", "v", "Te"):
            assert np.array_equal(a[key], g[key]), (k, key)
        ao = alone.observables()
        assert len(ao) == len(g["obs"]) == 13
        for p, q in zip(ao, g["obs"]):
            assert np.array_equal(p["M"], q["M"]) and p["E_ex"] == q["E_ex"]
        alone.close()
    b.close()
