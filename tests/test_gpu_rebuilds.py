"""Parity with the oracle across Verlet-list rebuilds during stepping.

The list holds every atom within rc + skin and is rebuilt when an atom has
moved more than half the skin since the last build; the oracle finds the
pairs within rc afresh at every step.  With a 0.05 A skin and 600 K
velocities the GPU rebuilds its lists every few tens of steps, so each
comparison below follows at least three builds after the initial one:
binning by the kick (unsorted bins) and binning only for a rebuild (sorted
bins) on the multi-kernel step, and the persistent per-run kernel of a
batch.  FP64 against the oracle at 1e-10 per component (reading R23).
"""
import sys
from dataclasses import replace

import pytest

from oracle import oracle as O
from paper_2608_18541_amd import inputs as I
from tests.gpu_util import compare_states

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


def _case():
    spec = replace(I.fe_bcc_spec(L=6, seed=31, run_id=2, alpha=0.05), skin=0.05)
    return spec, I.initial_state(spec, "tilt", T_lattice=600.0)


@pytest.fixture(scope="module")
def oracle_states():
    spec, st = _case()
    o = O.Oracle(spec, st.species, st.spins, st.vel)
    out = {}
    for n in (90, 180):
        o.step(n - o.step_count)
        out[n] = o.state()
    return out


@pytest.mark.parametrize("bin_mode", [1, 2])
def test_multi_kernel_parity_across_rebuilds(N, oracle_states, bin_mode):
    spec, st = _case()
    _log("rebuilds: bcc 6^3 skin 0.05 600 K bin_mode=%d" % bin_mode)
    g = N.System(spec, st, precision=N.SL_FP64)
    g.set_tuning(bin_mode=bin_mode)
    for n in (90, 180):
        g.step(n - g.info()[2])
        stats = g.stats()
        errs, bad = compare_states(g.state(), oracle_states[n], spec.box, 1e-10)
        assert not bad, (n, errs)
    assert stats["list_rebuilds"] >= 4, stats        # the initial build and three more
    g.close()


def test_persistent_kernel_parity_across_rebuilds(N, oracle_states):
    spec, st = _case()
    _log("rebuilds: bcc 6^3 skin 0.05 600 K, persistent batch run")
    b = N.Batch(precision=N.SL_FP64, max_runs=2)
    b.set_tuning(persist_block=512)
    slot = b.add(spec, st, 180)
    b.advance(90)
    errs, bad = compare_states(b.get(slot), oracle_states[90], spec.box, 1e-10)
    assert not bad, errs
    b.advance(90)
    stats = b.stats(slot)
    errs, bad = compare_states(b.get(slot), oracle_states[180], spec.box, 1e-10)
    assert not bad, errs
    assert stats["list_rebuilds"] >= 4 and stats["steps"] == 180, stats
    b.close()
