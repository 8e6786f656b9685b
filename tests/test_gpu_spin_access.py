"""The LDS-staged colour pass of bcc runs with one species and constant
exchange (tuning spin_access 1): a block stages the neighbour rows of a tile
of 2 x 2 (or 4 x 4) rows in LDS and runs the same site arithmetic as the
pass that gathers per site (spin_access 0).

* Bit for bit against that pass, FP32 and FP64, frozen and live lattices,
  one and two exchange shells, with merged sweeps on (its passes 2.. take
  the chosen access) and off; for the staged rows on every tile shape: 4 x 4
  rows in 256-thread blocks (rows shorter than 64 sites), 4 x 4 rows in
  1024-thread blocks and 2 x 2 rows (longer rows, by what fits in LDS).
* FP64 against the oracle at 1e-10 per component (reading R23), with the
  staged rows, across the list rebuilds of a hot live lattice.
* A batch of runs of two sizes against the runs alone.
"""
import sys
from dataclasses import replace

import numpy as np
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


def _run(N, spec, st, prec, mode, steps, merge=1):
    g = N.System(spec, st, precision=prec, obs_every=10)
    g.set_tuning(spin_access=mode, merge_sweeps=merge)
    for k in (3, steps - 3):
        g.step(k)
    out = g.state()
    obs = g.observables()
    g.close()
    return out, obs


@pytest.mark.parametrize("mode", [1])
@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("case", ["frozen_two_shells", "live_two_shells", "frozen_one_shell",
                                  "live_unmerged"])
def test_access_mode_bitwise(N, mode, prec, case):
    # 8^3 cells: 4 sites per colour row, whole 16-byte vectors in FP32 and
    # FP64, 4 x 4 tiles
    spec = I.fe_bcc_spec(L=8, seed=71, run_id=1)
    if case.startswith("frozen"):
        spec = replace(spec, lattice_mode=0)
    if case.endswith("one_shell"):
        spec = replace(spec, n_shells=1)
    merge = 0 if case == "live_unmerged" else 1
    st = I.initial_state(spec, "tilt", T_lattice=600.0)
    _log("access mode %d bitwise: %s prec %d" % (mode, case, prec))
    a, oa = _run(N, spec, st, prec, mode, 60, merge)
    b, ob = _run(N, spec, st, prec, 0, 60, merge)
    for k in ("s", "x", "v", "Te"):
        assert np.array_equal(a[k], b[k]), (case, k)
    assert len(oa) == len(ob)
    for p, q in zip(oa, ob):
        assert np.array_equal(p["M"], q["M"]) and p["E_ex"] == q["E_ex"]


@pytest.mark.parametrize("prec,ncell", [(1, (128, 128, 128)), (1, (256, 8, 4)), (0, (256, 8, 4)),
                                        (1, (32, 8, 8))])
def test_access_mode_bitwise_long_rows(N, prec, ncell):
    # frozen lattices with long colour rows: 4 x 4 tiles in 1024-thread
    # blocks (FP32 128^3 with 64 sites per row, FP32 rows of 128 sites), 2 x 2
    # tiles where those do not fit in LDS (FP64 rows of 128 sites), and 4 x 4
    # tiles in 256-thread blocks for rows of 16 sites; one launch per pass
    spec = replace(I.fe_bcc_spec(L=8, lattice_mode=0, seed=72, run_id=0), ncell=ncell)
    st = I.initial_state(spec, "tilt")
    _log("staged rows bitwise: %s prec %d" % (str(ncell), prec))
    b, _ = _run(N, spec, st, prec, 0, 12, merge=0)
    a, _ = _run(N, spec, st, prec, 1, 12, merge=0)
    assert np.array_equal(a["s"], b["s"])


@pytest.mark.parametrize("mode", [1])
def test_access_mode_against_oracle(N, mode):
    # a hot live lattice with a thin skin (several list rebuilds), FP64
    spec = replace(I.fe_bcc_spec(L=8, seed=73, run_id=2), skin=0.05)
    st = I.initial_state(spec, "tilt", T_lattice=900.0)
    _log("access mode %d against the oracle: bcc 8^3 FP64" % mode)
    g = N.System(spec, st, precision=N.SL_FP64, obs_every=10)
    g.set_tuning(spin_access=mode)
    o = O.Oracle(spec, st.species, st.spins, st.vel)
    for chunk in (7, 53, 60):
        g.step(chunk)
        o.step(chunk)
        errs, bad = compare_states(g.state(), o.state(), spec.box, 1e-10)
        assert not bad, (chunk, errs)
    assert g.stats()["list_rebuilds"] >= 3, g.stats()
    g.close()


@pytest.mark.parametrize("mode", [1])
@pytest.mark.parametrize("prec", [0, 1])
def test_access_mode_batch_equals_alone(N, mode, prec):
    # a batch of bcc runs of two sizes (8^3 and 16^3 cells, 4 x 4 tiles of
    # both in one launch) on the multi-kernel step with the staged pass: each
    # run keeps the bits it has alone with the gathering pass
    runs = []
    for k, L in enumerate((8, 16, 8)):
        spec = replace(I.fe_bcc_spec(L=L, seed=80 + k, run_id=k), lattice_mode=0 if k == 1 else 1)
        runs.append((spec, I.initial_state(spec, "tilt", T_lattice=500.0)))
    _log("access mode %d batch: prec %d" % (mode, prec))
    b = N.Batch(precision=prec, max_runs=3)
    b.set_tuning(persist_block=0, spin_access=mode)
    slots = [b.add(sp, st, 40, obs_every=10) for sp, st in runs]
    b.advance(40)
    for (sp, st), s in zip(runs, slots):
        g = b.get(s)
        a, _ = _run(N, sp, st, prec, 0, 40)
        for key in ("s", "x", "v"):
            assert np.array_equal(a[key], g[key]), (sp.ncell, key)
    b.close()
