"""The fused schedule (tuning fuse_force): in the folded chunks of a single
run with a live lattice, each step kicks the atoms in colour pass 0 and runs
the force kernel in the launch of colour pass 1; the chunk's last step (a
sample step) keeps its force kernel after the sweep.  The schedule changes
which launch carries the work, not the work: it must give the bits of the
unfused schedule in every launch shape, across list rebuilds, with binning
by separate launches, and in both precisions.  Against the oracle the
default (fused) schedule is held by the rebuild and full-size windows.
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


def _case(name):
    if name == "alloy_laser":
        # laser-heated sc alloy, 3^3 electron grid updated every step
        spec = I.gdfeco_sc_spec(L=12, tn=3, alpha=0.05, S0=0.6, t0=0.005, fwhm=0.005, seed=8, run_id=3)
        return spec, I.initial_state(spec, "afm"), 10
    # bcc Fe with a 0.05 A skin at 600 K: a list rebuild every few tens of steps
    spec = replace(I.fe_bcc_spec(L=6, seed=31, run_id=2, alpha=0.05), skin=0.05)
    return spec, I.initial_state(spec, "tilt", T_lattice=600.0), 20


SHAPES = [
    {},                                            # automatic: 64-thread colour passes, 4 lanes per atom
    {"atom_lanes": 1},
    {"atom_lanes": 2},
    {"spin_block": 128},
    {"spin_block": 256},
    {"spin_block": 64, "atom_block": 128, "atom_lanes": 2},
    {"bin_mode": 2},                               # binning launches between the kick and the forces
    {"spin_spt": 2},                               # two sites per thread in the colour passes
    {"spin_spt": 2, "spin_block": 128},
]


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("case", ["alloy_laser", "bcc_rebuilds"])
@pytest.mark.parametrize("shape", range(len(SHAPES)))
def test_fused_equals_unfused(N, case, prec, shape):
    spec, st, every = _case(case)
    tun = SHAPES[shape]
    _log("case: %s prec=%d shape=%s" % (case, prec, tun))
    ref = N.System(spec, st, precision=prec, obs_every=every)
    ref.set_tuning(fuse_force=0, **tun)
    fz = N.System(spec, st, precision=prec, obs_every=every)
    fz.set_tuning(fuse_force=1, **tun)
    for chunk in (7, 23, 15, 40, 1, 34):
        ref.step(chunk)
        fz.step(chunk)
        a, b = ref.state(), fz.state()
        for k in ("s", "x", "v", "Te"):
            assert np.array_equal(a[k], b[k]), (case, chunk, k)
    # the same schedules with every launch timed: only the fused one has
    # colour passes carrying the force kernel (class 5)
    _, cr = ref.step_profiled(2 * every)
    _, cf = fz.step_profiled(2 * every)
    assert cr[5] == 0 and cf[5] == 2 * (every - 1), (cr, cf)
    assert cf[1] == 2 and cr[1] == 2 * every, (cr, cf)
    a, b = ref.state(), fz.state()
    for k in ("s", "x", "v", "Te"):
        assert np.array_equal(a[k], b[k]), (case, "profiled", k)
    oa, ob = ref.observables(), fz.observables()
    assert [o["step"] for o in oa] == [o["step"] for o in ob]
    for x, y in zip(oa, ob):
        for k in ("E_ex", "E_z", "KE", "PE", "m_abs", "Te_mean"):
            assert x[k] == y[k], (case, x["step"], k)
    sr, sf = ref.stats(), fz.stats()
    assert sr["list_rebuilds"] == sf["list_rebuilds"]
    if case == "bcc_rebuilds":
        assert sf["list_rebuilds"] >= 4, sf
    ref.close()
    fz.close()


def test_fused_rebuild_window_against_oracle(N):
    """The fused schedule (the default, checked in the tuning) in chunks of
    20 steps against the oracle over 150 steps that cross at least three
    list rebuilds, FP64 at 1e-10 per component."""
    spec, st, every = _case("bcc_rebuilds")
    _log("fused: bcc 6^3 skin 0.05 600 K against the oracle")
    g = N.System(spec, st, precision=N.SL_FP64, obs_every=every)
    assert g.tuning()["fuse_force"] == 1
    g.step(150)
    stats = g.stats()
    o = O.Oracle(spec, st.species, st.spins, st.vel)
    o.step(150)
    errs, bad = compare_states(g.state(), o.state(), spec.box, 1e-10)
    assert not bad, errs
    assert stats["list_rebuilds"] >= 4, stats
    g.close()


def test_fuse_knob_rejects_other_values(N):
    spec, st, every = _case("alloy_laser")
    g = N.System(spec, st, precision=0, obs_every=every)
    with pytest.raises(N.SLError) as e:
        g.set_tuning(fuse_force=2)
    assert e.value.code == N.SL_EINVAL
    assert g.tuning()["fuse_force"] == 1
    g.close()


@pytest.mark.parametrize("prec", [0, 1])
def test_fused_batch_run_ends_inside_a_chunk(N, prec):
    """A batch's only run (multi-kernel, so it folds and fuses) reaches its
    target at step 37 inside a chunk of 10: the steps after it in the chunk
    skip their kick and force work, the chunk's end moves the counter to 37,
    and the run has the bits of the unfused system stepped 37 times."""
    spec, st, every = _case("alloy_laser")
    _log("fused: batch run ending at step 37, prec=%d" % prec)
    b = N.Batch(precision=prec, max_runs=1)
    b.set_tuning(persist_block=0)
    slot = b.add(spec, st, 37, obs_every=every)
    b.advance(60)
    g = b.get(slot)
    assert b.stats(slot)["steps"] == 37
    ref = N.System(spec, st, precision=prec, obs_every=every)
    ref.set_tuning(fuse_force=0)
    ref.step(37)
    a = ref.state()
    for k in ("s", "x", "v", "Te"):
        assert np.array_equal(a[k], g[k]), k
    assert [o["step"] for o in g["obs"]] == [0, 10, 20, 30]
    b.close()
    ref.close()


def test_fused_set_state_mid_run(N):
    """A checkpoint restored into a running system (lists, cells and forces
    recomputed) continues with the same bits under both schedules."""
    spec, st, every = _case("bcc_rebuilds")
    _log("fused: set_state after 25 steps")
    out = []
    for fz in (0, 1):
        g = N.System(spec, st, precision=N.SL_FP64, obs_every=every)
        g.set_tuning(fuse_force=fz)
        g.step(25)
        a = g.state()
        g.set_state(x=a["x"], v=a["v"], s=a["s"])
        g.step(55)
        out.append(g.state())
        g.close()
    for k in ("s", "x", "v"):
        assert np.array_equal(out[0][k], out[1][k]), k


def _poke_nan(alloc, block, fp32):
    import torch
    t = alloc._live[block]
    off = block - t.data_ptr()
    b = np.array([np.nan], dtype=np.float32 if fp32 else np.float64).view(np.uint8).copy()
    t[off:off + b.size] = torch.from_numpy(b).to(t.device)
    torch.cuda.synchronize()


def test_fused_watchdog_stops_the_run(N):
    """A NaN written into the spins of a batch's only run between advances
    (the fused schedule): the run stops with SL_ENUMERIC and its watchdog
    bit before its target, and the advance after it returns."""
    spec, st, every = _case("alloy_laser")
    _log("fused: watchdog on a single folded run")
    b = N.Batch(precision=0, max_runs=1)
    b.set_tuning(persist_block=0)
    h0 = len(b._alloc.history)
    slot = b.add(spec, st, 120, obs_every=every)
    block = b._alloc.history[h0][0]
    b.advance(40)
    b.synchronize()
    _poke_nan(b._alloc, block, False)
    b.advance(80)
    with pytest.raises(N.SLError) as e:
        b.synchronize()
    assert e.value.code == N.SL_ENUMERIC
    s = b.stats(slot)
    assert s["error"] & 16 and s["steps"] < 120, s
    b.close()


@pytest.mark.parametrize("prec", [0, 1])
def test_fused_batch_of_runs_merging_together(N, prec):
    """Three live runs on the multi-kernel step merging together (unfolded:
    each step ends in k_finalize, which clears the bins and flags): the fused
    schedule gives the bits of the unfused one and of each run alone."""
    specs = [replace(I.gdfeco_sc_spec(L=10, tn=2, alpha=0.03, S0=0.6, t0=0.005, fwhm=0.005,
                                      seed=60 + k, run_id=k), skin=0.1) for k in range(3)]
    states = [I.initial_state(sp, "afm", T_lattice=600.0) for sp in specs]
    _log("fused: batch of three merging runs, prec=%d" % prec)
    got = []
    for fz in (0, 1):
        b = N.Batch(precision=prec, max_runs=3)
        b.set_tuning(persist_block=0, fuse_force=fz)
        slots = [b.add(sp, st, 90, obs_every=10) for sp, st in zip(specs, states)]
        b.advance(23)
        _, cnt = b.advance_profiled(27)
        assert (cnt[5] > 0) == (fz == 1), cnt
        b.advance(60)
        got.append([b.get(s) for s in slots])
        b.close()
    for k, sp in enumerate(specs):
        for key in ("s", "x", "v", "Te"):
            assert np.array_equal(got[0][k][key], got[1][k][key]), (k, key)
        alone = N.System(sp, states[k], precision=prec, obs_every=10)
        alone.step(90)
        a = alone.state()
        for key in ("s", "x", "v", "Te"):
            assert np.array_equal(a[key], got[1][k][key]), (k, key)
        assert [o["step"] for o in got[1][k]["obs"]] == list(range(0, 91, 10))
        alone.close()


def test_fused_unfolded_single_run_with_diffusion(N):
    """A single run whose diffusing electron grid keeps its own launches (no
    folding) still merges and fuses: same bits as unfused, against the
    oracle within 1e-10 after 40 steps."""
    spec = replace(I.gdfeco_sc_spec(L=8, tn=2, alpha=0.05, S0=0.6, t0=0.005, fwhm=0.005,
                                    kappa_e=I.w_per_mk_to_metal(80.0), n_sub=2, seed=71, run_id=1),
                   tn=(2, 2, 4))
    st = I.initial_state(spec, "afm")
    _log("fused: unfolded single run with diffusion")
    out = []
    for fz in (0, 1):
        g = N.System(spec, st, precision=N.SL_FP64, obs_every=10)
        g.set_tuning(fuse_force=fz)
        g.step(13)
        _, cnt = g.step_profiled(17)
        assert (cnt[5] > 0) == (fz == 1), cnt
        g.step(10)
        out.append(g.state())
        g.close()
    for key in ("s", "x", "v", "Te"):
        assert np.array_equal(out[0][key], out[1][key]), key
    o = O.Oracle(spec, st.species, st.spins, st.vel)
    o.step(40)
    errs, bad = compare_states(out[1], o.state(), spec.box, 1e-10)
    assert not bad, errs
