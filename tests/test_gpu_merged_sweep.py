"""Merged colour sweeps: a step that leaves its last colour-0 half step to the
next step's colour pass 0 (two rotations in one pass, same neighbours) must
give the bits of the unmerged schedule.

A run sampled every step cannot merge (no chunk length in 2..64 divides 1),
so it is the unmerged reference; the same run sampled every 10 steps merges
in chunks of 10.  Advances of uneven length start and stop inside chunks,
and a batch run reaches its target inside a chunk.
"""
import sys
from dataclasses import replace

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


def _cases():
    # bcc Fe, fixed 300 K electrons (the deferred half step reads T_e itself)
    yield "bcc_fixed_Te", I.fe_bcc_spec(L=6), "tilt"
    # laser-heated sc alloy, live lattice, electron grid updated every step
    # (the deferred half step reads the previous step's T_e)
    yield "alloy_laser_live", I.gdfeco_sc_spec(L=12, tn=3, alpha=0.05, S0=0.6, t0=0.005,
                                               fwhm=0.005), "afm"
    # uniaxial anisotropy: the field depends on the site's own spin, so the
    # merged pass's second rotation takes it from the first one's result
    yield "alloy_anisotropy", replace(
        I.gdfeco_sc_spec(L=12, tn=3, alpha=0.05, S0=0.6, t0=0.005, fwhm=0.005),
        K=(2.0e-3, 1.0e-3, 0.0, 0.0)), "afm"
    # the stepped T_e profile on a frozen lattice (the production runs):
    # the deferred half step reads the stage of its own step
    yield "alloy_stepped_profile", replace(
        I.gdfeco_sc_spec(L=12, tn=3, alpha=0.05, lattice_mode=0, K=(2.0e-3, 1.0e-3, 0.0, 0.0)),
        ttm_mode=2, step_T=(1100.0, 550.0, 300.0), step_end=(0.0042, 0.0097)), "afm"
    # diffusing electrons heated in a top slab: four diffusion sub-steps per
    # step in one tiled launch, the previous step's T_e kept by the grid update
    yield "alloy_diffusing", replace(
        I.gdfeco_sc_spec(L=12, tn=3, alpha=0.05, S0=0.6, t0=0.005, fwhm=0.005,
                         kappa_e=I.w_per_mk_to_metal(80.0), n_sub=4, profile=1, depth=10.0),
        tn=(3, 3, 6)), "afm"
    # the fcc production model (coloured by basis site, odd cell counts)
    yield "fcc_production", replace(
        I.gdfeco_fcc_spec(L=5, alpha=0.05, K=(2.0e-3, 1.0e-3, 0.0, 0.0)),
        ttm_mode=2, step_T=(1100.0, 550.0, 300.0), step_end=(0.0042, 0.0097)), "afm"


def _samples(sysobj, every):
    return {o["step"]: o for o in sysobj.observables() if (o["step"] % every) == 0}


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("case", ["bcc_fixed_Te", "alloy_laser_live", "alloy_anisotropy",
                                  "alloy_stepped_profile", "alloy_diffusing", "fcc_production"])
def test_merged_sweep_equals_unmerged(N, case, prec):
    name, spec, init = next(c for c in _cases() if c[0] == case)
    st = I.initial_state(spec, init)
    _log("case: %s prec=%d" % (name, prec))
    ref = N.System(spec, st, precision=prec, obs_every=1)
    mrg = N.System(spec, st, precision=prec, obs_every=10)
    for chunk in (7, 23, 15, 40, 1, 34):
        ref.step(chunk)
        mrg.step(chunk)
        a, b = ref.state(), mrg.state()
        for k in ("s", "x", "v", "Te"):
            assert np.array_equal(a[k], b[k]), (name, chunk, k)
    # samples at steps 10, 20, ...: the merged run's samples see complete sweeps
    sa, sb = _samples(ref, 10), _samples(mrg, 10)
    assert sorted(sb) == list(range(0, 121, 10))
    for stp, o in sb.items():
        r = sa[stp]
        for k in ("E_ex", "E_z", "KE", "PE", "m_abs", "Te_mean"):
            assert r[k] == o[k], (name, stp, k)
        assert np.array_equal(np.array(r["M"]), np.array(o["M"])), (name, stp)
    ref.close()
    mrg.close()


def test_run_ending_inside_a_chunk(N):
    """A batch's only multi-kernel run reaches its target at step 37 while the
    engine steps chunks of 10: the half step deferred by step 36 is applied
    by the next pass 0 although the run no longer steps."""
    spec = I.gdfeco_sc_spec(L=12, tn=3, alpha=0.05, S0=0.6, t0=0.005, fwhm=0.005, seed=3, run_id=2)
    st = I.initial_state(spec, "afm")
    b = N.Batch(precision=0, max_runs=1)
    slot = b.add(spec, st, 37, obs_every=10)
    b.advance(60)
    g = b.get(slot)
    ref = N.System(spec, st, precision=0, obs_every=1)
    ref.step(37)
    a = ref.state()
    for k in ("s", "x", "v", "Te"):
        assert np.array_equal(a[k], g[k]), k
    assert [o["step"] for o in g["obs"]] == [0, 10, 20, 30]
    b.close()
    ref.close()


def test_merge_knob_same_bits(N):
    """merge_sweeps 0 (one launch per colour pass) and 1 at the same sample
    interval: identical trajectories and samples; other values rejected."""
    spec = I.gdfeco_sc_spec(L=12, tn=3, alpha=0.05, S0=0.6, t0=0.005, fwhm=0.005, seed=5, run_id=4)
    st = I.initial_state(spec, "afm")
    out = []
    for m in (0, 1):
        g = N.System(spec, st, precision=1, obs_every=20)
        g.set_tuning(merge_sweeps=m)
        g.step(13)
        g.step(90)
        out.append((g.state(), g.observables()))
        if m == 1:
            before = g.tuning()
            with pytest.raises(N.SLError) as e:
                g.set_tuning(merge_sweeps=2)
            assert e.value.code == N.SL_EINVAL and g.tuning() == before
        g.close()
    for k in ("s", "x", "v", "Te"):
        assert np.array_equal(out[0][0][k], out[1][0][k]), k
    assert [o["step"] for o in out[0][1]] == [o["step"] for o in out[1][1]]
    for a, b in zip(out[0][1], out[1][1]):
        assert a["E_ex"] == b["E_ex"] and a["m_abs"] == b["m_abs"] and a["Te_mean"] == b["Te_mean"]


def test_negative_electron_energy_inside_a_chunk(N):
    """Electrons at 600 K with a hundredth of the alloy's heat capacity over
    a lattice at 0 K give their energy away within about twenty steps (the
    oracle meets a negative energy density after 18), until one step's
    transfer exceeds what is left: the run stops with a negative electron
    energy.  Stepped one by one (samples every step) it stops at the step
    whose end met it.  In chunks of ten, where a step's end runs with the
    next step's first colour pass, an end inside the chunk stops the run
    one step later; the chunk's own last end stops it at once."""
    spec = I.gdfeco_sc_spec(L=6, tn=2, gamma_e=I.j_per_m3k2_to_metal(2.25), Te0=600.0, seed=9,
                           run_id=1)
    st = I.initial_state(spec, "afm", T_lattice=0.0)
    steps = []
    for every in (1, 10):
        _log("case: negative energy, obs_every=%d" % every)
        g = N.System(spec, st, precision=0, obs_every=every)
        with pytest.raises(N.SLError) as e:
            g.step(200)
            g.synchronize()
        assert e.value.code == N.SL_ENUMERIC and "negative electron energy" in str(e.value)
        steps.append(g.stats()["steps"])
        g.close()
    u, f = steps
    assert 10 < u < 40, steps
    assert f == u + (1 if u % 10 else 0), steps


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("fuse", [0, 1])
def test_batch_runs_merge_together(N, prec, fuse):
    """Three sc alloys added together to a batch on the multi-kernel step
    (same colour count, sample interval 10) advance in merged chunks: one
    colour pass without the kick per step instead of two, except at a
    chunk's last step (with the force kernel beside colour pass 1: no
    colour pass alone but a chunk's last step's two).  Each run keeps the
    bits it has alone stepped one by one; two of them reach their targets
    inside a chunk."""
    specs = [I.gdfeco_sc_spec(L=L, tn=2, alpha=0.02 * (k + 1), S0=0.6, t0=0.005, fwhm=0.005,
                              seed=20 + k, run_id=k) for k, L in enumerate((8, 10, 12))]
    states = [I.initial_state(sp, "afm") for sp in specs]
    targets = [37, 50, 44]
    _log("case: batch of 3 sc alloys, prec=%d" % prec)
    b = N.Batch(precision=prec, max_runs=4)
    b.set_tuning(persist_block=0, fuse_force=fuse)
    slots = [b.add(sp, st, t, obs_every=10) for sp, st, t in zip(specs, states, targets)]
    b.advance(23)
    # a shorter merged chunk of 7 steps up to step 30, then two chunks of 10:
    # unfused, one colour pass without the kick per step, plus the last
    # step's closing pass in each chunk; fused, every colour pass 0 carries
    # the kick and every colour pass 1 but a chunk's last the force kernel
    avg, cnt = b.advance_profiled(27)
    if fuse:
        assert cnt[0] == 2 * 3 and cnt[2] == 27 and cnt[5] == 27 - 3 and cnt[1] == 3, cnt
    else:
        assert cnt[0] == (7 + 1) + 2 * 11 and cnt[5] == 0, cnt
    for sp, st, t, s in zip(specs, states, targets, slots):
        g = b.get(s)
        ref = N.System(sp, st, precision=prec, obs_every=1)
        ref.step(t)
        a = ref.state()
        for k in ("s", "x", "v", "Te"):
            assert np.array_equal(a[k], g[k]), (t, k)
        want = [o for o in ref.observables() if o["step"] % 10 == 0]
        assert [o["step"] for o in g["obs"]] == [o["step"] for o in want]
        for o, r in zip(g["obs"], want):
            assert o["E_ex"] == r["E_ex"] and o["m_abs"] == r["m_abs"] and o["Te_mean"] == r["Te_mean"]
        ref.close()
    b.close()


def test_batch_run_added_out_of_phase_steps_unmerged(N):
    """A run added to a merging batch at a step that is not a chunk boundary
    of the others: the batch steps unmerged (two colour passes without the
    kick per step) and every run keeps its bits alone."""
    specs = [I.gdfeco_sc_spec(L=8, tn=2, alpha=0.03, S0=0.6, t0=0.005, fwhm=0.005,
                              seed=40 + k, run_id=k) for k in range(3)]
    states = [I.initial_state(sp, "afm") for sp in specs]
    _log("case: batch, third run added after 25 steps")
    b = N.Batch(precision=0, max_runs=4)
    b.set_tuning(persist_block=0)
    slots = [b.add(specs[k], states[k], 60, obs_every=10) for k in range(2)]
    b.advance(25)
    slots.append(b.add(specs[2], states[2], 40, obs_every=10))
    avg, cnt = b.advance_profiled(20)      # phases 5 and 0 modulo 10: no chunk fits
    assert cnt[0] == 2 * 20, cnt
    b.advance(20)
    for sp, st, t, s in zip(specs, states, (60, 60, 40), slots):
        g = b.get(s)
        ref = N.System(sp, st, precision=0, obs_every=1)
        ref.step(t)
        a = ref.state()
        for k in ("s", "x", "v", "Te"):
            assert np.array_equal(a[k], g[k]), (t, k)
        ref.close()
    b.close()
