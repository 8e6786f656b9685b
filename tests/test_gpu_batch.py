"""Batched runs and the FP32 path on the GPU.

* a run inside a batch (any mix of sizes, lattices, targets, admission
  times) is bitwise identical to the same run alone, in FP64 and FP32;
* slots and the memory budget are enforced;
* FP32 agrees with FP64 statistically and stays close over short windows.
"""
import math
import sys
from dataclasses import replace

import numpy as np
import pytest

from oracle import oracle as O
from paper_2608_18541_amd import inputs as I
from tests.gpu_util import compare_states

pytestmark = pytest.mark.gpu

KB = 8.617333262e-5
MUB = 5.7883818060e-5


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


def _mixed_runs():
    runs = []
    for k, L in enumerate((6, 8, 10)):
        spec = I.gdfeco_sc_spec(L=L, tn=2, alpha=0.02 * (k + 1), S0=0.3, t0=0.002, fwhm=0.002,
                                seed=100 + k, run_id=k)
        runs.append((spec, I.initial_state(spec, "afm")))
    spec = I.fe_bcc_spec(L=6, seed=7, run_id=9)
    runs.append((spec, I.initial_state(spec, "tilt")))
    spec = I.fe_bcc_spec(L=4, lattice_mode=0, seed=8, run_id=10, Te0=500.0)
    runs.append((spec, I.initial_state(spec, "random")))
    # diffusing electrons: this run's step ends in its own launches, the
    # others' in the force kernel
    spec = replace(I.gdfeco_sc_spec(L=12, alpha=0.05, S0=0.6, t0=0.005, fwhm=0.005,
                                    kappa_e=I.w_per_mk_to_metal(80.0), n_sub=4, profile=1,
                                    depth=10.0, seed=12, run_id=11), tn=(3, 3, 6))
    runs.append((spec, I.initial_state(spec, "afm")))
    # a production run (frozen lattice, anisotropy, stepped T_e with both
    # stage ends inside the window): it advances in the persistent executor
    spec = replace(I.gdfeco_sc_spec(L=8, tn=2, alpha=0.05, lattice_mode=0, seed=13, run_id=12,
                                    K=(2.0e-3, 1.0e-3, 0.0, 0.0)),
                   ttm_mode=2, step_T=(1100.0, 550.0, 300.0), step_end=(0.0021, 0.0047))
    runs.append((spec, I.initial_state(spec, "afm")))
    return runs


@pytest.mark.parametrize("prec", [0, 1])
def test_batch_equals_alone_bitwise(N, prec):
    runs = _mixed_runs()
    targets = [37, 50, 64, 45, 70, 55, 66]
    _log("batch: %d runs prec=%d" % (len(runs), prec))
    b = N.Batch(precision=prec, max_runs=8)
    slots = [b.add(sp, st, t, obs_every=5) for (sp, st), t in zip(runs, targets)]
    b.advance(30)
    b.advance(40)          # every run reaches its target inside this call
    for (sp, st), t, s in zip(runs, targets, slots):
        alone = N.System(sp, st, precision=prec, obs_every=5)
        alone.step(t)
        a = alone.state()
        g = b.get(s)
        for k in ("s", "x", "v", "Te"):
            assert np.array_equal(a[k], g[k]), (s, k)
        oa = alone.observables()
        assert [o["step"] for o in g["obs"]] == [o["step"] for o in oa]
        assert all(x["E_ex"] == y["E_ex"] for x, y in zip(oa, g["obs"]))
        alone.close()
    info = b.runs()
    assert [r["steps_done"] for r in info] == targets


def test_late_admission_and_removal(N):
    """Continuous batching: a run admitted while others are mid-flight, and
    a slot reused after removal, still match their solo trajectories."""
    runs = _mixed_runs()
    b = N.Batch(precision=1, max_runs=2)
    s0 = b.add(*runs[0], 100)
    b.advance(24)
    s1 = b.add(*runs[1], 30)
    b.advance(30)
    g1 = b.get(s1)
    b.remove(s1)
    s2 = b.add(*runs[3], 20)
    with pytest.raises(N.SLError) as e:
        b.add(*runs[2], 10)
    assert e.value.code == N.SL_EBUSY
    b.advance(46)
    g0, g2 = b.get(s0), b.get(s2)
    for (sp, st), steps, g in ((runs[0], 100, g0), (runs[1], 30, g1), (runs[3], 20, g2)):
        alone = N.System(sp, st, precision=1)
        alone.step(steps)
        a = alone.state()
        for k in ("s", "x", "v", "Te"):
            assert np.array_equal(a[k], g[k]), k


def test_memory_budget(N):
    spec, st = _mixed_runs()[1]
    fp = N.footprint_bytes(spec, precision=1, obs_capacity=4096)
    b = N.Batch(precision=1, max_runs=8, mem_budget=int(2.5 * fp))
    assert b.add(spec, st, 10) is not None
    assert b.add(spec, st, 10) is not None
    assert b.try_add(spec, st, 10) is None
    used, budget = b.memory()
    assert used == 2 * fp and budget == int(2.5 * fp)


def _isolated_spins(prec, mu, T, Bz):
    """32^3 sc lattice with J = 0: 32768 independent spins."""
    spec = I.SystemSpec(lattice=0, ncell=(32, 32, 32), a=3.0, n_species=1, mu=(mu, 0, 0, 0),
                        mass=(55.845, 0, 0, 0), n_shells=1,
                        J=(((0.0,) * 4,) * 4, ((0.0,) * 4,) * 4), B=(0.0, 0.0, Bz), alpha=0.5,
                        lattice_mode=0, dt=5e-4, tn=(1, 1, 1), ttm_mode=0, Te0=T, seed=31)
    st = I.InitialState(species=np.zeros(spec.n_sites, dtype=np.int8),
                        spins=np.tile([0.0, 0.0, 1.0], (spec.n_sites, 1)), vel=None)
    return spec, st


@pytest.mark.parametrize("prec", [0, 1])
def test_langevin_function_on_gpu(N, prec):
    """Thermal equilibrium of the GPU path itself: <s_z> = coth x - 1/x for
    two moments, from 32768 independent spins (FP64 and FP32)."""
    T, Bz = 50.0, 67.0
    for mu in (2.2, 7.63):
        spec, st = _isolated_spins(prec, mu, T, Bz)
        g = N.System(spec, st, precision=prec, obs_every=50, obs_capacity=256)
        g.step(2000)
        g.observables()
        g.step(4000)
        obs = g.observables()
        mz = np.array([o["m"][2] for o in obs])
        x = mu * MUB * Bz / (KB * T)
        ref = 1.0 / math.tanh(x) - 1.0 / x
        assert abs(mz.mean() - ref) < 0.01, (prec, mu, mz.mean(), ref)


def test_fp32_short_window_close_to_oracle(N):
    """FP32 storage and spin arithmetic track the FP64 oracle closely over a
    short window (the difference is rounding, amplified by the dynamics)."""
    spec = I.fe_bcc_spec(L=6)
    st = I.initial_state(spec, "tilt")
    g = N.System(spec, st, precision=1)
    o = O.Oracle(spec, st.species, st.spins, st.vel)
    g.step(20)
    o.step(20)
    errs, bad = compare_states(g.state(), o.state(), spec.box, 2e-4)
    assert not bad, errs


def test_fp32_ensemble_matches_fp64(N):
    """Sublattice M_z(t) of a laser-heated alloy: FP32 and FP64 ensembles
    over the same 24 seeds agree within their statistical error bars; the
    FP32 - FP64 difference is reported."""
    nrun = 24
    steps, every = 1500, 100
    means = {}
    for prec in (0, 1):
        b = N.Batch(precision=prec, max_runs=nrun)
        slots = []
        for r in range(nrun):
            spec = I.gdfeco_sc_spec(L=10, tn=2, alpha=0.05, S0=0.08, t0=0.03, fwhm=0.02,
                                    seed=500, run_id=r)
            slots.append(b.add(spec, I.initial_state(spec, "afm"), steps, obs_every=every))
        b.advance(steps)
        traj = []
        for s in slots:
            obs = b.get(s)["obs"]
            traj.append([[o["M"][1][2], o["M"][0][2]] for o in obs])
        means[prec] = np.array(traj)           # [run, sample, (Gd, TM)]
    a, c = means[0], means[1]
    diff = a.mean(axis=0) - c.mean(axis=0)
    err = np.sqrt(a.var(axis=0, ddof=1) / nrun + c.var(axis=0, ddof=1) / nrun) + 1e-6
    _log("FP32-FP64 max |dM| = %.3e, max |dM|/err = %.2f" % (np.abs(diff).max(),
                                                           (np.abs(diff) / err).max()))
    assert np.all(np.abs(diff) < 4.0 * err + 2e-3)
    # the pulse did demagnetise the sublattices
    assert a[:, -1, 1].mean() < 0.97



def test_fp32_production_ensemble_matches_fp64(N):
    """The production mode (frozen lattice, anisotropy, stepped T_e) in the
    persistent executor: FP32 and FP64 ensembles of sublattice M_z(t) over
    the same 24 seeds agree within their statistical error bars."""
    nrun = 24
    steps, every = 1500, 100
    means = {}
    for prec in (0, 1):
        b = N.Batch(precision=prec, max_runs=nrun)
        slots = []
        for r in range(nrun):
            spec = replace(I.gdfeco_sc_spec(L=10, tn=2, alpha=0.05, lattice_mode=0, seed=600, run_id=r,
                                            K=(I.GDFECO_K, I.GDFECO_K, 0.0, 0.0)),
                           ttm_mode=2, step_T=(1100.0, 550.0, 300.0), step_end=(0.05, 0.1))
            slots.append(b.add(spec, I.initial_state(spec, "afm", exact_count=True), steps,
                               obs_every=every))
        b.advance(steps)
        traj = []
        for s in slots:
            obs = b.get(s)["obs"]
            traj.append([[o["M"][1][2], o["M"][0][2]] for o in obs])
        means[prec] = np.array(traj)           # [run, sample, (Gd, TM)]
    a, c = means[0], means[1]
    diff = a.mean(axis=0) - c.mean(axis=0)
    err = np.sqrt(a.var(axis=0, ddof=1) / nrun + c.var(axis=0, ddof=1) / nrun) + 1e-6
    _log("production FP32-FP64 max |dM| = %.3e, max |dM|/err = %.2f"
         % (np.abs(diff).max(), (np.abs(diff) / err).max()))
    assert np.all(np.abs(diff) < 4.0 * err + 2e-3)
    # the pulse demagnetised the TM sublattice (it starts at -1)
    assert a[:, :, 1].mean(axis=0).max() > -0.97

def test_fp32_fcc_production_ensemble_matches_fp64(N):
    """The same check on the paper's production lattice: fcc GdFeCo (5^3
    cells, 500 sites, exact-count alloy, Table 1 exchange, anisotropy,
    stepped T_e) in the persistent executor, FP32 against FP64 ensembles of
    sublattice M_z(t) over 24 seeds."""
    nrun = 24
    steps, every = 1500, 100
    means = {}
    for prec in (0, 1):
        b = N.Batch(precision=prec, max_runs=nrun)
        slots = []
        for r in range(nrun):
            spec = replace(I.gdfeco_fcc_spec(L=5, alpha=0.05, seed=610, run_id=r), tn=(2, 2, 2),
                           ttm_mode=2, step_T=(1400.0, 700.0, 300.0), step_end=(0.05, 0.1))
            slots.append(b.add(spec, I.initial_state(spec, "afm", exact_count=True), steps,
                               obs_every=every))
        b.advance(steps)
        traj = []
        for s in slots:
            obs = b.get(s)["obs"]
            traj.append([[o["M"][1][2], o["M"][0][2]] for o in obs])
        means[prec] = np.array(traj)           # [run, sample, (Gd, TM)]
    a, c = means[0], means[1]
    diff = a.mean(axis=0) - c.mean(axis=0)
    err = np.sqrt(a.var(axis=0, ddof=1) / nrun + c.var(axis=0, ddof=1) / nrun) + 1e-6
    _log("fcc production FP32-FP64 max |dM| = %.3e, max |dM|/err = %.2f"
         % (np.abs(diff).max(), (np.abs(diff) / err).max()))
    assert np.all(np.abs(diff) < 4.0 * err + 2e-3)
    # the pulse demagnetised the TM sublattice (it starts at -1)
    assert a[:, :, 1].mean(axis=0).max() > -0.97


def test_launch_shapes_are_bitwise_identical(N):
    """Every launch shape the autotuner may choose gives the same bits: a
    batch stepped under several settings (and then autotuned) equals the
    runs stepped alone with the default setting."""
    from paper_2608_18541_amd.autotune import autotune
    runs = _mixed_runs()[:4]
    for prec in (0, 1):
        b = N.Batch(precision=prec, max_runs=4)
        slots = [b.add(sp, st, 10_000) for sp, st in runs]
        shapes = [dict(spin_block=64, spin_spt=4, atom_block=128, graph_steps=8, persist_block=0,
                       xcd_order=1, bin_mode=2, atom_lanes=2),
                  dict(spin_block=128, spin_spt=2, atom_block=64, graph_steps=32,
                       persist_block=512, xcd_order=0, bin_mode=1, atom_lanes=1),
                  dict(spin_block=256, spin_spt=1, atom_block=256, graph_steps=1,
                       persist_block=0, xcd_order=1, bin_mode=2, atom_lanes=4),
                  dict(spin_block=256, spin_spt=1, atom_block=256, graph_steps=16,
                       persist_block=256, xcd_order=0, bin_mode=0, atom_lanes=1),
                  dict(spin_block=128, spin_spt=1, atom_block=128, graph_steps=8,
                       persist_block=1024, xcd_order=0, bin_mode=0, atom_lanes=2),
                  dict(spin_block=256, spin_spt=1, atom_block=256, graph_steps=4,
                       persist_block=0, xcd_order=0, bin_mode=1, atom_lanes=4)]
        for sh in shapes:
            b.set_tuning(**sh)
            b.advance(17)
        best = autotune(b, steps=8, use_cache=False)
        assert set(best) == {"spin_block", "spin_spt", "atom_block", "graph_steps",
                             "persist_block", "xcd_order", "bin_mode", "atom_lanes",
                             "merge_sweeps", "spin_access", "fuse_force"}
        info = {r["slot"]: r["steps_done"] for r in b.runs()}
        for (sp, st), s in zip(runs, slots):
            alone = N.System(sp, st, precision=prec)
            alone.step(info[s])
            a = alone.state()
            g = b.get(s)
            for k in ("s", "x", "v", "Te"):
                assert np.array_equal(a[k], g[k]), (prec, s, k)
            alone.close()
        b.close()


def test_full_phase_diagram_batch_sampled_runs(N):
    """The full 1280-run phase-diagram batch (16^3 alloys, the bench's launch
    configuration: persistent executor, FP32) for 60 steps: sampled runs
    from corners and the middle of the grid equal the same runs alone, bit
    for bit, and every run advanced exactly 60 steps."""
    from paper_2608_18541_amd import workloads as W
    runs = W.phase_diagram(L=16, n_seeds=20, n_steps=60)
    b = N.Batch(precision=1, max_runs=len(runs))
    slots = [b.add(r.spec, r.state, r.n_steps, obs_every=20, obs_capacity=8) for r in runs]
    _log("full batch: %d runs" % len(runs))
    b.advance(60)
    info = b.runs()
    assert len(info) == 1280 and all(r["steps_done"] == 60 for r in info)
    for k in (0, 639, 1279):
        g = b.get(slots[k])
        alone = N.System(runs[k].spec, runs[k].state, precision=1, obs_every=20, obs_capacity=8)
        alone.step(60)
        a = alone.state()
        for key in ("s", "x", "v", "Te"):
            assert np.array_equal(a[key], g[key]), (k, key)
        oa = alone.observables()
        assert [o["E_ex"] for o in oa] == [o["E_ex"] for o in g["obs"]]
        alone.close()
    b.close()


def test_large_bcc_fp32_invariants(N):
    """bcc Fe 64^3 (524288 atoms) with surface heating, FP32 as the bench
    runs it, through at least one list rebuild: unit spins, finite state,
    counters, and FP32 tracking FP64 over the first 20 steps."""
    spec = I.fe_large_spec()
    st = I.initial_state(spec, "tilt")
    g32 = N.System(spec, st, precision=1, obs_every=10, obs_capacity=64)
    g64 = N.System(spec, st, precision=0, obs_every=10, obs_capacity=64)
    g32.step(20)
    g64.step(20)
    a, c = g32.state(), g64.state()
    assert np.abs(np.linalg.norm(a["s"], axis=1) - 1.0).max() < 1e-6
    # FP32 vs FP64 is a statistical comparison: the typical site differs by
    # float rounding (about 1e-7 after 20 steps); a few sites amplify it
    ds = np.abs(a["s"] - c["s"])
    assert np.sqrt((ds ** 2).mean()) < 1e-5 and ds.max() < 1e-2
    vr = np.sqrt((c["v"] ** 2).mean())
    dv = np.abs(a["v"] - c["v"])
    assert np.sqrt((dv ** 2).mean()) < 1e-5 * vr and dv.max() < 1e-2 * vr
    g32.step(480)
    s = g32.stats()
    assert s["steps"] == 500 and s["list_rebuilds"] >= 1
    assert 0 < s["max_list"] <= s["list_capacity"]
    fin = g32.state()
    assert np.all(np.isfinite(fin["x"])) and np.all(np.isfinite(fin["v"]))
    assert np.abs(np.linalg.norm(fin["s"], axis=1) - 1.0).max() < 1e-6
    g32.close()
    g64.close()
