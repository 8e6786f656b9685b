"""The force kernel's lane split and the Verlet-list builds.

An atom's pair sums are four interleaved partial sums over its list, folded
in a fixed tree, and the list holds the 27 bins in a fixed order with each
bin's atoms in ascending index.  So one, two or four lanes per atom, bins
filled by the kick (unsorted) or sorted by a separate launch, and the
persistent executor must all give the same bits; with a skin this thin the
lists are rebuilt every few steps.  A wide skin overfills the per-bin
buffer of the unsorted build, whose second scan of a bin is counted and
checked against the oracle.
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


def _obs_array(obs):
    keys = ("E_ex", "E_z", "KE", "PE", "m_abs", "Tl", "Te_mean")
    return np.array([[o[k] for k in keys] + list(np.ravel(o["M"])) for o in obs])


SHAPES = [dict(atom_lanes=1, atom_block=256, bin_mode=2),
          dict(atom_lanes=1, atom_block=64, bin_mode=1),
          dict(atom_lanes=2, atom_block=128, bin_mode=1),
          dict(atom_lanes=2, atom_block=256, bin_mode=2),
          dict(atom_lanes=4, atom_block=256, bin_mode=1),
          dict(atom_lanes=4, atom_block=256, bin_mode=2),
          dict(atom_lanes=1, atom_block=256, bin_mode=0, persist_block=512),
          dict(atom_lanes=0, atom_block=128, spin_block=0, bin_mode=1)]


@pytest.mark.parametrize("prec", [0, 1])
def test_lane_split_and_list_builds_bitwise(N, prec):
    spec = replace(I.gdfeco_sc_spec(L=16, tn=4, S0=0.3, t0=0.002, fwhm=0.002, seed=11, run_id=3),
                   skin=0.05)
    st = I.initial_state(spec, "afm")
    ref = None
    for sh in SHAPES:
        _log("case: prec=%d shape=%s" % (prec, sh))
        g = N.System(spec, st, precision=prec, obs_every=10)
        g.set_tuning(**sh)
        g.step(120)
        s, obs, stats = g.state(), _obs_array(g.observables()), g.stats()
        g.close()
        assert stats["list_rebuilds"] >= 5, stats
        if ref is None:
            ref = (s, obs, stats)
            continue
        for k in ("s", "x", "v", "Te"):
            assert np.array_equal(s[k], ref[0][k]), (sh, k)
        assert np.array_equal(obs, ref[1]), sh
        assert stats["list_rebuilds"] == ref[2]["list_rebuilds"], (sh, stats)


def test_invalid_lane_split_rejected(N):
    spec = I.fe_bcc_spec(L=6)
    g = N.System(spec, I.initial_state(spec, "tilt"))
    before = g.tuning()
    for bad in (dict(atom_lanes=3), dict(atom_lanes=2, atom_block=64),
                dict(atom_lanes=4, atom_block=128)):
        with pytest.raises(N.SLError) as e:
            g.set_tuning(**bad)
        assert e.value.code == N.SL_EINVAL
        assert g.tuning() == before
    g.close()


def test_overfull_bins_against_oracle(N):
    """bcc Fe 8^3 with a 1 A skin: 7.6 A bins hold about 38 atoms, more than
    the 16 accepted atoms per bin the unsorted build keeps sorted, so a
    rebuild from unsorted bins scans such bins a second time.  3000 K
    velocities at a 1 fs step trigger rebuilds inside the 100-step window;
    the rescans are counted on the device.  FP64 against the oracle, and
    bitwise against the sorted-bin build."""
    spec = replace(I.fe_bcc_spec(L=8), skin=1.0, dt=1e-3)
    st = I.initial_state(spec, "tilt", T_lattice=3000.0)
    out = []
    for sh in (dict(bin_mode=1, atom_lanes=1), dict(bin_mode=2, atom_lanes=4, atom_block=256)):
        _log("case: bcc L=8 skin=1 3000 K shape=%s" % sh)
        g = N.System(spec, st, precision=0)
        g.set_tuning(**sh)
        g.step(100)
        out.append(g.state())
        stats = g.stats()
        assert stats["list_rebuilds"] >= 3 and stats["max_list"] > 16, stats
        if sh["bin_mode"] == 1:
            assert stats["list_rescans"] > 0, stats
        g.close()
    for k in ("s", "x", "v", "Te"):
        assert np.array_equal(out[0][k], out[1][k]), k
    o = O.Oracle(spec, st.species, st.spins, st.vel, disp=st.disp)
    o.step(100)
    errs, bad = compare_states(out[0], o.state(), spec.box, 1e-10)
    assert not bad, errs


def test_large_grid_bins_emptied_by_the_grid_update(N):
    """A live run whose electron grid is updated cell-parallel (17^3 = 4913
    cells) has its bins emptied by that launch.  Binning by the kick every
    step and binning only for a rebuild must build the same lists (stale
    bins would add wrong candidates or overflow), with a skin thin enough
    to rebuild every few steps; the first steps against the oracle."""
    spec = replace(I.gdfeco_sc_spec(L=18, tn=17, S0=0.3, t0=0.002, fwhm=0.002, seed=13, run_id=5),
                   skin=0.05)
    st = I.initial_state(spec, "afm")
    out = []
    for mode in (1, 2):
        _log("case: sc 18^3, 17^3 grid, bin_mode=%d" % mode)
        g = N.System(spec, st, precision=0, obs_every=10)
        g.set_tuning(bin_mode=mode)
        g.step(15)
        out.append(g.state())
        g.step(105)
        out.append(g.state())
        stats = g.stats()
        assert stats["list_rebuilds"] >= 4, stats
        g.close()
    for k in ("s", "x", "v", "Te"):
        assert np.array_equal(out[1][k], out[3][k]), k
    o = O.Oracle(spec, st.species, st.spins, st.vel, disp=st.disp)
    o.step(15)
    errs, bad = compare_states(out[0], o.state(), spec.box, 1e-10)
    assert not bad, errs
