"""Host-side helpers of bench.py and the ensemble statistics (CPU only)."""
import gc
import json
import math
import os
import sys

import numpy as np
import pytest

import bench
from paper_2608_18541_amd import inputs as I
from paper_2608_18541_amd.stats import homogeneity_chi2


def test_host_quiet_suspends_collection():
    assert gc.isenabled()
    with bench.host_quiet():
        assert not gc.isenabled()
    assert gc.isenabled()
    with pytest.raises(RuntimeError):
        with bench.host_quiet():
            raise RuntimeError("inside")
    assert gc.isenabled()


def test_algorithmic_bytes_per_unit():
    # own spin read + write, species, electron-cell id
    assert bench.bytes_per_unit("spin_pass", 0, 2, 0) == 51
    assert bench.bytes_per_unit("spin_pass", 1, 2, 0) == 27
    assert bench.bytes_per_unit("spin_pass", 0, 1, 0) == 50
    # u read, v read + write, F write, list 4 z, count, species, cell (sc, z = 18)
    assert bench.bytes_per_unit("atom_final", 0, 2, 18.0) == 175
    assert bench.bytes_per_unit("atom_final", 1, 2, 18.0) == 127


def test_launch_bytes_of_the_fused_launch():
    """Colour pass 1 carrying the force kernel moves the bytes of both: the
    colour's sites (half of an sc lattice) and every atom."""
    n, z = 32768, 18.0
    sp = bench.launch_bytes("spin_pass", 0, 2, z, n, 2)
    af = bench.launch_bytes("atom_final", 0, 2, z, n, 2)
    assert sp == 51 * n / 2 and af == 175 * n
    assert bench.launch_bytes("spin_force", 0, 2, z, n, 2) == sp + af == 6569984
    assert "spin_force" in bench.KERNELS and bench.KERNELS.index("spin_force") == 5


def _write_profile(tmp_path, name, digest, tuning=None, value=12345.0):
    lines = ["# test", "traffic_bytes_per_launch: %.0f" % value, "source_sha256: %s" % digest]
    if tuning is not None:
        lines.append("tuning: %s" % json.dumps(tuning))
    (tmp_path / name).write_text("\n".join(lines) + "\n")


def test_measured_traffic_only_for_current_kernels(tmp_path, monkeypatch):
    monkeypatch.setattr(bench, "PROFILES", str(tmp_path))
    digest = bench.source_digest()
    tun = {"spin_block": 256, "spin_spt": 2}
    _write_profile(tmp_path, "spin_pass_w1_traffic.txt", digest, tun, 627e6)
    _write_profile(tmp_path, "atom_final_w2_traffic.txt", "0" * 64, None, 7e6)
    assert bench.measured_traffic("spin_pass", "w1", tun) == 627e6
    assert bench.measured_traffic("spin_pass", "w1") == 627e6
    assert bench.measured_traffic("spin_pass", "w1", {"spin_block": 128, "spin_spt": 2}) is None
    assert bench.measured_traffic("atom_final", "w2") is None        # kernels changed since
    assert bench.measured_traffic("atom_final", "missing") is None


def test_committed_profiles_are_well_formed():
    """Every committed counter summary names the command that made it and
    carries the source digest of the kernels it was taken on (the bench uses
    its figures only while that digest is the current one) and its figure."""
    import glob
    paths = glob.glob(os.path.join(bench.PROFILES, "*_traffic.txt")) + \
        glob.glob(os.path.join(bench.PROFILES, "*_valu.txt"))
    assert paths
    for path in paths:
        kv = {}
        for line in open(path):
            if ":" in line and not line.startswith("#"):
                k, v = line.split(":", 1)
                kv[k.strip()] = v.strip()
        assert len(kv.get("source_sha256", "")) == 64, path
        assert any(k.startswith("command") for k in kv), path
        assert "traffic_bytes_per_launch" in kv or "valu_wave_instructions_per_site_step" in kv, path


def _positions(spec, uz_of_layer):
    Lx, Ly, Lz = spec.ncell
    nb = 2 if spec.lattice == 1 else 1
    out = np.zeros((spec.n_sites, 3))
    for i in range(spec.n_sites):
        b, cell = i % nb, i // nb
        x, y, z = cell % Lx, (cell // Lx) % Ly, cell // (Lx * Ly)
        off = 0.25 + 0.5 * b
        out[i] = [(x + off) * spec.a, (y + off) * spec.a, (z + off) * spec.a + uz_of_layer[z]]
    out[:, 2] %= Lz * spec.a
    return out


@pytest.mark.parametrize("lattice", [0, 1])
def test_strain_profile_of_a_standing_wave(lattice):
    """u_z = A sin(2 pi k / Lz) per layer k gives the central-difference
    strain A cos(2 pi k / Lz) sin(2 pi / Lz) / a; the ideal lattice none."""
    spec = I.fe_bcc_spec(L=6) if lattice == 1 else I.gdfeco_sc_spec(L=6, tn=2)
    Lz = spec.ncell[2]
    assert np.allclose(bench.strain_profile(spec, _positions(spec, np.zeros(Lz))), 0.0, atol=1e-15)
    A = 0.05
    k = np.arange(Lz)
    eps = bench.strain_profile(spec, _positions(spec, A * np.sin(2 * np.pi * k / Lz)))
    want = A * np.cos(2 * np.pi * k / Lz) * np.sin(2 * np.pi / Lz) / spec.a
    np.testing.assert_allclose(eps, want, atol=1e-12)


def test_homogeneity_chi2_against_the_exact_tail():
    scipy_stats = pytest.importorskip("scipy.stats")
    rng = np.random.default_rng(3)
    for cells, n in ((64, 20), (40, 50), (16, 200)):
        p = rng.uniform(0.1, 0.9, cells)
        ka, kb = rng.binomial(n, p), rng.binomial(n, p)
        chi2, dof, pval = homogeneity_chi2(ka, kb, n)
        # the statistic written out directly
        pp = (ka + kb) / (2.0 * n)
        m = (pp > 0) & (pp < 1)
        direct = np.sum((ka - kb)[m] ** 2 / (2.0 * n * pp[m] * (1 - pp[m])))
        assert math.isclose(chi2, direct, rel_tol=1e-12) and dof == int(m.sum())
        # Wilson-Hilferty tail within its stated accuracy at dof >= 10
        assert abs(pval - scipy_stats.chi2.sf(chi2, dof)) < 2e-3
    # cells at p = 0 or 1 carry no information; identical counts give chi2 0
    chi2, dof, pval = homogeneity_chi2([0, 20, 5], [0, 20, 5], 20)
    assert chi2 == 0.0 and dof == 1 and pval > 0.3
    assert homogeneity_chi2([0, 20], [0, 20], 20) == (0.0, 0, 1.0)


def test_more_than_one_gpu_is_refused(monkeypatch, capsys):
    monkeypatch.setattr(sys, "argv", ["bench.py", "--gpus", "2"])
    assert bench.main() == 2
    assert "one GPU" in capsys.readouterr().err


def test_production_diagram_grid():
    """The production grid: T0 800-2900 K in steps of 300 K (rows), d = 1-8
    (columns), seeds innermost; frozen lattice, literature anisotropy, zero
    field, stage ends scaling with d; every run its own run_id."""
    from paper_2608_18541_amd import workloads as W
    runs = W.production_diagram(L=4, n_seeds=2, n_steps=100, base_ends=(0.05, 0.15))
    assert len(runs) == 128
    assert len({r.spec.run_id for r in runs}) == 128
    for k, r in enumerate(runs):
        T0 = 800.0 + 300.0 * (k // 16)
        d = 1.0 + (k // 2) % 8
        sp = r.spec
        assert sp.step_T == (T0, T0 / 2, 300.0) and r.tag == (T0, d)
        assert np.allclose(sp.step_end, (0.05 * d, 0.15 * d), rtol=0, atol=1e-15)
        assert sp.ttm_mode == 2 and sp.lattice_mode == 0 and sp.alpha == 0.01
        assert sp.K[:2] == (5.0384e-5, 5.0384e-5) and tuple(sp.B) == (0.0, 0.0, 0.0)


def test_production_run_follows_its_profile_in_the_oracle():
    """A production spec with stage ends at steps 4 and 10: the oracle's grid
    holds T0, then T0 / 2, then 300 K."""
    from oracle import oracle as O
    from paper_2608_18541_amd import workloads as W
    r = W.production_run(L=4, T0=1400.0, d=2.0, seed=5, run_id=3, n_steps=12,
                         base_ends=(0.0002, 0.0005))
    st = r.state
    orc = O.Oracle(r.spec, st.species, st.spins, st.vel)
    seen = []
    for _ in range(12):
        orc.step(1)
        seen.append(float(orc.state()["Te"][0]))
    assert seen[:3] == [1400.0] * 3 and seen[4:9] == [700.0] * 5 and seen[10:] == [300.0] * 2


def test_exact_count_alloy_matches_the_random_occupancy_prediction():
    """Exactly k Gd of N sites, drawn without replacement: the expected
    number of Gd-Gd nearest-neighbour bonds on a periodic sc L^3 lattice is
    3N k(k-1) / (N(N-1)), below the independent-site value 3N (k/N)^2; the
    mean over 3000 alloys lies within four standard errors of it (and more
    than four from the independent-site value), and every site is Gd with
    frequency near k/N."""
    L = 4
    M = 3000
    N = L ** 3
    k = int(round(0.25 * N))
    counts, freq = [], np.zeros(N)
    for r in range(M):
        sp = I.species_exact(N, k, seed=11, run_id=r).reshape(L, L, L)
        assert int(sp.sum()) == k
        freq += sp.ravel()
        g = sp.astype(np.int64)
        counts.append(int(sum((g * np.roll(g, 1, axis=ax)).sum() for ax in range(3))))
    counts = np.array(counts, dtype=np.float64)
    expect = 3 * N * k * (k - 1) / (N * (N - 1))
    se = counts.std(ddof=1) / math.sqrt(len(counts))
    assert abs(counts.mean() - expect) < 4 * se
    assert 3 * N * (k / N) ** 2 - expect > 4 * se       # the test tells the two apart
    f = freq / M
    assert abs(f.mean() - k / N) < 1e-12
    assert np.abs(f - k / N).max() < 0.04                  # binomial(3000, 1/4): sd 0.008
    with pytest.raises(ValueError):
        I.species_exact(10, 11, 1, 1)


def test_production_runs_have_exact_counts():
    from paper_2608_18541_amd import workloads as W
    r = W.production_run(L=6, T0=1100.0, d=6.0, seed=3, run_id=4, n_steps=10)
    assert int(r.state.species.sum()) == round(0.25 * 216)


def test_field_runs_layout():
    from paper_2608_18541_amd import workloads as W
    runs = W.field_runs(2900.0, 7.0, n_seeds=3, L=4, n_steps=10)
    assert [r.spec.B for r in runs] == [(0.0, 0.0, B) for B in (0.0, 0.5, 10.0) for _ in range(3)]
    assert len({r.spec.run_id for r in runs}) == 9
    r = runs[4]
    assert r.spec.ttm_mode == 2 and r.spec.lattice_mode == 0 and r.exact_count
    assert r.spec.step_T == (2900.0, 1450.0, 300.0) and r.tag == (2900.0, 7.0, 0.5)
    # the field opposes the reversal: Gd (and the net moment) start along +z
    st = r.state
    gd = st.species == 1
    assert np.all(st.spins[gd, 2] == 1.0) and np.all(st.spins[~gd, 2] == -1.0)
    mu = np.where(gd, 7.63, 1.92)
    assert (mu * st.spins[:, 2]).sum() > 0
