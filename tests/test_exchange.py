"""The radial exchange function and its re-derivation (host side) against the
paper's worked example and the conditions that define it."""
import math

import numpy as np
import pytest

from paper_2608_18541_amd import exchange as X


def test_fcc_worked_example():
    """fcc with a = 3.6 A: r1 = 2.5456 A gives x1 = 0.6458, J2 = 0.4050 and
    J3 = 3.1677 A (the values printed with the re-derivation, four places)."""
    r1 = X.nearest_neighbour_distance("fcc", 3.6)
    assert abs(r1 - 2.5456) < 5e-5
    x1, J2, J3 = X.rederive_radial_exchange(r1)
    assert abs(x1 - 0.6458) < 5e-5
    assert abs(J2 - 0.4050) < 5e-5
    assert abs(J3 - 3.1677) < 5e-5


@pytest.mark.parametrize("lattice,a", [("fcc", 3.6), ("bcc", 2.8665), ("sc", 3.52)])
def test_maximum_at_r1_with_the_nominal_value(lattice, a):
    """The two defining conditions on each lattice: J(r1) = J1 and the
    extremum at r1 (a maximum: J falls on both sides), by the analytic
    derivative and by central differences."""
    J1 = 0.01762
    r1 = X.nearest_neighbour_distance(lattice, a)
    _, J2, J3 = X.rederive_radial_exchange(r1)
    assert abs(X.radial_exchange(r1, J1, J2, J3) - J1) < 1e-15
    assert abs(X.radial_exchange_dr(r1, J1, J2, J3)) < 1e-15
    h = 1e-4
    fd = (X.radial_exchange(r1 + h, J1, J2, J3) - X.radial_exchange(r1 - h, J1, J2, J3)) / (2 * h)
    assert abs(fd) < 1e-9
    for dr in (-0.3, -0.05, 0.05, 0.3):
        assert X.radial_exchange(r1 + dr, J1, J2, J3) < J1


def test_derivative_against_central_differences():
    J1, J2, J3 = 0.02, 0.3, 2.2
    r = np.linspace(0.8, 5.0, 43)
    h = 1e-5
    fd = (X.radial_exchange(r + h, J1, J2, J3) - X.radial_exchange(r - h, J1, J2, J3)) / (2 * h)
    assert np.allclose(X.radial_exchange_dr(r, J1, J2, J3), fd, rtol=0, atol=1e-10)


def test_shape_is_lattice_independent():
    """x1 and J2 do not depend on r1; J3 scales with it; the fraction of J1
    delivered at a given r / r1 is the same on every lattice."""
    a = X.rederive_radial_exchange(2.0)
    b = X.rederive_radial_exchange(3.0)
    assert a[0] == b[0] and a[1] == b[1]
    assert abs(b[2] / a[2] - 1.5) < 1e-15
    for q in (0.9, 1.1, 1.3):
        fa = X.radial_exchange(q * 2.0, 1.0, a[1], a[2])
        fb = X.radial_exchange(q * 3.0, 1.0, b[1], b[2])
        assert abs(fa - fb) < 1e-14


def test_a_parameterisation_off_r1_delivers_less_than_j1():
    """A shape whose maximum sits at another distance gives less than J1 at
    r1: the function's maximum value is J1 only at x1, so any other r
    falls short (the effect the re-derivation removes)."""
    x1, J2, _ = X.rederive_radial_exchange(1.0)
    r1 = X.nearest_neighbour_distance("fcc", 3.6)
    J3_bcc = X.rederive_radial_exchange(X.nearest_neighbour_distance("bcc", 2.8665))[2]
    frac = X.radial_exchange(r1, 1.0, J2, J3_bcc)
    assert 0.0 < frac < 1.0
    x = (r1 / J3_bcc) ** 2
    assert abs(frac - 4 * x * (1 - J2 * x) * math.exp(-x)) < 1e-15


def test_cutoff_between_the_first_two_fcc_shells():
    """The 3.4 A cutoff of the fcc runs lies between r1 = a / sqrt(2) and
    r2 = a, so only nearest neighbours couple."""
    r1 = X.nearest_neighbour_distance("fcc", 3.6)
    assert r1 < 3.4 < 3.6


def test_bad_arguments():
    with pytest.raises(ValueError):
        X.rederive_radial_exchange(0.0)
    with pytest.raises(ValueError):
        X.nearest_neighbour_distance("hcp", 3.0)


def test_shell_table_of_the_frozen_lattice():
    """With the re-derived shape every nearest-neighbour pair gets exactly its
    amplitude, a shell beyond the cutoff gets zero, and a shell inside it
    gets J(r2) for every pair, in proportion to the amplitudes."""
    J1 = np.zeros((4, 4))
    J1[0, 0], J1[0, 1], J1[1, 0], J1[1, 1] = 0.01762, -0.006803, -0.006803, 0.007864
    a = 2.8665
    r1, r2 = X.shell_distances("bcc", a)
    assert abs(r1 - a * math.sqrt(3) / 2) < 1e-15 and r2 == a
    _, J2, J3 = X.rederive_radial_exchange(r1)
    t1, t2 = X.shell_exchange_table("bcc", a, J1, J2, J3, cutoff=0.5 * (r1 + r2), n_shells=2)
    assert np.allclose(np.array(t1), J1, rtol=1e-15, atol=0)
    assert np.all(np.array(t2) == 0.0)
    _, u2 = X.shell_exchange_table("bcc", a, J1, J2, J3, cutoff=3.0, n_shells=2)
    f2 = float(X.radial_exchange(r2, 1.0, J2, J3))
    assert 0.0 < f2 < 1.0
    assert np.allclose(np.array(u2), f2 * J1, rtol=1e-15, atol=0)
    with pytest.raises(ValueError):
        X.shell_exchange_table("bcc", a, np.ones((3, 3)), J2, J3, 3.0, 1)
    bad = J1.copy()
    bad[0, 1] = 0.0
    with pytest.raises(ValueError):
        X.shell_exchange_table("bcc", a, bad, J2, J3, 3.0, 1)


def test_shell_table_drives_the_oracle_like_the_direct_constants():
    """A sc alloy whose exchange comes from J(r) with the re-derived shape
    takes the same steps in the oracle as the alloy with its constants
    given directly."""
    from dataclasses import replace
    from oracle import oracle as O
    from paper_2608_18541_amd import inputs as I
    spec = I.gdfeco_sc_spec(L=4, tn=1, alpha=0.05, lattice_mode=0)
    J1 = np.array(spec.J[0], dtype=np.float64)
    _, J2, J3 = X.rederive_radial_exchange(spec.a)
    (t1,) = X.shell_exchange_table("sc", spec.a, J1, J2, J3, cutoff=0.5 * (1 + math.sqrt(2)) * spec.a,
                                   n_shells=1)
    spec_r = replace(spec, J=(t1, spec.J[1]))
    st = I.initial_state(spec, "afm")
    a = O.Oracle(spec, st.species, st.spins, st.vel)
    b = O.Oracle(spec_r, st.species, st.spins, st.vel)
    a.step(5)
    b.step(5)
    assert np.allclose(a.state()["s"], b.state()["s"], rtol=0, atol=1e-12)
