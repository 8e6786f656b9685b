"""Seeded synthetic inputs: workload presets and initial states.

This module holds no step of the dynamics.  It turns the published workload
descriptions (lattice, species, moments, couplings, two-temperature
parameters) into plain numbers in metal units (Angstrom, ps, eV, amu, K, T)
and draws seeded initial states, so that the HIP library and the test
oracle start from identical inputs.

Workload shapes follow the paper's validation systems: a bcc-Fe block with
a Morse lattice (Results A), the Gd25(FeCo)75 random alloy with
antiferromagnetic Fe-Gd coupling (Methods D, Table 1), ensembles of
independent realizations (Methods F) and mixed-size request streams.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field, replace
from typing import List, Optional

import numpy as np

# --- unit conversions of input parameters (CODATA 2018) ----------------------
EV = 1.602176634e-19            # J per eV
KB_EV = 8.617333262e-5          # eV / K
AMU_KG = 1.66053906660e-27
# 1 amu (A/ps)^2 in eV
MVV2E = AMU_KG * 1.0e4 / EV

LATTICE_SC = 0
LATTICE_BCC = 1
LATTICE_FCC = 2

SPECIES_TM = 0                  # transition metal (Fe/Co merged)
SPECIES_GD = 1


def joule_to_ev(j: float) -> float:
    return j / EV


def w_per_m3k_to_metal(g: float) -> float:
    """W m^-3 K^-1 -> eV ps^-1 A^-3 K^-1."""
    return g / EV * 1.0e-12 * 1.0e-30


def j_per_m3k2_to_metal(g: float) -> float:
    """J m^-3 K^-2 -> eV A^-3 K^-2."""
    return g / EV * 1.0e-30


def w_per_m3_to_metal(s: float) -> float:
    """W m^-3 -> eV ps^-1 A^-3."""
    return s / EV * 1.0e-12 * 1.0e-30


def w_per_mk_to_metal(k: float) -> float:
    """W m^-1 K^-1 -> eV ps^-1 A^-1 K^-1."""
    return k / EV * 1.0e-12 * 1.0e-10


@dataclass
class SystemSpec:
    """Everything that defines one run, in metal units."""
    lattice: int = LATTICE_BCC
    ncell: tuple = (6, 6, 6)
    a: float = 2.8665
    n_species: int = 1
    mu: tuple = (2.2, 0.0, 0.0, 0.0)            # Bohr magnetons
    mass: tuple = (55.845, 0.0, 0.0, 0.0)       # amu
    n_shells: int = 2
    # J[shell][si][sj] in eV
    J: tuple = (((0.022, 0, 0, 0), (0, 0, 0, 0), (0, 0, 0, 0), (0, 0, 0, 0)),
                ((0.011, 0, 0, 0), (0, 0, 0, 0), (0, 0, 0, 0), (0, 0, 0, 0)))
    B: tuple = (0.0, 0.0, 1.0)
    K: tuple = (0.0, 0.0, 0.0, 0.0)             # uniaxial anisotropy along z, eV/atom
    alpha: float = 0.1
    noise_mode: int = 0
    mu_ref: float = 0.0
    lattice_mode: int = 1                       # 0 frozen, 1 live
    morse: tuple = (0.4174, 1.3885, 2.845, 5.0)  # D eV, a 1/A, r0 A, rc A
    skin: float = 0.5
    dt: float = 1.0e-4                          # ps (0.1 fs)
    seed: int = 1234
    run_id: int = 0
    # electron-temperature grid
    tn: tuple = (3, 3, 3)
    ttm_mode: int = 0                           # 0 fixed field, 1 two-temperature
    Te0: float = 300.0
    gamma_e: float = 0.0
    G_el: float = 0.0
    kappa_e: float = 0.0
    n_sub: int = 1
    S0: float = 0.0
    t0: float = 0.0
    fwhm: float = 0.0
    profile: int = 0
    depth: float = 0.0
    # ttm_mode 2: stepped T_e(t), stage temperatures (K) and ends of stages 1, 2 (ps)
    step_T: tuple = (0.0, 0.0, 0.0)
    step_end: tuple = (0.0, 0.0)
    # radial exchange (live lattices): J holds the amplitudes J1 of
    # J(r) = 4 J1 x (1 - J2 x) e^{-x}, x = (r / J3)^2; exch_r[shell] = (J2, J3 A)
    exch_radial: int = 0
    exch_r: tuple = ((0.0, 0.0), (0.0, 0.0))

    @property
    def nbasis(self) -> int:
        return {LATTICE_SC: 1, LATTICE_BCC: 2, LATTICE_FCC: 4}[self.lattice]

    @property
    def n_sites(self) -> int:
        L = self.ncell
        return self.nbasis * L[0] * L[1] * L[2]

    @property
    def box(self) -> tuple:
        return tuple(self.a * L for L in self.ncell)

    @property
    def n_tcells(self) -> int:
        return self.tn[0] * self.tn[1] * self.tn[2]


@dataclass
class InitialState:
    species: np.ndarray          # int8 [n]
    spins: np.ndarray            # float64 [n, 3]
    vel: np.ndarray              # float64 [n, 3]  A/ps
    disp: Optional[np.ndarray] = None   # float64 [n, 3] A from ideal sites


def _rng(seed: int, run_id: int, stream: int) -> np.random.Generator:
    return np.random.default_rng(np.random.SeedSequence([int(seed), int(run_id), int(stream)]))


# --- initial-state generators ---------------------------------------------------

def species_bernoulli(n: int, p: float, seed: int, run_id: int) -> np.ndarray:
    """Random binary alloy: each site independently Gd with probability p."""
    rng = _rng(seed, run_id, 4)
    return (rng.random(n) < p).astype(np.int8)


def species_exact(n: int, n_gd: int, seed: int, run_id: int) -> np.ndarray:
    """Random binary alloy with exactly n_gd Gd sites, drawn uniformly without
    replacement (every set of n_gd sites equally likely), as the production
    alloys are placed."""
    if not 0 <= n_gd <= n:
        raise ValueError("n_gd must lie in [0, n]")
    rng = _rng(seed, run_id, 4)
    out = np.zeros(n, dtype=np.int8)
    out[rng.choice(n, size=n_gd, replace=False)] = 1
    return out


def spins_tilted(n: int, max_deg: float, seed: int, run_id: int) -> np.ndarray:
    """Unit spins uniform on the spherical cap within max_deg of +z."""
    rng = _rng(seed, run_id, 2)
    cmin = math.cos(math.radians(max_deg))
    c = 1.0 - rng.random(n) * (1.0 - cmin)
    phi = rng.random(n) * 2.0 * math.pi
    sn = np.sqrt(np.maximum(0.0, 1.0 - c * c))
    s = np.stack([sn * np.cos(phi), sn * np.sin(phi), c], axis=1)
    return s / np.linalg.norm(s, axis=1, keepdims=True)


def spins_antiparallel(species: np.ndarray) -> np.ndarray:
    """Gd along +z, transition metal along -z."""
    s = np.zeros((species.shape[0], 3))
    s[:, 2] = np.where(species == SPECIES_GD, 1.0, -1.0)
    return s


def spins_random(n: int, seed: int, run_id: int) -> np.ndarray:
    rng = _rng(seed, run_id, 2)
    s = rng.standard_normal((n, 3))
    return s / np.linalg.norm(s, axis=1, keepdims=True)


def maxwell_velocities(masses: np.ndarray, T: float, seed: int, run_id: int) -> np.ndarray:
    """Gaussian velocities at temperature T with the centre-of-mass motion
    removed and the kinetic energy rescaled to exactly (3N-3)/2 k_B T."""
    n = masses.shape[0]
    rng = _rng(seed, run_id, 3)
    sd = np.sqrt(KB_EV * T / (masses * MVV2E))
    v = rng.standard_normal((n, 3)) * sd[:, None]
    p = (masses[:, None] * v).sum(axis=0)
    v -= p / masses.sum()
    if T <= 0.0 or n < 2:
        return np.zeros_like(v)
    ke = 0.5 * (masses[:, None] * MVV2E * v * v).sum()
    target = 0.5 * (3 * n - 3) * KB_EV * T
    return v * math.sqrt(target / ke)


# --- workload presets --------------------------------------------------------------

def fe_bcc_spec(L: int = 6, **kw) -> SystemSpec:
    """bcc Fe, a = 2.8665 A, mu = 2.2 mu_B, J1 = 22 meV, J2 = 11 meV,
    alpha = 0.1, B = 1 T along z, Morse lattice, fixed 300 K grid."""
    s = SystemSpec(lattice=LATTICE_BCC, ncell=(L, L, L), a=2.8665, n_species=1,
                   mu=(2.2, 0, 0, 0), mass=(55.845, 0, 0, 0), n_shells=2,
                   J=(((0.022, 0, 0, 0), (0,) * 4, (0,) * 4, (0,) * 4),
                      ((0.011, 0, 0, 0), (0,) * 4, (0,) * 4, (0,) * 4)),
                   B=(0.0, 0.0, 1.0), alpha=0.1, lattice_mode=1,
                   morse=(0.4174, 1.3885, 2.845, 5.0), skin=0.5, dt=1.0e-4,
                   tn=(3, 3, 3), ttm_mode=0, Te0=300.0)
    return replace(s, **kw)


GDFECO_J_TMTM = joule_to_ev(2.835e-21)
GDFECO_J_GDGD = joule_to_ev(1.26e-21)
GDFECO_J_TMGD = joule_to_ev(-1.09e-21)
# uniaxial easy-axis anisotropy of both species, eV per atom (parameter table)
GDFECO_K = 5.0384e-5


def gdfeco_sc_spec(L: int = 32, alpha: float = 0.01, S0: float = 0.0, tn: int = 8,
                   **kw) -> SystemSpec:
    """Gd25(FeCo)75 on a simple-cubic lattice, a = 3.52 A: moments 1.92 / 7.63
    mu_B, nearest-neighbour exchange TM-TM, Gd-Gd and antiferromagnetic TM-Gd,
    B = 0, the Morse lattice of the Fe block (same potential and mass for
    both species), two-temperature grid with C_e = gamma_e T_e,
    gamma_e = 225 J m^-3 K^-2, G_el = 6.6e17 W m^-3 K^-1, 50 fs laser."""
    J1 = ((GDFECO_J_TMTM, GDFECO_J_TMGD, 0, 0), (GDFECO_J_TMGD, GDFECO_J_GDGD, 0, 0),
          (0,) * 4, (0,) * 4)
    s = SystemSpec(lattice=LATTICE_SC, ncell=(L, L, L), a=3.52, n_species=2,
                   mu=(1.92, 7.63, 0, 0), mass=(55.845, 55.845, 0, 0), n_shells=1,
                   J=(J1, ((0,) * 4,) * 4), B=(0.0, 0.0, 0.0), alpha=alpha,
                   lattice_mode=1, morse=(0.4174, 1.3885, 2.845, 5.0), skin=0.5,
                   dt=1.0e-4, tn=(tn, tn, tn), ttm_mode=1, Te0=300.0,
                   gamma_e=j_per_m3k2_to_metal(225.0),
                   G_el=w_per_m3k_to_metal(6.6e17), kappa_e=0.0, n_sub=1,
                   S0=S0, t0=0.1, fwhm=0.05, profile=0)
    return replace(s, **kw)


# the production GdFeCo model's literature exchange amplitudes (eV, the
# parameter table): nearest neighbours of the fcc lattice
GDFECO_FCC_J_FEFE = 0.01762
GDFECO_FCC_J_GDGD = 0.007864
GDFECO_FCC_J_FEGD = -0.006803


def gdfeco_fcc_spec(L: int = 13, alpha: float = 0.01, **kw) -> SystemSpec:
    """The production Gd25(FeCo)75 model (Methods, GdFeCo model; the
    parameter table): random binary alloy on an fcc lattice, a = 3.6 A,
    L^3 cells (13^3: 8788 sites), moments 1.92 / 7.63 mu_B, nearest-neighbour
    exchange Fe-Fe 17.62 meV, Gd-Gd 7.864 meV, Fe-Gd -6.803 meV (the radial
    exchange function re-derived to equal J_1 at the nearest-neighbour
    distance, so on the frozen lattice each bond is one constant), uniaxial
    anisotropy 5.0384e-5 eV on both species, damping 0.01, no field, frozen
    lattice, one electron cell.  The temperature profile is set by the
    caller (production_spec in workloads)."""
    J1 = ((GDFECO_FCC_J_FEFE, GDFECO_FCC_J_FEGD, 0, 0), (GDFECO_FCC_J_FEGD, GDFECO_FCC_J_GDGD, 0, 0),
          (0,) * 4, (0,) * 4)
    s = SystemSpec(lattice=LATTICE_FCC, ncell=(L, L, L), a=3.6, n_species=2,
                   mu=(1.92, 7.63, 0, 0), mass=(55.845, 55.845, 0, 0), n_shells=1,
                   J=(J1, ((0,) * 4,) * 4), B=(0.0, 0.0, 0.0),
                   K=(GDFECO_K, GDFECO_K, 0.0, 0.0), alpha=alpha, lattice_mode=0,
                   morse=(0.4174, 1.3885, 2.845, 5.0), skin=0.5, dt=1.0e-4, tn=(1, 1, 1),
                   ttm_mode=0, Te0=300.0)
    return replace(s, **kw)


def initial_state(spec: SystemSpec, kind: str = "tilt", p_gd: float = 0.25,
                  T_lattice: float = 300.0, exact_count: bool = False) -> InitialState:
    """Seeded initial state for a spec.  kind: 'tilt' (within 10 degrees of
    +z), 'afm' (Gd +z, TM -z) or 'random'.  An alloy has each site Gd with
    probability p_gd, or, with exact_count, exactly round(p_gd n) Gd sites."""
    n = spec.n_sites
    if spec.n_species > 1 and exact_count:
        species = species_exact(n, int(round(p_gd * n)), spec.seed, spec.run_id)
    elif spec.n_species > 1:
        species = species_bernoulli(n, p_gd, spec.seed, spec.run_id)
    else:
        species = np.zeros(n, dtype=np.int8)
    if kind == "tilt":
        spins = spins_tilted(n, 10.0, spec.seed, spec.run_id)
    elif kind == "afm":
        spins = spins_antiparallel(species)
    elif kind == "random":
        spins = spins_random(n, spec.seed, spec.run_id)
    else:
        raise ValueError(kind)
    masses = np.asarray(spec.mass, dtype=np.float64)[species.astype(np.int64)]
    if spec.lattice_mode == 1 and T_lattice > 0:
        vel = maxwell_velocities(masses, T_lattice, spec.seed, spec.run_id)
    else:
        vel = np.zeros((n, 3))
    return InitialState(species=species, spins=spins, vel=vel)


# --- laser amplitude ---------------------------------------------------------------

def peak_te_0d(S0_si, gamma_e: float, C_l: float, G: float, t0: float, fwhm: float,
               T0: float = 300.0, dt: float = 2.0e-16):
    """Peak electron temperature of the zero-dimensional two-temperature
    model gamma_e T_e dT_e/dt = -G (T_e - T_l) + S(t), C_l dT_l/dt =
    G (T_e - T_l) (SI units), classical RK4, vectorised over S0_si."""
    S0 = np.atleast_1d(np.asarray(S0_si, dtype=np.float64))

    def rhs(t, Te, Tl):
        S = S0 * math.exp(-4.0 * math.log(2.0) * (t - t0) ** 2 / fwhm ** 2)
        q = G * (Te - Tl)
        return (S - q) / (gamma_e * Te), q / C_l
    Te = np.full_like(S0, T0)
    Tl = np.full_like(S0, T0)
    peak = Te.copy()
    t = 0.0
    t_end = t0 + 4.0 * fwhm
    while t < t_end:
        a1, b1 = rhs(t, Te, Tl)
        a2, b2 = rhs(t + dt / 2, Te + dt / 2 * a1, Tl + dt / 2 * b1)
        a3, b3 = rhs(t + dt / 2, Te + dt / 2 * a2, Tl + dt / 2 * b2)
        a4, b4 = rhs(t + dt, Te + dt * a3, Tl + dt * b3)
        Te = Te + dt / 6 * (a1 + 2 * a2 + 2 * a3 + a4)
        Tl = Tl + dt / 6 * (b1 + 2 * b2 + 2 * b3 + b4)
        t += dt
        peak = np.maximum(peak, Te)
    return peak


def calibrate_laser(targets, fwhm_s: float, t0_s: float, gamma_e: float = 225.0,
                    C_l: float = 3.1e6, G: float = 6.6e17):
    """Peak source power densities (W m^-3) for which the zero-dimensional
    two-temperature model reaches each target peak T_e (vectorised
    bisection)."""
    tg = np.atleast_1d(np.asarray(targets, dtype=np.float64))
    lo = np.zeros_like(tg)
    hi = np.full_like(tg, 1.0e24)
    for _ in range(56):
        mid = 0.5 * (lo + hi)
        below = peak_te_0d(mid, gamma_e, C_l, G, t0_s, fwhm_s) < tg
        lo = np.where(below, mid, lo)
        hi = np.where(below, hi, mid)
    return 0.5 * (lo + hi)


_S0_CACHE = {}


def laser_S0_many(targets, fwhm_ps: float, t0_ps: float) -> np.ndarray:
    """Calibrated source amplitudes in eV ps^-1 A^-3 (cached per target)."""
    tg = [round(float(x), 6) for x in np.atleast_1d(targets)]
    key0 = (round(fwhm_ps, 9), round(t0_ps, 9))
    todo = sorted(set(x for x in tg if (key0, x) not in _S0_CACHE))
    if todo:
        vals = calibrate_laser(todo, fwhm_ps * 1e-12, t0_ps * 1e-12)
        for x, v in zip(todo, vals):
            _S0_CACHE[(key0, x)] = w_per_m3_to_metal(float(v))
    return np.array([_S0_CACHE[(key0, x)] for x in tg])


def laser_S0_metal(target_peak: float, fwhm_ps: float, t0_ps: float) -> float:
    return float(laser_S0_many([target_peak], fwhm_ps, t0_ps)[0])


def cfg1_S0() -> float:
    """32^3 alloy workload: 50 fs FWHM pulse centred at 100 fs, peak
    T_e about 1800 K."""
    return laser_S0_metal(1800.0, 0.05, 0.1)


def fe_large_spec(L: int = 64, tn: int = 32, **kw) -> SystemSpec:
    """bcc Fe L^3 cells with the Fe-block exchange and Morse lattice, tn^3
    grid with the alloy's two-temperature constants, kappa_e = 80 W/m/K
    (4 diffusion sub-steps), 100 fs pulse absorbed in the top 10 nm with
    peak T_e about 1500 K (surface heating)."""
    t0, fwhm = 0.2, 0.1
    s = fe_bcc_spec(L=L, tn=(tn, tn, tn), ttm_mode=1, Te0=300.0,
                    gamma_e=j_per_m3k2_to_metal(225.0), G_el=w_per_m3k_to_metal(6.6e17),
                    kappa_e=w_per_mk_to_metal(80.0), n_sub=4,
                    S0=laser_S0_metal(1500.0, fwhm, t0), t0=t0, fwhm=fwhm, profile=1,
                    depth=100.0)
    return replace(s, **kw)
