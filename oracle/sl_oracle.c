/*
 * sl_oracle.c -- plain FP64 CPU oracle for one timestep of three-temperature
 * atomistic spin-lattice dynamics (stochastic LLG spins driven by the local
 * electron temperature of a two-temperature grid, a velocity-Verlet lattice,
 * and the finite-difference electron-temperature grid).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the correctness reference for the
 * HIP path.  It shares no code, header, table or constant with the product
 * library; only the test-suite, the smoke check and the CPU-baseline leg of
 * the benchmark may load it.  Every routine is written for clarity, not
 * speed: pair forces take every pair closer than the cutoff (minimum image),
 * found through a cell list rebuilt at every evaluation and pinned against
 * the loop over all pairs; every spin is updated one at a time, and all
 * arithmetic is double precision.
 *
 * Units (LAMMPS "metal"): Angstrom, picosecond, eV, amu, Kelvin, Tesla.
 *
 * Paper sections followed (arXiv 2608.18541):
 *   - Methods A, Eq. (1): Landau-Lifshitz form of the LLG equation for the
 *     unit spin s_i with precession vector omega_i and damping alpha.
 *   - Methods C: the effective field H_i = -(1/mu_i) dH/ds_i, so the
 *     deterministic torque scales as 1/mu_i, and the fluctuation-dissipation
 *     theorem then makes the noise amplitude scale as 1/sqrt(mu_i).
 *   - Methods B, Eq. (2): the Langevin bath temperature of each spin is the
 *     electron temperature of the grid cell that contains the atom.
 *   - Methods A/B: spins and lattice advance together; the electron grid is
 *     heated by a laser source and loses energy to the lattice.
 * Readings of points the paper leaves open are listed next to the code that
 * takes them.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ---------------------------------------------------------------- constants
 * CODATA 2018 values in metal units. */
static const double OR_KB = 8.617333262e-5;      /* eV / K                 */
static const double OR_HBAR = 6.582119569e-4;    /* eV ps                  */
static const double OR_MUB = 5.7883818060e-5;    /* eV / T                 */
/* 1 amu * (Angstrom/ps)^2 expressed in eV:
 * 1.66053906660e-27 kg * 1e4 m^2/s^2 / 1.602176634e-19 J/eV */
static const double OR_MVV2E = 1.66053906660e-27 * 1.0e4 / 1.602176634e-19;
static const double OR_PI = 3.14159265358979323846;

/* Gyromagnetic ratio of a g = 2 spin, rad / (ps T). */
static double or_gamma(void) { return 2.0 * OR_MUB / OR_HBAR; }

/* ------------------------------------------------------------ Philox4x32-10
 * Counter-based generator of Salmon, Moraes, Dror and Shaw (SC'11): ten
 * rounds of two 32x32->64 multiplies, the key advanced by the Weyl
 * constants between rounds.  Written from the published definition. */
void or_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
        uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c1 ^ k0;
        uint32_t n2 = hi0 ^ c3 ^ k1;
        c0 = n0;
        c1 = lo1;
        c2 = n2;
        c3 = lo0;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* Three standard normals for (seed, run) and counter (id, step, stream):
 * four Philox words become uniforms on the open interval (0,1) as
 * (w + 1/2) 2^-32, then two Box-Muller pairs; the fourth normal is unused. */
void or_normals3(uint32_t seed, uint32_t run, uint32_t id, int64_t step, uint32_t stream,
                 double nrm[3])
{
    uint32_t key[2] = {seed, run};
    uint64_t st = (uint64_t)step;
    uint32_t ctr[4] = {id, (uint32_t)(st & 0xFFFFFFFFu), (uint32_t)(st >> 32), stream};
    uint32_t w[4];
    or_philox4x32_10(ctr, key, w);
    double u[4];
    for (int k = 0; k < 4; ++k) u[k] = ((double)w[k] + 0.5) * (1.0 / 4294967296.0);
    double r0 = sqrt(-2.0 * log(u[0]));
    double r1 = sqrt(-2.0 * log(u[2]));
    nrm[0] = r0 * cos(2.0 * OR_PI * u[1]);
    nrm[1] = r0 * sin(2.0 * OR_PI * u[1]);
    nrm[2] = r1 * cos(2.0 * OR_PI * u[3]);
}

/* ------------------------------------------------------------------ system */
typedef struct {
    int32_t n;               /* number of atoms (= spins)                       */
    int32_t n_colours;       /* colours of the spin update order               */
    const int32_t* colour;   /* [n] colour of each spin; no bond inside a colour */
    const int32_t* ctr_id;   /* [n] first Philox counter word of each atom       */
    const int32_t* species;  /* [n] species index                              */
    int32_t n_species;
    const double* mu_s;      /* [n_species] moment, Bohr magnetons            */
    const double* mass_s;    /* [n_species] mass, amu                          */
    const int32_t* nbr_off;  /* [n+1] exchange neighbours of atom i are         */
    const int32_t* nbr_j;    /*   nbr_j[nbr_off[i] .. nbr_off[i+1]) with         */
    const double* nbr_J;     /*   coupling nbr_J (eV); each bond appears twice   */
    const double* x0;        /* [n*3] positions, Angstrom                      */
    const double* v0;        /* [n*3] velocities, Angstrom/ps (NULL = 0)        */
    const double* s0;        /* [n*3] unit spins                               */
    double box[3];           /* periodic box lengths, Angstrom                 */
    double B[3];             /* applied field, Tesla                           */
    double alpha;            /* Gilbert damping                                */
    double dt;               /* ps                                             */
    int32_t noise_mode;      /* 0: variance ~ 1/mu (FDT); 1: amplitude ~ 1/mu  */
    double mu_ref;           /* reference moment of noise_mode 1               */
    uint32_t seed, run_id;
    int32_t lattice_live;    /* 0: positions frozen; 1: velocity Verlet        */
    double morse[4];         /* D (eV), a (1/Angstrom), r0 (A), cutoff rc (A)   */
    int32_t tn[3];           /* electron-temperature grid cells per dimension   */
    int32_t ttm_mode;        /* 0: fixed T_e field; 1: two-temperature update;
                                2: prescribed stepped T_e(t)                   */
    const double* Te0;       /* [tn0*tn1*tn2] initial T_e, K, x fastest        */
    double gamma_e;          /* C_e = gamma_e T_e, eV / (Angstrom^3 K^2)        */
    double G_el;             /* electron-phonon coupling, eV/(ps Angstrom^3 K)  */
    double kappa_e;          /* electron conductivity, eV/(ps Angstrom K)       */
    int32_t n_sub;           /* diffusion sub-cycles per step                  */
    double S0, t0, fwhm;     /* laser: peak power density eV/(ps A^3), centre and FWHM (ps) */
    int32_t profile;         /* 0: uniform; 1: cells with centre z > box_z - depth */
    double depth;            /* Angstrom                                       */
    const double* K_s;       /* [n_species] uniaxial anisotropy along z, eV per atom
                                (energy -K s_z^2), or NULL for none           */
    double step_T[3];        /* ttm_mode 2: stage temperatures, K              */
    double step_end[2];      /* ttm_mode 2: ends of stages 1 and 2, ps         */
    int32_t exch_radial;     /* 1: nbr_J holds amplitudes J1 of the radial
                                exchange J(r) = 4 J1 x (1 - J2 x) e^{-x},
                                x = (r / J3)^2, at the bond's current length  */
    double exch_r[2][2];     /* per shell: J2, J3 (Angstrom)                   */
    const int32_t* nbr_sh;   /* [nnz] shell of each neighbour entry (or NULL)  */
} or_desc;

typedef struct {
    double t;
    int64_t step;
    double M[4][3];          /* mean spin per species                          */
    double m[3];             /* mean spin of all atoms                         */
    double m_abs;
    double E_ex, E_z, KE, PE, E_e;
    double Te_mean, Te_max, Tl;
    double Tspin[4];
} or_obs;

typedef struct {
    or_desc d;
    int32_t n, ncell;
    double *s, *x, *v, *F;   /* [n][3]                                         */
    double *mu, *mass;       /* [n]                                            */
    double* K;               /* [n] anisotropy constant, eV                    */
    int32_t *colour, *ctr_id, *species, *nbr_off, *nbr_j, *nbr_sh;
    double* nbr_J;
    double *Te, *dE;         /* [ncell]                                        */
    int64_t step;
    int32_t err;
} or_system;

static void* or_copy(const void* src, size_t bytes)
{
    void* p = malloc(bytes ? bytes : 1);
    if (src && bytes) memcpy(p, src, bytes);
    else memset(p, 0, bytes ? bytes : 1);
    return p;
}

static double or_wrap(double x, double L) { return x - L * floor(x / L); }

/* Minimum-image separation of two positions. */
static void or_min_image(const double* xi, const double* xj, const double* box, double d[3])
{
    for (int k = 0; k < 3; ++k) {
        double dk = xj[k] - xi[k];
        d[k] = dk - box[k] * round(dk / box[k]);
    }
}

/* Index of the electron-temperature cell containing a position: the grid
 * spans the periodic box, cell = floor(wrapped coordinate / cell width). */
static int32_t or_cell_of(const or_system* S, const double* x)
{
    int32_t idx[3];
    for (int k = 0; k < 3; ++k) {
        double h = S->d.box[k] / S->d.tn[k];
        int32_t c = (int32_t)floor(or_wrap(x[k], S->d.box[k]) / h);
        if (c >= S->d.tn[k]) c = S->d.tn[k] - 1;
        if (c < 0) c = 0;
        idx[k] = c;
    }
    return (idx[2] * S->d.tn[1] + idx[1]) * S->d.tn[0] + idx[0];
}

/* ----------------------------------------------------------- Morse lattice
 * Pair energy shifted so that it vanishes at the cutoff; pairs interact when
 * their minimum-image distance is below the cutoff. */
static double or_morse_energy(const double* m, double r)
{
    double D = m[0], a = m[1], r0 = m[2], rc = m[3];
    double Vr = D * (exp(-2.0 * a * (r - r0)) - 2.0 * exp(-a * (r - r0)));
    double Vc = D * (exp(-2.0 * a * (rc - r0)) - 2.0 * exp(-a * (rc - r0)));
    return Vr - Vc;
}

/* -dV/dr */
static double or_morse_force(const double* m, double r)
{
    double D = m[0], a = m[1], r0 = m[2];
    return 2.0 * a * D * (exp(-2.0 * a * (r - r0)) - exp(-a * (r - r0)));
}

/* The interacting pairs: every unordered pair {i, j}, i < j, whose
 * minimum-image distance is below the cutoff, as (i, j) entries of `pairs`
 * (2 * count ints, malloc'd; the caller frees).  method 0 tests all pairs;
 * method 1 finds the same set with a cell list built for this call: the box
 * is cut into floor(L_d / rc) >= 3 bins per axis (bins at least rc wide), so
 * the two atoms of a pair closer than rc sit in the same or adjacent bins,
 * and the 27 bins around an atom are distinct; with fewer than 3 bins along
 * an axis, all pairs are tested. */
static int64_t or_pairs(const double* x, int32_t n, const double* box, double rc, int method,
                        int32_t** pairs)
{
    int32_t nb[3];
    int use_bins = method == 1;
    for (int k = 0; k < 3; ++k) {
        nb[k] = (int32_t)floor(box[k] / rc);
        if (nb[k] < 3) use_bins = 0;
    }
    int64_t cap = 1024, cnt = 0;
    int32_t* out = (int32_t*)malloc(sizeof(int32_t) * 2 * cap);
    if (!use_bins) {
        for (int32_t i = 0; i < n; ++i)
            for (int32_t j = i + 1; j < n; ++j) {
                double d[3];
                or_min_image(&x[3 * i], &x[3 * j], box, d);
                if (sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]) >= rc) continue;
                if (cnt == cap) { cap *= 2; out = (int32_t*)realloc(out, sizeof(int32_t) * 2 * cap); }
                out[2 * cnt] = i; out[2 * cnt + 1] = j; ++cnt;
            }
        *pairs = out;
        return cnt;
    }
    /* bin of every atom, then the atoms of each bin in ascending index */
    int64_t nbins = (int64_t)nb[0] * nb[1] * nb[2];
    int32_t* bin = (int32_t*)malloc(sizeof(int32_t) * (n > 0 ? n : 1));
    int32_t* start = (int32_t*)calloc((size_t)nbins + 1, sizeof(int32_t));
    int32_t* list = (int32_t*)malloc(sizeof(int32_t) * (n > 0 ? n : 1));
    for (int32_t i = 0; i < n; ++i) {
        int32_t c[3];
        for (int k = 0; k < 3; ++k) {
            c[k] = (int32_t)floor(or_wrap(x[3 * i + k], box[k]) / (box[k] / nb[k]));
            if (c[k] >= nb[k]) c[k] = nb[k] - 1;
            if (c[k] < 0) c[k] = 0;
        }
        bin[i] = (c[2] * nb[1] + c[1]) * nb[0] + c[0];
        start[bin[i] + 1] += 1;
    }
    for (int64_t b = 0; b < nbins; ++b) start[b + 1] += start[b];
    int32_t* fill = (int32_t*)malloc(sizeof(int32_t) * (size_t)(nbins > 0 ? nbins : 1));
    for (int64_t b = 0; b < nbins; ++b) fill[b] = start[b];
    for (int32_t i = 0; i < n; ++i) list[fill[bin[i]]++] = i;
    free(fill);
    for (int32_t i = 0; i < n; ++i) {
        int32_t bx = bin[i] % nb[0], by = (bin[i] / nb[0]) % nb[1], bz = bin[i] / (nb[0] * nb[1]);
        for (int dz = -1; dz <= 1; ++dz)
            for (int dy = -1; dy <= 1; ++dy)
                for (int dx = -1; dx <= 1; ++dx) {
                    int32_t ox = (bx + dx + nb[0]) % nb[0], oy = (by + dy + nb[1]) % nb[1];
                    int32_t oz = (bz + dz + nb[2]) % nb[2];
                    int32_t b = (oz * nb[1] + oy) * nb[0] + ox;
                    for (int32_t q = start[b]; q < start[b + 1]; ++q) {
                        int32_t j = list[q];
                        if (j <= i) continue;
                        double d[3];
                        or_min_image(&x[3 * i], &x[3 * j], box, d);
                        if (sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]) >= rc) continue;
                        if (cnt == cap) { cap *= 2; out = (int32_t*)realloc(out, sizeof(int32_t) * 2 * cap); }
                        out[2 * cnt] = i; out[2 * cnt + 1] = j; ++cnt;
                    }
                }
    }
    free(bin); free(start); free(list);
    *pairs = out;
    return cnt;
}

/* Morse forces (into F, [n][3]) and the shifted pair energy of positions x,
 * over the pairs found by `method` (see or_pairs).  Pure function of its
 * arguments: also the test hook that pins the cell list to all pairs. */
double or_pair_forces(const double* x, int32_t n, const double* box, const double* morse, int method,
                      double* F)
{
    int32_t* pairs = NULL;
    int64_t np = or_pairs(x, n, box, morse[3], method, &pairs);
    double pe = 0.0;
    if (F) memset(F, 0, sizeof(double) * 3 * n);
    for (int64_t q = 0; q < np; ++q) {
        int32_t i = pairs[2 * q], j = pairs[2 * q + 1];
        double d[3];
        or_min_image(&x[3 * i], &x[3 * j], box, d);
        double r = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
        pe += or_morse_energy(morse, r);
        if (!F) continue;
        double f = or_morse_force(morse, r);   /* force on j along d/r */
        for (int k = 0; k < 3; ++k) {
            double fk = f * d[k] / r;
            F[3 * j + k] += fk;
            F[3 * i + k] -= fk;
        }
    }
    free(pairs);
    return pe;
}

/* The system's forces use the cell list (the same pair set as all pairs). */
static void or_compute_forces(or_system* S)
{
    (void)or_pair_forces(S->x, S->n, S->d.box, S->d.morse, 1, S->F);
}

/* Total pair energy of the current positions (eV). */
static double or_potential_energy(const or_system* S)
{
    return or_pair_forces(S->x, S->n, S->d.box, S->d.morse, 1, NULL);
}

/* ------------------------------------------------------------- spin update */

/* Radial exchange function of a bond of shell sh at distance r (Methods A;
 * the re-derivation of the radial exchange function):
 * J(r) = 4 J1 x (1 - J2 x) exp(-x), x = (r / J3)^2, and its derivative
 * dJ/dr = dJ/dx 2 r / J3^2 with dJ/dx = 4 J1 exp(-x) (1 - x - J2 x (2 - x)). */
static double or_radial_J(const or_system* S, int32_t sh, double J1, double r)
{
    double J2 = S->d.exch_r[sh][0], J3 = S->d.exch_r[sh][1];
    double x = (r / J3) * (r / J3);
    return 4.0 * J1 * x * (1.0 - J2 * x) * exp(-x);
}

static double or_radial_dJdr(const or_system* S, int32_t sh, double J1, double r)
{
    double J2 = S->d.exch_r[sh][0], J3 = S->d.exch_r[sh][1];
    double x = (r / J3) * (r / J3);
    double dJdx = 4.0 * J1 * exp(-x) * (1.0 - x - J2 * x * (2.0 - x));
    return dJdx * 2.0 * r / (J3 * J3);
}

/* Coupling of neighbour entry q of atom i: the constant, or the radial
 * function at the pair's current minimum-image distance. */
static double or_bond_J(const or_system* S, int32_t i, int32_t q)
{
    if (!S->d.exch_radial) return S->nbr_J[q];
    double d[3];
    or_min_image(&S->x[3 * i], &S->x[3 * S->nbr_j[q]], S->d.box, d);
    double r = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
    return or_radial_J(S, S->nbr_sh[q], S->nbr_J[q], r);
}

/* Exchange field sum_j J_ij s_j (eV) from the current spins. */
static void or_exchange_sum(const or_system* S, int32_t i, double h[3])
{
    h[0] = h[1] = h[2] = 0.0;
    for (int32_t q = S->nbr_off[i]; q < S->nbr_off[i + 1]; ++q) {
        int32_t j = S->nbr_j[q];
        double J = or_bond_J(S, i, q);
        for (int k = 0; k < 3; ++k) h[k] += J * S->s[3 * j + k];
    }
}

/* Exchange force on every atom (radial exchange only; zero otherwise):
 * F_i = -grad_i of -sum_bonds J(r_ij) s_i.s_j = sum_j (s_i.s_j) dJ/dr (x_i - x_j)/r,
 * each bond entered from both of its atoms. */
static void or_exchange_forces(const or_system* S, double* F)
{
    memset(F, 0, sizeof(double) * 3 * S->n);
    if (!S->d.exch_radial) return;
    for (int32_t i = 0; i < S->n; ++i)
        for (int32_t q = S->nbr_off[i]; q < S->nbr_off[i + 1]; ++q) {
            int32_t j = S->nbr_j[q];
            double d[3];
            or_min_image(&S->x[3 * i], &S->x[3 * j], S->d.box, d);     /* x_j - x_i */
            double r = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
            double ss = S->s[3 * i] * S->s[3 * j] + S->s[3 * i + 1] * S->s[3 * j + 1] +
                        S->s[3 * i + 2] * S->s[3 * j + 2];
            double c = ss * or_radial_dJdr(S, S->nbr_sh[q], S->nbr_J[q], r) / r;
            for (int k = 0; k < 3; ++k) F[3 * i + k] -= c * d[k];
        }
}

/* Exact solution of Eq. (1) over a time tau for a precession vector omega
 * (rad/ps) held constant.  Writing theta for the angle between s and the
 * unit axis e = omega/|omega|: the transverse part rotates right-handedly
 * about e by phi = |omega| tau / (1 + alpha^2), and the damping term makes
 * tan(theta/2) decay by exp(-alpha phi).  Reduces to a rotation when
 * alpha = 0.  The result is renormalised to unit length. */
void or_llg_exact_flow(double s[3], const double w[3], double alpha, double tau)
{
    double wn = sqrt(w[0] * w[0] + w[1] * w[1] + w[2] * w[2]);
    if (wn == 0.0) return;
    double e[3] = {w[0] / wn, w[1] / wn, w[2] / wn};
    double u = s[0] * e[0] + s[1] * e[1] + s[2] * e[2];
    double sp[3] = {s[0] - u * e[0], s[1] - u * e[1], s[2] - u * e[2]};
    double spn = sqrt(sp[0] * sp[0] + sp[1] * sp[1] + sp[2] * sp[2]);
    if (spn == 0.0) return;                      /* s parallel to the axis */
    double phi = wn * tau / (1.0 + alpha * alpha);
    /* polar angle */
    double theta = atan2(spn, u);
    double theta_new = 2.0 * atan(tan(0.5 * theta) * exp(-alpha * phi));
    /* rotate the transverse unit vector about e by phi */
    double ex[3] = {e[1] * sp[2] - e[2] * sp[1], e[2] * sp[0] - e[0] * sp[2],
                    e[0] * sp[1] - e[1] * sp[0]};
    double c = cos(phi), sn = sin(phi);
    double out[3];
    for (int k = 0; k < 3; ++k) {
        double rot = (c * sp[k] + sn * ex[k]) / spn;
        out[k] = cos(theta_new) * e[k] + sin(theta_new) * rot;
    }
    double on = sqrt(out[0] * out[0] + out[1] * out[1] + out[2] * out[2]);
    for (int k = 0; k < 3; ++k) s[k] = out[k] / on;
}

/* Standard deviation (Tesla) of each Cartesian component of the thermal
 * field of atom i at bath temperature T.  The fluctuation-dissipation
 * theorem for Eq. (1) with a white-noise field gives the variance
 * 2 alpha k_B T / (gamma mu_i mu_B dt) per step (Methods C: the variance
 * carries 1/mu_i, so the amplitude goes as 1/sqrt(mu_i)).  noise_mode 1 is
 * the negative control of Methods C, in which the amplitude instead goes as
 * 1/mu_i (equal to the FDT value at mu_i = mu_ref). */
static double or_noise_sigma(const or_system* S, int32_t i, double T)
{
    if (T <= 0.0 || S->d.alpha == 0.0) return 0.0;
    double var = 2.0 * S->d.alpha * OR_KB * T / (or_gamma() * S->mu[i] * OR_MUB * S->d.dt);
    double sig = sqrt(var);
    if (S->d.noise_mode == 1) sig *= sqrt(S->d.mu_ref / S->mu[i]);
    return sig;
}

/* One spin step: thermal fields drawn once per atom and step (held over the
 * whole step), then the colours are swept forward with half steps and back
 * again, the last colour of the forward sweep and the first of the backward
 * sweep being one update of a full step (two half-step exact flows with the
 * same held field compose to one full-step flow). */
static void or_spin_step(or_system* S)
{
    int32_t n = S->n, C = S->d.n_colours;
    double* xi = (double*)malloc(sizeof(double) * 3 * n);
    for (int32_t i = 0; i < n; ++i) {
        double T = S->Te[or_cell_of(S, &S->x[3 * i])];
        double sig = or_noise_sigma(S, i, T);
        double nu[3];
        or_normals3(S->d.seed, S->d.run_id, (uint32_t)S->ctr_id[i], S->step, 0u, nu);
        for (int k = 0; k < 3; ++k) xi[3 * i + k] = sig * nu[k];
    }
    const double g = or_gamma();
    for (int32_t pass = 0; pass < 2 * C - 1; ++pass) {
        int32_t colour = pass < C ? pass : 2 * C - 2 - pass;
        double tau = (pass == C - 1) ? S->d.dt : 0.5 * S->d.dt;
        for (int32_t i = 0; i < n; ++i) {
            if (S->colour[i] != colour) continue;
            double h[3];
            or_exchange_sum(S, i, h);
            /* uniaxial anisotropy: -dE/ds of E = -K s_z^2 is 2 K s_z along z,
             * from the spin this update starts from */
            h[2] += 2.0 * S->K[i] * S->s[3 * i + 2];
            double w[3];
            for (int k = 0; k < 3; ++k) {
                double H = h[k] / (S->mu[i] * OR_MUB) + S->d.B[k];   /* Tesla */
                w[k] = g * (H + xi[3 * i + k]);
            }
            or_llg_exact_flow(&S->s[3 * i], w, S->d.alpha, tau);
        }
    }
    free(xi);
}

/* ---------------------------------------------------------- lattice update */

/* Velocity Verlet with the spins held at their values after the sweep:
 * half kick, drift (wrapped into the box), new forces, half kick.  The force
 * is the pair force plus, with radial exchange, the bonds' exchange force
 * (S->F keeps the pair force of the current positions). */
static void or_lattice_step(or_system* S)
{
    int32_t n = S->n;
    double dt = S->d.dt;
    double* Fe = (double*)malloc(sizeof(double) * 3 * (n > 0 ? n : 1));
    or_exchange_forces(S, Fe);
    for (int32_t i = 0; i < n; ++i)
        for (int k = 0; k < 3; ++k)
            S->v[3 * i + k] += 0.5 * dt * (S->F[3 * i + k] + Fe[3 * i + k]) / (S->mass[i] * OR_MVV2E);
    for (int32_t i = 0; i < n; ++i)
        for (int k = 0; k < 3; ++k)
            S->x[3 * i + k] = or_wrap(S->x[3 * i + k] + dt * S->v[3 * i + k], S->d.box[k]);
    or_compute_forces(S);
    or_exchange_forces(S, Fe);
    for (int32_t i = 0; i < n; ++i)
        for (int k = 0; k < 3; ++k)
            S->v[3 * i + k] += 0.5 * dt * (S->F[3 * i + k] + Fe[3 * i + k]) / (S->mass[i] * OR_MVV2E);
    free(Fe);
}

/* Electron-phonon exchange as an exact Ornstein-Uhlenbeck step on the
 * velocities at the electron temperature of the atom's cell.  The friction
 * rate Gamma = G_el / (3 n_atoms k_B) gives the same mean power
 * G_el (T_e - T_l) per volume as the textbook two-temperature coupling.
 * The electrons of the cell lose the mean energy the step hands to each of
 * its atoms given the atom's velocity, (1 - c1^2)(3/2 k_B T_e - m v^2 / 2):
 * summed over the cell this is the volumetric coupling with the cell's
 * instantaneous atomic temperature, conserving energy on average without
 * feeding the per-step noise into the (small) electron heat capacity. */
static void or_eph_step(or_system* S)
{
    int32_t n = S->n;
    double vol = S->d.box[0] * S->d.box[1] * S->d.box[2];
    double Gamma = S->d.G_el / (3.0 * ((double)n / vol) * OR_KB);
    double c1 = exp(-Gamma * S->d.dt);
    for (int32_t i = 0; i < n; ++i) {
        int32_t c = or_cell_of(S, &S->x[3 * i]);
        double T = S->Te[c];
        double eta[3];
        or_normals3(S->d.seed, S->d.run_id, (uint32_t)S->ctr_id[i], S->step, 1u, eta);
        double amp = sqrt((1.0 - c1 * c1) * OR_KB * T / (S->mass[i] * OR_MVV2E));
        double vv = 0.0;
        for (int k = 0; k < 3; ++k) {
            double v = S->v[3 * i + k];
            vv += v * v;
            S->v[3 * i + k] = c1 * v + amp * eta[k];
        }
        double ke = 0.5 * S->mass[i] * OR_MVV2E * vv;
        S->dE[c] += (1.0 - c1 * c1) * (1.5 * OR_KB * T - ke);
    }
}

/* Laser power density (eV / (ps Angstrom^3)) at cell-centre height z and
 * time t: a Gaussian pulse of the given FWHM centred on t0. */
static double or_laser(const or_system* S, double zc, double t)
{
    if (S->d.S0 == 0.0 || S->d.fwhm <= 0.0) return 0.0;
    double f = 1.0;
    if (S->d.profile == 1) f = (zc > S->d.box[2] - S->d.depth) ? 1.0 : 0.0;
    double dtl = t - S->d.t0;
    return S->d.S0 * f * exp(-4.0 * log(2.0) * dtl * dtl / (S->d.fwhm * S->d.fwhm));
}

/* Finite-difference two-temperature update of the electron energy density
 * e = gamma_e T_e^2 / 2: n_sub explicit diffusion sub-steps with the
 * periodic 7-point Laplacian, then the laser energy at the mid-step time and
 * the energy handed to the atoms of each cell. */
static int or_ttm_step(or_system* S)
{
    const int32_t* tn = S->d.tn;
    int32_t nc = S->ncell;
    double h[3] = {S->d.box[0] / tn[0], S->d.box[1] / tn[1], S->d.box[2] / tn[2]};
    double Vc = h[0] * h[1] * h[2];
    double ge = S->d.gamma_e;
    double* e = (double*)malloc(sizeof(double) * nc);
    double* lap = (double*)malloc(sizeof(double) * nc);
    for (int32_t c = 0; c < nc; ++c) e[c] = 0.5 * ge * S->Te[c] * S->Te[c];
    double dts = S->d.dt / (S->d.n_sub > 0 ? S->d.n_sub : 1);
    if (S->d.kappa_e != 0.0) {
        for (int32_t sub = 0; sub < S->d.n_sub; ++sub) {
            for (int32_t k = 0; k < tn[2]; ++k)
                for (int32_t j = 0; j < tn[1]; ++j)
                    for (int32_t i = 0; i < tn[0]; ++i) {
                        int32_t c = (k * tn[1] + j) * tn[0] + i;
                        int32_t ip = (k * tn[1] + j) * tn[0] + (i + 1) % tn[0];
                        int32_t im = (k * tn[1] + j) * tn[0] + (i + tn[0] - 1) % tn[0];
                        int32_t jp = (k * tn[1] + (j + 1) % tn[1]) * tn[0] + i;
                        int32_t jm = (k * tn[1] + (j + tn[1] - 1) % tn[1]) * tn[0] + i;
                        int32_t kp = (((k + 1) % tn[2]) * tn[1] + j) * tn[0] + i;
                        int32_t km = (((k + tn[2] - 1) % tn[2]) * tn[1] + j) * tn[0] + i;
                        double T = S->Te[c];
                        lap[c] = (S->Te[ip] - 2.0 * T + S->Te[im]) / (h[0] * h[0]) +
                                 (S->Te[jp] - 2.0 * T + S->Te[jm]) / (h[1] * h[1]) +
                                 (S->Te[kp] - 2.0 * T + S->Te[km]) / (h[2] * h[2]);
                    }
            for (int32_t c = 0; c < nc; ++c) {
                e[c] += dts * S->d.kappa_e * lap[c];
                if (e[c] < 0.0) { free(e); free(lap); return -1; }
                S->Te[c] = sqrt(2.0 * e[c] / ge);
            }
        }
    }
    double tmid = (S->step + 0.5) * S->d.dt;
    for (int32_t k = 0; k < tn[2]; ++k) {
        double zc = (k + 0.5) * h[2];
        double src = or_laser(S, zc, tmid);
        for (int32_t j = 0; j < tn[1]; ++j)
            for (int32_t i = 0; i < tn[0]; ++i) {
                int32_t c = (k * tn[1] + j) * tn[0] + i;
                e[c] += S->d.dt * src - S->dE[c] / Vc;
                if (e[c] < 0.0) { free(e); free(lap); return -1; }
                S->Te[c] = sqrt(2.0 * e[c] / ge);
            }
    }
    free(e);
    free(lap);
    return 0;
}

/* ------------------------------------------------------------------ public */

or_system* or_create(const or_desc* d)
{
    or_system* S = (or_system*)calloc(1, sizeof(or_system));
    S->d = *d;
    int32_t n = d->n;
    S->n = n;
    S->ncell = d->tn[0] * d->tn[1] * d->tn[2];
    S->s = (double*)or_copy(d->s0, sizeof(double) * 3 * n);
    S->x = (double*)or_copy(d->x0, sizeof(double) * 3 * n);
    S->v = (double*)or_copy(d->v0, sizeof(double) * 3 * n);
    S->F = (double*)or_copy(NULL, sizeof(double) * 3 * n);
    S->colour = (int32_t*)or_copy(d->colour, sizeof(int32_t) * n);
    S->ctr_id = (int32_t*)or_copy(d->ctr_id, sizeof(int32_t) * n);
    S->species = (int32_t*)or_copy(d->species, sizeof(int32_t) * n);
    S->nbr_off = (int32_t*)or_copy(d->nbr_off, sizeof(int32_t) * (n + 1));
    int32_t nnz = S->nbr_off[n];
    S->nbr_j = (int32_t*)or_copy(d->nbr_j, sizeof(int32_t) * nnz);
    S->nbr_J = (double*)or_copy(d->nbr_J, sizeof(double) * nnz);
    S->nbr_sh = (int32_t*)or_copy(d->nbr_sh, sizeof(int32_t) * nnz);
    S->mu = (double*)malloc(sizeof(double) * n);
    S->mass = (double*)malloc(sizeof(double) * n);
    S->K = (double*)malloc(sizeof(double) * n);
    for (int32_t i = 0; i < n; ++i) {
        S->mu[i] = d->mu_s[S->species[i]];
        S->mass[i] = d->mass_s[S->species[i]];
        S->K[i] = d->K_s != NULL ? d->K_s[S->species[i]] : 0.0;
        for (int k = 0; k < 3; ++k) S->x[3 * i + k] = or_wrap(S->x[3 * i + k], d->box[k]);
    }
    S->Te = (double*)or_copy(d->Te0, sizeof(double) * S->ncell);
    S->dE = (double*)or_copy(NULL, sizeof(double) * S->ncell);
    /* the description's pointers are not kept */
    S->d.colour = S->d.ctr_id = S->d.species = S->d.nbr_off = S->d.nbr_j = NULL;
    S->d.nbr_J = S->d.x0 = S->d.v0 = S->d.s0 = S->d.Te0 = NULL;
    S->d.nbr_sh = NULL;
    S->d.mu_s = S->d.mass_s = NULL;
    if (d->lattice_live) or_compute_forces(S);
    return S;
}

void or_destroy(or_system* S)
{
    if (!S) return;
    free(S->s); free(S->x); free(S->v); free(S->F); free(S->mu); free(S->mass); free(S->K);
    free(S->colour); free(S->ctr_id); free(S->species); free(S->nbr_off); free(S->nbr_j);
    free(S->nbr_J); free(S->nbr_sh); free(S->Te); free(S->dE);
    free(S);
}

/* One timestep n -> n+1: spins (bath temperature T_e^n of the cell holding
 * x^n), then the lattice, then the electron-phonon step and the electron
 * grid.  Returns 0, or -1 if an electron energy density went negative. */
int or_step(or_system* S, int64_t nsteps)
{
    for (int64_t it = 0; it < nsteps; ++it) {
        if (S->err) return -1;
        or_spin_step(S);
        if (S->d.lattice_live) or_lattice_step(S);
        if (S->d.ttm_mode == 1) {
            memset(S->dE, 0, sizeof(double) * S->ncell);
            if (S->d.lattice_live) or_eph_step(S);
            if (or_ttm_step(S) != 0) { S->err = 1; return -1; }
        } else if (S->d.ttm_mode == 2) {
            /* prescribed stepped profile: every cell at T_e(t_{n+1}) */
            double t = (double)(S->step + 1) * S->d.dt;
            double T = t < S->d.step_end[0] ? S->d.step_T[0]
                     : (t < S->d.step_end[1] ? S->d.step_T[1] : S->d.step_T[2]);
            for (int32_t c = 0; c < S->ncell; ++c) S->Te[c] = T;
        }
        S->step += 1;
    }
    return 0;
}

void or_get_state(const or_system* S, double* x, double* v, double* s, double* F, double* Te)
{
    int32_t n = S->n;
    if (x) memcpy(x, S->x, sizeof(double) * 3 * n);
    if (v) memcpy(v, S->v, sizeof(double) * 3 * n);
    if (s) memcpy(s, S->s, sizeof(double) * 3 * n);
    if (F) memcpy(F, S->F, sizeof(double) * 3 * n);
    if (Te) memcpy(Te, S->Te, sizeof(double) * S->ncell);
}

void or_set_spins(or_system* S, const double* s) { memcpy(S->s, s, sizeof(double) * 3 * S->n); }

/* Exchange forces of the current state ([n][3]; zero without radial exchange). */
void or_get_exchange_forces(const or_system* S, double* F) { or_exchange_forces(S, F); }

/* Replaces the positions (test hook: finite differences of the energy). */
void or_set_positions(or_system* S, const double* x)
{
    for (int32_t i = 0; i < 3 * S->n; ++i) S->x[i] = or_wrap(x[i], S->d.box[i % 3]);
}

int64_t or_get_step(const or_system* S) { return S->step; }

/* Observables of the current state, each from its definition. */
void or_observables(const or_system* S, or_obs* o)
{
    int32_t n = S->n;
    memset(o, 0, sizeof(*o));
    o->step = S->step;
    o->t = S->step * S->d.dt;
    double cnt[4] = {0, 0, 0, 0};
    double num[4] = {0, 0, 0, 0}, den[4] = {0, 0, 0, 0};
    for (int32_t i = 0; i < n; ++i) {
        int32_t sp = S->species[i];
        const double* s = &S->s[3 * i];
        double h[3];
        or_exchange_sum(S, i, h);
        cnt[sp] += 1.0;
        for (int k = 0; k < 3; ++k) {
            o->M[sp][k] += s[k];
            o->m[k] += s[k];
        }
        o->E_ex += -0.5 * (s[0] * h[0] + s[1] * h[1] + s[2] * h[2]);
        o->E_z += -S->mu[i] * OR_MUB * (S->d.B[0] * s[0] + S->d.B[1] * s[1] + S->d.B[2] * s[2]) -
                  S->K[i] * s[2] * s[2];
        double ht[3];
        for (int k = 0; k < 3; ++k) ht[k] = h[k] + S->mu[i] * OR_MUB * S->d.B[k];
        ht[2] += 2.0 * S->K[i] * s[2];
        double cr[3] = {s[1] * ht[2] - s[2] * ht[1], s[2] * ht[0] - s[0] * ht[2],
                        s[0] * ht[1] - s[1] * ht[0]};
        num[sp] += cr[0] * cr[0] + cr[1] * cr[1] + cr[2] * cr[2];
        den[sp] += s[0] * ht[0] + s[1] * ht[1] + s[2] * ht[2];
        const double* v = &S->v[3 * i];
        o->KE += 0.5 * S->mass[i] * OR_MVV2E * (v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
    }
    for (int sp = 0; sp < 4; ++sp) {
        if (cnt[sp] > 0)
            for (int k = 0; k < 3; ++k) o->M[sp][k] /= cnt[sp];
        o->Tspin[sp] = den[sp] != 0.0 ? num[sp] / (2.0 * OR_KB * den[sp]) : 0.0;
    }
    for (int k = 0; k < 3; ++k) o->m[k] /= n;
    o->m_abs = sqrt(o->m[0] * o->m[0] + o->m[1] * o->m[1] + o->m[2] * o->m[2]);
    if (S->d.lattice_live) o->PE = or_potential_energy(S);
    o->Tl = 2.0 * o->KE / (3.0 * n * OR_KB);
    double h[3] = {S->d.box[0] / S->d.tn[0], S->d.box[1] / S->d.tn[1], S->d.box[2] / S->d.tn[2]};
    double Vc = h[0] * h[1] * h[2];
    o->Te_max = 0.0;
    for (int32_t c = 0; c < S->ncell; ++c) {
        double T = S->Te[c];
        o->Te_mean += T / S->ncell;
        if (T > o->Te_max) o->Te_max = T;
        o->E_e += 0.5 * S->d.gamma_e * T * T * Vc;
    }
}
