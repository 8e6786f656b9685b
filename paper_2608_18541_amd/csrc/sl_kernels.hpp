// sl_kernels.hpp -- HIP kernels of one spin-lattice timestep (gfx950).
//
// Every launch covers all active runs of an engine: block b reads
// work[b] = {run, first item} and works on a tile of consecutive items of
// that run, so one run alone and the same run inside a batch execute
// identical arithmetic in identical order (bitwise-equal trajectories).
//
// Per step, in stream order:
//   k_spin_pass  x (2C-1)  colour sweep 0..C-1 (half steps), C-2..0, the
//                          middle colour taking one full step; the launch of
//                          pass 1 also carries the lattice's half kick +
//                          drift, electron-cell id, skin check and binning
//                          (they read no spin, and the cell ids of the new
//                          positions go to the third of three buffers).  In
//                          a merged chunk a step leaves its last pass
//                          (colour 0, half step) to the next step's pass 0,
//                          which applies it before its own: 2C-2 passes per
//                          step; when the chunk is folded, extra blocks of
//                          pass 0 also end the previous step (small electron
//                          grid, bins, flags) while its spin blocks compute
//                          the new T_e of their cells from the same inputs.
//                          In the fused schedule of merged chunks pass 0
//                          carries the kick and pass 1 is k_spin_force,
//                          which also runs k_atom_final's work, for every
//                          step but a chunk's last
//   k_nbr_bin, k_nbr_sort  binning for a rebuild (large engines; exit at
//                          once unless a rebuild is flagged)
//   k_atom_final           Verlet-list rebuild of its own atoms when flagged,
//                          Morse forces, half kick, electron-phonon
//                          Ornstein-Uhlenbeck step and its mean energy per
//                          electron cell, observable partials
//   k_ttm_tile             all explicit electron diffusion sub-steps of a
//                          step in one launch, tiled with halos in LDS (runs
//                          with kappa_e > 0), or
//   k_ttm_diffuse x n_sub  one launch per sub-step when a tile and its halo
//                          do not fit
//   k_grid                 laser source and electron-phonon energy per
//                          cell of large grids
//   k_finalize             one block per run: small grids, the observable
//                          sample, the step counter (in a folded chunk only
//                          after its last step)
// or, for runs small enough to live in LDS, k_persist: one block per run
// advancing many steps in one launch.  A run is initialised (and restored
// from a checkpoint) by k_init_lattice, k_nbr_bin, k_nbr_sort, k_nbr_build,
// k_atom_final and k_finalize in their initialisation phase.
#pragma once

#include "sl_device.hpp"
#include "../../include/spinlattice.h"

namespace sl {

constexpr int kBlock = 256;
constexpr int NQ = 24;      // observable partial sums per wave of 64 atoms
static_assert(NQ % 3 == 0, "samples reduce three quantities at a time");
constexpr int kLdsCells = 2048;   // electron grids up to this size are summed in LDS
constexpr int kSmallGrid = 4096;  // larger electron grids update cell-parallel (k_grid)

// Numerical errors of a run (RunState.err).  ERR_NUMERIC is the watchdog: a
// spin update whose input was not a finite unit vector, or a kick that left a
// non-finite velocity or displacement.  A run with an error stops stepping.
enum { ERR_NEG_E = 1, ERR_BIN = 2, ERR_NBR = 4, ERR_DE = 8, ERR_NUMERIC = 16 };
enum { PHASE_STEP = 0, PHASE_INIT = 1 };

struct RunState {
    int64_t step;
    int64_t target;
    int32_t err;
    int32_t rebuild;
    int64_t n_samples;
    int32_t bad_atom;    // first atom that overflowed a neighbour table (+1), for diagnostics
    int32_t bad_count;
    int64_t bad_step;
    int64_t n_rebuild;   // Verlet-list builds so far, the initial one included
    int32_t max_list;    // longest list built so far
    int32_t bin_over;    // a bin overflowed while binning this step
    int32_t pending;     // the last half step (colour 0) of step `step - 1` is deferred
                         // to the next colour pass 0, which applies it first
    int32_t chunk_done;  // steps of the current folded chunk that have ended
    int32_t neg_at;      // 1 + position in the current folded chunk of the first step
                         // end that met a negative electron energy (0: none)
    int32_t n_rescan;    // bins scanned again by a list build from unsorted bins
                         // (more than kBinKeep accepted atoms)
    int32_t force_done;  // force blocks that have finished a colour pass carrying the
                         // force kernel on a list-rebuild step (the last one clears the
                         // bins and the rebuild flags, then this count)
};

// Wrapped absolute position of an atom, padded to a 16/32-byte vector so a
// neighbour's position is one load.
template <typename T> struct alignas(4 * sizeof(T)) Pos4 {
    T x, y, z, w;
};

template <typename T> struct RunDev {
    Geom g;
    int32_t lattice, n, n_species, n_shells, live, ttm_mode, obs_every, obs_cap;
    int32_t aniso;       // some species has a uniaxial anisotropy (Kd, kan below)
    int32_t noisy;       // some species has a thermal field (sig > 0)
    int32_t bin_step;    // 1: atoms are binned by the kick every step, 0: only for a rebuild
    int32_t eta_drawn;   // 1: the kick draws the electron-phonon normals into eta for the
                         // force kernel (which then gives an atom several lanes)
    uint32_t seed, run_id;
    T a, box[3], inv_box[3];
    T alpha, dt, tau_half, inv1pa2, gam;
    T B[3];
    T inv_mumb[4];       // 1 / (mu mu_B), T/eV
    T sig[4];            // thermal-field std per sqrt(K), T
    T J[2][4][4];        // eV
    T hdtm[4];           // dt / (2 m) in A/ps per eV/A
    T ou_c1, ou_amp[4];  // exp(-Gamma dt); sqrt((1 - c1^2) k_B / m) per sqrt(K)
    double ou_1mc2;      // 1 - c1^2
    T m_e[4];            // m in eV ps^2 / A^2
    T mD, ma, mr0, rc2, Vc;
    T mk1, mk0;          // single precision: exp(-a (r - r0)) = exp2(mk1 r + mk0)
    T skin_half2, rlist2;
    double mumb[4];      // mu mu_B, eV/T
    double Bd[3];
    double cnt[4];       // sites per species
    // electron grid
    int32_t tn[3], ncell, n_sub, profile;
    int32_t dtile[3], dntile[3];     // diffusion tiles (cells per axis, tiles per axis);
                                     // dtile[0] == 0: one launch per sub-step instead
    double th[3], gamma_e, kappa_e, S0, t0, fwhm, Vcell, depth, dtd;
    double dcoef[3];     // (dt / n_sub) kappa_e / h_d^2 per axis
    double two_ge;       // 2 / gamma_e
    // neighbour bins
    int32_t nbin[3], nbins, bin_cap, max_nbr;
    T binw[3];
    // device arrays
    T *sx, *sy, *sz, *ux, *uy, *uz, *vx, *vy, *vz, *fx, *fy, *fz, *rx, *ry, *rz;
    Pos4<T>* pos;                    // wrap(ideal site + u), refreshed by k_kick_drift
    int8_t* species;
    uint16_t* cellb[3];              // electron-cell id of x^n in cellb[n mod 3]
    int32_t *nbr, *nbr_n;
    int32_t *bin_n, *bin_atoms;      // [nbins], [nbins][bin_cap]
    double *Te, *ee, *Te_alt;        // T_e, energy density, diffusion ping-pong buffer
    unsigned long long* dE;
    unsigned long long* dE_alt;      // second electron-phonon sum buffer (folded chunks)
    double* partial;
    int32_t n_part;
    sl_obs* ring;
    RunState* st;
    int32_t* any_rebuild;            // engine-wide: a run flagged a list rebuild this step
    T* eta;                          // [3][n]: the step's electron-phonon normals (live
                                     // runs), drawn by the kick for the force kernel
    // uniaxial anisotropy along z per species (energy -K s_z^2), kept last so
    // that the fields every kernel reads keep their places
    double Kd[4];                    // K, eV
    T kan[4];                        // its field per unit s_z, 2 K / (mu mu_B), T
    double stT[3], stEnd[2];         // stepped T_e profile (grid mode 2): K, ps
    // radial exchange: J[shell] holds the amplitudes J1 of
    // J(r) = J1 4 x (1 - J2 x) e^{-x}, x = (r / J3)^2, per shell
    int32_t radial;
    T rJ2[2], rinvJ3sq[2];           // J2 and 1 / J3^2 per shell
};

// ------------------------------------------------------- memory access
// Element i of a global array through its base pointer and a 32-bit byte
// offset: with a wave-uniform base the load or store is issued with the base
// in scalar registers and one 32-bit vector offset per lane.  Every array
// read this way is below 4 GiB (the host limits the atom count).
#define SL_GLOBAL __attribute__((address_space(1)))
#define SL_LDS __attribute__((address_space(3)))

template <typename X> __device__ __forceinline__ X gld(const X* base, uint32_t i)
{
    return *(const SL_GLOBAL X*)((const SL_GLOBAL char*)base + i * (uint32_t)sizeof(X));
}
template <typename X> __device__ __forceinline__ void gst(X* base, uint32_t i, X v)
{
    *(SL_GLOBAL X*)((SL_GLOBAL char*)base + i * (uint32_t)sizeof(X)) = v;
}

// positions move as one 16- or 32-byte vector
template <typename T> struct Vec4 {
    typedef T type __attribute__((ext_vector_type(4)));
};
template <typename T> __device__ __forceinline__ Pos4<T> gld(const Pos4<T>* base, uint32_t i)
{
    typedef typename Vec4<T>::type V4;
    const V4 v = *(const SL_GLOBAL V4*)((const SL_GLOBAL char*)base + i * (uint32_t)sizeof(Pos4<T>));
    return Pos4<T>{v.x, v.y, v.z, v.w};
}
template <typename T> __device__ __forceinline__ void gst(Pos4<T>* base, uint32_t i, Pos4<T> p)
{
    typedef typename Vec4<T>::type V4;
    V4 v = {p.x, p.y, p.z, p.w};
    *(SL_GLOBAL V4*)((SL_GLOBAL char*)base + i * (uint32_t)sizeof(Pos4<T>)) = v;
}
template <typename T> __device__ __forceinline__ Pos4<T> sld(const Pos4<T>* base, uint32_t i)
{
    typedef typename Vec4<T>::type V4;
    const V4 v = ((const SL_LDS V4*)base)[i];
    return Pos4<T>{v.x, v.y, v.z, v.w};
}
template <typename T> __device__ __forceinline__ void sst(Pos4<T>* base, uint32_t i, Pos4<T> p)
{
    typedef typename Vec4<T>::type V4;
    V4 v = {p.x, p.y, p.z, p.w};
    ((SL_LDS V4*)base)[i] = v;
}
template <typename X> __device__ __forceinline__ X sld(const X* base, uint32_t i)
{
    return ((const SL_LDS X*)base)[i];
}
template <typename X> __device__ __forceinline__ void sst(X* base, uint32_t i, X v)
{
    ((SL_LDS X*)base)[i] = v;
}

struct InGlobal {
    template <typename X> static __device__ __forceinline__ X ld(const X* b, uint32_t i)
    {
        return gld(b, i);
    }
    template <typename X> static __device__ __forceinline__ void st(X* b, uint32_t i, X v)
    {
        gst(b, i, v);
    }
};
struct InLds {
    template <typename X> static __device__ __forceinline__ X ld(const X* b, uint32_t i)
    {
        return sld(b, i);
    }
    template <typename X> static __device__ __forceinline__ void st(X* b, uint32_t i, X v)
    {
        sst(b, i, v);
    }
};

// ----------------------------------------------------------- views
// Where the hot arrays of a run live while a kernel works on it: the run's
// global arrays (the multi-kernel step) or copies in LDS (the persistent
// per-run kernel; positions there too when they fit).  Every per-site,
// per-atom and per-cell computation below takes a view, so both executors
// run literally the same arithmetic.
template <typename T, typename M, typename P> struct View {
    using Mem = M;      // spins, species, cell ids, T_e, observable rows
    using PosMem = P;   // wrapped positions
    T *sx, *sy, *sz;
    const int8_t* species;
    uint16_t* cell;
    Pos4<T>* pos;
    double* Te;
    double* partial;
};

template <typename T> using GView = View<T, InGlobal, InGlobal>;

// The cell-id buffer of x^n.  Three buffers: a launch that drifts the atoms
// to x^{n+1} may run beside colour passes that still read the cells of x^n
// and x^{n-1}.
__host__ __device__ inline int cell_slot(int64_t n)
{
    const int r = (int)(n % 3);
    return r < 0 ? r + 3 : r;
}

// View of the run's global arrays with the electron-cell ids of x^n.
template <typename T> __device__ inline GView<T> global_view(const RunDev<T>& R, int64_t n)
{
    return GView<T>{R.sx, R.sy, R.sz, R.species, R.cellb[cell_slot(n)], R.pos, R.Te, R.partial};
}

template <typename T, typename VW>
__device__ __forceinline__ int species_of(const RunDev<T>& R, const VW& V, uint32_t idx)
{
    return R.n_species > 1 ? (int)VW::Mem::ld(V.species, idx) : 0;
}

// One of four per-species values by the bits of k (0..3): two levels of
// register selects, no branches.
template <typename T> __device__ __forceinline__ T select4(int k, T a, T b, T c, T d)
{
    const T ab = (k & 1) ? b : a;
    const T cd = (k & 1) ? d : c;
    return (k & 2) ? cd : ab;
}

// Offsets, inside one colour block, of the sites around cell (x, y, z):
// the half-x index of x-1, x, x+1 and the row (y) and plane (z) offsets of
// the three neighbouring rows and planes, periodic.  A neighbour at
// (x', y', z') of colour k' sits at k' H + xh(x') + row(y') + plane(z').
struct Around {
    uint32_t xm, x0, xp, ym, y0, yp, zm, z0, zp;
};

__device__ __forceinline__ Around around(const Geom& g, uint32_t x, uint32_t xh, uint32_t y,
                                         uint32_t z)
{
    const uint32_t Lxh = (uint32_t)g.Lxh, Ly = (uint32_t)g.Ly, Lz = (uint32_t)g.Lz;
    const uint32_t row = Lxh, plane = Lxh * Ly;
    Around a;
    a.x0 = xh;
    if (g.par) {
        // x = 2 xh + parity: x - 1 leaves the pair when x is even, x + 1 when odd
        a.xm = (x & 1u) ? xh : (xh == 0 ? Lxh - 1 : xh - 1);
        a.xp = (x & 1u) ? (xh == Lxh - 1 ? 0 : xh + 1) : xh;
    } else {
        // full rows (fcc): x itself
        a.xm = xh == 0 ? Lxh - 1 : xh - 1;
        a.xp = xh == Lxh - 1 ? 0 : xh + 1;
    }
    a.y0 = __umul24(y, row);
    a.ym = y == 0 ? __umul24(Ly - 1, row) : a.y0 - row;
    a.yp = y == Ly - 1 ? 0 : a.y0 + row;
    a.z0 = __umul24(z, plane);
    a.zm = z == 0 ? __umul24(Lz - 1, plane) : a.z0 - plane;
    a.zp = z == Lz - 1 ? 0 : a.z0 + plane;
    return a;
}

// Exchange sum h = sum_j J_ij s_j (eV) over the neighbour shells of the
// site of colour k at (x, y, z).  Neighbour colours follow from k alone
// (uniform over a colour pass), so each neighbour is one offset into the
// spin arrays of its colour.  All loads are issued before the arithmetic;
// the coupling J[shell][sp][sj] is selected in registers.
//   simple cubic: the 6 sites at +-a along an axis;
//   bcc: first shell the 8 sites of the other basis at (+-a/2)^3 in the
//   order (x0|x1, y0|y1, z0|z1) with x fastest, then the 6 second-shell
//   sites of the same basis at -x, +x, -y, +y, -z, +z;
//   fcc: the 12 sites at (+-a/2, +-a/2, 0) and its permutations, four in
//   each other sublattice b': along the two axes on which b and b' differ in
//   their half shifts the neighbour lies half a constant either way (the
//   same cell and the one below when b is not shifted there, the same cell
//   and the one above when it is), on the third axis in the same cell.
template <int LAT> struct Bonds {
    static constexpr int NB = LAT == SL_LATTICE_SC ? 6 : (LAT == SL_LATTICE_FCC ? 12 : 14);
    uint32_t col[NB], off[NB];   // neighbour q: colour block and offset inside it
    int sh[NB];                  // its shell
    int nn;                      // bonds in use (bcc: 8 with one shell)
};

template <int LAT, typename T>
__device__ __forceinline__ Bonds<LAT> bond_list(const RunDev<T>& R, int k, const Around& a)
{
    constexpr int NN = Bonds<LAT>::NB;
    Bonds<LAT> B;
    const int p = k & 1;
    if (LAT == SL_LATTICE_SC) {
        B.nn = 6;
        const uint32_t o[6] = {a.xm + a.y0 + a.z0, a.xp + a.y0 + a.z0, a.x0 + a.ym + a.z0,
                               a.x0 + a.yp + a.z0, a.x0 + a.y0 + a.zm, a.x0 + a.y0 + a.zp};
#pragma unroll
        for (int q = 0; q < NN; ++q) {
            B.col[q] = (uint32_t)(1 - p);
            B.off[q] = o[q];
            B.sh[q] = 0;
        }
    } else if (LAT == SL_LATTICE_FCC) {
        B.nn = 12;
        const uint32_t hb = basis_half_bits(4, k);
        // per axis: [0] and [1] the two cells of a shifted axis, [2] the same cell
        const uint32_t X[3] = {(hb & 1u) ? a.x0 : a.xm, (hb & 1u) ? a.xp : a.x0, a.x0};
        const uint32_t Y[3] = {(hb & 2u) ? a.y0 : a.ym, (hb & 2u) ? a.yp : a.y0, a.y0};
        const uint32_t Z[3] = {(hb & 4u) ? a.z0 : a.zm, (hb & 4u) ? a.zp : a.z0, a.z0};
#pragma unroll
        for (int q = 0; q < NN; ++q) {
            const int t = q >> 2, u = q & 3;
            const int bp = t < k ? t : t + 1;                 // the other sublattice
            const uint32_t d = hb ^ basis_half_bits(4, bp);   // its two shifted axes
            const int ax = d & 1u, ay = (d >> 1) & 1u, az = (d >> 2) & 1u;
            const int sx = ax ? (u & 1) : 2;
            const int sy = ay ? (ax ? (u >> 1) & 1 : u & 1) : 2;
            const int sz = az ? (u >> 1) & 1 : 2;
            B.col[q] = (uint32_t)bp;
            B.off[q] = X[sx] + Y[sy] + Z[sz];
            B.sh[q] = 0;
        }
    } else {
        B.nn = R.n_shells > 1 ? 14 : 8;
        const int b = k >> 1;
        const uint32_t X[2] = {b == 0 ? a.xm : a.x0, b == 0 ? a.x0 : a.xp};
        const uint32_t Y[2] = {b == 0 ? a.ym : a.y0, b == 0 ? a.y0 : a.yp};
        const uint32_t Z[2] = {b == 0 ? a.zm : a.z0, b == 0 ? a.z0 : a.zp};
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const int mx = q & 1, my = (q >> 1) & 1, mz = q >> 2;
            // cell shift sum is mx+my+mz (b = 1) or that minus 3 (b = 0)
            B.col[q] = (uint32_t)(2 * (1 - b) + ((p + mx + my + mz + (1 - b)) & 1));
            B.off[q] = X[mx] + Y[my] + Z[mz];
            B.sh[q] = 0;
        }
        const uint32_t o2[6] = {a.xm + a.y0 + a.z0, a.xp + a.y0 + a.z0, a.x0 + a.ym + a.z0,
                                a.x0 + a.yp + a.z0, a.x0 + a.y0 + a.zm, a.x0 + a.y0 + a.zp};
#pragma unroll
        for (int q = 8; q < NN; ++q) {
            B.col[q] = (uint32_t)(2 * b + (1 - p));
            B.off[q] = o2[(q - 8) % 6];
            B.sh[q] = 1;
        }
    }
    return B;
}

// Radial exchange (Methods A and the re-derivation of the radial exchange
// function): a bond's coupling is its amplitude J1 times
// f(x) = 4 x (1 - J2 x) e^{-x}, x = (r / J3)^2, at the bond's current
// minimum-image length r (J2, J3 per shell); (1/r) df/dr = 2 g(x) / J3^2 with
// g(x) = df/dx = 4 e^{-x} (1 - x - J2 x (2 - x)).
template <typename T> __device__ __forceinline__ T radial_f(const RunDev<T>& R, int sh, T r2)
{
    const T x = r2 * R.rinvJ3sq[sh];
    return T(4) * x * (T(1) - R.rJ2[sh] * x) * expo(-x);
}
template <typename T> __device__ __forceinline__ T radial_dfr(const RunDev<T>& R, int sh, T r2)
{
    const T x = r2 * R.rinvJ3sq[sh];
    const T g = T(4) * expo(-x) * (T(1) - x - R.rJ2[sh] * x * (T(2) - x));
    return T(2) * R.rinvJ3sq[sh] * g;
}

template <typename T, typename VW>
__device__ __forceinline__ V3<T> separation(const RunDev<T>& R, const VW& V, const Pos4<T>& pi,
                                            uint32_t j);

// h = sum_q J_q s_q over NN neighbour spins already loaded, in bond order:
// the coupling of bond q by its shell sh[q] (and the neighbour's species
// sj[q]; times the radial factor fr[q] with radial exchange).  Every colour
// pass sums the field here, whichever memory its neighbours came from.
template <typename T, bool MULTI, bool RADIAL, int NN>
__device__ __forceinline__ V3<T> exchange_accum(const RunDev<T>& R, const int* sh, const T* ax,
                                                const T* ay, const T* az, const int* sj,
                                                const T* fr, int sp)
{
    T row[2][4];
#pragma unroll
    for (int s2 = 0; s2 < 2; ++s2)
#pragma unroll
        for (int t = 0; t < 4; ++t)
            row[s2][t] = MULTI ? select4(sp, R.J[s2][0][t], R.J[s2][1][t], R.J[s2][2][t], R.J[s2][3][t])
                               : R.J[s2][0][0];
    V3<T> h{T(0), T(0), T(0)};
#pragma unroll
    for (int q = 0; q < NN; ++q) {
        T Jv = !MULTI ? row[sh[q]][0]
               : sh[q] == 0 ? select4(sj[q], row[0][0], row[0][1], row[0][2], row[0][3])
                            : select4(sj[q], row[1][0], row[1][1], row[1][2], row[1][3]);
        if constexpr (RADIAL) Jv *= fr[q];
        h.x += Jv * ax[q];
        h.y += Jv * ay[q];
        h.z += Jv * az[q];
    }
    return h;
}

// The exchange sum over the first NN bonds of B (a compile-time count, so
// that no term is selected per lane).
template <typename T, typename VW, int LAT, bool MULTI, bool RADIAL, int NN>
__device__ __forceinline__ V3<T> exchange_sum_n(const RunDev<T>& R, const VW& V, int k, const Around& a,
                                                const Bonds<LAT>& B, int sp)
{
    using M = typename VW::Mem;
    const uint32_t H = (uint32_t)R.g.H;
    T ax[NN], ay[NN], az[NN];
    int sj[NN];
#pragma unroll
    for (int q = 0; q < NN; ++q) {
        const uint32_t cb = B.col[q] * H;
        ax[q] = M::ld(V.sx + cb, B.off[q]);
        ay[q] = M::ld(V.sy + cb, B.off[q]);
        az[q] = M::ld(V.sz + cb, B.off[q]);
        sj[q] = MULTI ? (int)M::ld(V.species + cb, B.off[q]) : 0;
    }
    T fr[NN];
    if constexpr (RADIAL) {
        const Pos4<T> pi = VW::PosMem::ld(V.pos, (uint32_t)k * H + a.x0 + a.y0 + a.z0);
#pragma unroll
        for (int q = 0; q < NN; ++q) {
            const V3<T> d = separation(R, V, pi, B.col[q] * H + B.off[q]);
            fr[q] = radial_f(R, B.sh[q], d.x * d.x + d.y * d.y + d.z * d.z);
        }
    }
    return exchange_accum<T, MULTI, RADIAL, NN>(R, B.sh, ax, ay, az, sj, fr, sp);
}

template <typename T, typename VW, int LAT, bool MULTI, bool RADIAL = false>
__device__ __forceinline__ V3<T> exchange_sum_t(const RunDev<T>& R, const VW& V, int k, const Around& a,
                                                int sp)
{
    const Bonds<LAT> B = bond_list<LAT>(R, k, a);
    // bcc with one shell uses the first 8 bonds (a branch uniform per run)
    if constexpr (LAT == SL_LATTICE_BCC) {
        if (B.nn < Bonds<LAT>::NB) return exchange_sum_n<T, VW, LAT, MULTI, RADIAL, 8>(R, V, k, a, B, sp);
    }
    return exchange_sum_n<T, VW, LAT, MULTI, RADIAL, Bonds<LAT>::NB>(R, V, k, a, B, sp);
}

// The radial bonds' force on the atom at site (k, a) with spin s and wrapped
// position pi: minus the gradient of -sum_j J(r_ij) s.s_j, i.e.
// F = -sum_j (s . s_j) J1_ij (1/r) df/dr (x_j - x_i).
template <typename T, typename VW, int LAT>
__device__ __forceinline__ V3<T> exchange_force_t(const RunDev<T>& R, const VW& V, int k, const Around& a,
                                                  int sp, const V3<T>& s, const Pos4<T>& pi)
{
    using M = typename VW::Mem;
    constexpr int NN = Bonds<LAT>::NB;
    const uint32_t H = (uint32_t)R.g.H;
    const Bonds<LAT> B = bond_list<LAT>(R, k, a);
    V3<T> F{T(0), T(0), T(0)};
#pragma unroll
    for (int q = 0; q < NN; ++q) {
        if (q < B.nn) {
            const uint32_t j = B.col[q] * H + B.off[q];
            const T sx = M::ld(V.sx, j), sy = M::ld(V.sy, j), sz = M::ld(V.sz, j);
            const int sj = (int)M::ld(V.species, j);
            const V3<T> d = separation(R, V, pi, j);
            const T J1 = B.sh[q] == 0 ? select4(sp, select4(sj, R.J[0][0][0], R.J[0][0][1], R.J[0][0][2], R.J[0][0][3]),
                                                select4(sj, R.J[0][1][0], R.J[0][1][1], R.J[0][1][2], R.J[0][1][3]),
                                                select4(sj, R.J[0][2][0], R.J[0][2][1], R.J[0][2][2], R.J[0][2][3]),
                                                select4(sj, R.J[0][3][0], R.J[0][3][1], R.J[0][3][2], R.J[0][3][3]))
                                      : select4(sp, select4(sj, R.J[1][0][0], R.J[1][0][1], R.J[1][0][2], R.J[1][0][3]),
                                                select4(sj, R.J[1][1][0], R.J[1][1][1], R.J[1][1][2], R.J[1][1][3]),
                                                select4(sj, R.J[1][2][0], R.J[1][2][1], R.J[1][2][2], R.J[1][2][3]),
                                                select4(sj, R.J[1][3][0], R.J[1][3][1], R.J[1][3][2], R.J[1][3][3]));
            const T c = (s.x * sx + s.y * sy + s.z * sz) * J1 *
                        radial_dfr(R, B.sh[q], d.x * d.x + d.y * d.y + d.z * d.z);
            F.x -= c * d.x;
            F.y -= c * d.y;
            F.z -= c * d.z;
        }
    }
    return F;
}

// Dispatch on the run's lattice and species count (uniform per run); runs
// with radial exchange take the species-resolved instantiation.
template <typename T, typename VW, bool RADIAL_OK = true>
__device__ __forceinline__ V3<T> exchange_sum(const RunDev<T>& R, const VW& V, int k, const Around& a,
                                              int sp)
{
    if (RADIAL_OK && R.radial) {
        if (R.lattice == SL_LATTICE_SC) return exchange_sum_t<T, VW, SL_LATTICE_SC, true, true>(R, V, k, a, sp);
        if (R.lattice == SL_LATTICE_FCC) return exchange_sum_t<T, VW, SL_LATTICE_FCC, true, true>(R, V, k, a, sp);
        return exchange_sum_t<T, VW, SL_LATTICE_BCC, true, true>(R, V, k, a, sp);
    }
    if (R.lattice == SL_LATTICE_SC)
        return R.n_species > 1 ? exchange_sum_t<T, VW, SL_LATTICE_SC, true>(R, V, k, a, sp)
                               : exchange_sum_t<T, VW, SL_LATTICE_SC, false>(R, V, k, a, sp);
    if (R.lattice == SL_LATTICE_FCC)
        return R.n_species > 1 ? exchange_sum_t<T, VW, SL_LATTICE_FCC, true>(R, V, k, a, sp)
                               : exchange_sum_t<T, VW, SL_LATTICE_FCC, false>(R, V, k, a, sp);
    return R.n_species > 1 ? exchange_sum_t<T, VW, SL_LATTICE_BCC, true>(R, V, k, a, sp)
                           : exchange_sum_t<T, VW, SL_LATTICE_BCC, false>(R, V, k, a, sp);
}

template <typename T, typename VW>
__device__ __forceinline__ V3<T> exchange_force(const RunDev<T>& R, const VW& V, int k, const Around& a,
                                                int sp, const V3<T>& s, const Pos4<T>& pi)
{
    if (R.lattice == SL_LATTICE_SC) return exchange_force_t<T, VW, SL_LATTICE_SC>(R, V, k, a, sp, s, pi);
    if (R.lattice == SL_LATTICE_FCC) return exchange_force_t<T, VW, SL_LATTICE_FCC>(R, V, k, a, sp, s, pi);
    return exchange_force_t<T, VW, SL_LATTICE_BCC>(R, V, k, a, sp, s, pi);
}

// sqrt of a cell temperature in the storage precision
__device__ __forceinline__ double sqrt_te(double Te, double) { return sqrt(Te); }
__device__ __forceinline__ float sqrt_te(double Te, float) { return __builtin_amdgcn_sqrtf((float)Te); }

// Cell coordinates of offset l inside a colour block.
struct Cell3 {
    uint32_t x, xh, y, z;
};
__device__ __forceinline__ Cell3 cell_of(const Geom& g, int k, uint32_t l)
{
    Cell3 c;
    const uint32_t r = fdiv(l, g.divLxh);
    c.xh = l - __umul24(r, (uint32_t)g.Lxh);
    c.z = fdiv(r, g.divLy);
    c.y = r - __umul24(c.z, (uint32_t)g.Ly);
    c.x = g.par ? 2 * c.xh + (((uint32_t)k + c.y + c.z) & 1u) : c.xh;
    return c;
}

// Ideal position of a site: its cell corner, the basis shift and a quarter
// lattice constant along each axis (so that no ideal site lies on a face of
// the electron grid).
template <typename T> __device__ inline V3<T> ideal_site(const RunDev<T>& R, const Site& s)
{
    const uint32_t hb = basis_half_bits(R.g.nb, s.b);
    const T ox = (hb & 1u) ? T(0.75) : T(0.25);
    const T oy = (hb & 2u) ? T(0.75) : T(0.25);
    const T oz = (hb & 4u) ? T(0.75) : T(0.25);
    return {((T)s.x + ox) * R.a, ((T)s.y + oy) * R.a, ((T)s.z + oz) * R.a};
}

// Minimum image of a separation |d| < 1.5 box: the nearest lattice
// translate, d - box rint(d / box) (one product, one rounding, one fused
// multiply-add; d itself whenever |d| < box / 2).
__device__ inline float min_image(float d, float box, float inv_box)
{
    return __builtin_fmaf(-box, __builtin_rintf(d * inv_box), d);
}
__device__ inline double min_image(double d, double box, double inv_box)
{
    return __builtin_fma(-box, __builtin_rint(d * inv_box), d);
}

// Separation x_j - x_i (minimum image) from the wrapped positions.
template <typename T, typename VW>
__device__ __forceinline__ V3<T> separation(const RunDev<T>& R, const VW& V, const Pos4<T>& pi,
                                            uint32_t j)
{
    const Pos4<T> pj = VW::PosMem::ld(V.pos, j);
    V3<T> d{pj.x - pi.x, pj.y - pi.y, pj.z - pi.z};
    d.x = min_image(d.x, R.box[0], R.inv_box[0]);
    d.y = min_image(d.y, R.box[1], R.inv_box[1]);
    d.z = min_image(d.z, R.box[2], R.inv_box[2]);
    return d;
}

// Morse force factor f = -dV/dr / r at separation^2 r2 (and r).  The
// single-precision path uses the hardware reciprocal square root and
// exponential (exp2 of one fused multiply-add); double precision stays
// correctly rounded.
__device__ inline float morse_f(const RunDev<float>& R, float r2, float* r_out)
{
    const float ir = __builtin_amdgcn_rsqf(r2);
    const float r = r2 * ir;
    *r_out = r;
    const float e1 = __builtin_amdgcn_exp2f(__builtin_fmaf(r, R.mk1, R.mk0));
    return 2.0f * R.ma * R.mD * (e1 * e1 - e1) * ir;
}
__device__ inline double morse_f(const RunDev<double>& R, double r2, double* r_out)
{
    const double r = sqrt(r2);
    *r_out = r;
    const double e1 = exp(-R.ma * (r - R.mr0));
    return 2.0 * R.ma * R.mD * (e1 * e1 - e1) / r;
}

template <typename T> __device__ inline T wrap_box(T x, T L)
{
    return x - L * floor(x / L);
}

// Wrapped position of atom idx from its ideal site and displacement.
template <typename T> __device__ inline V3<T> position(const RunDev<T>& R, const Site& s, uint32_t idx)
{
    V3<T> r = ideal_site(R, s);
    return {wrap_box(r.x + gld(R.ux, idx), R.box[0]), wrap_box(r.y + gld(R.uy, idx), R.box[1]),
            wrap_box(r.z + gld(R.uz, idx), R.box[2])};
}

template <typename T> __device__ inline int electron_cell(const RunDev<T>& R, const V3<T>& p)
{
    int c[3];
    const T pv[3] = {p.x, p.y, p.z};
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        int k = (int)floor((double)pv[d] / R.th[d]);
        c[d] = k < 0 ? 0 : (k >= R.tn[d] ? R.tn[d] - 1 : k);
    }
    return (c[2] * R.tn[1] + c[1]) * R.tn[0] + c[0];
}

template <typename T> __device__ inline int bin_of(const RunDev<T>& R, const V3<T>& p, int* b3)
{
    const T pv[3] = {p.x, p.y, p.z};
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        int k = (int)(pv[d] / R.binw[d]);
        b3[d] = k < 0 ? 0 : (k >= R.nbin[d] ? R.nbin[d] - 1 : k);
    }
    return (b3[2] * R.nbin[1] + b3[1]) * R.nbin[0] + b3[0];
}

template <typename T> __device__ inline bool run_active(const RunDev<T>& R, int64_t* step)
{
    const RunState* st = R.st;
    *step = st->step;
    return st->err == 0 && st->step < st->target;
}

// Folded chunks (a single run on the multi-kernel step): the run's step
// counter holds the chunk's first step until the chunk ends, and a kernel
// at position k of the chunk works on step counter + k.  The electron
// temperatures and electron-phonon sums of position k live in the first or
// second buffer by the parity of k (a fixed grid keeps one buffer).
template <typename T> __device__ inline int64_t step_at(const RunDev<T>& R, int fold_k)
{
    return R.st->step + (fold_k > 0 ? fold_k : 0);
}
// Whether no error stops the run at position k of a folded chunk (k < 0:
// outside one).  The end of step k - 1 runs in the same launch as the first
// colour pass of step k, so a negative electron energy it meets is recorded
// with its position and stops the run from step k + 1 on: every kernel of
// step k reads the same answer whenever the record is written.
__device__ inline bool fold_ok(const RunState* st, int k)
{
    if (st->err != 0) return false;
    if (k < 0) return true;
    const int32_t neg = st->neg_at;
    return neg == 0 || neg > k;
}
// End of a folded chunk: a recorded negative energy becomes the run's error.
__device__ inline void fold_close(RunState* st)
{
    if (st->neg_at != 0) st->err |= ERR_NEG_E;
    st->neg_at = 0;
    st->chunk_done = 0;
}
template <typename T> __device__ inline double* te_buf(const RunDev<T>& R, int fold_k)
{
    return (R.ttm_mode == 1 && fold_k > 0 && (fold_k & 1)) ? R.Te_alt : R.Te;
}
template <typename T> __device__ inline unsigned long long* de_buf(const RunDev<T>& R, int fold_k)
{
    return (fold_k > 0 && (fold_k & 1)) ? R.dE_alt : R.dE;
}
// Whether the bins of a run are emptied by the cell-parallel grid update
// (live runs with a large electron grid) instead of the step end.
template <typename T> __device__ inline bool empties_bins_in_grid(const RunDev<T>& R)
{
    return R.live && R.ttm_mode == 1 && R.ncell > kSmallGrid;
}
// Whether the grid update keeps the step's T_e in the second buffer for a
// deferred spin half step: unless sub-step launches use it for diffusion.
template <typename T> __device__ inline bool keeps_prev_te(const RunDev<T>& R)
{
    return R.kappa_e == 0.0 || R.dtile[0] > 0;
}
// Grid mode 2: the prescribed stepped T_e of step n, at t = n dt.
template <typename T> __device__ inline double te_stepped(const RunDev<T>& R, int64_t n)
{
    const double t = (double)n * R.dtd;
    return t < R.stEnd[0] ? R.stT[0] : (t < R.stEnd[1] ? R.stT[1] : R.stT[2]);
}

// ------------------------------------------------------------ spins
// Update of site l of a colour: field from the current neighbours, thermal
// field from the step's Philox block (drawn whenever the run has a thermal
// field; its amplitude is zero in cells at T_e = 0), exact flow over tau.
// With `has_prev` (colour pass 0 only), the deferred last half step of the
// previous step comes first: the same neighbours, hence the same exchange
// field, with that step's noise, T_e and electron cells.  Two rotations in
// one pass give the same bits as the two passes they replace.
struct PrevHalf {
    const uint16_t* cell;    // electron cells of the previous step's positions
    const double* Te;        // the previous step's electron temperatures
    // folded chunks: this step's T_e is not written yet (the end of the
    // previous step runs in the same launch), so a site computes its cell's
    // value from the previous step's T_e and electron-phonon sum
    const unsigned long long* dE;   // non-null: compute T_e of this step
};

template <typename T>
__device__ inline double cell_energy(const RunDev<T>& R, double e0, unsigned long long raw, int c,
                                     int64_t step);
template <typename T> __device__ inline double cell_e0(const RunDev<T>& R, double T0);
__device__ inline double cell_temp(double e, double ge);

// The rest of a site update once its exchange sum h (eV) is known: the
// field, the thermal field of each rotation and the exact flows, from the
// site's own spin s; returns the new spin.  `bad` is set by the watchdog.
template <typename T, typename VW, int LAT, bool MULTI, bool ANISO>
__device__ __forceinline__ V3<T> site_rotate(const RunDev<T>& R, const VW& V, int colour, T tau,
                                             const Cell3& c, uint32_t idx, int sp, const V3<T>& h,
                                             V3<T> s, int64_t step, bool cur, bool has_prev,
                                             const PrevHalf& prev, bool& bad)
{
    using M = typename VW::Mem;
    const T imu = MULTI ? select4(sp, R.inv_mumb[0], R.inv_mumb[1], R.inv_mumb[2], R.inv_mumb[3])
                        : R.inv_mumb[0];
    const T H0x = h.x * imu + R.B[0];
    const T H0y = h.y * imu + R.B[1];
    const T H0z = h.z * imu + R.B[2];
    const int b = LAT == SL_LATTICE_BCC ? (colour >> 1) : (LAT == SL_LATTICE_FCC ? colour : 0);
    const uint32_t canon =
        __umul24(__umul24(c.z, (uint32_t)R.g.Ly) + c.y, (uint32_t)R.g.Lx) * (uint32_t)R.g.nb +
        c.x * (uint32_t)R.g.nb + (uint32_t)b;
    // one exact rotation over tau_ with the thermal field of step stp at T_e
    auto rotate = [&](V3<T> s0, int64_t stp, double Te, T tau_) {
        T Hx = H0x, Hy = H0y, Hz = H0z;
        // uniaxial anisotropy: 2 K s_z / (mu mu_B) along z, from the spin
        // this rotation starts from (a merged pass's second rotation sees the
        // first one's result)
        if constexpr (ANISO)
            Hz += (MULTI ? select4(sp, R.kan[0], R.kan[1], R.kan[2], R.kan[3]) : R.kan[0]) * s0.z;
        if (R.noisy) {
            const Normals3<T> nu = normals3<T>(R.seed, R.run_id, canon, stp, 0u);
            const T sg = MULTI ? select4(sp, R.sig[0], R.sig[1], R.sig[2], R.sig[3]) : R.sig[0];
            const T amp = Te > 0.0 ? sg * sqrt_te(Te, T(0)) : T(0);
            Hx += amp * nu.a;
            Hy += amp * nu.b;
            Hz += amp * nu.c;
        }
        const V3<T> wv{R.gam * Hx, R.gam * Hy, R.gam * Hz};
        return llg_flow(s0, wv, R.alpha, tau_, R.inv1pa2, bad);
    };
    if (has_prev) {
        const double Te = R.noisy ? gld(prev.Te, (uint32_t)gld(prev.cell, idx)) : 0.0;
        s = rotate(s, step - 1, Te, R.tau_half);
    }
    if (cur) {
        double Te = 0.0;
        if (R.noisy) {
            const uint32_t cc = (uint32_t)M::ld(V.cell, idx);
            if (prev.dE != nullptr)
                Te = cell_temp(cell_energy(R, cell_e0(R, gld(prev.Te, cc)), gld(prev.dE, cc), (int)cc,
                                           step - 1),
                               R.gamma_e);
            else
                Te = M::ld(V.Te, cc);
        }
        s = rotate(s, step, Te, tau);
    }
    return s;
}

template <typename T, typename VW, int LAT, bool MULTI, bool ANISO, bool RADIAL = false>
__device__ __forceinline__ void spin_site_t(const RunDev<T>& R, const VW& V, int colour, T tau,
                                            uint32_t l, int64_t step, bool cur = true,
                                            bool has_prev = false, PrevHalf prev = {})
{
    using M = typename VW::Mem;
    const Cell3 c = cell_of(R.g, colour, l);
    const Around a = around(R.g, c.x, c.xh, c.y, c.z);
    const uint32_t kH = (uint32_t)colour * (uint32_t)R.g.H;
    const uint32_t idx = kH + l;
    const int sp = MULTI ? (int)M::ld(V.species, idx) : 0;
    const V3<T> h = exchange_sum_t<T, VW, LAT, MULTI, RADIAL>(R, V, colour, a, sp);
    bool bad = false;   // the watchdog: a spin that was not a finite unit vector
    V3<T> s{M::ld(V.sx + kH, l), M::ld(V.sy + kH, l), M::ld(V.sz + kH, l)};
    s = site_rotate<T, VW, LAT, MULTI, ANISO>(R, V, colour, tau, c, idx, sp, h, s, step, cur,
                                              has_prev, prev, bad);
    M::st(V.sx + kH, l, s.x);
    M::st(V.sy + kH, l, s.y);
    M::st(V.sz + kH, l, s.z);
    if (bad) atomicOr(&R.st->err, ERR_NUMERIC);
}

// Dispatch on the run's lattice, species count, anisotropy and exchange form
// (uniform per run).  Runs with anisotropy or radial exchange take their
// own instantiations, so the others keep the site update's code unchanged.
template <typename T, typename VW, bool ANISO, bool RADIAL>
__device__ __forceinline__ void spin_site_lat(const RunDev<T>& R, const VW& V, int colour, T tau,
                                              uint32_t l, int64_t step, bool cur, bool has_prev,
                                              PrevHalf prev)
{
    const bool multi = RADIAL || R.n_species > 1;
    if (R.lattice == SL_LATTICE_SC) {
        if (multi) spin_site_t<T, VW, SL_LATTICE_SC, true, ANISO, RADIAL>(R, V, colour, tau, l, step, cur, has_prev, prev);
        else if constexpr (!RADIAL) spin_site_t<T, VW, SL_LATTICE_SC, false, ANISO>(R, V, colour, tau, l, step, cur, has_prev, prev);
    } else if (R.lattice == SL_LATTICE_FCC) {
        if (multi) spin_site_t<T, VW, SL_LATTICE_FCC, true, ANISO, RADIAL>(R, V, colour, tau, l, step, cur, has_prev, prev);
        else if constexpr (!RADIAL) spin_site_t<T, VW, SL_LATTICE_FCC, false, ANISO>(R, V, colour, tau, l, step, cur, has_prev, prev);
    } else {
        if (multi) spin_site_t<T, VW, SL_LATTICE_BCC, true, ANISO, RADIAL>(R, V, colour, tau, l, step, cur, has_prev, prev);
        else if constexpr (!RADIAL) spin_site_t<T, VW, SL_LATTICE_BCC, false, ANISO>(R, V, colour, tau, l, step, cur, has_prev, prev);
    }
}

// RADIAL_OK: the kernel may meet runs with radial exchange (engines without
// any compile the dispatch without those instantiations).
template <typename T, typename VW, bool RADIAL_OK = true>
__device__ __forceinline__ void spin_site(const RunDev<T>& R, const VW& V, int colour, T tau,
                                          uint32_t l, int64_t step, bool cur = true,
                                          bool has_prev = false, PrevHalf prev = {})
{
    if (RADIAL_OK && R.radial) {
        if constexpr (RADIAL_OK) {
            if (R.aniso) spin_site_lat<T, VW, true, true>(R, V, colour, tau, l, step, cur, has_prev, prev);
            else spin_site_lat<T, VW, false, true>(R, V, colour, tau, l, step, cur, has_prev, prev);
        }
    } else if (R.aniso) {
        spin_site_lat<T, VW, true, false>(R, V, colour, tau, l, step, cur, has_prev, prev);
    } else {
        spin_site_lat<T, VW, false, false>(R, V, colour, tau, l, step, cur, has_prev, prev);
    }
}

template <typename T> __device__ inline void pass_colour(const RunDev<T>& R, int pass, int* colour, T* tau)
{
    const int C = R.g.C;
    *colour = pass < C ? pass : 2 * C - 2 - pass;
    *tau = (pass == C - 1) ? R.dt : R.tau_half;
}

// ------------------------------------------------------------ lattice
// The atom of internal index i: its site, the offsets around it and its
// species.
template <typename T, typename VW>
__device__ __forceinline__ Around around_atom(const RunDev<T>& R, const Site& si, uint32_t i)
{
    const uint32_t l = i - (uint32_t)si.k * (uint32_t)R.g.H;
    return around(R.g, (uint32_t)si.x, l - __umul24(fdiv(l, R.g.divLxh), (uint32_t)R.g.Lxh),
                  (uint32_t)si.y, (uint32_t)si.z);
}

// First half kick of an atom of a run with radial exchange: the stored pair
// force (at x^n) plus the bonds' exchange force at x^n with the spins the
// sweep just produced, so that with the kick and drift after the sweep a
// step is the symmetric splitting spins -> lattice with the spins held.  The
// wrapped positions are read only (the drift writes them in a later launch
// or phase).
template <typename T, typename VW>
__device__ __forceinline__ void half_kick_radial(const RunDev<T>& R, const VW& V, uint32_t i)
{
    using M = typename VW::Mem;
    const Site si = decode_site(R.g, i);
    const int sp = species_of(R, V, i);
    const V3<T> s{M::ld(V.sx, i), M::ld(V.sy, i), M::ld(V.sz, i)};
    const V3<T> Fe = exchange_force(R, V, si.k, around_atom<T, VW>(R, si, i), sp, s,
                                    VW::PosMem::ld(V.pos, i));
    const T k = select4(sp, R.hdtm[0], R.hdtm[1], R.hdtm[2], R.hdtm[3]);
    gst(R.vx, i, gld(R.vx, i) + k * (gld(R.fx, i) + Fe.x));
    gst(R.vy, i, gld(R.vy, i) + k * (gld(R.fy, i) + Fe.y));
    gst(R.vz, i, gld(R.vz, i) + k * (gld(R.fz, i) + Fe.z));
}

// Half kick and drift of atom i (step phase), then its electron cell and
// wrapped position; returns whether it moved more than half the skin since
// its list was built.  `kicked`: the half kick was applied already
// (half_kick_radial), only the drift remains.
template <typename T, typename VW>
__device__ __forceinline__ bool kick_drift_atom(const RunDev<T>& R, const VW& V, uint32_t i, int phase,
                                                bool kicked = false)
{
    const Site s = decode_site(R.g, i);
    bool far = false;
    if (phase == PHASE_STEP) {
        const int sp = species_of(R, V, i);
        const T k = select4(sp, R.hdtm[0], R.hdtm[1], R.hdtm[2], R.hdtm[3]);
        T vx = gld(R.vx, i), vy = gld(R.vy, i), vz = gld(R.vz, i);
        if (!kicked) {
            vx += k * gld(R.fx, i);
            vy += k * gld(R.fy, i);
            vz += k * gld(R.fz, i);
        }
        T ux = gld(R.ux, i) + R.dt * vx;
        T uy = gld(R.uy, i) + R.dt * vy;
        T uz = gld(R.uz, i) + R.dt * vz;
        gst(R.vx, i, vx); gst(R.vy, i, vy); gst(R.vz, i, vz);
        gst(R.ux, i, ux); gst(R.uy, i, uy); gst(R.uz, i, uz);
        // watchdog: a non-finite velocity or displacement (from a non-finite
        // force) stops the run
        if (!(fabs(vx) + fabs(vy) + fabs(vz) + fabs(ux) + fabs(uy) + fabs(uz) < T(1.0e30)))
            atomicOr(&R.st->err, ERR_NUMERIC);
        const T dx = ux - gld(R.rx, i), dy = uy - gld(R.ry, i), dz = uz - gld(R.rz, i);
        far = dx * dx + dy * dy + dz * dz > R.skin_half2;
    }
    const V3<T> p = position(R, s, i);
    VW::Mem::st(V.cell, i, (uint16_t)electron_cell(R, p));
    if (R.live) VW::PosMem::st(V.pos, i, Pos4<T>{p.x, p.y, p.z, T(0)});
    return far;
}

// Atom i into the bin of its wrapped position (any order within a bin).  An
// overflow is only flagged: it is an error if the list is rebuilt from
// these bins.
template <typename T, typename VW>
__device__ inline void nbr_bin_atom(const RunDev<T>& R, const VW& V, uint32_t i)
{
    const Pos4<T> pi = VW::PosMem::ld(V.pos, i);
    int b3[3];
    const int bin = bin_of(R, V3<T>{pi.x, pi.y, pi.z}, b3);
    const int slot = atomicAdd(&R.bin_n[bin], 1);
    if (slot < R.bin_cap)
        R.bin_atoms[(size_t)bin * R.bin_cap + slot] = (int32_t)i;
    else
        atomicOr(&R.st->bin_over, 1);
}

// Sorts a bin's atoms by index (insertion sort of a short list); with every
// bin sorted the list build takes each bin in order.
template <typename T> __device__ inline void nbr_sort_bin(const RunDev<T>& R, int bin)
{
    int cnt = R.bin_n[bin];
    cnt = cnt < R.bin_cap ? cnt : R.bin_cap;
    int32_t* a = R.bin_atoms + (size_t)bin * R.bin_cap;
    for (int p = 1; p < cnt; ++p) {
        const int v = a[p];
        int q = p - 1;
        while (q >= 0 && a[q] > v) {
            a[q + 1] = a[q];
            --q;
        }
        a[q + 1] = v;
    }
}

// Raised by the list build when it finds an overflowed bin.
template <typename T> __device__ inline void raise_bin_overflow(const RunDev<T>& R)
{
    if (atomicCAS(&R.st->bad_atom, 0, -1) == 0) {
        R.st->bad_count = R.bin_cap;
        R.st->bad_step = R.st->step;
    }
    atomicOr(&R.st->err, ERR_BIN);
}

// Verlet list of atom i: every atom within rc + skin in its own and the 26
// surrounding bins, bins in a fixed order and atoms in ascending index
// within a bin (so the list, and the order of the force sum, do not depend
// on the order in which atoms were binned).  The list is stored
// column-major, entry q of atom i at nbr[q n + i].
// Verlet list of atom i: the 27 bins around it in a fixed order, each bin's
// atoms within r_list in ascending index, so the list does not depend on
// the order in which atoms entered the bins.  From sorted bins the atoms
// are appended as scanned; from unsorted bins (binned by atomics) a bin's
// accepted atoms are kept sorted in a small per-thread LDS buffer and
// appended when the bin is done (in windows of kBinKeep when it holds more).
// `keep` (unsorted bins only) is the thread's buffer in LDS: slot t at
// keep[t * kBlock], so the threads of a wave touch consecutive words.
constexpr int kBinKeep = 16;

template <typename T, typename VW, bool SORTED_BINS = false>
__device__ inline void nbr_build_atom(const RunDev<T>& R, const VW& V, uint32_t i,
                                      int* keep = nullptr)
{
    const V3<T> ui{gld(R.ux, i), gld(R.uy, i), gld(R.uz, i)};
    const Pos4<T> pi = VW::PosMem::ld(V.pos, i);
    int b3[3];
    bin_of(R, V3<T>{pi.x, pi.y, pi.z}, b3);
    int count = 0;
    const size_t n = (size_t)R.n;
    int32_t* col = R.nbr + i;
    auto append = [&](int jv) {
        if (count < R.max_nbr) col[(size_t)count * n] = jv;
        ++count;
    };
    for (int dz = -1; dz <= 1; ++dz) {
        const int bz = wrapi(b3[2] + dz, R.nbin[2]);
        for (int dy = -1; dy <= 1; ++dy) {
            const int by = wrapi(b3[1] + dy, R.nbin[1]);
            for (int dx = -1; dx <= 1; ++dx) {
                const int bx = wrapi(b3[0] + dx, R.nbin[0]);
                const int bin = (bz * R.nbin[1] + by) * R.nbin[0] + bx;
                int cnt = R.bin_n[bin];
                cnt = cnt < R.bin_cap ? cnt : R.bin_cap;
                const int32_t* a = R.bin_atoms + (size_t)bin * R.bin_cap;
                // candidates four at a time: indices, then positions, then the
                // distance tests (padding slots repeat atom i itself).  Unsorted:
                // a pass keeps the kBinKeep smallest accepted indices above
                // `lo` in ascending order and appends them; a bin with more
                // accepted atoms is scanned again above the last one appended.
                int lo = -1;
                for (bool more = true; more;) {
                    int m = 0, mtot = 0;
                    for (int q0 = 0; q0 < cnt; q0 += 4) {
                        int jj[4];
#pragma unroll
                        for (int u = 0; u < 4; ++u) jj[u] = q0 + u < cnt ? a[q0 + u] : (int)i;
                        V3<T> d[4];
#pragma unroll
                        for (int u = 0; u < 4; ++u) d[u] = separation(R, V, pi, (uint32_t)jj[u]);
#pragma unroll
                        for (int u = 0; u < 4; ++u) {
                            const T r2 = d[u].x * d[u].x + d[u].y * d[u].y + d[u].z * d[u].z;
                            if (jj[u] == (int)i || !(r2 < R.rlist2)) continue;
                            if (SORTED_BINS) {
                                append(jj[u]);
                                continue;
                            }
                            if (jj[u] <= lo) continue;
                            ++mtot;
                            if (m == kBinKeep &&
                                jj[u] > sld(keep, (uint32_t)(kBinKeep - 1) * kBlock))
                                continue;
                            // insertion into the ascending keep[0..m); when
                            // full, the largest entry drops out
                            int t = m < kBinKeep ? m : kBinKeep - 1;
                            for (; t > 0; --t) {
                                const int prev = sld(keep, (uint32_t)(t - 1) * kBlock);
                                if (prev < jj[u]) break;
                                sst(keep, (uint32_t)t * kBlock, prev);
                            }
                            sst(keep, (uint32_t)t * kBlock, jj[u]);
                            m += m < kBinKeep ? 1 : 0;
                        }
                    }
                    if (SORTED_BINS) break;
                    for (int t = 0; t < m; ++t) append(sld(keep, (uint32_t)t * kBlock));
                    more = mtot > kBinKeep;
                    if (more) {
                        lo = sld(keep, (uint32_t)(kBinKeep - 1) * kBlock);
                        atomicAdd(&R.st->n_rescan, 1);
                    }
                }
            }
        }
    }
    // one address for all atoms: only counts above the value already seen
    // reach the atomic (the maximum does not depend on which do)
    if (count > *(volatile int32_t*)&R.st->max_list) atomicMax(&R.st->max_list, count);
    if (count > R.max_nbr) {
        if (atomicCAS(&R.st->bad_atom, 0, (int)i + 1) == 0) {
            R.st->bad_count = count;
            R.st->bad_step = R.st->step;
        }
        atomicOr(&R.st->err, ERR_NBR);
        count = R.max_nbr;
    }
    gst(R.nbr_n, i, (int32_t)count);
    gst(R.rx, i, ui.x);
    gst(R.ry, i, ui.y);
    gst(R.rz, i, ui.z);
}

// An atom's contribution to an observable sample.  The NQ slots of a row are
// derived from it one at a time (obs_slot), so a wave never holds all of
// them at once.
struct ObsTerms {
    double s0, s1, s2;   // spin
    double eex, ez;      // exchange (bonds once) and Zeeman energy, eV
    double ke, pe;       // kinetic and Morse energy, eV
    double num, den;     // |s x h_tot|^2 and s . h_tot of the spin temperature
    int sp;              // species
};

// Slot k of a row: species-resolved spin sums (0-11), energies (12-15),
// spin-temperature numerators (16-19) and denominators (20-23).
__device__ __forceinline__ double obs_slot(const ObsTerms& o, int k)
{
    if (k < 12) return o.sp == k / 3 ? (k % 3 == 0 ? o.s0 : (k % 3 == 1 ? o.s1 : o.s2)) : 0.0;
    if (k == 12) return o.eex;
    if (k == 13) return o.ez;
    if (k == 14) return o.ke;
    if (k == 15) return o.pe;
    if (k < 20) return o.sp == k - 16 ? o.num : 0.0;
    return o.sp == k - 20 ? o.den : 0.0;
}

// Lane exchange inside aligned groups of four lanes (DPP quad permutation:
// MASK 1 swaps neighbours, MASK 2 swaps pairs).
template <int MASK> __device__ __forceinline__ uint32_t quad_xor_u32(uint32_t v)
{
    static_assert(MASK == 1 || MASK == 2, "quad lane masks");
    constexpr int ctrl = MASK == 1 ? 0xB1 : 0x4E;   // quad_perm [1,0,3,2] / [2,3,0,1]
    return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, ctrl, 0xF, 0xF, false);
}
template <int MASK> __device__ __forceinline__ float quad_xor(float v)
{
    return __builtin_bit_cast(float, quad_xor_u32<MASK>(__builtin_bit_cast(uint32_t, v)));
}
template <int MASK> __device__ __forceinline__ double quad_xor(double v)
{
    const uint64_t b = __builtin_bit_cast(uint64_t, v);
    const uint64_t lo = quad_xor_u32<MASK>((uint32_t)b);
    const uint64_t hi = quad_xor_u32<MASK>((uint32_t)(b >> 32));
    return __builtin_bit_cast(double, lo | (hi << 32));
}

// Pair sums over an atom's Verlet list are defined as four interleaved
// partial sums -- entry k goes to partial k mod 4, in ascending k -- folded
// as (p0 + p1) + (p2 + p3).  One lane may hold all four partials, or LPA
// lanes of a quad hold 4/LPA each (lane j of the group: partials j, j + LPA,
// ...): the sums, and so every result, are bitwise the same for LPA = 1, 2
// and 4.  `p` holds this lane's partials; every lane of the group returns
// the folded sum.
template <int LPA, typename X> __device__ __forceinline__ X fold_partials(const X (&p)[4 / LPA])
{
    if constexpr (LPA == 1) {
        return (p[0] + p[1]) + (p[2] + p[3]);
    } else if constexpr (LPA == 2) {
        // lane 0 holds p0, p2 and lane 1 holds p1, p3 (addition commutes, so
        // both lanes form the same bits)
        return (p[0] + quad_xor<1>(p[0])) + (p[1] + quad_xor<1>(p[1]));
    } else {
        const X s = p[0] + quad_xor<1>(p[0]);   // p0 + p1 on lanes 0, 1; p2 + p3 on 2, 3
        return s + quad_xor<2>(s);
    }
}

// Walks this lane's share of atom i's Verlet list within the Morse cutoff:
// entries k = j, j + LPA, ... in chunks of CH (all index loads, then all
// position loads, then the arithmetic: two memory round trips per chunk;
// column k of the list starts at nbr + k n).  With CH LPA a multiple of 4,
// entry q of a chunk belongs to partial (k mod 4), which is this lane's
// slot q mod (4 / LPA), whatever the chunk: f(slot, r^2, d), d = x_j - x_i.
template <typename T, typename VW, int LPA, int CH = 8, typename F>
__device__ __forceinline__ void walk_list(const RunDev<T>& R, const VW& V, uint32_t i, int j,
                                          const Pos4<T>& pi, F&& f)
{
    constexpr int NA = 4 / LPA;
    static_assert((CH * LPA) % 4 == 0, "chunks must keep the partial of each entry");
    const int nn = gld(R.nbr_n, i);
    const size_t n = (size_t)R.n;
    for (int k0 = j; k0 < nn; k0 += CH * LPA) {
        uint32_t jj[CH];
#pragma unroll
        for (int q8 = 0; q8 < CH; ++q8) {
            const int k = k0 + q8 * LPA;
            jj[q8] = k < nn ? (uint32_t)gld(R.nbr + (size_t)k * n, i) : i;
        }
        T dx[CH], dy[CH], dz[CH];
#pragma unroll
        for (int q8 = 0; q8 < CH; ++q8) {
            const V3<T> d = separation(R, V, pi, jj[q8]);
            dx[q8] = d.x;
            dy[q8] = d.y;
            dz[q8] = d.z;
        }
#pragma unroll
        for (int q8 = 0; q8 < CH; ++q8) {
            const T r2 = dx[q8] * dx[q8] + dy[q8] * dy[q8] + dz[q8] * dz[q8];
            if (k0 + q8 * LPA < nn && r2 < R.rc2) f(q8 % NA, r2, dx[q8], dy[q8], dz[q8]);
        }
    }
}

// Forces on atom i at the new positions, the second half kick, the
// electron-phonon Ornstein-Uhlenbeck step (its mean energy added to
// acc[cell - acc_first], fixed point) and, on sample steps, the atom's
// observable terms.  LPA lanes of a quad share the atom (lane `j` of the
// group): they split its neighbour list, fold the pair sums, and then all
// compute the rest while only lane 0 stores.
template <typename T, typename VW, int LPA = 1, bool RADIAL = false>
__device__ __forceinline__ void atom_final_atom(const RunDev<T>& R, const VW& V, uint32_t i,
                                                int phase, int64_t step, bool obs,
                                                unsigned long long* acc, ObsTerms& o, int j = 0,
                                                uint32_t acc_first = 0, const T* drawn = nullptr)
{
    static_assert(LPA == 1 || LPA == 2 || LPA == 4, "lanes per atom");
    constexpr int NA = 4 / LPA;   // partial sums held by one lane
    using M = typename VW::Mem;
    const bool lead = j == 0;
    // drawn: the step's electron-phonon normals, already drawn by the kick
    // (loaded first, so that their latency overlaps the list walk)
    const bool pre = drawn != nullptr && phase == PHASE_STEP && R.ttm_mode == 1 && R.live;
    Normals3<T> kept{T(0), T(0), T(0)};
    if (pre) kept = Normals3<T>{gld(drawn, i), gld(drawn + R.n, i), gld(drawn + 2 * R.n, i)};
    const Site si = decode_site(R.g, i);
    const int sp = species_of(R, V, i);
    if (R.live) {
        const Pos4<T> pi = VW::PosMem::ld(V.pos, i);
        T px[NA], py[NA], pz[NA];
#pragma unroll
        for (int a = 0; a < NA; ++a) px[a] = py[a] = pz[a] = T(0);
        walk_list<T, VW, LPA>(R, V, i, j, pi, [&](int a, T r2, T dx, T dy, T dz) {
            T r;
            // -dV/dr along +d pushes j; the force on i is its opposite
            const T f = morse_f(R, r2, &r);
            px[a] -= f * dx;
            py[a] -= f * dy;
            pz[a] -= f * dz;
        });
        const T Fx = fold_partials<LPA>(px), Fy = fold_partials<LPA>(py), Fz = fold_partials<LPA>(pz);
        double pe = 0.0;
        if (obs) {
            // the Morse energy (sample steps only: a second walk keeps the
            // force loop's registers free of it), bonds counted once
            double ppe[NA];
#pragma unroll
            for (int a = 0; a < NA; ++a) ppe[a] = 0.0;
            walk_list<T, VW, LPA, 4>(R, V, i, j, pi, [&](int a, T r2, T, T, T) {
                T r;
                (void)morse_f(R, r2, &r);
                const double e1 = exp(-(double)R.ma * ((double)r - (double)R.mr0));
                ppe[a] += 0.5 * ((double)R.mD * (e1 * e1 - 2.0 * e1) - (double)R.Vc);
            });
            pe = fold_partials<LPA>(ppe);
        }
        T vx = gld(R.vx, i), vy = gld(R.vy, i), vz = gld(R.vz, i);
        const T me = select4(sp, R.m_e[0], R.m_e[1], R.m_e[2], R.m_e[3]);
        if (phase == PHASE_STEP) {
            const T k = select4(sp, R.hdtm[0], R.hdtm[1], R.hdtm[2], R.hdtm[3]);
            if (RADIAL && R.radial) {
                // the bonds' exchange force at x^{n+1} with this step's spins
                // (the stored force stays the pair force alone)
                const V3<T> s{M::ld(V.sx, i), M::ld(V.sy, i), M::ld(V.sz, i)};
                const V3<T> Fe = exchange_force(R, V, si.k, around_atom<T, VW>(R, si, i), sp, s, pi);
                vx += k * (Fx + Fe.x);
                vy += k * (Fy + Fe.y);
                vz += k * (Fz + Fe.z);
            } else {
                vx += k * Fx;
                vy += k * Fy;
                vz += k * Fz;
            }
            if (R.ttm_mode == 1) {
                const uint32_t c = M::ld(V.cell, i);
                const double Te = M::ld(V.Te, c);
                const uint32_t canon =
                    (((uint32_t)si.z * R.g.Ly + si.y) * R.g.Lx + si.x) * R.g.nb + si.b;
                const Normals3<T> eta = pre ? kept : normals3<T>(R.seed, R.run_id, canon, step, 1u);
                const T oa = select4(sp, R.ou_amp[0], R.ou_amp[1], R.ou_amp[2], R.ou_amp[3]);
                const T amp = oa * sqrt_te(Te, T(0));
                const T nx = R.ou_c1 * vx + amp * eta.a;
                const T ny = R.ou_c1 * vy + amp * eta.b;
                const T nz = R.ou_c1 * vz + amp * eta.c;
                // mean energy the step hands to this atom given its velocity
                const double ke = 0.5 * (double)me *
                                  ((double)vx * vx + (double)vy * vy + (double)vz * vz);
                const double dE = R.ou_1mc2 * (1.5 * kKB * Te - ke);
                if (fabs(dE) < 1.0e3) {
                    const long long fixp = llrint(dE * kFIX);
                    if (lead) atomicAdd(&acc[c - acc_first], (unsigned long long)fixp);
                } else if (lead) {
                    atomicOr(&R.st->err, ERR_DE);
                }
                vx = nx;
                vy = ny;
                vz = nz;
            }
            if (lead) {
                gst(R.vx, i, vx);
                gst(R.vy, i, vy);
                gst(R.vz, i, vz);
            }
        }
        if (lead) {
            gst(R.fx, i, Fx);
            gst(R.fy, i, Fy);
            gst(R.fz, i, Fz);
        }
        if (obs) {
            o.ke = 0.5 * (double)me * ((double)vx * vx + (double)vy * vy + (double)vz * vz);
            o.pe = pe;
        }
    }
    if (obs) {
        const double s0 = M::ld(V.sx, i), s1 = M::ld(V.sy, i), s2 = M::ld(V.sz, i);
        const V3<T> h = exchange_sum<T, VW, RADIAL>(R, V, si.k, around_atom<T, VW>(R, si, i), sp);
        const double h0 = h.x, h1 = h.y, h2 = h.z;
        const double mb = select4(sp, R.mumb[0], R.mumb[1], R.mumb[2], R.mumb[3]);
        o.eex = -0.5 * (s0 * h0 + s1 * h1 + s2 * h2);
        // single-site energy and field: Zeeman and uniaxial anisotropy
        const double kk = select4(sp, R.Kd[0], R.Kd[1], R.Kd[2], R.Kd[3]);
        o.ez = -mb * (R.Bd[0] * s0 + R.Bd[1] * s1 + R.Bd[2] * s2) - kk * s2 * s2;
        const double t0 = h0 + mb * R.Bd[0];
        const double t1 = h1 + mb * R.Bd[1];
        const double t2 = h2 + mb * R.Bd[2] + 2.0 * kk * s2;
        const double c0 = s1 * t2 - s2 * t1, c1 = s2 * t0 - s0 * t2, c2 = s0 * t1 - s1 * t0;
        o.num = c0 * c0 + c1 * c1 + c2 * c2;
        o.den = s0 * t0 + s1 * t1 + s2 * t2;
        o.s0 = s0;
        o.s1 = s1;
        o.s2 = s2;
        o.sp = sp;
    }
}

// Fixed-order wave reduction of the row slots, one slot at a time; lane 0
// writes the row of the wave's 64 consecutive atoms (row = first atom / 64),
// so samples do not depend on the block size.
__device__ inline void wave_write_row(const ObsTerms& o, double* partial, int i_first, int n)
{
    double* row = partial + (size_t)(i_first >> 6) * NQ;
    const bool writer = (threadIdx.x & 63) == 0 && i_first < n;
#pragma unroll
    for (int k = 0; k < NQ; ++k) {
        double x = obs_slot(o, k);
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) x += __shfl_down(x, off, 64);
        if (writer) row[k] = x;
    }
}

// ------------------------------------------------------- electron grid
template <typename T> __device__ inline double laser_power(const RunDev<T>& R, double zc, double t)
{
    if (R.S0 == 0.0 || R.fwhm <= 0.0) return 0.0;
    if (R.profile == 1 && !(zc > (double)R.box[2] - R.depth)) return 0.0;
    const double d = t - R.t0;
    return R.S0 * exp(-4.0 * 0.69314718055994530942 * d * d / (R.fwhm * R.fwhm));
}

// Electron energy density of a cell after one explicit diffusion sub-step:
// e0 + (dt / n_sub) kappa_e times the 7-point Laplacian of T at the cell
// (its temperature Tc and its six neighbours'), with the per-axis factors
// (dt / n_sub) kappa_e / h^2 precomputed.  The first sub-step of a step
// starts from e0 = gamma_e Tc^2 / 2 (diffuse_e0); the cell's temperature
// after it is sqrt(2 e / gamma_e) (diffuse_temp).
template <typename T>
__device__ inline double diffuse_energy(const RunDev<T>& R, double Tc, double xp, double xm, double yp,
                                     double ym, double zp, double zm, double e0)
{
    return e0 + R.dcoef[0] * (xp - 2.0 * Tc + xm) + R.dcoef[1] * (yp - 2.0 * Tc + ym) +
           R.dcoef[2] * (zp - 2.0 * Tc + zm);
}
template <typename T> __device__ inline double diffuse_temp(const RunDev<T>& R, double e)
{
    return sqrt(R.two_ge * (e > 0.0 ? e : 0.0));
}
template <typename T>
__device__ inline double diffuse_e0(const RunDev<T>& R, double Tc)
{
    return 0.5 * R.gamma_e * Tc * Tc;
}

// One sub-step of cell c with the periodic Laplacian of src, written to dst.
template <typename T>
__device__ inline void diffuse_cell(const RunDev<T>& R, const double* src, double* dst, int c, int sub)
{
    const int n0 = R.tn[0], n1 = R.tn[1], n2 = R.tn[2];
    const int i = c % n0, j = (c / n0) % n1, k = c / (n0 * n1);
    const int ip = (i + 1) % n0, im = (i + n0 - 1) % n0;
    const int jp = (j + 1) % n1, jm = (j + n1 - 1) % n1;
    const int kp = (k + 1) % n2, km = (k + n2 - 1) % n2;
    const int row = (k * n1 + j) * n0;
    const double Tc = src[c];
    const double e0 = sub == 0 ? diffuse_e0(R, Tc) : R.ee[c];
    const double e = diffuse_energy(R, Tc, src[row + ip], src[row + im], src[(k * n1 + jp) * n0 + i],
                                    src[(k * n1 + jm) * n0 + i], src[(kp * n1 + j) * n0 + i],
                                    src[(km * n1 + j) * n0 + i], e0);
    R.ee[c] = e;
    if (!(e >= 0.0)) atomicOr(&R.st->err, ERR_NEG_E);   // negative or not a number
    dst[c] = diffuse_temp(R, e);
}

// Laser source and electron-phonon energy of one cell (two-temperature
// mode): e = (after diffusion, or gamma_e T^2 / 2) + dt S(z, t + dt/2)
// - dE / V, T_e = sqrt(2 e / gamma_e).  dE is the cell's fixed-point sum.
// cell_energy: the electron energy density of cell c after step `step`, from the density e0
// before it (gamma_e T^2 / 2 when the electrons do not diffuse), the laser
// source at mid-step and the cell's electron-phonon sum (fixed point).
template <typename T>
__device__ inline double cell_energy(const RunDev<T>& R, double e0, unsigned long long raw, int c,
                                     int64_t step)
{
    const int k = c / (R.tn[0] * R.tn[1]);
    const double tmid = ((double)step + 0.5) * R.dtd;
    const double src = laser_power(R, (k + 0.5) * R.th[2], tmid);
    const double de = (double)(long long)raw / kFIX;
    return e0 + R.dtd * src - de / R.Vcell;
}
template <typename T> __device__ inline double cell_e0(const RunDev<T>& R, double T0)
{
    return 0.5 * R.gamma_e * T0 * T0;
}
__device__ inline double cell_temp(double e, double ge)
{
    return sqrt(2.0 * (e > 0.0 ? e : 0.0) / ge);
}

// neg_k >= 0: the update ends a step inside a folded chunk at position
// neg_k, where a negative energy is recorded by position (fold_ok).
template <typename T>
__device__ inline void cell_update_from(const RunDev<T>& R, double T0, unsigned long long raw, double* Te,
                                        unsigned long long* dEsum, int c, int64_t step,
                                        double* Te_prev = nullptr, int neg_k = -1)
{
    const double ge = R.gamma_e;
    if (Te_prev != nullptr) Te_prev[c] = T0;   // kept for a deferred spin half step
    const double e0 = R.kappa_e != 0.0 ? R.ee[c] : cell_e0(R, T0);
    if (dEsum != nullptr) dEsum[c] = 0ull;
    const double e = cell_energy(R, e0, raw, c, step);
    R.ee[c] = e;
    if (!(e >= 0.0)) {   // negative or not a number
        if (neg_k >= 0) atomicCAS(&R.st->neg_at, 0, neg_k + 1);
        else atomicOr(&R.st->err, ERR_NEG_E);
    }
    Te[c] = cell_temp(e, ge);
}

template <typename T>
__device__ inline void cell_update(const RunDev<T>& R, double* Te, unsigned long long* dEsum, int c,
                                   int64_t step, double* Te_prev = nullptr)
{
    cell_update_from(R, Te[c], dEsum[c], Te, dEsum, c, step, Te_prev);
}



// The observable sample of a run, computed by one block of any size: per-wave
// partial rows in order, electron-grid sums in a fixed-shape tree.
// `step_of_sample` is the step the sample describes.  `go` and `step` carry
// the run's state read once for the whole block.
struct SampleScratch {
    double red[3][kBlock];
    double tot[NQ];
    int64_t step;
    int32_t go, rebuild, done;
};

template <typename T, typename VW>
__device__ inline void write_sample(const RunDev<T>& R, const VW& V, SampleScratch& S,
                                    int64_t step_of_sample)
{
    // kBlock virtual threads whatever the block size (vt = tid, tid + B, ...),
    // so the order of every sum is that of a 256-thread block
    const int tid = threadIdx.x, B = blockDim.x;
    const int nc = R.ncell;
    // the per-wave rows: virtual thread t sums rows t, t + 256, ... in order,
    // then a fixed-shape tree over the virtual threads, three quantities at
    // a time
    for (int q0 = 0; q0 < NQ; q0 += 3) {
        for (int vt = tid; vt < kBlock; vt += B) {
            double a0 = 0.0, a1 = 0.0, a2 = 0.0;
            for (int bk = vt; bk < R.n_part; bk += kBlock) {
                const double* row = V.partial + (size_t)bk * NQ + q0;
                a0 += row[0];
                a1 += row[1];
                a2 += row[2];
            }
            S.red[0][vt] = a0;
            S.red[1][vt] = a1;
            S.red[2][vt] = a2;
        }
        __syncthreads();
        for (int off = kBlock / 2; off > 0; off >>= 1) {
            for (int vt = tid; vt < off; vt += B) {
                S.red[0][vt] += S.red[0][vt + off];
                S.red[1][vt] += S.red[1][vt + off];
                S.red[2][vt] += S.red[2][vt + off];
            }
            __syncthreads();
        }
        if (tid == 0) {
            S.tot[q0] = S.red[0][0];
            S.tot[q0 + 1] = S.red[1][0];
            S.tot[q0 + 2] = S.red[2][0];
        }
        __syncthreads();
    }
    for (int vt = tid; vt < kBlock; vt += B) {
        double eacc = 0.0, tacc = 0.0, tmax = 0.0;
        for (int c = vt; c < nc; c += kBlock) {
            const double Tc = V.Te[c];
            eacc += 0.5 * R.gamma_e * Tc * Tc * R.Vcell;
            tacc += Tc;
            tmax = Tc > tmax ? Tc : tmax;
        }
        S.red[0][vt] = eacc;
        S.red[1][vt] = tacc;
        S.red[2][vt] = tmax;
    }
    __syncthreads();
    for (int off = kBlock / 2; off > 0; off >>= 1) {
        for (int vt = tid; vt < off; vt += B) {
            S.red[0][vt] += S.red[0][vt + off];
            S.red[1][vt] += S.red[1][vt + off];
            S.red[2][vt] = S.red[2][vt] > S.red[2][vt + off] ? S.red[2][vt] : S.red[2][vt + off];
        }
        __syncthreads();
    }
    if (tid == 0) {
        RunState* st = R.st;
        const int64_t ns = st->n_samples;
        sl_obs* o = &R.ring[ns % R.obs_cap];
        o->t = (double)step_of_sample * R.dtd;
        o->step = step_of_sample;
        double m[3] = {0.0, 0.0, 0.0};
        for (int sp = 0; sp < 4; ++sp)
            for (int k = 0; k < 3; ++k) {
                m[k] += S.tot[3 * sp + k];
                o->M[sp][k] = R.cnt[sp] > 0.0 ? S.tot[3 * sp + k] / R.cnt[sp] : 0.0;
            }
        for (int k = 0; k < 3; ++k) o->m[k] = m[k] / (double)R.n;
        o->m_abs = sqrt(o->m[0] * o->m[0] + o->m[1] * o->m[1] + o->m[2] * o->m[2]);
        o->E_ex = S.tot[12];
        o->E_z = S.tot[13];
        o->KE = S.tot[14];
        o->PE = S.tot[15];
        o->E_e = S.red[0][0];
        o->Te_mean = S.red[1][0] / (double)nc;
        o->Te_max = S.red[2][0];
        o->Tl = 2.0 * S.tot[14] / (3.0 * (double)R.n * kKB);
        for (int sp = 0; sp < 4; ++sp)
            o->Tspin[sp] = S.tot[20 + sp] != 0.0 ? S.tot[16 + sp] / (2.0 * kKB * S.tot[20 + sp]) : 0.0;
        st->n_samples = ns + 1;
    }
    __syncthreads();
}

template <typename T> __device__ inline bool sample_due(const RunDev<T>& R, int phase, int64_t step)
{
    return R.obs_every > 0 && (phase == PHASE_INIT || ((step + 1) % R.obs_every) == 0);
}

// ==================================================== multi-kernel step
// The end of step k - 1 of a folded chunk, by the nf extra blocks of colour
// pass 0 of step k (k >= 1; this is block f of them, one thread per cell):
// the small electron grid from the buffers of position k - 1 into those of
// position k (the sums of position k - 1 are read by this pass's spin
// blocks and cleared by the force kernel of step k), and with `clear` the
// bins emptied (when no binning has filled them since they were last
// emptied they are empty already, so no block needs the rebuild flag that
// the first block clears) and the flags cleared.  Without `clear` the
// launch also kicks the atoms of step k, which bin and flag again: the
// force launch of step k - 1 has cleared them instead.  Chunks end on
// sample steps, so no sample falls here; the step counter moves at the
// chunk's end.
template <typename T>
__device__ inline void fold_end_step(const RunDev<T>& R, int k, int f, int nf, bool clear)
{
    RunState* st = R.st;
    const int64_t step = st->step + k - 1;
    if (!fold_ok(st, k - 1) || step >= st->target) return;
    const int t = f * (int)blockDim.x + (int)threadIdx.x, nt = nf * (int)blockDim.x;
    if (R.ttm_mode == 1) {
        const double* Tp = te_buf(R, k - 1);
        const unsigned long long* Ep = de_buf(R, k - 1);
        double* Tn = te_buf(R, k);
        for (int c = t; c < R.ncell; c += nt)
            cell_update_from(R, Tp[c], Ep[c], Tn, (unsigned long long*)nullptr, c, step, nullptr, k);
    }
    if (R.live && clear)
        for (int b = t; b < R.nbins; b += nt) R.bin_n[b] = 0;
    if (t == 0) {
        if (R.live && clear) {
            st->bin_over = 0;
            st->rebuild = 0;
        }
        st->chunk_done = k;
        if (clear) *R.any_rebuild = 0;
    }
}

// One atom of the kick table (a block of a colour pass beyond its spin
// blocks): half kick, drift, the electron cell of the new position (into
// the buffer of x^{n+1}, so the spin blocks of the launch still see the
// cells of x^n and x^{n-1}), the skin check and binning, and the step's
// electron-phonon normals when the force kernel gives an atom several
// lanes.  It reads no spin.
template <typename T>
__device__ __forceinline__ void kick_atom_step(const RunDev<T>* __restrict__ runs, int2 w, int fold_k,
                                               uint32_t lane)
{
    const RunDev<T>& R = runs[w.x];
    const int64_t step = step_at(R, fold_k);
    if (!fold_ok(R.st, fold_k) || step >= R.st->target || !R.live) return;
    const uint32_t i = (uint32_t)w.y + lane;
    if (i >= (uint32_t)R.n) return;
    const GView<T> V = global_view(R, step + 1);
    if (kick_drift_atom(R, V, i, PHASE_STEP, R.radial != 0) &&
        *(volatile int32_t*)&R.st->rebuild == 0) {
        atomicOr(&R.st->rebuild, 1);
        atomicOr(R.any_rebuild, 1);
    }
    if (R.bin_step) nbr_bin_atom(R, V, i);
    if (R.ttm_mode == 1 && R.eta_drawn) {
        // this step's electron-phonon normals for the force kernel, one
        // atom per lane (the force kernel gives an atom several)
        const Site si = decode_site(R.g, i);
        const uint32_t canon = (((uint32_t)si.z * R.g.Ly + si.y) * R.g.Lx + si.x) * R.g.nb + si.b;
        const Normals3<T> eta = normals3<T>(R.seed, R.run_id, canon, step, 1u);
        gst(R.eta, i, eta.a);
        gst(R.eta + R.n, i, eta.b);
        gst(R.eta + 2 * R.n, i, eta.c);
    }
}

// The sites of one tile of a colour pass: site first + k nt + lane of the
// colour, k < SPT.  `merge` (pass 0): apply the previous step's deferred
// last half step first.  LAT >= 0: the specialised site update of that
// lattice and species form (no anisotropy, constant exchange), which the
// engine takes when every run has that form.
template <typename T, int SPT, bool RADIAL, int LAT = -1, bool MULTI = false>
__device__ __forceinline__ void spin_pass_tile(const RunDev<T>* __restrict__ runs, int2 w, int pass,
                                               int merge, int fold_k, uint32_t lane, uint32_t nt)
{
    const RunDev<T>& R = runs[w.x];
    const RunState* st = R.st;
    const int64_t step = step_at(R, fold_k);
    const bool cur = fold_ok(st, fold_k) && step < st->target;
    // colour pass 0 of a merged step first applies the previous step's
    // deferred last half step (also when the run has just reached its
    // target): in a folded chunk whenever the previous step ran, otherwise
    // as recorded by the previous step's end
    const bool prev = merge && pass == 0 &&
                      (fold_k >= 0 ? fold_k >= 1 && fold_ok(st, fold_k - 1) && step - 1 < st->target
                                   : st->pending != 0);
    if (!cur && !prev) return;
    if (pass >= 2 * R.g.C - 1) return;
    int colour;
    T tau;
    pass_colour(R, pass, &colour, &tau);
    GView<T> V = global_view(R, step);
    if (fold_k >= 0) V.Te = te_buf(R, fold_k);
    // T_e of the previous step: in a folded chunk the previous position's
    // buffer (and this step's T_e is computed from it, its end running in
    // this launch); otherwise kept by the grid update (two-temperature or
    // prescribed) in the second buffer; a fixed grid never changes
    PrevHalf ph{R.cellb[cell_slot(step - 1)], R.ttm_mode != 0 ? R.Te_alt : R.Te, nullptr};
    if (fold_k >= 1 && pass == 0)
        ph = PrevHalf{R.cellb[cell_slot(step - 1)], te_buf(R, fold_k - 1),
                      R.ttm_mode == 1 ? de_buf(R, fold_k - 1) : nullptr};
#pragma unroll
    for (int k = 0; k < SPT; ++k) {
        const uint32_t l = (uint32_t)w.y + k * nt + lane;
        if (l < (uint32_t)R.g.H) {
            if constexpr (LAT >= 0)
                spin_site_t<T, GView<T>, LAT, MULTI, false>(R, V, colour, tau, l, step, cur, prev, ph);
            else
                spin_site<T, GView<T>, RADIAL>(R, V, colour, tau, l, step, cur, prev, ph);
        }
    }
}

// Colour pass `pass` over the sites of every active run.  Blocks from
// n_spin_blocks on take other work: the first n_fold of them end the
// previous step of a folded chunk (colour pass 0 at position k >= 1,
// fold_end_step), the rest kick the atoms of live runs (kick_atom_step).
// Those read no spin and the spin blocks read no lattice array.  LAT >= 0:
// the spin blocks take the specialised site update (spin_pass_tile).
template <typename T, int SPT, bool RADIAL = false, int LAT = -1, bool MULTI = false>
__global__ __launch_bounds__(kBlock) void k_spin_pass(const RunDev<T>* __restrict__ runs,
                                                      const int2* __restrict__ work, int pass,
                                                      const int2* __restrict__ work_kick,
                                                      int n_spin_blocks, int n_fold, int merge, int fold_k)
{
    const int e = (int)blockIdx.x - n_spin_blocks;
    if (e >= 0) {
        if (e < n_fold) {
            // the bins and flags are cleared here unless the launch also kicks
            fold_end_step(runs[work[0].x], fold_k, e, n_fold, (int)gridDim.x - n_spin_blocks == n_fold);
            return;
        }
        kick_atom_step(runs, work_kick[e - n_fold], fold_k, threadIdx.x);
        return;
    }
    spin_pass_tile<T, SPT, RADIAL, LAT, MULTI>(runs, work[blockIdx.x], pass, merge, fold_k, threadIdx.x,
                                               blockDim.x);
}

// First half kick of the atoms of runs with radial exchange (the atom table
// of the kick), after the colour sweep and before the drift: exchange forces
// at x^n with the new spins.  Other runs' blocks return.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_half_kick(const RunDev<T>* __restrict__ runs,
                                                      const int2* __restrict__ work_kick)
{
    const int2 w = work_kick[blockIdx.x];
    const RunDev<T>& R = runs[w.x];
    const int64_t step = R.st->step;
    if (!R.radial || !R.live || R.st->err != 0 || step >= R.st->target) return;
    const uint32_t i = (uint32_t)w.y + threadIdx.x;
    if (i < (uint32_t)R.n) half_kick_radial(R, global_view(R, step), i);
}

// A colour pass with nothing but the site updates (no kick or step-end
// blocks, no deferred half step), for engines whose runs on the multi-kernel
// step share one site-update form: one lattice, one or several species for
// all, no anisotropy, constant exchange.  The same device function as in
// k_spin_pass, compiled alone, so the kernel holds fewer registers (more
// waves per SIMD) and gives the same bits.
template <typename T, int SPT, int LAT, bool MULTI>
__device__ __forceinline__ void spin_lean_tile(const RunDev<T>* __restrict__ runs, int2 w, int pass,
                                               int fold_k, uint32_t lane, uint32_t nt)
{
    const RunDev<T>& R = runs[w.x];
    const RunState* st = R.st;
    const int64_t step = step_at(R, fold_k);
    if (!fold_ok(st, fold_k) || step >= st->target || pass >= 2 * R.g.C - 1) return;
    int colour;
    T tau;
    pass_colour(R, pass, &colour, &tau);
    GView<T> V = global_view(R, step);
    if (fold_k >= 0) V.Te = te_buf(R, fold_k);
#pragma unroll
    for (int k = 0; k < SPT; ++k) {
        const uint32_t l = (uint32_t)w.y + k * nt + lane;
        if (l < (uint32_t)R.g.H) spin_site_t<T, GView<T>, LAT, MULTI, false>(R, V, colour, tau, l, step);
    }
}

template <typename T, int SPT, int LAT, bool MULTI>
__global__ __launch_bounds__(kBlock) void k_spin_pass_lean(const RunDev<T>* __restrict__ runs,
                                                           const int2* __restrict__ work, int pass,
                                                           int fold_k)
{
    spin_lean_tile<T, SPT, LAT, MULTI>(runs, work[blockIdx.x], pass, fold_k, threadIdx.x, blockDim.x);
}

// ------------------------------------------------ LDS-staged colour pass
// A colour pass of bcc runs with one species and constant exchange (the
// runs the specialised pass takes) in which a block updates a tile of
// TY x TZ whole rows of its colour (rows y0 <= y < y0 + TY, planes
// z0 <= z < z0 + TZ, every x) from rows staged in LDS.  First the block
// copies, with 16-byte loads, every row its sites read: the other basis's
// two colours on (TY + 1)(TZ + 1) rows (the first shell lies half a cell
// away along every axis), the same basis's other colour on (TY + 2)(TZ + 2)
// rows (the second shell, one cell away along one axis) and its own
// colour's TY TZ rows.  Then each site gathers its 14 (or 8) neighbours from
// LDS and runs the pass's own field sum, in bond order, and rotation, so the
// results have the same bits as the pass that gathers from global memory.
// What changes is the memory instruction stream: one 16-byte load per four
// (FP32) or two (FP64) sites of a staged row instead of one 4- or 8-byte
// gather per neighbour component, about six times fewer load instructions.
// It is a launch shape to choose, not the default: at 256^3 in FP32 it ran
// slower than the gathering pass, because the staged rows (6.4 per computed
// row with 4 x 4 tiles) are the L2 traffic the gathers already draw through
// their L1, and a tile's LDS leaves room for one block per CU.
// Staged row slots: [0, 2 NA) the other basis's colours (colour 2(1 - b)
// first), [2 NA, 2 NA + NB) the second shell's colour, then the own rows;
// slot s holds its three spin components as rows of Lxh values at
// (3 s + comp) Lxh.
template <int TY, int TZ> struct TileRows {
    static constexpr int NA = (TY + 1) * (TZ + 1);
    static constexpr int NB = (TY + 2) * (TZ + 2);
    static constexpr int NOWN = TY * TZ;
    static constexpr int N = 2 * NA + NB + NOWN;
};

// Rows of the staged tile in LDS bytes, for the host's launch.
template <int TY, int TZ> __host__ __device__ constexpr uint32_t tile_lds_bytes(uint32_t Lxh, uint32_t tsize)
{
    return (uint32_t)TileRows<TY, TZ>::N * 3u * Lxh * tsize;
}

template <typename T, int TY, int TZ, int NT = kBlock>
__global__ __launch_bounds__(NT) void k_spin_tile_bcc(const RunDev<T>* __restrict__ runs,
                                                      const int4* __restrict__ work, int pass,
                                                      int fold_k)
{
    typedef TileRows<TY, TZ> TR;
    extern __shared__ __align__(16) unsigned char tile_smem[];
    T* rows = reinterpret_cast<T*>(tile_smem);
    __shared__ int32_t b_go;
    __shared__ uint32_t b_off[TR::N];
    const int4 w = work[blockIdx.x];   // run, first row y0, first plane z0
    const RunDev<T>& R = runs[w.x];
    const RunState* st = R.st;
    // the run's state, read once for the block: every thread takes the same
    // branch at the barrier even if another block raises an error meanwhile
    if (threadIdx.x == 0)
        b_go = fold_ok(st, fold_k) && step_at(R, fold_k) < st->target && pass < 2 * R.g.C - 1;
    __syncthreads();
    if (!b_go) return;
    const int64_t step = step_at(R, fold_k);
    int colour;
    T tau;
    pass_colour(R, pass, &colour, &tau);
    GView<T> V = global_view(R, step);
    if (fold_k >= 0) V.Te = te_buf(R, fold_k);
    const uint32_t Lxh = (uint32_t)R.g.Lxh, Ly = (uint32_t)R.g.Ly, Lz = (uint32_t)R.g.Lz;
    const uint32_t H = (uint32_t)R.g.H;
    const int b = colour >> 1, p = colour & 1;
    const int y0 = w.y, z0 = w.z;
    // ---- staging.  First each staged row's offset in its colour-major
    // arrays, once per block; then the rows themselves as 16-byte vectors,
    // consecutive lanes along a row, a group of spb rows per sweep of the
    // block (the host keeps Lxh <= NT vectors)
    if (threadIdx.x < (uint32_t)TR::N) {
        const int slot = (int)threadIdx.x;
        int col, gy, gz;
        if (slot < 2 * TR::NA) {
            const int cc = slot / TR::NA, q = slot - cc * TR::NA;
            const int lz = q / (TY + 1), ly = q - lz * (TY + 1);
            col = 2 * (1 - b) + cc;
            gy = y0 - (b == 0 ? 1 : 0) + ly;
            gz = z0 - (b == 0 ? 1 : 0) + lz;
        } else if (slot < 2 * TR::NA + TR::NB) {
            const int q = slot - 2 * TR::NA;
            const int lz = q / (TY + 2), ly = q - lz * (TY + 2);
            col = 2 * b + (1 - p);
            gy = y0 - 1 + ly;
            gz = z0 - 1 + lz;
        } else {
            const int q = slot - 2 * TR::NA - TR::NB;
            const int lz = q / TY, ly = q - lz * TY;
            col = colour;
            gy = y0 + ly;
            gz = z0 + lz;
        }
        gy = gy < 0 ? gy + (int)Ly : (gy >= (int)Ly ? gy - (int)Ly : gy);
        gz = gz < 0 ? gz + (int)Lz : (gz >= (int)Lz ? gz - (int)Lz : gz);
        b_off[slot] = (uint32_t)col * H + Lxh * ((uint32_t)gy + Ly * (uint32_t)gz);
    }
    __syncthreads();
    constexpr uint32_t VEC = 16u / (uint32_t)sizeof(T);
    typedef typename Vec4<float>::type F4;
    {
        const uint32_t e0 = threadIdx.x * VEC;
        const uint32_t slot0 = fdiv(e0, R.g.divLxh);          // first row of this lane
        const uint32_t j = e0 - slot0 * Lxh;                  // its vector in the row
        const uint32_t spb = fdiv(blockDim.x * VEC, R.g.divLxh);   // rows per sweep
        const uint32_t rstride = 3u * Lxh * (uint32_t)sizeof(T);   // bytes per staged row
        const uint32_t cstride = Lxh * (uint32_t)sizeof(T);        // bytes per component
        // up to U rows' loads in flight before their stores to LDS
        constexpr int U = NT >= 1024 ? 4 : 8;
        for (uint32_t base = slot0; slot0 < spb && base < (uint32_t)TR::N; base += U * spb) {
            F4 vx[U], vy[U], vz[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const uint32_t slot = base + (uint32_t)u * spb;
                if (slot < (uint32_t)TR::N) {
                    const uint32_t go = (b_off[slot] + j) * (uint32_t)sizeof(T);
                    vx[u] = *(const SL_GLOBAL F4*)((const SL_GLOBAL char*)V.sx + go);
                    vy[u] = *(const SL_GLOBAL F4*)((const SL_GLOBAL char*)V.sy + go);
                    vz[u] = *(const SL_GLOBAL F4*)((const SL_GLOBAL char*)V.sz + go);
                }
            }
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const uint32_t slot = base + (uint32_t)u * spb;
                if (slot < (uint32_t)TR::N) {
                    SL_LDS char* dst = (SL_LDS char*)rows + __umul24(slot, rstride) + j * (uint32_t)sizeof(T);
                    *(SL_LDS F4*)dst = vx[u];
                    *(SL_LDS F4*)(dst + cstride) = vy[u];
                    *(SL_LDS F4*)(dst + 2u * cstride) = vz[u];
                }
            }
        }
    }
    __syncthreads();
    // ---- the tile's sites
    const uint32_t nsite = (uint32_t)(TY * TZ) * Lxh;
    const bool two = R.n_shells > 1;
    const uint32_t L3 = 3u * Lxh;   // elements per staged row
    // each bond's staged row relative to the site's own row in its group
    // (uniform over the block: scalar products)
    uint32_t dq[14];
#pragma unroll
    for (int q = 0; q < 8; ++q) {
        const int mx = q & 1, my = (q >> 1) & 1, mz = q >> 2;
        const int cc = (p + mx + my + mz + (1 - b)) & 1;
        dq[q] = __builtin_amdgcn_readfirstlane((uint32_t)(cc * TR::NA + mz * (TY + 1) + my) * L3);
    }
    {
        const uint32_t c0 = (uint32_t)(2 * TR::NA + (TY + 2) + 1);
        const uint32_t dz = (uint32_t)(TY + 2);
        dq[8] = dq[9] = __builtin_amdgcn_readfirstlane(c0 * L3);
        dq[10] = __builtin_amdgcn_readfirstlane((c0 - 1u) * L3);
        dq[11] = __builtin_amdgcn_readfirstlane((c0 + 1u) * L3);
        dq[12] = __builtin_amdgcn_readfirstlane((c0 - dz) * L3);
        dq[13] = __builtin_amdgcn_readfirstlane((c0 + dz) * L3);
    }
    const uint32_t down = __builtin_amdgcn_readfirstlane((uint32_t)(2 * TR::NA + TR::NB) * L3);
    for (uint32_t t = threadIdx.x; t < nsite; t += blockDim.x) {
        const uint32_t r = fdiv(t, R.g.divLxh);
        const uint32_t xh = t - __umul24(r, Lxh);
        const int ty = (int)(r % TY), tz = (int)(r / TY);
        Cell3 c;
        c.xh = xh;
        c.y = (uint32_t)(y0 + ty);
        c.z = (uint32_t)(z0 + tz);
        c.x = 2 * xh + (((uint32_t)colour + c.y + c.z) & 1u);
        // the half-x indices of x - 1, x, x + 1 in a row (as the global pass)
        const uint32_t xm = (c.x & 1u) ? xh : (xh == 0 ? Lxh - 1 : xh - 1);
        const uint32_t xp = (c.x & 1u) ? (xh == Lxh - 1 ? 0 : xh + 1) : xh;
        const uint32_t X[2] = {b == 0 ? xm : xh, b == 0 ? xh : xp};
        // the site's row in each group: first shell, second shell, own
        const uint32_t rA = __umul24((uint32_t)(tz * (TY + 1) + ty), L3);
        const uint32_t rB = __umul24((uint32_t)(tz * (TY + 2) + ty), L3);
        const uint32_t rO = __umul24(r, L3);
        uint32_t at[14];   // each bond's element in the staged rows (component 0)
        int sh[14];
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            at[q] = rA + dq[q] + X[(q & 1)];
            sh[q] = 0;
        }
        at[8] = rB + dq[8] + xm;
        at[9] = rB + dq[9] + xp;
#pragma unroll
        for (int q = 10; q < 14; ++q) at[q] = rB + dq[q] + xh;
#pragma unroll
        for (int q = 8; q < 14; ++q) sh[q] = 1;
        T ax[14], ay[14], az[14];
        int sj[14];
        T fr[14];
#pragma unroll
        for (int q = 0; q < 14; ++q) {
            ax[q] = sld(rows, at[q]);
            ay[q] = sld(rows, at[q] + Lxh);
            az[q] = sld(rows, at[q] + 2u * Lxh);
            sj[q] = 0;
        }
        const V3<T> h = two ? exchange_accum<T, false, false, 14>(R, sh, ax, ay, az, sj, fr, 0)
                            : exchange_accum<T, false, false, 8>(R, sh, ax, ay, az, sj, fr, 0);
        const uint32_t own = rO + down + xh;
        V3<T> s{sld(rows, own), sld(rows, own + Lxh), sld(rows, own + 2u * Lxh)};
        const uint32_t l = xh + __umul24(Lxh, c.y + __umul24(Ly, c.z));
        const uint32_t kH = (uint32_t)colour * H;
        bool bad = false;
        s = site_rotate<T, GView<T>, SL_LATTICE_BCC, false, false>(R, V, colour, tau, c, kH + l, 0, h, s,
                                                                   step, true, false, PrevHalf{}, bad);
        gst(V.sx + kH, l, s.x);
        gst(V.sy + kH, l, s.y);
        gst(V.sz + kH, l, s.z);
        if (bad) atomicOr(&R.st->err, ERR_NUMERIC);
    }
}

// Initialisation of the lattice arrays of one run: electron cells and
// wrapped positions of the current positions, the cell ids into all three
// buffers (a frozen lattice never rewrites them).  In steps the kick is
// carried by a colour pass.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_init_lattice(const RunDev<T>* __restrict__ runs,
                                                         const int2* __restrict__ work)
{
    const int2 w = work[blockIdx.x];
    const RunDev<T>& R = runs[w.x];
    const int64_t step = R.st->step;
    const uint32_t i = (uint32_t)w.y + threadIdx.x;
    if (i >= (uint32_t)R.n) return;
    kick_drift_atom(R, global_view(R, step), i, PHASE_INIT);
    const uint16_t c = gld(R.cellb[cell_slot(step)], i);
    gst(R.cellb[cell_slot(step + 1)], i, c);
    gst(R.cellb[cell_slot(step + 2)], i, c);
}

// Binning on its own, for a rebuild: at initialisation, and every step for
// runs whose kick does not bin.  Blocks stride over the n_work entries of
// the atom table; in steps (any_rebuild given) the launch is capped and
// exits at once unless some run flagged a rebuild.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_nbr_bin(const RunDev<T>* __restrict__ runs,
                                                    const int2* __restrict__ work, int phase,
                                                    int fold_k, int n_work,
                                                    const int32_t* __restrict__ any_rebuild)
{
    if (any_rebuild != nullptr && *any_rebuild == 0) return;
    for (int e = (int)blockIdx.x; e < n_work; e += (int)gridDim.x) {
        const int2 w = work[e];
        const RunDev<T>& R = runs[w.x];
        if (!R.live || R.st->rebuild == 0 || !fold_ok(R.st, fold_k)) continue;
        if (phase == PHASE_STEP && (R.bin_step || step_at(R, fold_k) >= R.st->target)) continue;
        const uint32_t i = (uint32_t)w.y + threadIdx.x;
        if (i < (uint32_t)R.n) nbr_bin_atom(R, global_view(R, 0), i);
    }
}

// Sorts the bins filled by k_nbr_bin for a rebuild (thread i of a run takes
// bins i, i + n, ...): at initialisation, and in steps of runs whose kick
// does not bin.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_nbr_sort(const RunDev<T>* __restrict__ runs,
                                                     const int2* __restrict__ work, int phase,
                                                     int fold_k, int n_work,
                                                     const int32_t* __restrict__ any_rebuild)
{
    if (any_rebuild != nullptr && *any_rebuild == 0) return;
    for (int e = (int)blockIdx.x; e < n_work; e += (int)gridDim.x) {
        const int2 w = work[e];
        const RunDev<T>& R = runs[w.x];
        if (!R.live || R.st->rebuild == 0 || !fold_ok(R.st, fold_k)) continue;
        if (phase == PHASE_STEP && (R.bin_step || step_at(R, fold_k) >= R.st->target)) continue;
        for (uint32_t b = (uint32_t)w.y + threadIdx.x; b < (uint32_t)R.nbins; b += (uint32_t)R.n)
            nbr_sort_bin(R, (int)b);
    }
}

// The initial Verlet-list build (from bins sorted by k_nbr_sort); in steps
// the lists are rebuilt by k_atom_final.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_nbr_build(const RunDev<T>* __restrict__ runs,
                                                      const int2* __restrict__ work)
{
    const int2 w = work[blockIdx.x];
    const RunDev<T>& R = runs[w.x];
    if (!R.live || R.st->rebuild == 0 || R.st->err != 0) return;
    const bool first = w.y == 0 && threadIdx.x == 0;
    if (R.st->bin_over) {
        if (first) raise_bin_overflow(R);
        return;
    }
    if (first) R.st->n_rebuild += 1;
    const uint32_t i = (uint32_t)w.y + threadIdx.x;
    if (i < (uint32_t)R.n) nbr_build_atom<T, GView<T>, true>(R, global_view(R, 0), i);
}

// LDS of one block of the force kernel.  The list build's per-thread bin
// buffers and the per-cell sums are never live together (a barrier
// separates them): one region, 16 KB, so five 256-thread blocks fit a CU.
template <int LPA> struct ForceShared {
    ObsTerms ostage[LPA > 1 ? kBlock / LPA : 1];
    union {
        int keep[kBinKeep * kBlock];
        unsigned long long cacc[kLdsCells];
    } lds;
    int64_t b_step;
    int32_t b_go, b_rebuild, b_last;
    uint32_t b_lo[kBlock / 64], b_hi[kBlock / 64];   // per-wave cell ranges
};

// Forces, the second half kick, the electron-phonon step and the
// observable rows of the atoms of one entry w of the atom table.  In a step
// whose kick flagged a rebuild, each block first rebuilds the lists of its
// own atoms: positions and bins are final after the kick, and an atom's
// forces read only its own list.  `sorted_bins` tells how the bins were
// filled (unsorted by the kick, or sorted).  LPA lanes per atom: a block of
// B threads takes B / LPA consecutive atoms (a multiple of 64, so
// observable rows of 64 atoms never straddle blocks).  The run's state is
// read once for the block, so every wave takes the same branch at the
// barriers even when another block raises an error meanwhile.
template <typename T, int LPA, bool RADIAL>
__device__ __forceinline__ void atom_final_block(const RunDev<T>* __restrict__ runs, int2 w, int phase,
                                                 int sorted_bins, int fold_k, ForceShared<LPA>& S)
{
    ObsTerms* const ostage = S.ostage;
    unsigned long long* const cacc = S.lds.cacc;
    int* const keep = S.lds.keep;
    int64_t& b_step = S.b_step;
    int32_t& b_go = S.b_go;
    int32_t& b_rebuild = S.b_rebuild;
    uint32_t* const b_lo = S.b_lo;
    uint32_t* const b_hi = S.b_hi;
    const RunDev<T>& R = runs[w.x];
    RunState* st = R.st;
    // the run's state, read once for the block
    if (threadIdx.x == 0) {
        b_step = step_at(R, fold_k);
        b_go = phase != PHASE_STEP || (fold_ok(st, fold_k) && b_step < st->target);
        b_rebuild = phase == PHASE_STEP && R.live && st->rebuild != 0 ? (st->bin_over ? 2 : 1) : 0;
    }
    __syncthreads();
    const int64_t step = b_step;
    const uint32_t apb = blockDim.x / LPA;              // atoms of this block
    const uint32_t la = threadIdx.x / LPA;              // the thread's atom in the block
    const int lj = (int)(threadIdx.x % LPA);            // its lane in the atom's group
    const uint32_t i = (uint32_t)w.y + la;
    const bool obs = sample_due(R, phase, step);
    if (b_go && b_rebuild == 2) {
        if (w.y == 0 && threadIdx.x == 0) raise_bin_overflow(R);
    } else if (b_go && (R.live || obs)) {
        if (b_rebuild) {
            if (w.y == 0 && threadIdx.x == 0) st->n_rebuild += 1;
            // one thread per atom builds the lists of the block's atoms
            const uint32_t ib = (uint32_t)w.y + threadIdx.x;
            if (threadIdx.x < apb && ib < (uint32_t)R.n) {
                if (sorted_bins)
                    [[clang::always_inline]] nbr_build_atom<T, GView<T>, true>(R, global_view(R, 0), ib);
                else
                    [[clang::always_inline]] nbr_build_atom<T, GView<T>, false>(
                        R, global_view(R, 0), ib, keep + threadIdx.x);
            }
            __syncthreads();
        }
        // electron-phonon energy per cell: first summed in LDS over the span
        // of cells the block's atoms occupy (fixed point, so the order does
        // not matter), then one global atomic per touched cell; a block whose
        // span exceeds the LDS table adds to the global sums directly
        const bool eph = phase == PHASE_STEP && R.live && R.ttm_mode == 1;
        GView<T> V = global_view(R, phase == PHASE_INIT ? step : step + 1);
        unsigned long long* const dE = fold_k >= 0 ? de_buf(R, fold_k) : R.dE;
        if (fold_k >= 0) V.Te = te_buf(R, fold_k);
        if (eph && fold_k >= 1) {
            // the previous position's sums, read by this step's colour pass
            // 0, are cleared for position k + 1
            unsigned long long* const old = de_buf(R, fold_k - 1);
            const uint32_t nb = ((uint32_t)R.n + apb - 1) / apb;
            for (uint32_t c = (uint32_t)w.y / apb * blockDim.x + threadIdx.x; c < (uint32_t)R.ncell;
                 c += nb * blockDim.x)
                old[c] = 0ull;
        }
        uint32_t c_lo = 0, c_span = 0;
        if (eph) {
            const bool mine = i < (uint32_t)R.n;
            const uint32_t c = mine ? (uint32_t)gld(V.cell, i) : 0u;
            uint32_t lo = mine ? c : 0xFFFFFFFFu, hi = mine ? c : 0u;
#pragma unroll
            for (int off = 32; off > 0; off >>= 1) {
                lo = min(lo, (uint32_t)__shfl_xor((int)lo, off, 64));
                hi = max(hi, (uint32_t)__shfl_xor((int)hi, off, 64));
            }
            if ((threadIdx.x & 63) == 0) {
                b_lo[threadIdx.x >> 6] = lo;
                b_hi[threadIdx.x >> 6] = hi;
            }
            __syncthreads();
            lo = b_lo[0];
            hi = b_hi[0];
            for (int wv = 1; wv < (int)(blockDim.x >> 6); ++wv) {
                lo = min(lo, b_lo[wv]);
                hi = max(hi, b_hi[wv]);
            }
            c_lo = lo;
            c_span = hi >= lo ? hi - lo + 1 : 0;
        }
        const bool lds_acc = eph && c_span <= (uint32_t)kLdsCells;
        if (lds_acc) {
            for (uint32_t c = threadIdx.x; c < c_span; c += blockDim.x) cacc[c] = 0ull;
            __syncthreads();
        }
        ObsTerms o{};
        if (i < (uint32_t)R.n)
            atom_final_atom<T, GView<T>, LPA, RADIAL>(R, V, i, phase, step, obs, lds_acc ? cacc : dE, o, lj,
                                              lds_acc ? c_lo : 0u, R.eta_drawn ? R.eta : nullptr);
        if (lds_acc) {
            __syncthreads();
            for (uint32_t c = threadIdx.x; c < c_span; c += blockDim.x)
                if (cacc[c] != 0ull) atomicAdd(&dE[c_lo + c], cacc[c]);
        }
        if (obs) {
            if constexpr (LPA == 1) {
                wave_write_row(o, R.partial, (int)i - (int)(threadIdx.x & 63), R.n);
            } else {
                // a wave holds 64 / LPA atoms: stage the terms so that rows of
                // 64 atoms are reduced by one wave each, as with one lane per
                // atom
                if (lj == 0) ostage[la] = o;
                __syncthreads();
                if (threadIdx.x < apb)
                    wave_write_row(ostage[threadIdx.x], R.partial,
                                   w.y + (int)(threadIdx.x & ~63u), R.n);
            }
        }
    }
}

template <typename T, int LPA, bool RADIAL = false>
__global__ __launch_bounds__(kBlock) void k_atom_final(const RunDev<T>* __restrict__ runs,
                                                       const int2* __restrict__ work, int phase,
                                                       int sorted_bins, int fold_k)
{
    __shared__ ForceShared<LPA> S;
    atom_final_block<T, LPA, RADIAL>(runs, work[blockIdx.x], phase, sorted_bins, fold_k, S);
}

// Colour pass `pass` (no merged half step) beside the force kernel of the
// same step of a merged chunk, whose kick ran in colour pass 0.  The first
// n_atom_blocks blocks take the atom table (the force kernel, the longer
// chain, is dispatched first); the others take n_spin_tiles tiles of the
// spin table (spin_bt threads each, a multiple of 64, so every wave has one
// tile; SPT sites per thread) with the specialised site update of
// k_spin_pass_lean.  The force
// kernel reads spins only on sample steps, which end a chunk and never take
// this launch.  Unfolded, each step's k_finalize clears the bins and flags
// the kick set.  In a folded chunk (`clear`, a single run) the next step's
// kick runs beside the end of this step, so this launch clears them: on a
// step without a list rebuild the force blocks empty the bins in shares; on
// a rebuild step, when they read them, the last force block to finish does.
// (A count of finished blocks on every step cost about 10 ns per block: the
// atomics on one address serialise.)
template <typename T, int LPA, int LAT, bool MULTI, int SPT = 1>
__global__ __launch_bounds__(kBlock) void k_spin_force(const RunDev<T>* __restrict__ runs,
                                                       const int2* __restrict__ work_spin, int n_spin_tiles,
                                                       int spin_bt, int n_atom_blocks,
                                                       const int2* __restrict__ work_atom, int pass,
                                                       int sorted_bins, int fold_k, int clear)
{
    __shared__ ForceShared<LPA> S;
    if ((int)blockIdx.x >= n_atom_blocks) {
        const int per = (int)blockDim.x / spin_bt;
        const int t = __builtin_amdgcn_readfirstlane(((int)blockIdx.x - n_atom_blocks) * per +
                                                     (int)threadIdx.x / spin_bt);
        if (t < n_spin_tiles)
            spin_lean_tile<T, SPT, LAT, MULTI>(runs, work_spin[t], pass, fold_k,
                                               threadIdx.x % (uint32_t)spin_bt, (uint32_t)spin_bt);
        return;
    }
    const int2 w = work_atom[blockIdx.x];
    atom_final_block<T, LPA, false>(runs, w, PHASE_STEP, sorted_bins, fold_k, S);
    const RunDev<T>& R = runs[w.x];
    RunState* st = R.st;
    if (!clear || !R.live) return;
    if (S.b_rebuild == 0) {
        // no list is built in this launch, so no block reads the bins or
        // the overflow flag: each force block empties its share of the bins
        // the kick filled (the rebuild flags are clear)
        const int nb = n_atom_blocks, f = (int)blockIdx.x;
        const int per = (R.nbins + nb - 1) / nb;
        const int hi = min(R.nbins, (f + 1) * per);
        if (R.bin_step)
            for (int b = f * per + (int)threadIdx.x; b < hi; b += blockDim.x) R.bin_n[b] = 0;
        if (f == 0 && threadIdx.x == 0) st->bin_over = 0;
        return;
    }
    // a rebuild step: every block reads the bins and flags, so the last one
    // to finish clears them.  No memory fence: a block's reads have returned
    // (their values were used) before its barrier and count; the clearing
    // stores reach the next launch at the kernel boundary; and a device
    // fence would write back and invalidate the L2 of the block's XCD under
    // the blocks still running there.
    __syncthreads();
    if (threadIdx.x == 0) {
        const int before = atomicAdd(&st->force_done, 1);
        S.b_last = before == n_atom_blocks - 1;
    }
    __syncthreads();
    if (!S.b_last) return;
    for (int b = threadIdx.x; b < R.nbins; b += blockDim.x) R.bin_n[b] = 0;
    if (threadIdx.x == 0) {
        st->bin_over = 0;
        st->rebuild = 0;
        *R.any_rebuild = 0;
        st->force_done = 0;
    }
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_ttm_diffuse(const RunDev<T>* __restrict__ runs,
                                                        const int2* __restrict__ work, int sub)
{
    const int2 w = work[blockIdx.x];
    const RunDev<T>& R = runs[w.x];
    int64_t step;
    if (!run_active(R, &step)) return;
    if (R.ttm_mode != 1 || R.kappa_e == 0.0 || sub >= R.n_sub) return;
    const int c = w.y + (int)threadIdx.x;
    if (c >= R.ncell) return;
    diffuse_cell(R, (sub & 1) ? R.Te_alt : R.Te, (sub & 1) ? R.Te : R.Te_alt, c, sub);
}

// All diffusion sub-steps of one tile of a run's electron grid in one launch
// (temporal blocking).  The temperatures of the tile and of a halo n_sub
// cells deep (periodic images included) are staged in LDS.  Sub-step s
// updates the region that is still exact after it, one cell per side
// smaller each sub-step, so a halo cell is recomputed by every tile that
// needs it with the arithmetic of the tile that owns it.  Only the tile's
// own cells are written: their diffused energy density, which the grid
// update then takes.  No block writes the temperatures during the launch,
// so every halo reads the same grid.
// The region is at most kTileSide cells along x and y (tile + 2 n_sub), laid
// out padded to kTileSide so that a thread's cell column is (x, y) =
// (thread mod 16, thread / 16 mod 16); the block's kTileBlock / 256 thread
// layers split the z range.
constexpr int kTileSide = 16;
constexpr int kTileBlock = 1024;
template <typename T>
__global__ __launch_bounds__(kTileBlock) void k_ttm_tile(const RunDev<T>* __restrict__ runs,
                                                         const int2* __restrict__ work)
{
    extern __shared__ double tl[];
    __shared__ int32_t b_go;
    const int2 w = work[blockIdx.x];
    const RunDev<T>& R = runs[w.x];
    if (threadIdx.x == 0) {
        int64_t step;
        b_go = run_active(R, &step) ? 1 : 0;
    }
    __syncthreads();
    if (!b_go) return;
    const int h = R.n_sub;
    const int n0 = R.tn[0], n1 = R.tn[1], n2 = R.tn[2];
    const int t0 = R.dtile[0], t1 = R.dtile[1], t2 = R.dtile[2];
    const int a0 = w.y % R.dntile[0], a1 = (w.y / R.dntile[0]) % R.dntile[1],
              a2 = w.y / (R.dntile[0] * R.dntile[1]);
    const int D0 = t0 + 2 * h, D1 = t1 + 2 * h, D2 = t2 + 2 * h;
    constexpr int S = kTileSide, P = kTileSide * kTileSide;
    const int vol = P * D2;
    // grid coordinates of region cell (0, 0, 0), and the tile's own extent
    // (the last tile along an axis may be cut by the grid's edge)
    const int o0 = a0 * t0 - h, o1 = a1 * t1 - h, o2 = a2 * t2 - h;
    const int w0 = min(t0, n0 - a0 * t0), w1 = min(t1, n1 - a1 * t1), w2 = min(t2, n2 - a2 * t2);
    double* A = tl;
    double* B = tl + vol;
    double* const E = tl + 2 * vol;
    const int x = (int)threadIdx.x & (S - 1), y = ((int)threadIdx.x / S) & (S - 1);
    const int zg = (int)threadIdx.x / P, nz = (int)blockDim.x / P;
    if (x < D0 && y < D1) {
        const int gx = ((o0 + x) % n0 + n0) % n0, gy = ((o1 + y) % n1 + n1) % n1;
        for (int z = zg; z < D2; z += nz) {
            const int gz = ((o2 + z) % n2 + n2) % n2;
            A[z * P + y * S + x] = R.Te[(gz * n1 + gy) * n0 + gx];
        }
    }
    __syncthreads();
    const bool own_col = x >= h && x < h + w0 && y >= h && y < h + w1;
    for (int sub = 0; sub < h; ++sub) {
        const int lo = sub + 1;
        if (x >= lo && x < D0 - lo && y >= lo && y < D1 - lo) {
            for (int z = lo + zg; z < D2 - lo; z += nz) {
                const int r = z * P + y * S + x;
                const double Tc = A[r];
                const double e0 = sub == 0 ? diffuse_e0(R, Tc) : E[r];
                const double e = diffuse_energy(R, Tc, A[r + 1], A[r - 1], A[r + S], A[r - S], A[r + P],
                                                A[r - P], e0);
                E[r] = e;
                B[r] = diffuse_temp(R, e);
                if (own_col && z >= h && z < h + w2 && !(e >= 0.0)) atomicOr(&R.st->err, ERR_NEG_E);
            }
        }
        __syncthreads();
        double* const t = A;
        A = B;
        B = t;
    }
    if (own_col)
        for (int z = h + zg; z < h + w2; z += nz)
            R.ee[((a2 * t2 + z - h) * n1 + (a1 * t1 + y - h)) * n0 + (a0 * t0 + x - h)] = E[z * P + y * S + x];
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_grid(const RunDev<T>* __restrict__ runs,
                                                 const int2* __restrict__ work)
{
    const int2 w = work[blockIdx.x];
    const RunDev<T>& R = runs[w.x];
    int64_t step;
    if (!run_active(R, &step) || R.ttm_mode == 0 || R.ncell <= kSmallGrid) return;
    const int c = w.y + (int)threadIdx.x;
    if (c < R.ncell) {
        if (R.ttm_mode == 2) {
            // the prescribed profile (the previous step's value kept for a
            // deferred spin half step)
            R.Te_alt[c] = R.Te[c];
            R.Te[c] = te_stepped(R, step + 1);
        } else {
            cell_update(R, R.Te, R.dE, c, step, keeps_prev_te(R) ? R.Te_alt : nullptr);
        }
    }
    // the bins filled this step, emptied here for such runs (spread over the
    // grid's blocks rather than by the one block of the step end)
    if (empties_bins_in_grid(R) && (R.bin_step || R.st->rebuild != 0)) {
        const int span = (R.ncell + kBlock - 1) / kBlock * kBlock;
        for (int b = c; b < R.nbins; b += span) R.bin_n[b] = 0;
    }
}


// End of a step of one run, by one block: small electron grids, the
// observable sample, the bins emptied and the rebuild flag cleared,
// step + 1.  The run's state is read once for the block (the grid update
// may raise an error while other waves have yet to look, and every wave
// must take the same branch at the barriers).
// `deferred`: this step's last colour half step is left to the next step's
// colour pass 0 (recorded in the run state for it).
// fold_k >= 0: the last step (position fold_k) of a folded chunk, whose
// electron temperatures and sums are in that position's buffers; the step
// counter moves to the end of the chunk, or, when the run stopped inside
// it, past the last step that ended, whose temperatures are moved to the
// first buffer.
template <typename T>
__device__ inline void end_step(const RunDev<T>& R, SampleScratch& S, int phase, int deferred = 0,
                                int fold_k = -1)
{
    RunState* st = R.st;
    const int tid = threadIdx.x;
    const bool grid = phase == PHASE_STEP && R.ttm_mode == 1 && R.ncell <= kSmallGrid;
    const double* const srcT = fold_k >= 0 ? te_buf(R, fold_k) : R.Te;
    unsigned long long* const srcE = fold_k >= 0 ? de_buf(R, fold_k) : R.dE;
    // this thread's first two cells of a small grid, loaded before the state
    // is known (they were written by earlier launches) so that the two
    // memory round trips overlap
    double pT[2] = {0.0, 0.0};
    unsigned long long pE[2] = {0ull, 0ull};
#pragma unroll
    for (int q = 0; q < 2; ++q) {
        const int c = tid + q * (int)blockDim.x;
        if (grid && c < R.ncell) {
            pT[q] = srcT[c];
            pE[q] = srcE[c];
        }
    }
    // the binning launches of this step have read the engine's rebuild word
    if (blockIdx.x == 0 && tid == 0) *R.any_rebuild = 0;
    if (tid == 0) {
        S.step = phase == PHASE_STEP ? step_at(R, fold_k) : st->step;
        S.go = phase != PHASE_STEP || (fold_ok(st, fold_k) && S.step < st->target);
        S.rebuild = st->rebuild;
        S.done = st->chunk_done;
    }
    __syncthreads();
    if (!S.go) {
        if (phase != PHASE_STEP) return;
        if (fold_k >= 0 && R.ttm_mode == 1) {
            // stopped inside a folded chunk after S.done steps
            for (int c = tid; c < R.ncell; c += blockDim.x) {
                if (S.done & 1) R.Te[c] = R.Te_alt[c];
                R.dE[c] = 0ull;
                R.dE_alt[c] = 0ull;
            }
        }
        if (tid == 0) {
            st->pending = 0;
            if (fold_k >= 0) {
                st->step += S.done;
                fold_close(st);
            }
        }
        return;
    }
    const int64_t step = S.step;
    if (phase == PHASE_STEP && R.ttm_mode == 2 && R.ncell <= kSmallGrid) {
        // the prescribed profile (the previous step's value kept for a
        // deferred spin half step)
        const double Tn = te_stepped(R, step + 1);
        for (int c = tid; c < R.ncell; c += blockDim.x) {
            R.Te_alt[c] = R.Te[c];
            R.Te[c] = Tn;
        }
        __syncthreads();
    }
    if (grid) {
        double* const keep_prev = keeps_prev_te(R) ? R.Te_alt : nullptr;
        int q = 0;
        for (int c = tid; c < R.ncell; c += blockDim.x, ++q) {
            if (q < 2)
                cell_update_from(R, pT[q & 1], pE[q & 1], R.Te, srcE, c, step, keep_prev);
            else
                cell_update_from(R, srcT[c], srcE[c], R.Te, srcE, c, step, keep_prev);
        }
        __syncthreads();
    }
    if (sample_due(R, phase, step))
        write_sample(R, global_view(R, step), S, phase == PHASE_INIT ? step : step + 1);
    // the bins filled this step have been read by the list build: empty them
    // for the next binning (runs with a large grid: emptied by k_grid)
    if (R.live && (R.bin_step || S.rebuild != 0 || phase == PHASE_INIT) &&
        (phase == PHASE_INIT || !empties_bins_in_grid(R)))
        for (int b = tid; b < R.nbins; b += blockDim.x) R.bin_n[b] = 0;
    __syncthreads();
    if (tid == 0) {
        if (R.live) {
            st->bin_over = 0;
            st->rebuild = 0;
        }
        if (phase == PHASE_STEP) {
            st->pending = deferred;
            st->step = step + 1;
            if (fold_k >= 0) fold_close(st);
        }
    }
}

// One block per run.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_finalize(const RunDev<T>* __restrict__ runs,
                                                     const int* __restrict__ run_list, int phase,
                                                     int deferred, int fold_k)
{
    __shared__ SampleScratch S;
    end_step(runs[run_list[blockIdx.x]], S, phase, deferred, fold_k);
}

// ======================================================= launch tables
// Writes a single run's launch tables into `base` (then the run list and
// the persistent list, one int each, at `ints`).
static __global__ __launch_bounds__(kBlock) void k_fill_tables(int2* __restrict__ base, int* __restrict__ ints,
                                                        TableFill f)
{
    for (int32_t e = (int32_t)(blockIdx.x * blockDim.x + threadIdx.x); e < f.n_int2;
         e += (int32_t)(gridDim.x * blockDim.x)) {
        int k = 0;
        while (k < 5 && e >= f.off[k] + f.m[k]) ++k;
        base[e] = fill_entry(f, k, e - f.off[k], f.slot);
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        ints[0] = f.rl_n > 0 ? f.slot : 0;
        ints[1] = f.pl_n > 0 ? f.slot : 0;
    }
}

// The per-run launch flags of a run's device descriptor (kick binning,
// normals drawn by the kick), written without a host copy.
template <typename T>
__global__ void k_set_run_flags(RunDev<T>* runs, int slot, int32_t bin_step, int32_t eta_drawn)
{
    runs[slot].bin_step = bin_step;
    runs[slot].eta_drawn = eta_drawn;
}

// ==================================================== persistent kernel
// One block advances one run by up to `nsteps` steps in a single launch.
// Spins, species, electron-cell ids, the electron grid, the per-cell
// electron-phonon sums and the observable rows live in LDS (positions too
// when they fit); phases are separated by block barriers only.  The
// arithmetic of every site, atom and cell is that of the multi-kernel step,
// so a run gives the same bits on either executor.
struct PersistLayout {
    uint32_t off_s, off_species, off_cell, off_pos, off_Te, off_Te2, off_acc, off_part, bytes;
    int32_t pos_in_lds;
    int32_t part_in_lds;   // the observable rows (else the run's global rows: they are
                           // written and read on sample steps only)
};

template <typename T>
__host__ __device__ inline PersistLayout persist_layout(int n, int ncell, int n_part, bool live,
                                                        int n_species, uint32_t lds_max)
{
    PersistLayout L{};
    uint32_t o = 0;
    auto take = [&](uint32_t bytes) {
        const uint32_t at = o;
        o += (bytes + 15u) & ~15u;
        return at;
    };
    L.off_s = take(3u * (uint32_t)n * (uint32_t)sizeof(T));
    L.off_species = n_species > 1 ? take((uint32_t)n) : 0u;
    L.off_cell = take(2u * (uint32_t)n);
    L.off_Te = take(8u * (uint32_t)ncell);
    L.off_Te2 = take(8u * (uint32_t)ncell);
    L.off_acc = take(8u * (uint32_t)ncell);
    L.part_in_lds = 0;
    L.off_part = 0;
    const uint32_t part_bytes = 8u * NQ * (uint32_t)n_part;
    if (o + part_bytes <= lds_max) {
        L.off_part = take(part_bytes);
        L.part_in_lds = 1;
    }
    L.pos_in_lds = 0;
    L.off_pos = 0;
    if (live && L.part_in_lds && o + (uint32_t)n * (uint32_t)sizeof(Pos4<T>) <= lds_max) {
        L.off_pos = take((uint32_t)n * (uint32_t)sizeof(Pos4<T>));
        L.pos_in_lds = 1;
    }
    L.bytes = o;
    return L;
}

struct PersistShared {
    SampleScratch S;
    int flag_rebuild;
    int flag_stop;
};

// The run's steps inside one block: load the LDS copies, step, write back.
template <typename T, typename VW, bool RADIAL>
__device__ __forceinline__ void persist_run(const RunDev<T>& R, const VW& V, double* Te2,
                                            unsigned long long* acc, PersistShared& P, int nsteps,
                                            bool pos_in_lds)
{
    RunState* st = R.st;
    const int tid = threadIdx.x, B = blockDim.x;
    const int n = R.n, nc = R.ncell;
    // load the run into LDS
    const uint16_t* cell_in = R.cellb[cell_slot(st->step)];
    for (int i = tid; i < n; i += B) {
        V.sx[i] = gld(R.sx, i);
        V.sy[i] = gld(R.sy, i);
        V.sz[i] = gld(R.sz, i);
        V.cell[i] = gld(cell_in, i);
        if (R.n_species > 1) const_cast<int8_t*>(V.species)[i] = gld(R.species, i);
        if (pos_in_lds) V.pos[i] = gld(R.pos, i);
    }
    for (int c = tid; c < nc; c += B) {
        V.Te[c] = gld(R.Te, c);
        acc[c] = 0ull;
    }
    for (int k = tid; k < R.n_part * NQ; k += B) V.partial[k] = 0.0;
    int64_t step = st->step;
    const int64_t target = st->target;
    // A step that raises an error is abandoned where the multi-kernel step
    // would abandon it: the rest of the step is skipped and the step
    // counter keeps the step's number.
    auto error_raised = [&]() {
        __syncthreads();
        if (tid == 0) P.flag_stop = st->err != 0 ? 1 : 0;
        __syncthreads();
        return P.flag_stop != 0;
    };
    const bool run = !error_raised() && step < target;
    for (int it = 0; run && it < nsteps && step < target; ++it) {
        if (tid == 0) P.flag_rebuild = 0;
        // spins: the colour sweep
        for (int pass = 0; pass < 2 * R.g.C - 1; ++pass) {
            __syncthreads();
            int colour;
            T tau;
            pass_colour(R, pass, &colour, &tau);
            for (int l = tid; l < R.g.H; l += B) spin_site<T, VW, RADIAL>(R, V, colour, tau, (uint32_t)l, step);
        }
        __syncthreads();
        // lattice: kick and drift, list rebuild when flagged
        if (R.live) {
            if constexpr (RADIAL) {
                if (R.radial) {
                    // the exchange forces read the positions of x^n: all of
                    // them before any drift
                    for (int i = tid; i < n; i += B) half_kick_radial(R, V, (uint32_t)i);
                    __syncthreads();
                }
            }
            for (int i = tid; i < n; i += B)
                if (kick_drift_atom(R, V, (uint32_t)i, PHASE_STEP, R.radial != 0))
                    atomicOr(&P.flag_rebuild, 1);
            if (tid == 0) st->step = step;   // read by the overflow diagnostics
            __syncthreads();
            if (P.flag_rebuild) {
                for (int i = tid; i < n; i += B) nbr_bin_atom(R, V, (uint32_t)i);
                __syncthreads();
                if (tid == 0 && st->bin_over) raise_bin_overflow(R);
                if (error_raised()) break;
                if (tid == 0) st->n_rebuild += 1;
                for (int b = tid; b < R.nbins; b += B) nbr_sort_bin(R, b);
                __syncthreads();
                for (int i = tid; i < n; i += B)
                    nbr_build_atom<T, VW, true>(R, V, (uint32_t)i);
                if (error_raised()) break;
                for (int b = tid; b < R.nbins; b += B) R.bin_n[b] = 0;
            }
        }
        // forces, electron-phonon step, observable rows
        const bool obs = sample_due(R, PHASE_STEP, step);
        if (R.live || obs) {
            for (int base = 0; base < n; base += B) {
                const int i = base + tid;
                ObsTerms o{};
                if (i < n) atom_final_atom<T, VW, 1, RADIAL>(R, V, (uint32_t)i, PHASE_STEP, step, obs, acc, o);
                if (obs) wave_write_row(o, V.partial, i - (tid & 63), n);
            }
        }
        if (error_raised()) break;
        // electron grid
        if (R.ttm_mode == 1) {
            if (R.kappa_e != 0.0) {
                for (int sub = 0; sub < R.n_sub; ++sub) {
                    for (int c = tid; c < nc; c += B)
                        diffuse_cell(R, (sub & 1) ? Te2 : V.Te, (sub & 1) ? V.Te : Te2, c, sub);
                    __syncthreads();
                }
            }
            for (int c = tid; c < nc; c += B) cell_update(R, V.Te, acc, c, step);
            if (error_raised()) break;
        } else if (R.ttm_mode == 2) {
            const double Tn = te_stepped(R, step + 1);
            for (int c = tid; c < nc; c += B) V.Te[c] = Tn;
            __syncthreads();
        }
        if (obs) write_sample(R, V, P.S, step + 1);
        ++step;
    }
    __syncthreads();
    // write the run back (cell ids of the current positions to the current
    // step's buffer)
    uint16_t* cell_out = R.cellb[cell_slot(step)];
    for (int i = tid; i < n; i += B) {
        gst(R.sx, i, V.sx[i]);
        gst(R.sy, i, V.sy[i]);
        gst(R.sz, i, V.sz[i]);
        gst(cell_out, i, V.cell[i]);
        if (pos_in_lds) gst(R.pos, i, V.pos[i]);
    }
    for (int c = tid; c < nc; c += B) gst(R.Te, c, V.Te[c]);
    if (tid == 0) {
        st->step = step;
        st->rebuild = 0;
    }
}

// MAXT: the largest block the instantiation is compiled for (512: up to 256
// registers per lane; 1024: up to 128, with some spilling).
template <typename T, int MAXT, bool RADIAL = false>
__global__ __launch_bounds__(MAXT) void k_persist(const RunDev<T>* __restrict__ runs,
                                                   const int* __restrict__ run_list, int nsteps,
                                                   uint32_t lds_max)
{
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ PersistShared P;
    const RunDev<T>& R = runs[run_list[blockIdx.x]];
    const int n = R.n;
    const PersistLayout L = persist_layout<T>(n, R.ncell, R.n_part, R.live != 0, R.n_species, lds_max);
    T* sx = reinterpret_cast<T*>(smem + L.off_s);
    const int8_t* species =
        R.n_species > 1 ? reinterpret_cast<const int8_t*>(smem + L.off_species) : R.species;
    uint16_t* cell = reinterpret_cast<uint16_t*>(smem + L.off_cell);
    double* Te = reinterpret_cast<double*>(smem + L.off_Te);
    double* Te2 = reinterpret_cast<double*>(smem + L.off_Te2);
    unsigned long long* acc = reinterpret_cast<unsigned long long*>(smem + L.off_acc);
    double* partial = L.part_in_lds ? reinterpret_cast<double*>(smem + L.off_part) : R.partial;
    if (L.pos_in_lds) {
        const View<T, InLds, InLds> V{sx, sx + n, sx + 2 * n, species, cell,
                                      reinterpret_cast<Pos4<T>*>(smem + L.off_pos), Te, partial};
        persist_run<T, View<T, InLds, InLds>, RADIAL>(R, V, Te2, acc, P, nsteps, true);
    } else {
        const View<T, InLds, InGlobal> V{sx, sx + n, sx + 2 * n, species, cell, R.pos, Te, partial};
        persist_run<T, View<T, InLds, InGlobal>, RADIAL>(R, V, Te2, acc, P, nsteps, false);
    }
}

}  // namespace sl
