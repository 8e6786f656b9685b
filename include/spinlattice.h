/*
 * spinlattice.h -- C ABI of the MI355X (gfx950) three-temperature
 * atomistic spin-lattice step.
 *
 * One timestep n -> n+1 of a run (arXiv 2608.18541):
 *   1. spins: stochastic Landau-Lifshitz-Gilbert update, Eq. (1) of
 *      Methods A, with the effective field H_i = -(1/mu_i) dH/ds_i
 *      (Heisenberg exchange over the lattice neighbour shells plus Zeeman)
 *      and a Langevin field whose variance is 2 alpha k_B T_e / (gamma mu_i
 *      mu_B dt) (Methods C: deterministic torque ~ 1/mu_i, noise amplitude
 *      ~ 1/sqrt(mu_i)); T_e is the electron temperature of the grid cell
 *      that contains the atom (Eq. (2), Methods B).  The spins are swept in
 *      checkerboard colours, forward with half steps and back again, every
 *      colour update being the exact constant-field flow of Eq. (1);
 *   2. lattice: velocity Verlet with a Morse pair potential cut (and
 *      shifted) at rc (the live lattice of Methods A);
 *   3. electron-phonon exchange: an Ornstein-Uhlenbeck velocity step at the
 *      cell's T_e with friction G_el / (3 n k_B); the cell's electrons lose
 *      the mean energy the step hands to its atoms given their velocities,
 *      (1 - c1^2)(3/2 k_B T_e - m v^2/2) per atom (Methods B: both baths
 *      read the same T_e grid; the coupling is the two-temperature term
 *      with the cell's atomic temperature);
 *   4. electron grid: explicit finite differences of
 *      d(gamma_e T_e^2/2)/dt = kappa_e lap T_e + S(z,t) - (e-ph power), with
 *      a Gaussian laser source S (Methods B).
 * Noise is Philox4x32-10 keyed by (seed, run id) at counter (canonical site,
 * step, stream), so a run's trajectory does not depend on what else runs.
 *
 * Units: Angstrom, ps, eV, amu, K, Tesla, Bohr magnetons.
 * Arrays exchanged with the caller are host memory in canonical site order
 * ((z*Ly + y)*Lx + x)*nb + b (nb = 1 sc, 2 bcc, 4 fcc; see sl_system_desc);
 * vectors are [n][3] row-major doubles.  Host pointers are borrowed for the
 * duration of the call.  The library owns all device memory, obtained from
 * the caller's allocator when one is given (else hipMalloc).  Streams are
 * borrowed, never destroyed.  A handle is not thread-safe.
 *
 * Every entry point returns SL_OK or a negative status and never throws;
 * sl_last_error() returns a message for the calling thread's last failure.
 */
#ifndef SPINLATTICE_H
#define SPINLATTICE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t sl_status;
enum {
    SL_OK = 0,
    SL_EINVAL = -1,    /* invalid argument; nothing was changed            */
    SL_ENOMEM = -2,    /* device memory or the batch memory budget exceeded */
    SL_EHIP = -3,      /* a HIP runtime call failed                         */
    SL_ENUMERIC = -4,  /* a run hit a numerical error; it is frozen and the
                          other runs of a batch go on.  Detected on the
                          device: a negative or non-finite electron energy,
                          a neighbour-table overflow, an electron-phonon
                          energy out of range, and the watchdog -- a spin
                          that is not a finite unit vector when it is
                          updated (|s|^2 off by more than about 1e-4 before
                          the renormalisation of the update), or a kick
                          that leaves a non-finite velocity or
                          displacement.  Reported by the next call that
                          waits (sl_synchronize, sl_get_state, ...)        */
    SL_EBUSY = -5      /* no free slot in a batch                           */
};

enum { SL_LATTICE_SC = 0, SL_LATTICE_BCC = 1, SL_LATTICE_FCC = 2 };
enum { SL_FP64 = 0, SL_FP32 = 1 };

/* Device-memory provider (e.g. PyTorch's caching allocator).  alloc returns
 * at least `bytes` bytes of device memory aligned to 256 bytes or NULL. */
typedef struct sl_allocator {
    void* ctx;
    void* (*alloc)(void* ctx, size_t bytes);
    void (*free)(void* ctx, void* ptr);
} sl_allocator;

/* One run.  Shell k couples the sites at the k-th neighbour distance of the
 * ideal lattice with J[k][species_i][species_j] (eV, H = -sum_bonds J s_i.s_j,
 * negative J antiferromagnetic).  Supported: sc with 1 shell, bcc with 1 or
 * 2 shells (the shells the checkerboard colouring keeps bond-free inside a
 * colour), fcc with 1 shell (the 12 nearest neighbours; coloured by basis
 * site, so no two neighbours share a colour).  Every ncell[d] must be
 * >= 2, and even for sc and bcc.  Basis sites: bcc b = 0 corner, 1 body
 * centre; fcc b = 0 corner, 1, 2, 3 the centres of the xy, xz and yz faces;
 * every site sits a quarter lattice constant above its ideal point along
 * each axis. */
typedef struct sl_system_desc {
    int32_t lattice;          /* SL_LATTICE_SC, SL_LATTICE_BCC or SL_LATTICE_FCC   */
    int32_t ncell[3];         /* unit cells per dimension                         */
    double a;                 /* lattice constant, Angstrom                       */
    int32_t n_species;        /* 1..4                                             */
    const int8_t* species;    /* [n] species of each site, or NULL (all 0)        */
    double mu[4];             /* moment per species, mu_B (> 0)                   */
    double mass[4];           /* mass per species, amu (> 0 when live)            */
    int32_t n_shells;         /* 1 or 2                                           */
    double J[2][4][4];        /* eV                                               */
    double B[3];              /* applied field, T                                 */
    double K[4];              /* uniaxial anisotropy per species along z, eV per
                                 atom: energy -K s_z^2, field 2 K s_z / (mu mu_B) */
    double alpha;             /* Gilbert damping (>= 0)                           */
    int32_t noise_mode;       /* 0: FDT noise ~ 1/sqrt(mu);
                                 1: control ~ 1/mu (equal at mu_ref)             */
    double mu_ref;            /* mu_B, used by noise_mode 1                       */
    int32_t lattice_mode;     /* 0: positions frozen at the sites; 1: live        */
    double morse[4];          /* D (eV), alpha (1/A), r0 (A), cutoff rc (A)       */
    double skin;              /* neighbour-list skin, A (> 0 when live)           */
    double dt;                /* ps (> 0)                                         */
    uint32_t seed, run_id;    /* Philox key                                       */
    int32_t precision;        /* SL_FP64 or SL_FP32 (storage and spin arithmetic)  */
    int32_t obs_every;        /* record observables every k steps (0: never)     */
    int32_t obs_capacity;     /* ring of samples kept on the device (>= 1)        */
    const double* spin0;      /* [n][3] unit spins (required, |s| within 1e-6)    */
    const double* vel0;       /* [n][3] A/ps or NULL (zero)                       */
    const double* disp0;      /* [n][3] displacement from the ideal site, A, or NULL */
    void* stream;             /* hipStream_t to run on, or NULL (library stream)  */
    const sl_allocator* alloc;/* or NULL (hipMalloc)                              */
    /* Radial exchange (Methods A; the re-derivation of the radial exchange
     * function), live lattices only.  0: J[k] are the bonds' constants.  1:
     * J[k][a][b] is the amplitude J1 of J(r) = 4 J1 x (1 - J2 x) e^{-x},
     * x = (r / J3)^2, evaluated at a bond's current (minimum-image) length,
     * and the bond exerts the force -dJ/dr (s_i . s_j) on its two atoms.  The
     * bonds stay those of the ideal lattice's shells (the radial function
     * sets their strength).  A step then applies the first half kick (pair
     * and exchange forces at the old positions with the swept spins) after
     * the whole colour sweep; such runs do not merge colour sweeps. */
    int32_t exch_radial;      /* 0 or 1                                           */
    double exch_r[2][2];      /* per shell: J2 (dimensionless), J3 (A, > 0)       */
} sl_system_desc;

/* Electron-temperature grid over the periodic box, cell (i,j,k) at index
 * (k*n1 + j)*n0 + i; cell c holds the atoms whose wrapped position p has
 * floor(p_d / (box_d / n_d)) = c_d.  mode 0 keeps T_e fixed (no
 * electron-phonon step); mode 1 runs the two-temperature update; mode 2
 * prescribes a uniform stepped T_e(t): step_T[0] before step_end[0],
 * step_T[1] before step_end[1], step_T[2] after (the heat-pulse profile of
 * the production runs; no electron-phonon step), step n using
 * T_e(n dt). */
typedef struct sl_ttm_desc {
    int32_t n[3];             /* cells per dimension (product <= 65535)           */
    int32_t mode;             /* 0 fixed field, 1 two-temperature                 */
    double Te0;               /* uniform initial T_e, K (if Te_init is NULL)      */
    const double* Te_init;    /* [n0*n1*n2] K, or NULL                            */
    double gamma_e;           /* C_e = gamma_e T_e, eV A^-3 K^-2 (> 0 in mode 1)  */
    double G_el;              /* eV ps^-1 A^-3 K^-1                                */
    double kappa_e;           /* eV ps^-1 A^-1 K^-1                               */
    int32_t n_sub;            /* diffusion sub-steps per step (>= 1)              */
    double S0;                /* peak laser power density, eV ps^-1 A^-3          */
    double t0, fwhm;          /* pulse centre and FWHM, ps                        */
    int32_t profile;          /* 0 uniform; 1 cells whose centre z > box_z - depth */
    double depth;             /* A                                                */
    double step_T[3];         /* mode 2: T_e of the three stages, K (>= 0)        */
    double step_end[2];       /* mode 2: ends of stages 1 and 2, ps (ascending)   */
} sl_ttm_desc;

/* One observable sample, taken after a step (and once at step 0). */
typedef struct sl_obs {
    double t;                 /* ps                                               */
    int64_t step;
    double M[4][3];           /* mean spin per species                            */
    double m[3];              /* mean spin of all sites                           */
    double m_abs;
    double E_ex, E_z;         /* exchange energy; single-site energy (Zeeman and
                                 uniaxial anisotropy), eV                        */
    double KE, PE;            /* lattice kinetic and Morse energy, eV             */
    double E_e;               /* electron energy sum gamma_e T_e^2/2 V_cell, eV    */
    double Te_mean, Te_max;   /* K                                                */
    double Tl;                /* 2 KE / (3 n k_B), K                              */
    double Tspin[4];          /* sum |s x h|^2 / (2 k_B sum s.h) per species, K    */
} sl_obs;

typedef struct sl_system_s* sl_system;

/* Creates a run on the device (Methods A and D: the lattice, its spins and
 * atoms; the GdFeCo model for fcc alloys): copies the description and initial state,
 * builds the neighbour tables, computes the initial forces and (if
 * obs_every > 0) records the step-0 sample.  The electron grid starts as
 * one fixed cell at T_e = 0 until sl_set_ttm_grid is called.
 * SL_EINVAL for any invalid field (listed above) or a box shorter than
 * 3 (rc + skin) in a live dimension; *out is set only on success. */
sl_status sl_init_system(const sl_system_desc* desc, sl_system* out);

/* Replaces the electron-temperature grid of Methods B (fields above).  Only before the
 * first sl_step.  SL_EINVAL when an explicit diffusion sub-step would be
 * unstable for the initial grid: kappa_e (dt/n_sub) sum_d 2/h_d^2 >
 * gamma_e min T_e (h_d the cell widths; the linearised diffusivity is
 * kappa_e / (gamma_e T_e)). */
sl_status sl_set_ttm_grid(sl_system h, const sl_ttm_desc* ttm);

/* Enqueues n_steps timesteps on the run's stream and returns (asynchronous).
 * One step is the splitting of Methods A-C: the colour sweep of spin updates
 * (Eqs. (1)-(2)), the lattice's velocity Verlet step, the electron-phonon
 * step and the two-temperature grid update (Methods B), then a sample.
 * The first call after creation, a checkpoint restore or a tuning change
 * allocates the launch tables (through the system's allocator) and captures
 * a HIP graph of the steps. */
sl_status sl_step(sl_system h, int64_t n_steps);

/* For callers that cannot allocate device memory -- code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation: enqueues
 * n_steps timesteps exactly as sl_step does (the same kernels in the same
 * order, so the same results bit for bit), but allocates and frees nothing.
 * The launch tables are written, by a kernel on the run's stream, into a
 * static device buffer of SL_NOALLOC_SCRATCH_BYTES that every GPU the
 * library runs on holds until the process ends, and every step is launched
 * directly instead of through a HIP graph.  SL_EINVAL, with nothing
 * enqueued, when the system's tables exceed the buffer (about half a million
 * thread blocks: a few 10^7 sites) or for n_steps < 0.  Every call on a GPU
 * rewrites that GPU's one buffer, so calls whose work overlaps on one GPU
 * (systems stepped on different streams, other host threads) race: the
 * caller serialises them, e.g. on one stream.  Asynchronous like sl_step. */
#define SL_NOALLOC_SCRATCH_BYTES (4u << 20)
sl_status sl_step_noalloc(sl_system h, int64_t n_steps);

/* Waits for the run's stream.  SL_ENUMERIC if the run hit a numerical error
 * (the failure detection of the conventions above: a negative or non-finite
 * electron energy, a spin that was not a finite unit vector, a non-finite
 * velocity or displacement, a neighbour table overflow); the run is frozen
 * at the step where it was found. */
sl_status sl_synchronize(sl_system h);

/* The observables of Methods G and Results A (sublattice magnetisation,
 * energies, the three temperatures).
 * Waits, then copies up to max_samples observable samples not yet returned,
 * oldest first, into out (host).  Samples older than the device ring
 * capacity are lost; *n_out is the number copied. */
sl_status sl_observables(sl_system h, sl_obs* out, int64_t max_samples, int64_t* n_out);

/* The dynamical state of Methods A and B (positions, velocities, spins,
 * electron temperatures).
 * Waits, then copies the state to host arrays in canonical order (any
 * pointer may be NULL): positions wrapped into the box [n][3], velocities
 * [n][3], spins [n][3], electron temperatures [cells]. */
sl_status sl_get_state(sl_system h, double* x, double* v, double* s, double* Te);

/* Checkpoint restore of the state of Methods A and B.
 * Waits, then replaces parts of the state from host arrays in canonical
 * order (checkpoint restore; any pointer may be NULL to keep the current
 * values): positions [n][3] in A (any periodic image; stored as the
 * minimum-image displacement from the ideal site), velocities [n][3] in A/ps
 * (ignored for a frozen lattice), spins [n][3] (unit vectors within 1e-6),
 * electron temperatures [cells] in K.  Species, parameters, the step counter
 * (so the Philox noise continues) and the returned samples are kept.
 * Electron-cell ids, neighbour lists and forces are recomputed for the new
 * positions exactly as at initialisation, and with obs_every > 0 one sample
 * of the new state is recorded at the current step.  Synchronous.
 * SL_EINVAL, with the state unchanged, for a non-unit spin, a non-finite
 * position or velocity, or a negative or non-finite temperature. */
sl_status sl_set_state(sl_system h, const double* x, const double* v, const double* s,
                       const double* Te);

/* Device-side counters of one run. */
typedef struct {
    int64_t steps;            /* completed steps                                     */
    int64_t samples;          /* observable samples recorded (returned or not)       */
    int64_t list_rebuilds;    /* Verlet-list builds, the initial one included
                                 (0 for a frozen lattice)                            */
    int32_t max_list;         /* longest neighbour list built so far                 */
    int32_t list_capacity;    /* entries per atom the list holds (0: frozen lattice) */
    int32_t list_rescans;     /* bins scanned a second time by list builds from
                                 unsorted bins (more than 16 accepted atoms)        */
    int32_t error;            /* the run's error bits (0: none; nonzero: frozen)     */
} sl_run_stats;

/* Waits, then reads the run's counters (the neighbour lists of the live
 * lattice of Methods A, the error bits).  SL_EINVAL for a null output. */
sl_status sl_stats(sl_system h, sl_run_stats* out);

/* Number of sites, electron cells and completed steps (host view). */
sl_status sl_info(sl_system h, int64_t* n_sites, int64_t* n_cells, int64_t* steps);

/* Device bytes a run with this description would hold (the admission test
 * of batches of replicas, Methods F). */
sl_status sl_footprint_bytes(const sl_system_desc* desc, const sl_ttm_desc* ttm,
                             size_t* bytes);

/* Measurement, no passage of the method: the steps of sl_step, with timings.
 * Runs n_steps (at most 4096) launching every kernel directly, each timed
 * by HIP events stamped by its own dispatch; returns the average device time
 * (ms) per launch of each kernel class and the launch counts: 0 spin colour
 * pass, 1 neighbour-list rebuild (when due), lattice forces and
 * electron-phonon step, 2 colour pass carrying the lattice's kick, drift
 * and binning (live lattices), 3 binning for a rebuild (large engines),
 * electron grid and end-of-step reductions, 4 persistent kernel (one launch
 * for all steps), 5 colour pass 1 carrying the force kernel of class 1
 * (tuning fuse_force). */
sl_status sl_step_profiled(sl_system h, int64_t n_steps, double avg_ms[6], int64_t launches[6]);

/* Launch shape of the step kernels (no passage of the method: a choice of
 * the implementation).  Every choice performs the same
 * arithmetic in the same order for each site, atom and cell, so results are
 * bitwise identical; only the speed changes (an autotuner picks it). */
typedef struct sl_tuning {
    int32_t spin_block;       /* threads per block of the colour passes: 64, 128,
                                 256, or 0 automatic (the largest giving at least
                                 256 blocks per pass)                          */
    int32_t spin_spt;         /* sites per thread in a colour pass: 1, 2, 4          */
    int32_t atom_block;       /* threads per block of the lattice kernels: 64..256   */
    int32_t graph_steps;      /* steps captured per HIP graph replay: 1..256;
                                 runs that merge their sweeps replay chunks
                                 instead (the largest common divisor of their
                                 sample intervals up to 64, or graph_steps when
                                 none takes samples)                          */
    int32_t persist_block;    /* 0: all runs on the multi-kernel step; 256, 512 or
                                 1024: runs that fit in LDS advance in a persistent
                                 kernel, one block of this many threads per run
                                 (batches default to 1024 in FP32 and 512 in FP64,
                                 single systems to 0)                               */
    int32_t xcd_order;        /* 1: work tables ordered so that each of the 8 XCDs
                                 receives one contiguous range of tiles (its L2
                                 then holds their neighbours); 0: round-robin    */
    int32_t bin_mode;         /* neighbour binning: 1 by the kick every step, 2 by a
                                 separate launch only when a list is rebuilt, 0
                                 automatic (1 up to 2^20 live atoms)             */
    int32_t atom_lanes;       /* lanes sharing one atom's neighbour list in the
                                 force kernel: 1, 2 or 4 (atom_block / atom_lanes
                                 atoms per block, at least 64), 0 automatic (4 up
                                 to 2^16 atoms on the multi-kernel step, 2 up to
                                 2^17, then 1).  The pair sums are four
                                 interleaved partial sums over the list in every
                                 case, hence the same bits                   */
    int32_t merge_sweeps;     /* 1 (default): the runs on the multi-kernel step
                                 (a system, or batch runs with one colour count
                                 at the same step modulo the chunk length)
                                 apply the last colour half step of a step
                                 together with the next step's first, in chunks
                                 ending on every sample step; a single run with
                                 at most 4096 non-diffusing electron cells also
                                 ends each step of a chunk inside the next
                                 step's first colour pass.  0: one launch per
                                 colour pass and a step end per step.  Same bits
                                 either way, except that a negative electron
                                 energy met at a folded step end stops the run
                                 one step later (SL_ENUMERIC either way)      */
    int32_t spin_access;      /* how the colour passes of bcc runs with one species
                                 and constant exchange that carry no lattice
                                 kick and no deferred half step read their
                                 neighbours.  0 (default): every site gathers
                                 them from global memory, which measured
                                 fastest.  1: a block stages the neighbour
                                 rows of a tile of 4 x 4 (or 2 x 2) rows in
                                 LDS with 16-byte loads (when the tile divides
                                 the rows and planes and a row holds whole
                                 16-byte vectors; otherwise 0 runs).  Same
                                 bits either way                              */
    int32_t fuse_force;       /* 1 (default): in the merged chunks (merge_sweeps)
                                 of multi-kernel runs with constant exchange and
                                 no anisotropy, a live lattice among them (one or
                                 two sites per thread, atom_block a multiple of
                                 the colour-pass block), each step kicks the atoms
                                 in colour pass 0 and runs the force kernel in
                                 the launch of colour pass 1, but for the
                                 chunk's last step: one launch fewer per step.  0: the kick rides with
                                 colour pass 1 and the force kernel follows the
                                 sweep.  Same bits either way                 */
} sl_tuning;

/* Waits for the stream, then applies a launch shape (SL_EINVAL if out of
 * range; nothing changes then). */
sl_status sl_set_tuning(sl_system h, const sl_tuning* t);
sl_status sl_get_tuning(sl_system h, sl_tuning* t);

void sl_destroy(sl_system h);

/* Message of the calling thread's last failed call ("" if none). */
const char* sl_last_error(void);

/* -------------------------------------------------------------- batching
 * Many independent runs advance together: every kernel launch covers all
 * active runs (Methods F: replicas share nothing), and each run sees exactly
 * the arithmetic it would see alone, so its trajectory is bitwise the same.
 * Runs join and leave between advances (continuous batching). */
typedef struct sl_batch_s* sl_batch;

typedef struct sl_batch_desc {
    int32_t precision;        /* SL_FP64 or SL_FP32 for every run of the batch    */
    int32_t max_runs;         /* slots                                            */
    size_t mem_budget;        /* device bytes the runs may hold (0: unlimited)    */
    int32_t graph_steps;      /* steps captured per HIP graph replay (0: default) */
    void* stream;             /* hipStream_t or NULL                              */
    const sl_allocator* alloc;
} sl_batch_desc;

typedef struct sl_run_info {
    int32_t slot;
    int32_t status;           /* SL_OK or SL_ENUMERIC                             */
    int64_t steps_done;
    int64_t steps_target;
    int64_t n_samples;        /* samples recorded so far                          */
} sl_run_info;

/* An empty batch of replica slots (Methods F). */
sl_status sl_batch_create(const sl_batch_desc* desc, sl_batch* out);

/* Admits a replica (Methods F; its setup as sl_init_system and
 * sl_set_ttm_grid) that will take n_steps steps (desc->precision, stream and
 * alloc are ignored: the batch's apply).  SL_EBUSY when no slot is free,
 * SL_ENOMEM when its footprint does not fit the remaining budget. */
sl_status sl_batch_add(sl_batch b, const sl_system_desc* desc, const sl_ttm_desc* ttm,
                       int64_t n_steps, int32_t* slot);

/* Enqueues up to n_steps steps (as sl_step: Methods A-C) for every active
 * run (a run stops at its target).  Asynchronous. */
sl_status sl_batch_advance(sl_batch b, int64_t n_steps);

/* Waits, then reads the counters of the run in a slot (as sl_stats).
 * SL_EINVAL for a slot not in use. */
sl_status sl_batch_stats(sl_batch b, int32_t slot, sl_run_stats* out);

/* Host view of the slots in use (no wait): fills up to cap entries. */
sl_status sl_batch_runs(sl_batch b, sl_run_info* info, int32_t cap, int32_t* n_out);

/* Waits, then returns a run's state and samples (as sl_get_state and
 * sl_observables; NULL pointers skip). */
sl_status sl_batch_get(sl_batch b, int32_t slot, double* x, double* v, double* s, double* Te,
                       sl_obs* obs, int64_t max_samples, int64_t* n_obs);

/* Releases a slot and its device memory (waits for the stream first). */
sl_status sl_batch_remove(sl_batch b, int32_t slot);

/* As sl_batch_advance, launching every kernel directly with HIP events
 * around each; returns the average device time (ms) per launch of each
 * kernel class (as sl_step_profiled) and the launch counts. */
sl_status sl_batch_advance_profiled(sl_batch b, int64_t n_steps, double avg_ms[6],
                                    int64_t launches[6]);

/* Launch shape of a batch (as sl_set_tuning / sl_get_tuning). */
sl_status sl_batch_set_tuning(sl_batch b, const sl_tuning* t);
sl_status sl_batch_get_tuning(sl_batch b, sl_tuning* t);

/* Bytes of the budget in use. */
sl_status sl_batch_memory(sl_batch b, size_t* used, size_t* budget);

sl_status sl_batch_synchronize(sl_batch b);

void sl_batch_destroy(sl_batch b);

#ifdef __cplusplus
}
#endif

#endif /* SPINLATTICE_H */
