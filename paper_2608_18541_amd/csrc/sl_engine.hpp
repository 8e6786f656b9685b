// sl_engine.hpp -- the host runtime of the spin-lattice step: validation,
// run sizing, and the engine that owns runs and launches the kernels.  The
// engine template is instantiated once per precision in its own translation
// unit (sl_engine_fp32.hip, sl_engine_fp64.hip); the C ABI (spinlattice.hip)
// reaches it through the Engine interface and the two factories.
//
// An engine owns up to max_runs independent runs of one precision.  Each run
// lives in its own device allocation (spins, displacements, velocities,
// forces, neighbour tables, electron grid, observable ring); a device table
// of run descriptors plus block->(run, offset) work tables let every kernel
// launch cover all active runs.  A single system is an engine with one run.
// Steps are replayed from a captured HIP graph of graph_steps steps, or, for
// runs on the multi-kernel step, of chunks of steps whose adjacent colour-0
// half steps share one pass (chunk length dividing the sample interval, so
// that every sample sees complete sweeps).
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_ext.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/spinlattice.h"
#include "sl_kernels.hpp"

namespace slrt {

// message of the calling thread's last failure (defined with the C ABI)
extern thread_local std::string g_err;

inline sl_status fail(sl_status code, const std::string& msg)
{
    g_err = msg;
    return code;
}

#define SL_HIP(call)                                                                    \
    do {                                                                                \
        hipError_t e_ = (call);                                                         \
        if (e_ != hipSuccess)                                                           \
            return fail(SL_EHIP, std::string(#call) + ": " + hipGetErrorString(e_));    \
    } while (0)

// ------------------------------------------------------------ allocation
struct DevAlloc {
    sl_allocator a{};
    bool custom = false;
    void* get(size_t bytes)
    {
        if (bytes == 0) bytes = 256;
        if (custom) return a.alloc(a.ctx, bytes);
        void* p = nullptr;
        if (hipMalloc(&p, bytes) != hipSuccess) return nullptr;
        return p;
    }
    void put(void* p)
    {
        if (!p) return;
        if (custom)
            a.free(a.ctx, p);
        else
            (void)hipFree(p);
    }
};

inline size_t align256(size_t v) { return (v + 255) & ~size_t(255); }

constexpr int64_t kPersistChunk = 4096;   // steps per persistent launch

template <typename X> struct ident {
    using type = X;
};

// Kernel launch; when profiling, through HIP's extended launch, whose start
// and stop events are stamped by the dispatch itself (the kernel's own
// duration, as a kernel trace reports it, without the queue overhead that
// events recorded around the launch would add).
template <typename... KA>
inline void launch(void (*k)(KA...), dim3 grid, dim3 block, uint32_t shmem, hipStream_t st, hipEvent_t e0,
            hipEvent_t e1, typename ident<KA>::type... args)
{
    if (e0)
        hipExtLaunchKernelGGL(k, grid, block, shmem, st, e0, e1, 0, args...);
    else
        hipLaunchKernelGGL(k, grid, block, shmem, st, args...);
}

// Workgroups are dispatched round-robin over the accelerator's 8 XCDs
// (block b runs on XCD b mod 8), each with its own L2.  Reordering a work
// table so that every XCD receives one contiguous range of tiles keeps the
// neighbouring rows and planes of a tile in the same L2.  Any order gives the
// same results; only the cache traffic changes.
constexpr size_t kXcds = sl::kXcdCount;
template <typename E> inline void xcd_order(std::vector<E>& t)
{
    const size_t m = t.size();
    if (m < 2 * kXcds) return;
    const size_t per = (m + kXcds - 1) / kXcds;
    std::vector<E> o;
    o.reserve(m);
    for (size_t j = 0; j < per; ++j)
        for (size_t x = 0; x < kXcds; ++x) {
            const size_t src = x * per + j;   // only the last j can run past the end
            if (src < m) o.push_back(t[src]);
        }
    t.swap(o);
}

// Carves typed sub-arrays out of one allocation.
struct Carver {
    size_t off = 0;
    char* base = nullptr;
    template <typename U> U* take(size_t count)
    {
        size_t o = off;
        off += align256(count * sizeof(U));
        return base ? reinterpret_cast<U*>(base + o) : nullptr;
    }
};

// ------------------------------------------------------------ validation
// Ideal position of a site (as the kernels place it): cell corner, basis
// shift and a quarter lattice constant along each axis.
inline void ideal_position(const sl::Geom& g, const sl::Site& s, double a, double r0[3])
{
    const uint32_t hb = sl::basis_half_bits(g.nb, s.b);
    const int c[3] = {s.x, s.y, s.z};
    for (int k = 0; k < 3; ++k) r0[k] = (c[k] + ((hb >> k) & 1u ? 0.75 : 0.25)) * a;
}

// basis sites per cubic cell
inline int basis_count(int lattice)
{
    return lattice == SL_LATTICE_BCC ? 2 : (lattice == SL_LATTICE_FCC ? 4 : 1);
}

inline std::string validate_desc(const sl_system_desc* d)
{
    if (!d) return "null description";
    if (d->lattice != SL_LATTICE_SC && d->lattice != SL_LATTICE_BCC && d->lattice != SL_LATTICE_FCC)
        return "lattice must be 0 (sc), 1 (bcc) or 2 (fcc)";
    for (int k = 0; k < 3; ++k) {
        if (d->ncell[k] < 2) return "every ncell must be >= 2";
        // the checkerboard colourings need even counts; fcc colours by basis
        if (d->lattice != SL_LATTICE_FCC && (d->ncell[k] & 1)) return "every ncell must be even (sc, bcc)";
    }
    const int64_t nb = basis_count(d->lattice);
    const int64_t n = nb * (int64_t)d->ncell[0] * d->ncell[1] * d->ncell[2];
    // per-atom arrays are addressed with 32-bit byte offsets (32 B per atom
    // at most)
    if (n >= (1ll << 27)) return "too many sites (at most 2^27 - 1)";
    if (d->ncell[0] > 1024 || d->ncell[1] > 1024 || d->ncell[2] > 1024) return "ncell above 1024";
    if (!(d->a > 0.0)) return "lattice constant must be positive";
    if (d->n_species < 1 || d->n_species > 4) return "n_species must be 1..4";
    for (int s = 0; s < d->n_species; ++s) {
        if (!(d->mu[s] > 0.0)) return "every moment must be positive";
        if (d->lattice_mode == 1 && !(d->mass[s] > 0.0)) return "every mass must be positive";
    }
    if (d->lattice == SL_LATTICE_SC && d->n_shells != 1) return "sc supports one exchange shell";
    if (d->lattice == SL_LATTICE_FCC && d->n_shells != 1) return "fcc supports one exchange shell";
    if (d->lattice == SL_LATTICE_BCC && (d->n_shells < 1 || d->n_shells > 2)) return "bcc supports one or two shells";
    if (!(d->alpha >= 0.0)) return "alpha must be >= 0";
    if (d->noise_mode != 0 && d->noise_mode != 1) return "noise_mode must be 0 or 1";
    if (d->noise_mode == 1 && !(d->mu_ref > 0.0)) return "noise_mode 1 needs mu_ref > 0";
    if (!(d->dt > 0.0)) return "dt must be positive";
    if (d->precision != SL_FP64 && d->precision != SL_FP32) return "precision must be 0 or 1";
    if (d->obs_every < 0) return "obs_every must be >= 0";
    if (d->obs_every > 0 && d->obs_capacity < 1) return "obs_capacity must be >= 1";
    if (!d->spin0) return "spin0 is required";
    if (d->species)
        for (int64_t i = 0; i < n; ++i)
            if (d->species[i] < 0 || d->species[i] >= d->n_species) return "species out of range";
    for (int64_t i = 0; i < n; ++i) {
        const double* s = d->spin0 + 3 * i;
        double nn = std::sqrt(s[0] * s[0] + s[1] * s[1] + s[2] * s[2]);
        if (!(std::fabs(nn - 1.0) <= 1e-6)) return "initial spins must be unit vectors";
    }
    if (d->lattice_mode != 0 && d->lattice_mode != 1) return "lattice_mode must be 0 or 1";
    if (d->exch_radial != 0 && d->exch_radial != 1) return "exch_radial must be 0 or 1";
    if (d->exch_radial) {
        if (d->lattice_mode != 1) return "radial exchange needs a live lattice";
        for (int k = 0; k < d->n_shells; ++k)
            if (!(d->exch_r[k][1] > 0.0) || !std::isfinite(d->exch_r[k][0]))
                return "radial exchange needs J3 > 0 and a finite J2 per shell";
    }
    if (d->lattice_mode == 1) {
        if (!(d->morse[3] > 0.0) || !(d->skin > 0.0)) return "Morse cutoff and skin must be positive";
        const double reach = d->morse[3] + d->skin;
        for (int k = 0; k < 3; ++k)
            if (d->ncell[k] * d->a < 3.0 * reach) return "box must be at least 3 (rc + skin) along every axis";
    }
    return "";
}

inline std::string validate_ttm(const sl_ttm_desc* t, const sl_system_desc* d)
{
    if (!t) return "null grid";
    int64_t nc = 1;
    for (int k = 0; k < 3; ++k) {
        if (t->n[k] < 1) return "grid cells must be >= 1";
        nc *= t->n[k];
    }
    if (nc > 65535) return "at most 65535 electron cells";
    if (t->mode < 0 || t->mode > 2) return "grid mode must be 0, 1 or 2";
    if (t->mode == 2) {
        for (int k = 0; k < 3; ++k)
            if (!(t->step_T[k] >= 0.0)) return "stepped temperatures must be >= 0";
        if (!(t->step_end[0] <= t->step_end[1])) return "stage ends must be ascending";
    }
    double tmin = t->Te0;
    if (t->Te_init) {
        tmin = t->Te_init[0];
        for (int64_t c = 0; c < nc; ++c) {
            if (!(t->Te_init[c] >= 0.0)) return "temperatures must be >= 0";
            tmin = std::min(tmin, t->Te_init[c]);
        }
    } else if (!(t->Te0 >= 0.0)) {
        return "temperatures must be >= 0";
    }
    if (t->mode == 1) {
        if (!(t->gamma_e > 0.0)) return "gamma_e must be positive in two-temperature mode";
        if (t->n_sub < 1) return "n_sub must be >= 1";
        if (!(t->G_el >= 0.0) || !(t->kappa_e >= 0.0)) return "G_el and kappa_e must be >= 0";
        if (t->kappa_e > 0.0) {
            double s = 0.0;
            for (int k = 0; k < 3; ++k) {
                const double h = d->ncell[k] * d->a / t->n[k];
                s += 2.0 / (h * h);
            }
            if (t->kappa_e * (d->dt / t->n_sub) * s > t->gamma_e * tmin)
                return "explicit electron diffusion unstable: raise n_sub";
        }
        if (t->profile != 0 && t->profile != 1) return "profile must be 0 or 1";
    }
    return "";
}

inline sl_ttm_desc default_ttm()
{
    sl_ttm_desc t{};
    t.n[0] = t.n[1] = t.n[2] = 1;
    t.mode = 0;
    t.Te0 = 0.0;
    t.n_sub = 1;
    return t;
}

// ------------------------------------------------------------ run sizing
struct Sizes {
    int64_t n;
    int nbx[3], nbins, bin_cap, max_nbr, ncell, n_part;
};

inline Sizes run_sizes(const sl_system_desc* d, const sl_ttm_desc* t)
{
    Sizes z{};
    const int nb = basis_count(d->lattice);
    z.n = (int64_t)nb * d->ncell[0] * d->ncell[1] * d->ncell[2];
    z.ncell = t->n[0] * t->n[1] * t->n[2];
    z.n_part = (int)((z.n + 63) / 64);   // one row of observable partials per wave
    if (d->lattice_mode == 1) {
        const double reach = d->morse[3] + d->skin;
        const double vol_site = std::pow(d->a, 3) / nb;
        double w3 = 1.0;
        z.nbins = 1;
        for (int k = 0; k < 3; ++k) {
            const double L = d->ncell[k] * d->a;
            z.nbx[k] = std::max(3, (int)std::floor(L / reach));
            w3 *= L / z.nbx[k];
            z.nbins *= z.nbx[k];
        }
        // capacities bound the densest packing the pair potential allows:
        // close packing at the Morse minimum, sqrt(2)/r0^3 atoms per A^3
        // (a strained lattice may collapse locally towards it) or the
        // lattice density if that is larger, with a margin for thermal
        // compression
        const double r0 = std::max(d->morse[2], 0.5);
        const double dens = std::max(1.4142135623730951 / (r0 * r0 * r0), 1.0 / vol_site);
        z.bin_cap = (int)std::ceil(2.0 * w3 * dens) + 8;
        const double sphere = 4.18879020478639 * reach * reach * reach * dens;
        z.max_nbr = (int)std::ceil(1.6 * sphere + 8.0);
    }
    return z;
}

template <typename T> inline size_t main_bytes(const sl_system_desc* d, const Sizes& z)
{
    Carver c;
    const size_t n = (size_t)z.n;
    const bool live = d->lattice_mode == 1;
    c.take<T>(n); c.take<T>(n); c.take<T>(n);                       // spins
    c.take<T>(n); c.take<T>(n); c.take<T>(n);                       // displacements
    if (live) {
        for (int k = 0; k < 9; ++k) c.take<T>(n);                   // v, F, reference u
        c.take<int32_t>(n * (size_t)z.max_nbr);
        c.take<int32_t>(n);
        c.take<int32_t>((size_t)z.nbins);
        c.take<int32_t>((size_t)z.nbins * z.bin_cap);
    }
    if (live) c.take<sl::Pos4<T>>(n);
    c.take<int8_t>(n);
    c.take<uint16_t>(n);                                            // cell ids, three buffers
    c.take<uint16_t>(n);
    c.take<uint16_t>(n);
    c.take<double>((size_t)z.n_part * sl::NQ);
    c.take<sl_obs>((size_t)std::max(1, d->obs_capacity));
    c.take<sl::RunState>(1);
    if (live) c.take<T>(3 * n);                                     // electron-phonon normals
    return c.off;
}

inline size_t grid_bytes(const Sizes& z)
{
    Carver c;
    c.take<double>(z.ncell); c.take<double>(z.ncell); c.take<double>(z.ncell);
    c.take<unsigned long long>(z.ncell);
    c.take<unsigned long long>(z.ncell);
    return c.off;
}

// ------------------------------------------------------------ engine
struct Run {
    bool used = false;
    sl_system_desc d{};
    sl_ttm_desc t{};
    Sizes z{};
    int64_t steps = 0;          // host view of completed steps
    int64_t target = 0;
    int64_t samples_read = 0;
    void* main = nullptr;
    void* grid = nullptr;
    size_t footprint = 0;
    std::vector<int32_t> canon;  // canonical index of each internal site
    std::vector<double> te_init;
};

class Engine {
public:
    virtual ~Engine() = default;
    virtual sl_status add(const sl_system_desc* d, const sl_ttm_desc* t, int64_t target, int* slot) = 0;
    virtual sl_status set_grid(int slot, const sl_ttm_desc* t) = 0;
    virtual sl_status advance(int64_t n) = 0;
    virtual sl_status advance_noalloc(int64_t n, char* scratch, size_t cap) = 0;
    virtual sl_status get(int slot, double* x, double* v, double* s, double* Te, sl_obs* obs,
                          int64_t max_samples, int64_t* n_obs) = 0;
    virtual sl_status set_state(int slot, const double* x, const double* v, const double* s,
                                const double* Te) = 0;
    virtual sl_status remove(int slot) = 0;
    virtual sl_status stats(int slot, sl_run_stats* out) = 0;
    virtual sl_status sync() = 0;
    virtual sl_status profiled(int64_t n, double avg[6], int64_t cnt[6]) = 0;
    std::vector<Run> runs;
    DevAlloc alloc;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    hipStream_t cap_stream = nullptr;
    size_t budget = 0, used_bytes = 0;
    int graph_steps = 16;
    int precision = SL_FP64;
    // launch shape (every choice gives bitwise-identical results)
    int spin_block = 0, spin_spt = 1, atom_block = 256;   // spin_block 0: by the site count
    int spin_eff = 256;             // the colour-pass block size in use
    int persist_block = 0;          // 0: every run on the multi-kernel step
    int xcd_ord = 0;                // 1: XCD-contiguous work tables
    int bin_mode = 0;               // 0 automatic, 1 kick bins every step, 2 rebuild only
    int atom_lanes = 0;             // lanes per atom in k_atom_final (0: by the atom count)
    int merge_sweeps = 1;           // 1: merge adjacent colour half steps when possible
    int spin_access = 0;            // colour-pass neighbour access: 0 gathers per site,
                                    // 1 LDS-staged rows (where they apply)
    int fuse_force = 1;             // 1: merged chunks kick in colour pass 0 and run the
                                    // force kernel in the launch of colour pass 1
    int merge_g = 0;                // >= 2: steps per merged chunk of the multi-kernel runs
    int merge_run = -1;             // a stepping run among them (its step gives the chunk phase)
    std::vector<int> mk_runs;       // the runs on the multi-kernel step
    bool fold = false;              // chunks end each step inside the next one's colour pass 0
    int fold_blocks = 0;            // the blocks of colour pass 0 that end the previous step
    bool fused = false;             // fuse_force applies to the merged chunks
    int force_spin_blocks = 0;      // blocks of k_spin_force holding the colour pass (after
                                    // those of the atom table)
    int lanes_eff = 1;              // the lanes in use (tables are built for it)
    virtual sl_status retune() = 0;
    virtual sl_status init_device() = 0;
};

template <typename T> class EngineT final : public Engine {
public:
    using RD = sl::RunDev<T>;
    using T_ = T;

    EngineT(int max_runs) { runs.resize(max_runs); host_rd.resize(max_runs); }

    ~EngineT() override
    {
        if (stream) (void)hipStreamSynchronize(stream);
        drop_graph();
        for (size_t s = 0; s < runs.size(); ++s) release(s);
        for (void* p : tables) alloc.put(p);
        alloc.put(d_runs);
        if (d_any_rebuild) alloc.put(d_any_rebuild);
        if (cap_stream) (void)hipStreamDestroy(cap_stream);
        if (side_stream) (void)hipStreamDestroy(side_stream);
        if (ev_fork) (void)hipEventDestroy(ev_fork);
        if (ev_join) (void)hipEventDestroy(ev_join);
        if (own_stream && stream) (void)hipStreamDestroy(stream);
    }

    sl_status init_device() override
    {
        d_runs = static_cast<RD*>(alloc.get(sizeof(RD) * runs.size()));
        if (!d_runs) return fail(SL_ENOMEM, "device allocation of the run table failed");
        SL_HIP(hipMemset(d_runs, 0, sizeof(RD) * runs.size()));
        d_any_rebuild = static_cast<int32_t*>(alloc.get(256));
        if (!d_any_rebuild) return fail(SL_ENOMEM, "device allocation failed");
        SL_HIP(hipMemset(d_any_rebuild, 0, 256));
        SL_HIP(hipStreamCreateWithFlags(&cap_stream, hipStreamNonBlocking));
        SL_HIP(hipStreamCreateWithFlags(&side_stream, hipStreamNonBlocking));
        SL_HIP(hipEventCreateWithFlags(&ev_fork, hipEventDisableTiming));
        SL_HIP(hipEventCreateWithFlags(&ev_join, hipEventDisableTiming));
        // LDS available to the persistent kernel's dynamic buffer
        int dev = 0, per_block = 0;
        SL_HIP(hipGetDevice(&dev));
        SL_HIP(hipDeviceGetAttribute(&per_block, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
        const void* pk[4] = {reinterpret_cast<const void*>(&sl::k_persist<T, 512>),
                             reinterpret_cast<const void*>(&sl::k_persist<T, 1024>),
                             reinterpret_cast<const void*>(&sl::k_persist<T, 512, true>),
                             reinterpret_cast<const void*>(&sl::k_persist<T, 1024, true>)};
        int static_lds = 0;
        for (const void* f : pk) {
            hipFuncAttributes fa{};
            SL_HIP(hipFuncGetAttributes(&fa, f));
            static_lds = std::max(static_lds, (int)fa.sharedSizeBytes);
        }
        lds_max = per_block > static_lds ? (uint32_t)(per_block - static_lds) : 0u;
        for (const void* f : pk)
            SL_HIP(hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_max));
        const void* tk = reinterpret_cast<const void*>(&sl::k_ttm_tile<T>);
        hipFuncAttributes ta{};
        SL_HIP(hipFuncGetAttributes(&ta, tk));
        tile_lds_max = per_block > (int)ta.sharedSizeBytes ? (uint32_t)(per_block - (int)ta.sharedSizeBytes) : 0u;
        SL_HIP(hipFuncSetAttribute(tk, hipFuncAttributeMaxDynamicSharedMemorySize, (int)tile_lds_max));
        const void* sk[3] = {reinterpret_cast<const void*>(&sl::k_spin_tile_bcc<T, 2, 2>),
                             reinterpret_cast<const void*>(&sl::k_spin_tile_bcc<T, 4, 4>),
                             reinterpret_cast<const void*>(&sl::k_spin_tile_bcc<T, 4, 4, 1024>)};
        int sk_static = 0;
        for (const void* f : sk) {
            hipFuncAttributes fa{};
            SL_HIP(hipFuncGetAttributes(&fa, f));
            sk_static = std::max(sk_static, (int)fa.sharedSizeBytes);
        }
        stile_lds_max = per_block > sk_static ? (uint32_t)(per_block - sk_static) : 0u;
        for (const void* f : sk)
            SL_HIP(hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)stile_lds_max));
        return SL_OK;
    }

    // --------------------------------------------------------- add a run
    sl_status add(const sl_system_desc* d, const sl_ttm_desc* t, int64_t target, int* slot) override
    {
        std::string e = validate_desc(d);
        if (!e.empty()) return fail(SL_EINVAL, e);
        e = validate_ttm(t, d);
        if (!e.empty()) return fail(SL_EINVAL, e);
        int s = -1;
        for (size_t k = 0; k < runs.size(); ++k)
            if (!runs[k].used) { s = (int)k; break; }
        if (s < 0) return fail(SL_EBUSY, "no free slot");
        Sizes z = run_sizes(d, t);
        const size_t fp = main_bytes<T>(d, z) + grid_bytes(z);
        if (budget && used_bytes + fp > budget) return fail(SL_ENOMEM, "run does not fit the memory budget");
        Run& r = runs[s];
        r = Run{};
        r.d = *d;
        r.t = *t;
        r.z = z;
        r.target = target;
        r.main = alloc.get(main_bytes<T>(d, z));
        r.grid = alloc.get(grid_bytes(z));
        if (!r.main || !r.grid) {
            alloc.put(r.main);
            alloc.put(r.grid);
            r = Run{};
            return fail(SL_ENOMEM, "device allocation failed");
        }
        r.used = true;
        r.footprint = fp;
        used_bytes += fp;
        sl_status st = upload(s, d, t, target);
        if (st != SL_OK) {
            release(s);
            tables_dirty = true;
            return st;
        }
        *slot = s;
        return SL_OK;
    }

    sl_status set_grid(int s, const sl_ttm_desc* t) override
    {
        Run& r = runs[s];
        std::string e = validate_ttm(t, &r.d);
        if (!e.empty()) return fail(SL_EINVAL, e);
        if (r.steps != 0) return fail(SL_EINVAL, "the grid can only be set before the first step");
        SL_HIP(hipStreamSynchronize(stream));
        Sizes z = run_sizes(&r.d, t);
        void* g = alloc.get(grid_bytes(z));
        if (!g) return fail(SL_ENOMEM, "device allocation failed");
        alloc.put(r.grid);
        used_bytes -= r.footprint;
        r.grid = g;
        r.t = *t;
        r.z.ncell = z.ncell;
        r.footprint = main_bytes<T>(&r.d, r.z) + grid_bytes(r.z);
        used_bytes += r.footprint;
        fill_grid(s);
        sl::RunState rs{};
        rs.target = r.target;
        rs.rebuild = host_rd[s].live ? 1 : 0;
        SL_HIP(hipMemcpyAsync(host_rd[s].st, &rs, sizeof(rs), hipMemcpyHostToDevice, stream));
        if (host_rd[s].live)
            SL_HIP(hipMemsetAsync(host_rd[s].bin_n, 0, sizeof(int32_t) * host_rd[s].nbins, stream));
        r.samples_read = 0;
        return commit_and_init(s);
    }

    // --------------------------------------------------------- stepping
    sl_status advance(int64_t n) override
    {
        if (n < 0) return fail(SL_EINVAL, "negative step count");
        if (n == 0) return SL_OK;
        if (tables_dirty) {
            sl_status st = rebuild_tables();
            if (st != SL_OK) return st;
        }
        return advance_core(n, true);
    }

    // As advance(), with the launch tables in `scratch` (cap bytes of device
    // memory the engine does not own) and every step launched directly: no
    // device memory is allocated or freed and no graph is instantiated.  The
    // tables are written by a kernel from their closed form (a single run's
    // tables are arithmetic sequences, XCD-ordered or not), so the call holds
    // no host buffer that a captured graph would have to keep.  The engine's
    // own tables and graph, if any, are left as they were.
    sl_status advance_noalloc(int64_t n, char* scratch, size_t cap) override
    {
        if (n < 0) return fail(SL_EINVAL, "negative step count");
        Tables tb;
        std::vector<int> changed;
        plan_tables(tb, changed);
        sl::TableFill f{};
        const std::vector<int2>* tabs[6] = {&tb.ws, &tb.wa, &tb.wk, &tb.wc, &tb.wd, &tb.wt};
        const int xcd[6] = {xcd_ord, xcd_ord, xcd_ord, 0, 0, 0};
        // items per block of each table (the diffusion tiles are numbered)
        const int tiles[6] = {spin_eff * spin_spt, atom_block / lanes_eff, spin_eff, sl::kBlock,
                              sl::kBlock, 1};
        size_t off = 0;
        for (int k = 0; k < 6; ++k) {
            const std::vector<int2>& t = *tabs[k];
            f.off[k] = (int32_t)off;
            f.m[k] = (int32_t)t.size();
            f.xcd[k] = xcd[k];
            f.tile[k] = tiles[k];
            for (size_t q = 0; q < t.size(); ++q) {
                const int2 e = sl::fill_entry(f, k, (int32_t)q, t[q].x);
                if (e.x != t[q].x || e.y != t[q].y || (q > 0 && t[q].x != t[0].x))
                    return fail(SL_EINVAL, "sl_step_noalloc: only a single system's tables are built "
                                           "without allocation");
            }
            off += t.size();
        }
        f.slot = tb.rl.empty() ? (tb.pl.empty() ? 0 : tb.pl[0]) : tb.rl[0];
        f.n_int2 = (int32_t)off;
        if (tb.rl.size() > 1 || tb.pl.size() > 1)
            return fail(SL_EINVAL, "sl_step_noalloc: only a single system's tables are built "
                                   "without allocation");
        f.rl_n = (int32_t)tb.rl.size();
        f.pl_n = (int32_t)tb.pl.size();
        const size_t bytes = off * sizeof(int2) + 2 * sizeof(int);
        if (bytes > cap)
            return fail(SL_EINVAL, "sl_step_noalloc: the system's launch tables take " +
                                       std::to_string(bytes) + " bytes, more than the " +
                                       std::to_string(cap) + "-byte static buffer");
        if (n == 0) return SL_OK;
        int2* base = reinterpret_cast<int2*>(scratch);
        int* ints = reinterpret_cast<int*>(base + off);
        for (int s : changed)
            sl::k_set_run_flags<T_><<<1, 1, 0, stream>>>(d_runs, s, host_rd[s].bin_step,
                                                          host_rd[s].eta_drawn);
        const int fill_blocks = (int)std::min<size_t>((off + 2 + 255) / 256, 1024);
        sl::k_fill_tables<<<fill_blocks, 256, 0, stream>>>(base, ints, f);
        SL_HIP(hipGetLastError());
        // the launches below read the tables from the scratch buffer
        int2* keep_w[6] = {d_work_spin, d_work_atom, d_work_kick, d_work_cell, d_work_diff, d_work_tile};
        int* keep_rl = d_run_list;
        int* keep_pl = d_persist_list;
        const bool keep_graph = graph_ok;
        d_work_spin = base + f.off[0];
        d_work_atom = base + f.off[1];
        d_work_kick = base + f.off[2];
        d_work_cell = base + f.off[3];
        d_work_diff = base + f.off[4];
        d_work_tile = base + f.off[5];
        d_run_list = ints;
        d_persist_list = ints + 1;
        graph_ok = false;
        // (the LDS-staged pass's tile table is not built here: the
        // specialised pass, which gives the same bits, runs instead)
        stile_on = false;
        const sl_status st = advance_core(n, false);
        stile_on = true;
        d_work_spin = keep_w[0];
        d_work_atom = keep_w[1];
        d_work_kick = keep_w[2];
        d_work_cell = keep_w[3];
        d_work_diff = keep_w[4];
        d_work_tile = keep_w[5];
        d_run_list = keep_rl;
        d_persist_list = keep_pl;
        graph_ok = keep_graph;
        return st;
    }

    // The steps themselves, the tables being in place; with_graph: replay the
    // captured graph for whole chunks (capturing it first if needed).
    sl_status advance_core(int64_t n, bool with_graph)
    {
        if (active_blocks_atom == 0 && persist_runs == 0) return SL_OK;
        // the runs that live in LDS advance in persistent launches on a side
        // stream, concurrently with the multi-kernel step of the others
        if (persist_runs > 0) {
            SL_HIP(hipEventRecord(ev_fork, stream));
            SL_HIP(hipStreamWaitEvent(side_stream, ev_fork, 0));
            for (int64_t done = 0; done < n; done += kPersistChunk) {
                const int k = (int)std::min<int64_t>(kPersistChunk, n - done);
                launch_persist(side_stream, nullptr, nullptr, k);
            }
            SL_HIP(hipGetLastError());
            SL_HIP(hipEventRecord(ev_join, side_stream));
        }
        int64_t left = active_blocks_atom > 0 ? n : 0;
        const int G = graph_len();
        // a merged chunk shorter than the chunk length: replayed from a graph
        // kept per length, or launched directly
        auto short_chunk = [&](int len, bool free_end) -> sl_status {
            if (!with_graph) return enqueue_chunk(stream, nullptr, len, free_end);
            hipGraphExec_t ex = nullptr;
            sl_status st = chunk_graph(len, free_end, &ex);
            if (st != SL_OK) return st;
            SL_HIP(hipGraphLaunch(ex, stream));
            return SL_OK;
        };
        if (merge_g >= 2 && left > 0) {
            // a shorter merged chunk up to the next multiple of the chunk
            // length (it ends on no sample step: those are multiples of it)
            const int64_t head = std::min<int64_t>(chunk_head(), left);
            if (head > 0) {
                sl_status st = short_chunk((int)head, head < chunk_head());
                if (st != SL_OK) return st;
            }
            left -= head;
        }
        if (G > 1 && left >= G && with_graph) {
            if (!graph_ok) {
                sl_status st = capture();
                if (st != SL_OK) return st;
            }
            while (left >= G) {
                SL_HIP(hipGraphLaunch(exec, stream));
                left -= G;
            }
        } else if (G > 1 && merge_g >= 2) {
            for (; left >= G; left -= G) {
                sl_status st = enqueue_chunk(stream, nullptr);
                if (st != SL_OK) return st;
            }
        }
        if (merge_g >= 2 && left > 0) {
            // the rest as one shorter merged chunk from a chunk boundary
            sl_status st = short_chunk((int)left, true);
            if (st != SL_OK) return st;
            left = 0;
        }
        for (int64_t k = 0; k < left; ++k) enqueue_step(stream, nullptr);
        SL_HIP(hipGetLastError());
        if (persist_runs > 0) SL_HIP(hipStreamWaitEvent(stream, ev_join, 0));
        for (auto& r : runs)
            if (r.used) r.steps = std::min(r.target, r.steps + n);
        return SL_OK;
    }

    sl_status profiled(int64_t n, double avg[6], int64_t cnt[6]) override
    {
        if (n > kPersistChunk) return fail(SL_EINVAL, "profile at most 4096 steps per call");
        if (tables_dirty) {
            sl_status st = rebuild_tables();
            if (st != SL_OK) return st;
        }
        std::vector<hipEvent_t> ev;
        std::vector<int> cls;
        Prof p{&ev, &cls};
        if (persist_runs > 0) {
            sl_status st = timed(stream, &p, 4, [&](hipEvent_t a, hipEvent_t b) {
                launch_persist(stream, a, b, (int)n);
            });
            if (st != SL_OK) return st;
        }
        // the schedule advance() uses: a shorter merged chunk up to a chunk
        // boundary, whole chunks, a shorter chunk for the rest
        int64_t left = active_blocks_atom > 0 ? n : 0;
        if (merge_g >= 2 && left > 0) {
            const int64_t head = std::min<int64_t>(chunk_head(), left);
            if (head > 0) {
                sl_status st = enqueue_chunk(stream, &p, (int)head, head < chunk_head());
                if (st != SL_OK) return st;
            }
            left -= head;
            for (; left >= merge_g; left -= merge_g) {
                sl_status st = enqueue_chunk(stream, &p);
                if (st != SL_OK) return st;
            }
            if (left > 0) {
                sl_status st = enqueue_chunk(stream, &p, (int)left, true);
                if (st != SL_OK) return st;
                left = 0;
            }
        }
        for (int64_t k = 0; k < left; ++k) {
            sl_status st = enqueue_step(stream, &p);
            if (st != SL_OK) return st;
        }
        SL_HIP(hipStreamSynchronize(stream));
        double tot[6] = {0, 0, 0, 0, 0, 0};
        int64_t c[6] = {0, 0, 0, 0, 0, 0};
        for (size_t k = 0; k + 1 < ev.size(); k += 2) {
            float ms = 0.f;
            SL_HIP(hipEventElapsedTime(&ms, ev[k], ev[k + 1]));
            tot[cls[k / 2]] += ms;
            c[cls[k / 2]] += 1;
        }
        for (auto e : ev) (void)hipEventDestroy(e);
        for (int k = 0; k < 6; ++k) {
            avg[k] = c[k] ? tot[k] / c[k] : 0.0;
            cnt[k] = c[k];
        }
        for (auto& r : runs)
            if (r.used) r.steps = std::min(r.target, r.steps + n);
        return SL_OK;
    }

    sl_status sync() override
    {
        SL_HIP(hipStreamSynchronize(stream));
        for (size_t s = 0; s < runs.size(); ++s) {
            if (!runs[s].used) continue;
            sl::RunState rs;
            SL_HIP(hipMemcpy(&rs, host_rd[s].st, sizeof(rs), hipMemcpyDeviceToHost));
            if (rs.err) return numeric_error((int)s, rs.err);
        }
        return SL_OK;
    }

    sl_status get(int s, double* x, double* v, double* sp, double* Te, sl_obs* obs,
                  int64_t max_samples, int64_t* n_obs) override
    {
        if (s < 0 || s >= (int)runs.size() || !runs[s].used) return fail(SL_EINVAL, "bad slot");
        SL_HIP(hipStreamSynchronize(stream));
        Run& r = runs[s];
        const RD& R = host_rd[s];
        const size_t n = (size_t)r.z.n;
        std::vector<T> buf(3 * n);
        auto fetch3 = [&](T* a, T* b, T* c) -> sl_status {
            SL_HIP(hipMemcpy(buf.data(), a, n * sizeof(T), hipMemcpyDeviceToHost));
            SL_HIP(hipMemcpy(buf.data() + n, b, n * sizeof(T), hipMemcpyDeviceToHost));
            SL_HIP(hipMemcpy(buf.data() + 2 * n, c, n * sizeof(T), hipMemcpyDeviceToHost));
            return SL_OK;
        };
        sl_status st;
        if (sp) {
            if ((st = fetch3(R.sx, R.sy, R.sz)) != SL_OK) return st;
            for (size_t i = 0; i < n; ++i)
                for (int k = 0; k < 3; ++k) sp[3 * (size_t)r.canon[i] + k] = (double)buf[k * n + i];
        }
        if (x) {
            if ((st = fetch3(R.ux, R.uy, R.uz)) != SL_OK) return st;
            for (size_t i = 0; i < n; ++i) {
                sl::Site site = sl::decode_site(R.g, (uint32_t)i);
                double r0[3];
                ideal_position(R.g, site, r.d.a, r0);
                for (int k = 0; k < 3; ++k) {
                    const double L = r.d.ncell[k] * r.d.a;
                    double p = r0[k] + (double)buf[k * n + i];
                    p -= L * std::floor(p / L);
                    x[3 * (size_t)r.canon[i] + k] = p;
                }
            }
        }
        if (v) {
            if (r.d.lattice_mode == 1) {
                if ((st = fetch3(R.vx, R.vy, R.vz)) != SL_OK) return st;
                for (size_t i = 0; i < n; ++i)
                    for (int k = 0; k < 3; ++k) v[3 * (size_t)r.canon[i] + k] = (double)buf[k * n + i];
            } else {
                std::memset(v, 0, sizeof(double) * 3 * n);
            }
        }
        if (Te) SL_HIP(hipMemcpy(Te, R.Te, sizeof(double) * r.z.ncell, hipMemcpyDeviceToHost));
        sl::RunState rs;
        SL_HIP(hipMemcpy(&rs, R.st, sizeof(rs), hipMemcpyDeviceToHost));
        if (obs && n_obs) {
            *n_obs = 0;
            const int cap = std::max(1, r.d.obs_capacity);
            int64_t first = std::max(r.samples_read, rs.n_samples - cap);
            int64_t cntv = std::min<int64_t>(max_samples, rs.n_samples - first);
            for (int64_t k = 0; k < cntv; ++k) {
                SL_HIP(hipMemcpy(obs + k, R.ring + ((first + k) % cap), sizeof(sl_obs),
                                 hipMemcpyDeviceToHost));
            }
            r.samples_read = first + cntv;
            *n_obs = cntv;
        }
        if (rs.err) return numeric_error(s, rs.err);
        return SL_OK;
    }

    // Replaces positions, velocities, spins and/or the electron grid of a run
    // (canonical host order, NULL keeps the current values), then recomputes
    // electron cells, neighbour lists and forces as at initialisation.
    sl_status set_state(int s, const double* x, const double* v, const double* sp,
                        const double* Te) override
    {
        if (s < 0 || s >= (int)runs.size() || !runs[s].used) return fail(SL_EINVAL, "bad slot");
        Run& r = runs[s];
        RD& R = host_rd[s];
        const size_t n = (size_t)r.z.n;
        for (size_t i = 0; sp && i < n; ++i) {
            const double nn = std::sqrt(sp[3 * i] * sp[3 * i] + sp[3 * i + 1] * sp[3 * i + 1] +
                                        sp[3 * i + 2] * sp[3 * i + 2]);
            if (!(std::fabs(nn - 1.0) <= 1e-6)) return fail(SL_EINVAL, "spins must be unit vectors");
        }
        for (size_t i = 0; x && i < 3 * n; ++i)
            if (!std::isfinite(x[i])) return fail(SL_EINVAL, "positions must be finite");
        for (size_t i = 0; v && i < 3 * n; ++i)
            if (!std::isfinite(v[i])) return fail(SL_EINVAL, "velocities must be finite");
        for (int c = 0; Te && c < r.z.ncell; ++c)
            if (!(Te[c] >= 0.0) || !std::isfinite(Te[c])) return fail(SL_EINVAL, "temperatures must be >= 0");
        SL_HIP(hipStreamSynchronize(stream));
        std::vector<T> a(n), b(n), c(n);
        auto put3 = [&](T* dx, T* dy, T* dz) -> sl_status {
            SL_HIP(hipMemcpyAsync(dx, a.data(), n * sizeof(T), hipMemcpyHostToDevice, stream));
            SL_HIP(hipMemcpyAsync(dy, b.data(), n * sizeof(T), hipMemcpyHostToDevice, stream));
            SL_HIP(hipMemcpyAsync(dz, c.data(), n * sizeof(T), hipMemcpyHostToDevice, stream));
            SL_HIP(hipStreamSynchronize(stream));
            return SL_OK;
        };
        sl_status st;
        if (sp) {
            for (size_t i = 0; i < n; ++i) {
                const size_t ci = (size_t)r.canon[i];
                a[i] = (T)sp[3 * ci];
                b[i] = (T)sp[3 * ci + 1];
                c[i] = (T)sp[3 * ci + 2];
            }
            if ((st = put3(R.sx, R.sy, R.sz)) != SL_OK) return st;
        }
        if (x) {
            // displacement from the ideal site, minimum image
            T* out[3] = {a.data(), b.data(), c.data()};
            for (size_t i = 0; i < n; ++i) {
                const sl::Site site = sl::decode_site(R.g, (uint32_t)i);
                double r0[3];
                ideal_position(R.g, site, r.d.a, r0);
                const size_t ci = (size_t)r.canon[i];
                for (int k = 0; k < 3; ++k) {
                    const double L = r.d.ncell[k] * r.d.a;
                    double d = x[3 * ci + k] - r0[k];
                    d -= L * std::nearbyint(d / L);
                    out[k][i] = (T)d;
                }
            }
            if ((st = put3(R.ux, R.uy, R.uz)) != SL_OK) return st;
        }
        if (v && R.live) {
            for (size_t i = 0; i < n; ++i) {
                const size_t ci = (size_t)r.canon[i];
                a[i] = (T)v[3 * ci];
                b[i] = (T)v[3 * ci + 1];
                c[i] = (T)v[3 * ci + 2];
            }
            if ((st = put3(R.vx, R.vy, R.vz)) != SL_OK) return st;
        }
        if (Te) {
            r.te_init.assign(Te, Te + r.z.ncell);
        } else {
            r.te_init.resize(r.z.ncell);
            SL_HIP(hipMemcpy(r.te_init.data(), R.Te, sizeof(double) * r.z.ncell, hipMemcpyDeviceToHost));
        }
        if (R.live) {
            sl::RunState rs;
            SL_HIP(hipMemcpy(&rs, R.st, sizeof(rs), hipMemcpyDeviceToHost));
            rs.rebuild = 1;
            SL_HIP(hipMemcpy(R.st, &rs, sizeof(rs), hipMemcpyHostToDevice));
        }
        return commit_and_init(s);
    }

    sl_status stats(int s, sl_run_stats* out) override
    {
        if (s < 0 || s >= (int)runs.size() || !runs[s].used) return fail(SL_EINVAL, "bad slot");
        if (!out) return fail(SL_EINVAL, "null output");
        SL_HIP(hipStreamSynchronize(stream));
        sl::RunState rs;
        SL_HIP(hipMemcpy(&rs, host_rd[s].st, sizeof(rs), hipMemcpyDeviceToHost));
        out->steps = rs.step;
        out->samples = rs.n_samples;
        out->list_rebuilds = rs.n_rebuild;
        out->max_list = rs.max_list;
        out->list_capacity = host_rd[s].live ? host_rd[s].max_nbr : 0;
        out->list_rescans = rs.n_rescan;
        out->error = rs.err;
        return SL_OK;
    }

    sl_status remove(int s) override
    {
        if (s < 0 || s >= (int)runs.size() || !runs[s].used) return fail(SL_EINVAL, "bad slot");
        SL_HIP(hipStreamSynchronize(stream));
        release(s);
        tables_dirty = true;
        drop_graph();
        return SL_OK;
    }

    sl_status retune() override
    {
        SL_HIP(hipStreamSynchronize(stream));
        tables_dirty = true;
        drop_graph();
        return SL_OK;
    }

    sl_status n_samples(int s, int64_t* out)
    {
        sl::RunState rs;
        SL_HIP(hipMemcpy(&rs, host_rd[s].st, sizeof(rs), hipMemcpyDeviceToHost));
        *out = rs.n_samples;
        return SL_OK;
    }

private:
    struct Prof {
        std::vector<hipEvent_t>* ev;
        std::vector<int>* cls;
    };

    std::vector<RD> host_rd;
    RD* d_runs = nullptr;
    std::vector<void*> tables;
    int2* d_work_spin = nullptr;
    int2* d_work_atom = nullptr;
    int2* d_work_kick = nullptr;     // atoms of live runs, in tiles of the colour-pass block
    int2* d_work_cell = nullptr;
    int2* d_work_diff = nullptr;
    int2* d_work_tile = nullptr;
    int32_t* d_any_rebuild = nullptr;   // a run flagged a list rebuild this step (device word)
    static constexpr int kBinGrid = 2048;   // blocks of a step's binning launches
    int* d_run_list = nullptr;
    int active_runs = 0;
    int active_blocks_spin = 0, active_blocks_atom = 0, active_blocks_kick = 0, active_blocks_cell = 0,
        active_blocks_diff = 0, active_blocks_tile = 0;
    int max_sub = 0;
    bool any_live = false;
    bool any_radial = false;        // a run with radial exchange: kicks after the sweep
    bool persist_radial = false;    // a persistent run with radial exchange
    int lean_lat = -1;              // >= 0: the runs' lattice for the specialised colour pass
    int lean_multi = 0;             // ... and whether they have several species
    // the LDS-staged colour pass (bcc, one species, constant exchange):
    // 0 off, 1 tiles of 2 x 2 rows, 2 tiles of 4 x 4 rows, 3 tiles of 4 x 4
    // rows in 1024-thread blocks
    int stile = 0;
    bool stile_on = true;           // off while the allocation-free entry point steps
    int4* d_work_stile = nullptr;   // block: run, first row, first plane
    int active_blocks_stile = 0;
    uint32_t stile_bytes = 0;       // the LDS of its launch
    uint32_t stile_lds_max = 0;     // dynamic LDS available to it
    hipGraphExec_t exec = nullptr;
    bool graph_ok = false;
    // graphs of merged chunks shorter than merge_g, by length (a chunk's
    // launches depend on its length only; every kernel reads the steps from
    // the run state)
    std::vector<std::pair<int, hipGraphExec_t>> short_exec;   // by 2 len + free_end
    bool tables_dirty = true;
    // persistent executor: runs that fit in LDS, one block each
    hipStream_t side_stream = nullptr;
    hipEvent_t ev_fork = nullptr, ev_join = nullptr;
    uint32_t lds_max = 0;
    uint32_t tile_lds_max = 0;      // dynamic LDS available to k_ttm_tile
    uint32_t tile_bytes = 0;        // the LDS its launch takes (largest tile of the table)
    int* d_persist_list = nullptr;
    int persist_runs = 0;
    // the kick bins every step while the engine's live atoms are few (one
    // atomic per atom costs less than a launch); above that a separate
    // binning launch works only when a list is rebuilt
    static constexpr int64_t kBinEachStepMaxAtoms = int64_t(1) << 20;
    bool bin_each_step = true;
    uint32_t persist_bytes = 0;

    sl_status numeric_error(int s, int err)
    {
        sl::RunState rs{};
        (void)hipMemcpy(&rs, host_rd[s].st, sizeof(rs), hipMemcpyDeviceToHost);
        std::string m = "run in slot " + std::to_string(s) + " stopped:";
        if (rs.bad_atom > 0)
            m += " [atom " + std::to_string(rs.bad_atom - 1) + " count " +
                 std::to_string(rs.bad_count) + " at step " + std::to_string(rs.bad_step) +
                 ", list capacity " + std::to_string(host_rd[s].max_nbr) + ", bin capacity " +
                 std::to_string(host_rd[s].bin_cap) + "]";
        if (err & sl::ERR_NEG_E) m += " negative electron energy density (or not a number);";
        if (err & sl::ERR_NUMERIC)
            m += " non-finite or non-unit spin, or non-finite velocity or position;";
        if (err & sl::ERR_BIN) m += " neighbour bin overflow;";
        if (err & sl::ERR_NBR) m += " neighbour list overflow;";
        if (err & sl::ERR_DE) m += " electron-phonon energy out of range;";
        return fail(SL_ENUMERIC, m);
    }

    void drop_graph()
    {
        if (exec) (void)hipGraphExecDestroy(exec);
        exec = nullptr;
        graph_ok = false;
        for (auto& e : short_exec) (void)hipGraphExecDestroy(e.second);
        short_exec.clear();
    }

    void release(size_t s)
    {
        Run& r = runs[s];
        if (!r.used) return;
        alloc.put(r.main);
        alloc.put(r.grid);
        used_bytes -= r.footprint;
        r = Run{};
        host_rd[s] = RD{};
    }

    // Fills the host descriptor of slot s (device pointers into its blocks).
    void fill_main(int s)
    {
        Run& r = runs[s];
        const sl_system_desc* d = &r.d;
        RD R{};
        const int nb = basis_count(d->lattice);
        const bool fcc = d->lattice == SL_LATTICE_FCC;
        R.g.Lx = d->ncell[0];
        R.g.Ly = d->ncell[1];
        R.g.Lz = d->ncell[2];
        R.g.par = fcc ? 0 : 1;
        R.g.Lxh = fcc ? d->ncell[0] : d->ncell[0] / 2;
        R.g.H = fcc ? d->ncell[0] * d->ncell[1] * d->ncell[2] : d->ncell[0] * d->ncell[1] * d->ncell[2] / 2;
        R.g.nb = nb;
        R.g.C = fcc ? 4 : 2 * nb;
        R.g.divH = sl::make_fastdiv((uint32_t)R.g.H);
        R.g.divLxh = sl::make_fastdiv((uint32_t)R.g.Lxh);
        R.g.divLy = sl::make_fastdiv((uint32_t)R.g.Ly);
        R.lattice = d->lattice;
        R.n = (int32_t)r.z.n;
        R.n_species = d->n_species;
        R.n_shells = d->n_shells;
        R.live = d->lattice_mode;
        R.obs_every = d->obs_every;
        R.obs_cap = std::max(1, d->obs_capacity);
        R.seed = d->seed;
        R.run_id = d->run_id;
        R.a = (T)d->a;
        for (int k = 0; k < 3; ++k) {
            R.box[k] = (T)(d->ncell[k] * d->a);
            R.inv_box[k] = (T)(1.0 / (d->ncell[k] * d->a));
            R.B[k] = (T)d->B[k];
            R.Bd[k] = d->B[k];
        }
        R.alpha = (T)d->alpha;
        R.dt = (T)d->dt;
        R.tau_half = (T)(0.5 * d->dt);
        R.inv1pa2 = (T)(1.0 / (1.0 + d->alpha * d->alpha));
        R.gam = (T)sl::kGAMMA;
        std::vector<double> cnt(4, 0.0);
        if (d->species)
            for (int64_t i = 0; i < r.z.n; ++i) cnt[d->species[i]] += 1.0;
        else
            cnt[0] = (double)r.z.n;
        for (int sp = 0; sp < 4; ++sp) {
            const double mu = sp < d->n_species ? d->mu[sp] : 1.0;
            const double m = sp < d->n_species && d->mass[sp] > 0 ? d->mass[sp] : 1.0;
            R.inv_mumb[sp] = (T)(1.0 / (mu * sl::kMUB));
            R.mumb[sp] = mu * sl::kMUB;
            const double K = sp < d->n_species ? d->K[sp] : 0.0;
            R.Kd[sp] = K;
            R.kan[sp] = (T)(2.0 * K / (mu * sl::kMUB));
            if (K != 0.0) R.aniso = 1;
            double sig = std::sqrt(2.0 * d->alpha * sl::kKB / (sl::kGAMMA * mu * sl::kMUB * d->dt));
            if (d->noise_mode == 1) sig *= std::sqrt(d->mu_ref / mu);
            R.sig[sp] = (T)sig;
            R.hdtm[sp] = (T)(0.5 * d->dt / (m * sl::kMVV2E));
            R.m_e[sp] = (T)(m * sl::kMVV2E);
            R.cnt[sp] = cnt[sp];
        }
        R.noisy = 0;
        for (int sp = 0; sp < d->n_species; ++sp)
            if (R.sig[sp] > T(0)) R.noisy = 1;
        for (int sh = 0; sh < 2; ++sh)
            for (int a = 0; a < 4; ++a)
                for (int b = 0; b < 4; ++b) R.J[sh][a][b] = (T)d->J[sh][a][b];
        R.radial = d->exch_radial;
        for (int sh = 0; sh < 2; ++sh) {
            R.rJ2[sh] = (T)d->exch_r[sh][0];
            R.rinvJ3sq[sh] = d->exch_r[sh][1] > 0.0 ? (T)(1.0 / (d->exch_r[sh][1] * d->exch_r[sh][1])) : T(0);
        }
        R.mD = (T)d->morse[0];
        R.ma = (T)d->morse[1];
        R.mr0 = (T)d->morse[2];
        R.mk1 = (T)(-d->morse[1] * 1.4426950408889634);                 // -a log2(e)
        R.mk0 = (T)(d->morse[1] * d->morse[2] * 1.4426950408889634);    // a r0 log2(e)
        R.rc2 = (T)(d->morse[3] * d->morse[3]);
        R.Vc = (T)(d->morse[0] * (std::exp(-2.0 * d->morse[1] * (d->morse[3] - d->morse[2])) -
                                  2.0 * std::exp(-d->morse[1] * (d->morse[3] - d->morse[2]))));
        R.skin_half2 = (T)(0.25 * d->skin * d->skin);
        R.rlist2 = (T)((d->morse[3] + d->skin) * (d->morse[3] + d->skin));
        // carve the run block
        Carver c;
        c.base = static_cast<char*>(r.main);
        const size_t n = (size_t)r.z.n;
        R.sx = c.take<T>(n); R.sy = c.take<T>(n); R.sz = c.take<T>(n);
        R.ux = c.take<T>(n); R.uy = c.take<T>(n); R.uz = c.take<T>(n);
        if (R.live) {
            R.vx = c.take<T>(n); R.vy = c.take<T>(n); R.vz = c.take<T>(n);
            R.fx = c.take<T>(n); R.fy = c.take<T>(n); R.fz = c.take<T>(n);
            R.rx = c.take<T>(n); R.ry = c.take<T>(n); R.rz = c.take<T>(n);
            R.max_nbr = r.z.max_nbr;
            R.nbr = c.take<int32_t>(n * (size_t)r.z.max_nbr);
            R.nbr_n = c.take<int32_t>(n);
            R.nbins = r.z.nbins;
            R.bin_cap = r.z.bin_cap;
            for (int k = 0; k < 3; ++k) {
                R.nbin[k] = r.z.nbx[k];
                R.binw[k] = (T)(d->ncell[k] * d->a / r.z.nbx[k]);
            }
            R.bin_n = c.take<int32_t>((size_t)r.z.nbins);
            R.bin_atoms = c.take<int32_t>((size_t)r.z.nbins * r.z.bin_cap);
        }
        if (R.live) R.pos = c.take<sl::Pos4<T>>(n);
        R.species = c.take<int8_t>(n);
        for (int k = 0; k < 3; ++k) R.cellb[k] = c.take<uint16_t>(n);
        R.n_part = r.z.n_part;
        R.partial = c.take<double>((size_t)r.z.n_part * sl::NQ);
        R.ring = c.take<sl_obs>((size_t)R.obs_cap);
        R.st = c.take<sl::RunState>(1);
        R.eta = R.live ? c.take<T>(3 * n) : nullptr;
        R.any_rebuild = d_any_rebuild;
        host_rd[s] = R;
    }

    void fill_grid(int s)
    {
        Run& r = runs[s];
        RD& R = host_rd[s];
        const sl_ttm_desc* t = &r.t;
        const sl_system_desc* d = &r.d;
        R.ttm_mode = t->mode;
        for (int k = 0; k < 3; ++k) {
            R.tn[k] = t->n[k];
            R.th[k] = d->ncell[k] * d->a / t->n[k];
        }
        R.ncell = r.z.ncell;
        R.n_sub = std::max(1, t->n_sub);
        R.gamma_e = t->gamma_e;
        R.kappa_e = t->kappa_e;
        R.S0 = t->S0;
        R.t0 = t->t0;
        R.fwhm = t->fwhm;
        R.profile = t->profile;
        R.depth = t->depth;
        R.Vcell = R.th[0] * R.th[1] * R.th[2];
        R.dtd = d->dt;
        for (int k = 0; k < 3; ++k) R.dcoef[k] = d->dt / (double)R.n_sub * R.kappa_e / (R.th[k] * R.th[k]);
        R.two_ge = 2.0 / R.gamma_e;
        for (int k = 0; k < 3; ++k) R.stT[k] = t->step_T[k];
        for (int k = 0; k < 2; ++k) R.stEnd[k] = t->step_end[k];
        // diffusion tiles: the tile plus its halo of n_sub cells spans at most
        // 16 cells along every axis (k_ttm_tile's layout), and its three LDS
        // arrays must fit one block; otherwise one launch per sub-step.  The
        // tile's depth is halved (down to 2 cells) while the grid has fewer
        // than 256 tiles: more blocks and shorter columns per thread against
        // more recomputed halo
        for (int k = 0; k < 3; ++k) R.dtile[k] = R.dntile[k] = 0;
        if (t->mode == 1 && t->kappa_e != 0.0 && 2 * R.n_sub < sl::kTileSide) {
            int tt[3];
            for (int k = 0; k < 3; ++k) tt[k] = std::min(sl::kTileSide - 2 * R.n_sub, t->n[k]);
            auto bytes = [&]() {
                return 3.0 * 8.0 * sl::kTileSide * sl::kTileSide * (tt[2] + 2.0 * R.n_sub);
            };
            auto tiles = [&]() {
                int64_t m = 1;
                for (int k = 0; k < 3; ++k) m *= (t->n[k] + tt[k] - 1) / tt[k];
                return m;
            };
            while (tiles() < 256 && tt[2] > 2) tt[2] = (tt[2] + 1) / 2;
            while (bytes() > (double)tile_lds_max && tt[2] > 1) tt[2] = (tt[2] + 1) / 2;
            if (bytes() <= (double)tile_lds_max)
                for (int k = 0; k < 3; ++k) {
                    R.dtile[k] = tt[k];
                    R.dntile[k] = (t->n[k] + tt[k] - 1) / tt[k];
                }
        }
        // electron-phonon Ornstein-Uhlenbeck coefficients
        const double vol = (double)d->ncell[0] * d->ncell[1] * d->ncell[2] * std::pow(d->a, 3);
        const double Gamma = t->mode == 1 ? t->G_el / (3.0 * ((double)r.z.n / vol) * sl::kKB) : 0.0;
        const double c1 = std::exp(-Gamma * d->dt);
        R.ou_c1 = (T)c1;
        R.ou_1mc2 = 1.0 - c1 * c1;
        for (int sp = 0; sp < 4; ++sp) {
            const double m = sp < d->n_species && d->mass[sp] > 0 ? d->mass[sp] : 1.0;
            R.ou_amp[sp] = (T)std::sqrt((1.0 - c1 * c1) * sl::kKB / (m * sl::kMVV2E));
        }
        Carver c;
        c.base = static_cast<char*>(r.grid);
        R.Te = c.take<double>(r.z.ncell);
        R.ee = c.take<double>(r.z.ncell);
        R.Te_alt = c.take<double>(r.z.ncell);
        R.dE = c.take<unsigned long long>(r.z.ncell);
        R.dE_alt = c.take<unsigned long long>(r.z.ncell);

        // a stepped profile starts the grid at its value at t = 0
        const double te0 = t->mode != 2 ? t->Te0
                                         : (0.0 < t->step_end[0] ? t->step_T[0]
                                                                 : (0.0 < t->step_end[1] ? t->step_T[1]
                                                                                         : t->step_T[2]));
        std::vector<double> te(r.z.ncell, te0);
        if (t->Te_init) std::copy(t->Te_init, t->Te_init + r.z.ncell, te.begin());
        r.te_init = te;
        r.t.Te_init = nullptr;
    }

    sl_status upload(int s, const sl_system_desc* d, const sl_ttm_desc* t, int64_t target)
    {
        Run& r = runs[s];
        r.d.species = nullptr;
        r.d.spin0 = r.d.vel0 = r.d.disp0 = nullptr;
        r.d.stream = nullptr;
        r.d.alloc = nullptr;
        // species counts need the caller's array: fill with it, then drop it
        r.d.species = d->species;
        fill_main(s);
        r.d.species = nullptr;
        fill_grid(s);
        RD& R = host_rd[s];
        const size_t n = (size_t)r.z.n;
        r.canon.resize(n);
        for (size_t i = 0; i < n; ++i) {
            sl::Site site = sl::decode_site(R.g, (uint32_t)i);
            r.canon[i] = sl::canonical_of(R.g, site);
        }
        std::vector<T> a(n), b(n), c(n);
        auto put3 = [&](const double* src, T* dx, T* dy, T* dz) -> sl_status {
            for (size_t i = 0; i < n; ++i) {
                const size_t ci = (size_t)r.canon[i];
                a[i] = src ? (T)src[3 * ci + 0] : T(0);
                b[i] = src ? (T)src[3 * ci + 1] : T(0);
                c[i] = src ? (T)src[3 * ci + 2] : T(0);
            }
            SL_HIP(hipMemcpyAsync(dx, a.data(), n * sizeof(T), hipMemcpyHostToDevice, stream));
            SL_HIP(hipMemcpyAsync(dy, b.data(), n * sizeof(T), hipMemcpyHostToDevice, stream));
            SL_HIP(hipMemcpyAsync(dz, c.data(), n * sizeof(T), hipMemcpyHostToDevice, stream));
            SL_HIP(hipStreamSynchronize(stream));
            return SL_OK;
        };
        sl_status st;
        if ((st = put3(d->spin0, R.sx, R.sy, R.sz)) != SL_OK) return st;
        if ((st = put3(d->disp0, R.ux, R.uy, R.uz)) != SL_OK) return st;
        if (R.live) {
            if ((st = put3(d->vel0, R.vx, R.vy, R.vz)) != SL_OK) return st;
            if ((st = put3(nullptr, R.fx, R.fy, R.fz)) != SL_OK) return st;
            if ((st = put3(d->disp0, R.rx, R.ry, R.rz)) != SL_OK) return st;
            SL_HIP(hipMemsetAsync(R.bin_n, 0, sizeof(int32_t) * R.nbins, stream));
            SL_HIP(hipMemsetAsync(R.nbr_n, 0, sizeof(int32_t) * n, stream));
        }
        std::vector<int8_t> spc(n, 0);
        if (d->species)
            for (size_t i = 0; i < n; ++i) spc[i] = d->species[r.canon[i]];
        SL_HIP(hipMemcpyAsync(R.species, spc.data(), n, hipMemcpyHostToDevice, stream));
        sl::RunState rs{};
        rs.step = 0;
        rs.target = target;
        rs.rebuild = R.live ? 1 : 0;
        SL_HIP(hipMemcpyAsync(R.st, &rs, sizeof(rs), hipMemcpyHostToDevice, stream));
        SL_HIP(hipStreamSynchronize(stream));
        return commit_and_init(s);
    }

    // Copies the descriptor of slot s to the device, writes the initial
    // electron grid, computes electron-cell ids, neighbour lists, forces and
    // the step-0 sample of that run only, then rebuilds the work tables.
    sl_status commit_and_init(int s)
    {
        Run& r = runs[s];
        RD& R = host_rd[s];
        SL_HIP(hipMemcpyAsync(R.Te, r.te_init.data(), sizeof(double) * r.z.ncell,
                              hipMemcpyHostToDevice, stream));
        SL_HIP(hipMemsetAsync(R.dE, 0, sizeof(unsigned long long) * r.z.ncell, stream));
        SL_HIP(hipMemsetAsync(R.dE_alt, 0, sizeof(unsigned long long) * r.z.ncell, stream));
        SL_HIP(hipMemcpyAsync(d_runs + s, &R, sizeof(RD), hipMemcpyHostToDevice, stream));
        // single-run work tables for the initialisation launches
        std::vector<int2> wa;
        for (int st = 0; st < R.n; st += sl::kBlock) wa.push_back(make_int2(s, st));
        void* tmp = alloc.get(sizeof(int2) * wa.size() + 512);
        if (!tmp) return fail(SL_ENOMEM, "device allocation failed");
        int2* dwa = static_cast<int2*>(tmp);
        int* drl = reinterpret_cast<int*>(dwa + wa.size());
        const int one = s;
        SL_HIP(hipMemcpyAsync(drl, &one, sizeof(int), hipMemcpyHostToDevice, stream));
        SL_HIP(hipMemcpyAsync(dwa, wa.data(), sizeof(int2) * wa.size(), hipMemcpyHostToDevice, stream));
        const int ga = (int)wa.size();
        sl::k_init_lattice<T><<<ga, sl::kBlock, 0, stream>>>(d_runs, dwa);
        if (R.live) {
            sl::k_nbr_bin<T><<<ga, sl::kBlock, 0, stream>>>(d_runs, dwa, (int)sl::PHASE_INIT, -1,
                                                             (int)wa.size(), nullptr);
            sl::k_nbr_sort<T><<<ga, sl::kBlock, 0, stream>>>(d_runs, dwa, (int)sl::PHASE_INIT, -1,
                                                              (int)wa.size(), nullptr);
            sl::k_nbr_build<T><<<ga, sl::kBlock, 0, stream>>>(d_runs, dwa);
        }
        if (R.radial)
            sl::k_atom_final<T, 1, true><<<ga, sl::kBlock, 0, stream>>>(d_runs, dwa, sl::PHASE_INIT, 1, -1);
        else
            sl::k_atom_final<T, 1><<<ga, sl::kBlock, 0, stream>>>(d_runs, dwa, sl::PHASE_INIT, 1, -1);
        sl::k_finalize<T><<<1, sl::kBlock, 0, stream>>>(d_runs, drl, sl::PHASE_INIT, 0, -1);
        SL_HIP(hipGetLastError());
        SL_HIP(hipStreamSynchronize(stream));
        alloc.put(tmp);
        sl::RunState rs;
        SL_HIP(hipMemcpy(&rs, R.st, sizeof(rs), hipMemcpyDeviceToHost));
        if (rs.err) return numeric_error(s, rs.err);
        tables_dirty = true;
        drop_graph();
        return SL_OK;
    }

    // The launch tables of the current runs, as host arrays: block -> (run,
    // first item) of the colour passes (ws), the force kernel (wa), the kick
    // (wk), the cell-parallel grid update (wc), the diffusion sub-step
    // launches (wd) and tiles (wt); the runs on the multi-kernel step (rl) and
    // in the persistent kernel (pl).
    struct Tables {
        std::vector<int2> ws, wa, wk, wc, wd, wt;
        std::vector<int4> wst;      // LDS-staged colour-pass tiles
        std::vector<int> rl, pl;
    };

    sl_status rebuild_tables()
    {
        drop_graph();
        tables_dirty = false;
        Tables tb;
        std::vector<int> changed;
        plan_tables(tb, changed);
        for (int s : changed)
            SL_HIP(hipMemcpyAsync(d_runs + s, &host_rd[s], sizeof(RD), hipMemcpyHostToDevice, stream));
        return upload_tables(tb);
    }

    // Host part of a table rebuild: the launch plan (block sizes, lanes,
    // binning mode, merged chunks, block counts) and the tables.  Runs whose
    // per-run flags (binning by the kick, normals drawn by the kick) changed
    // are listed in `changed`: their host descriptors are updated here, their
    // device copies by the caller.
    void plan_tables(Tables& tb, std::vector<int>& changed)
    {
        std::vector<int2>& ws = tb.ws;
        std::vector<int2>& wa = tb.wa;
        std::vector<int2>& wk = tb.wk;
        std::vector<int2>& wc = tb.wc;
        std::vector<int2>& wd = tb.wd;
        std::vector<int2>& wt = tb.wt;
        std::vector<int>& rl = tb.rl;
        std::vector<int>& pl = tb.pl;
        any_live = false;
        max_sub = 0;
        tile_bytes = 0;
        persist_bytes = 0;
        // automatic launch shapes for the runs on the multi-kernel step: the
        // colour-pass block is the largest of 256, 128, 64 threads that still
        // gives at least one block per CU (256); lanes per atom give the force
        // launch about two waves per SIMD (4 lanes up to 64k atoms, 2 up to
        // 128k, then 1), within what the block size allows
        int64_t multi_atoms = 0, multi_sites = 0;
        for (size_t s = 0; s < runs.size(); ++s) {
            if (!runs[s].used) continue;
            const RD& R = host_rd[s];
            const bool fits =
                persist_block > 0 &&
                sl::persist_layout<T>(R.n, R.ncell, R.n_part, R.live != 0, R.n_species, lds_max)
                        .bytes <= lds_max;
            if (!fits) {
                multi_atoms += R.n;
                multi_sites += R.g.H;
            }
        }
        spin_eff = spin_block;
        if (spin_eff == 0) {
            spin_eff = 256;
            while (spin_eff > 64 && multi_sites < (int64_t)256 * spin_eff * spin_spt) spin_eff /= 2;
        }
        lanes_eff = atom_lanes;
        if (lanes_eff == 0) {
            lanes_eff = multi_atoms <= (int64_t(1) << 16) ? 4 : (multi_atoms <= (int64_t(1) << 17) ? 2 : 1);
            while (atom_block / lanes_eff < 64) lanes_eff /= 2;
        }
        for (size_t s = 0; s < runs.size(); ++s) {
            if (!runs[s].used) continue;
            const RD& R = host_rd[s];
            if (persist_block > 0) {
                const sl::PersistLayout L = sl::persist_layout<T>(R.n, R.ncell, R.n_part, R.live != 0,
                                                                  R.n_species, lds_max);
                if (L.bytes <= lds_max) {
                    pl.push_back((int)s);
                    persist_bytes = std::max(persist_bytes, L.bytes);
                    continue;
                }
            }
            for (int st = 0; st < R.g.H; st += spin_eff * spin_spt) ws.push_back(make_int2((int)s, st));
            const int atile = atom_block / lanes_eff;
            for (int st = 0; st < R.n; st += atile) wa.push_back(make_int2((int)s, st));
            if (R.live)
                for (int st = 0; st < R.n; st += spin_eff) wk.push_back(make_int2((int)s, st));
            if (R.ttm_mode != 0 && R.ncell > sl::kSmallGrid)
                for (int st = 0; st < R.ncell; st += sl::kBlock) wc.push_back(make_int2((int)s, st));
            rl.push_back((int)s);
            if (R.ttm_mode == 1 && R.kappa_e != 0.0 && R.dtile[0] > 0) {
                const int nt = R.dntile[0] * R.dntile[1] * R.dntile[2];
                for (int k = 0; k < nt; ++k) wt.push_back(make_int2((int)s, k));
                const uint32_t b = (uint32_t)(3 * 8 * sl::kTileSide * sl::kTileSide *
                                              (R.dtile[2] + 2 * R.n_sub));
                tile_bytes = std::max(tile_bytes, b);
            } else if (R.ttm_mode == 1 && R.kappa_e != 0.0) {
                for (int st = 0; st < R.ncell; st += sl::kBlock) wd.push_back(make_int2((int)s, st));
                max_sub = std::max(max_sub, R.n_sub);
            }
            any_live = any_live || R.live;
        }
        if (xcd_ord) {
            xcd_order(ws);
            xcd_order(wa);
            xcd_order(wk);
        }
        int64_t live_atoms = 0;
        for (int2 t : wk) live_atoms += std::min<int64_t>(spin_eff, host_rd[t.x].n - t.y);
        bin_each_step = bin_mode == 1 || (bin_mode == 0 && live_atoms <= kBinEachStepMaxAtoms);
        for (size_t s = 0; s < runs.size(); ++s) {
            if (!runs[s].used) continue;
            const int32_t want = bin_each_step ? 1 : 0;
            // with several lanes per atom in the force kernel, the kick draws
            // the electron-phonon normals once per atom for it
            const int32_t draw = lanes_eff > 1 ? 1 : 0;
            if (host_rd[s].bin_step != want || host_rd[s].eta_drawn != draw) {
                host_rd[s].bin_step = want;
                host_rd[s].eta_drawn = draw;
                changed.push_back((int)s);
            }
        }
        // adjacent colour-0 half steps of consecutive steps merge into one pass
        // when the grid update can keep each run's previous T_e in the second
        // buffer for the deferred half step (not when diffusion runs as
        // sub-step launches, which use that buffer) and chunks of merge_g
        // steps can end on every sample step (merge_g divides every obs_every);
        // chunks start at multiples of merge_g
        // Within a chunk each step's end (small electron grid, bins, flags)
        // also runs as extra blocks of the next step's colour pass 0, whose
        // spin blocks compute the new T_e of their sites from the same
        // inputs; the chunk's last step ends in k_finalize.  Larger grids
        // keep their cell-parallel update, and diffusing electrons (whose
        // new T_e depends on the neighbour cells) their own launches.
        merge_g = 0;
        merge_run = -1;
        fold = false;
        mk_runs = rl;
        any_radial = false;
        for (int s : rl) any_radial = any_radial || host_rd[s].radial != 0;
        // the specialised colour pass: every run on the multi-kernel step has
        // the same lattice and species flag, no anisotropy, constant exchange
        lean_lat = -1;
        lean_multi = 0;
        if (!rl.empty()) {
            const RD& R0 = host_rd[rl[0]];
            bool same = spin_spt <= 2;
            for (int s : rl) {
                const RD& R = host_rd[s];
                same = same && R.lattice == R0.lattice && (R.n_species > 1) == (R0.n_species > 1) &&
                       !R.aniso && !R.radial;
            }
            if (same) {
                lean_lat = R0.lattice;
                lean_multi = R0.n_species > 1 ? 1 : 0;
            }
        }
        // the LDS-staged colour pass: bcc runs with one species, tiles of
        // 4 x 4 rows (in 1024-thread blocks when rows have 64 sites or more,
        // else 2 x 2 rows in 256-thread blocks when those do not fit), when
        // the tile divides every run's rows and planes, a row holds whole
        // 16-byte vectors (at most one per thread of the block), the spin
        // arrays are 16-byte aligned and the rows fit in LDS
        stile = 0;
        stile_bytes = 0;
        if (spin_access == 1 && lean_lat == SL_LATTICE_BCC && !lean_multi && !rl.empty()) {
            const uint32_t vec = 16u / (uint32_t)sizeof(T);
            bool small = false;
            for (int s : rl) small = small || host_rd[s].g.Lxh < 64;
            // long rows: 4 x 4 tiles in 1024-thread blocks while they fit in
            // LDS (one block per CU), else 2 x 2 in 256-thread blocks
            auto fits = [&](int kind) {
                bool ok = true;
                for (int s : rl) {
                    const RD& R = host_rd[s];
                    const int t = kind == 1 ? 2 : 4;
                    const uint32_t nt = kind == 3 ? 1024u : (uint32_t)sl::kBlock;
                    const uint32_t b = kind == 1 ? sl::tile_lds_bytes<2, 2>((uint32_t)R.g.Lxh, sizeof(T))
                                                 : sl::tile_lds_bytes<4, 4>((uint32_t)R.g.Lxh, sizeof(T));
                    const auto al = [](const void* q) { return (reinterpret_cast<uintptr_t>(q) & 15u) == 0; };
                    ok = ok && R.g.Ly % t == 0 && R.g.Lz % t == 0 && (uint32_t)R.g.Lxh % vec == 0 &&
                         (uint32_t)R.g.Lxh <= nt * vec && al(R.sx) && al(R.sy) && al(R.sz) &&
                         b <= stile_lds_max;
                }
                return ok;
            };
            const int kind = small ? (fits(2) ? 2 : 0) : (fits(3) ? 3 : (fits(1) ? 1 : 0));
            const int t = kind == 1 ? 2 : 4;
            uint32_t bytes = 0;
            for (int s : rl)
                bytes = std::max(bytes, kind == 1 ? sl::tile_lds_bytes<2, 2>((uint32_t)host_rd[s].g.Lxh, sizeof(T))
                                                  : sl::tile_lds_bytes<4, 4>((uint32_t)host_rd[s].g.Lxh, sizeof(T)));
            if (kind > 0) {
                stile = kind;
                stile_bytes = bytes;
                for (int s : rl) {
                    const RD& R = host_rd[s];
                    for (int z0 = 0; z0 < R.g.Lz; z0 += t)
                        for (int y0 = 0; y0 < R.g.Ly; y0 += t) tb.wst.push_back(make_int4(s, y0, z0, 0));
                }
                // each XCD takes one contiguous range of tiles, so the rows two
                // neighbouring tiles both stage come through the same L2
                xcd_order(tb.wst);
            }
        }
        // runs with radial exchange kick after the whole sweep, so no step
        // may leave its last colour pass to the next one
        if (merge_sweeps && !rl.empty() && !any_radial) {
            // several runs merge together when they have the same colour count
            // (they defer the same pass), a common chunk length divides every
            // sample interval, and the runs still stepping are at the same
            // step modulo it (runs added together, advanced in whole chunks)
            bool ok = true, sampled = false;
            for (int s : rl) {
                const RD& R = host_rd[s];
                if ((R.ttm_mode == 1 && R.kappa_e != 0.0 && R.dtile[0] == 0) ||
                    R.g.C != host_rd[rl[0]].g.C)
                    ok = false;
                sampled = sampled || R.obs_every > 0;
            }
            int g = sampled ? 0 : graph_steps;
            for (int d = 64; sampled && d >= 2 && g == 0; --d) {
                bool all = true;
                for (int s : rl) all = all && (host_rd[s].obs_every <= 0 || host_rd[s].obs_every % d == 0);
                if (all) g = d;
            }
            int64_t phase = -1;
            for (int s : rl) {
                if (!ok || g < 2 || runs[s].steps >= runs[s].target) continue;
                if (phase < 0) {
                    phase = runs[s].steps % g;
                    merge_run = s;
                } else if (runs[s].steps % g != phase) {
                    ok = false;
                }
            }
            if (ok && g >= 2 && merge_run >= 0) {
                merge_g = g;
                const RD& R = host_rd[merge_run];
                if (rl.size() == 1) {
                    // (a prescribed profile is written at the step end in
                    // place, so it does not fold)
                    fold = R.ttm_mode != 2 &&
                           !(R.ttm_mode == 1 && (R.ncell > sl::kSmallGrid || R.kappa_e != 0.0));
                    // one thread per electron cell, four bins per thread
                    const int cells = R.ttm_mode == 1 ? R.ncell : 0;
                    const int bins = R.live ? (R.nbins + 3) / 4 : 0;
                    fold_blocks = std::max(1, (std::max(cells, bins) + spin_eff - 1) / spin_eff);
                }
            }
        }
        // the fused schedule (tuning fuse_force): merged chunks of runs with
        // the specialised site update (merging already excludes radial
        // exchange; at most two sites per thread), a live lattice among them,
        // and force blocks that hold whole colour-pass tiles
        fused = false;
        force_spin_blocks = 0;
        if (merge_g >= 2 && fuse_force && lean_lat >= 0 && atom_block % spin_eff == 0 && !wk.empty()) {
            fused = true;
            const int per = atom_block / spin_eff;
            force_spin_blocks = ((int)ws.size() + per - 1) / per;
        }
        active_blocks_spin = (int)ws.size();
        active_blocks_atom = (int)wa.size();
        active_blocks_kick = (int)wk.size();
        active_blocks_cell = (int)wc.size();
        active_blocks_diff = (int)wd.size();
        active_blocks_tile = (int)wt.size();
        active_blocks_stile = (int)tb.wst.size();
        active_runs = (int)rl.size();
        persist_runs = (int)pl.size();
        persist_radial = false;
        for (int s : pl) persist_radial = persist_radial || host_rd[s].radial != 0;
    }

    // Device copies of the tables, in memory from the engine's allocator.
    sl_status upload_tables(const Tables& tb)
    {
        for (void* p : tables) alloc.put(p);
        tables.clear();
        d_work_spin = d_work_atom = d_work_kick = d_work_cell = d_work_diff = d_work_tile = nullptr;
        d_work_stile = nullptr;
        d_run_list = nullptr;
        d_persist_list = nullptr;
        auto up = [&](const void* src, size_t bytes, void** dst) -> sl_status {
            if (bytes == 0) return SL_OK;
            void* p = alloc.get(bytes);
            if (!p) return fail(SL_ENOMEM, "device allocation failed");
            tables.push_back(p);
            SL_HIP(hipMemcpyAsync(p, src, bytes, hipMemcpyHostToDevice, stream));
            *dst = p;
            return SL_OK;
        };
        sl_status st;
        if ((st = up(tb.ws.data(), sizeof(int2) * tb.ws.size(), (void**)&d_work_spin)) != SL_OK) return st;
        if ((st = up(tb.wa.data(), sizeof(int2) * tb.wa.size(), (void**)&d_work_atom)) != SL_OK) return st;
        if ((st = up(tb.wk.data(), sizeof(int2) * tb.wk.size(), (void**)&d_work_kick)) != SL_OK) return st;
        if ((st = up(tb.wc.data(), sizeof(int2) * tb.wc.size(), (void**)&d_work_cell)) != SL_OK) return st;
        if ((st = up(tb.wd.data(), sizeof(int2) * tb.wd.size(), (void**)&d_work_diff)) != SL_OK) return st;
        if ((st = up(tb.wt.data(), sizeof(int2) * tb.wt.size(), (void**)&d_work_tile)) != SL_OK) return st;
        if ((st = up(tb.wst.data(), sizeof(int4) * tb.wst.size(), (void**)&d_work_stile)) != SL_OK) return st;
        if ((st = up(tb.rl.data(), sizeof(int) * tb.rl.size(), (void**)&d_run_list)) != SL_OK) return st;
        if ((st = up(tb.pl.data(), sizeof(int) * tb.pl.size(), (void**)&d_persist_list)) != SL_OK) return st;
        SL_HIP(hipStreamSynchronize(stream));
        return SL_OK;
    }

    int max_colours() const
    {
        int c = 0;
        for (size_t s = 0; s < runs.size(); ++s)
            if (runs[s].used) c = std::max(c, host_rd[s].g.C);
        return c;
    }

    template <typename F> sl_status timed(hipStream_t st, Prof* p, int cls, F&& launch)
    {
        if (!p) {
            launch(nullptr, nullptr);
            return SL_OK;
        }
        hipEvent_t a, b;
        SL_HIP(hipEventCreate(&a));
        SL_HIP(hipEventCreate(&b));
        launch(a, b);
        SL_HIP(hipGetLastError());
        p->ev->push_back(a);
        p->ev->push_back(b);
        p->cls->push_back(cls);
        return SL_OK;
    }

    // Binning for a rebuild, between the kick and the force kernel, in
    // engines whose kick does not bin: capped grids striding over the atom
    // table, which exit at once unless a run flagged a rebuild.
    sl_status enqueue_binning(hipStream_t st, Prof* p, int fold_k)
    {
        if (active_blocks_kick == 0 || bin_each_step) return SL_OK;
        // one thread per atom of the atom table's tiles
        const dim3 gb(std::min(active_blocks_atom, kBinGrid)), bt(atom_block / lanes_eff);
        sl_status e = timed(st, p, 3, [&](hipEvent_t a, hipEvent_t b) {
            launch(sl::k_nbr_bin<T>, gb, bt, 0, st, a, b, d_runs, d_work_atom, (int)sl::PHASE_STEP,
                   fold_k, active_blocks_atom, (const int32_t*)d_any_rebuild);
        });
        if (e != SL_OK) return e;
        return timed(st, p, 3, [&](hipEvent_t a, hipEvent_t b) {
            launch(sl::k_nbr_sort<T>, gb, bt, 0, st, a, b, d_runs, d_work_atom, (int)sl::PHASE_STEP,
                   fold_k, active_blocks_atom, (const int32_t*)d_any_rebuild);
        });
    }

    // One step of every run on the multi-kernel path.  Profiling classes:
    // 0 colour pass, 1 list rebuild (when flagged) and force / e-ph kernel,
    // 2 colour pass carrying the lattice kick and drift, 3 binning for a
    // rebuild, electron grid and end of step, 5 colour pass 1 carrying the
    // force kernel.
    // merge_first: colour pass 0 applies the previous step's deferred last
    // half step first; defer_last: this step's last colour pass is left to
    // the next step's pass 0.  The lattice kick rides on colour pass 1 (on
    // pass 0 in the fused schedule).
    // fold_k >= 0: position of the step in a folded chunk of chunk_len steps
    // (its pass 0 ends the previous step, and only the chunk's last step has
    // a k_finalize).  In the fused schedule (merged chunks) the force
    // kernel of every step but the chunk's last (a sample step, whose force
    // kernel reads the spins after the whole sweep) runs in the launch of
    // colour pass 1; free_end: the chunk ends off a chunk boundary, so on no
    // sample step, and its last step's force kernel does too.
    sl_status enqueue_step(hipStream_t st, Prof* p, bool merge_first = false, bool defer_last = false,
                           int fold_k = -1, int chunk_len = 0, bool free_end = false)
    {
        const int C = max_colours();
        // the atom table's tiles hold atom_block / atom_lanes atoms:
        // k_atom_final gives each atom_lanes threads
        const dim3 bs(spin_eff), ba(atom_block), bk(sl::kBlock);
        const bool kick0 = fused && chunk_len > 0;
        const bool force1 = kick0 && (defer_last || free_end);
        sl_status e;
        for (int pass = 0; pass < 2 * C - 1; ++pass) {
            if (defer_last && pass == 2 * C - 2) break;
            const int merge = merge_first && pass == 0 ? 1 : 0;
            if (force1 && pass == 1) {
                e = timed(st, p, 5, [&](hipEvent_t a, hipEvent_t b) {
                    if (lanes_eff == 4)
                        spin_force_lanes<4>(st, a, b, pass, fold_k);
                    else if (lanes_eff == 2)
                        spin_force_lanes<2>(st, a, b, pass, fold_k);
                    else
                        spin_force_lanes<1>(st, a, b, pass, fold_k);
                });
                if (e != SL_OK) return e;
                continue;
            }
            const bool kicks = kick0 ? pass == 0 : pass == 1 && active_blocks_kick > 0 && !any_radial;
            const int nf = pass == 0 && fold_k >= 1 ? fold_blocks : 0;
            const int nk = (kicks ? active_blocks_kick : 0) + nf;
            e = timed(st, p, kicks ? 2 : 0, [&](hipEvent_t a, hipEvent_t b) {
                const dim3 g(active_blocks_spin + nk);
                if (nk == 0 && merge == 0 && lean_lat >= 0) {
                    if (stile > 0 && stile_on) {
                        const dim3 gt(active_blocks_stile), bt2(sl::kBlock);
                        if (stile == 1)
                            launch(sl::k_spin_tile_bcc<T, 2, 2>, gt, bt2, stile_bytes, st, a, b, d_runs,
                                   d_work_stile, pass, fold_k);
                        else if (stile == 2)
                            launch(sl::k_spin_tile_bcc<T, 4, 4>, gt, bt2, stile_bytes, st, a, b, d_runs,
                                   d_work_stile, pass, fold_k);
                        else
                            launch(sl::k_spin_tile_bcc<T, 4, 4, 1024>, gt, dim3(1024), stile_bytes, st, a,
                                   b, d_runs, d_work_stile, pass, fold_k);
                        return;
                    }
                    launch_lean(g, bs, st, a, b, pass, fold_k);
                    return;
                }
                if (lean_lat >= 0) {
                    spin_pass_form(g, bs, st, a, b, pass, nf, merge, fold_k);
                    return;
                }
                if (any_radial) {
                    if (spin_spt == 4)
                        launch(sl::k_spin_pass<T, 4, true>, g, bs, 0, st, a, b, d_runs, d_work_spin, pass,
                               d_work_kick, active_blocks_spin, nf, merge, fold_k);
                    else if (spin_spt == 2)
                        launch(sl::k_spin_pass<T, 2, true>, g, bs, 0, st, a, b, d_runs, d_work_spin, pass,
                               d_work_kick, active_blocks_spin, nf, merge, fold_k);
                    else
                        launch(sl::k_spin_pass<T, 1, true>, g, bs, 0, st, a, b, d_runs, d_work_spin, pass,
                               d_work_kick, active_blocks_spin, nf, merge, fold_k);
                } else if (spin_spt == 4)
                    launch(sl::k_spin_pass<T, 4>, g, bs, 0, st, a, b, d_runs, d_work_spin, pass,
                           d_work_kick, active_blocks_spin, nf, merge, fold_k);
                else if (spin_spt == 2)
                    launch(sl::k_spin_pass<T, 2>, g, bs, 0, st, a, b, d_runs, d_work_spin, pass,
                           d_work_kick, active_blocks_spin, nf, merge, fold_k);
                else
                    launch(sl::k_spin_pass<T, 1>, g, bs, 0, st, a, b, d_runs, d_work_spin, pass,
                           d_work_kick, active_blocks_spin, nf, merge, fold_k);
            });
            if (e != SL_OK) return e;
            if (kick0 && pass == 0) {
                e = enqueue_binning(st, p, fold_k);
                if (e != SL_OK) return e;
            }
        }
        const dim3 ga(active_blocks_atom);
        if (any_radial && active_blocks_kick > 0) {
            // after the sweep: the exchange half kick of radial runs, then the
            // drift of every live run (a launch of kick blocks only)
            e = timed(st, p, 2, [&](hipEvent_t a, hipEvent_t b) {
                launch(sl::k_half_kick<T>, dim3(active_blocks_kick), bs, 0, st, a, b, d_runs, d_work_kick);
            });
            if (e != SL_OK) return e;
            e = timed(st, p, 2, [&](hipEvent_t a, hipEvent_t b) {
                launch(sl::k_spin_pass<T, 1>, dim3(active_blocks_kick), bs, 0, st, a, b, d_runs, d_work_spin,
                       1, d_work_kick, 0, 0, 0, -1);
            });
            if (e != SL_OK) return e;
        }
        if (!kick0) {
            e = enqueue_binning(st, p, fold_k);
            if (e != SL_OK) return e;
        }
        if (!force1) {
            e = timed(st, p, 1, [&](hipEvent_t a, hipEvent_t b) {
                const int sorted = bin_each_step ? 0 : 1;
                if (any_radial) {
                    if (lanes_eff == 4)
                        launch(sl::k_atom_final<T, 4, true>, ga, ba, 0, st, a, b, d_runs, d_work_atom,
                               (int)sl::PHASE_STEP, sorted, fold_k);
                    else if (lanes_eff == 2)
                        launch(sl::k_atom_final<T, 2, true>, ga, ba, 0, st, a, b, d_runs, d_work_atom,
                               (int)sl::PHASE_STEP, sorted, fold_k);
                    else
                        launch(sl::k_atom_final<T, 1, true>, ga, ba, 0, st, a, b, d_runs, d_work_atom,
                               (int)sl::PHASE_STEP, sorted, fold_k);
                } else if (lanes_eff == 4)
                    launch(sl::k_atom_final<T, 4>, ga, ba, 0, st, a, b, d_runs, d_work_atom,
                           (int)sl::PHASE_STEP, sorted, fold_k);
                else if (lanes_eff == 2)
                    launch(sl::k_atom_final<T, 2>, ga, ba, 0, st, a, b, d_runs, d_work_atom,
                           (int)sl::PHASE_STEP, sorted, fold_k);
                else
                    launch(sl::k_atom_final<T, 1>, ga, ba, 0, st, a, b, d_runs, d_work_atom,
                           (int)sl::PHASE_STEP, sorted, fold_k);
            });
            if (e != SL_OK) return e;
        }
        if (active_blocks_tile > 0) {
            e = timed(st, p, 3, [&](hipEvent_t a, hipEvent_t b) {
                launch(sl::k_ttm_tile<T>, dim3(active_blocks_tile), dim3(sl::kTileBlock), tile_bytes, st, a,
                       b, d_runs, d_work_tile);
            });
            if (e != SL_OK) return e;
        }
        for (int sub = 0; sub < max_sub; ++sub) {
            e = timed(st, p, 3, [&](hipEvent_t a, hipEvent_t b) {
                launch(sl::k_ttm_diffuse<T>, dim3(active_blocks_diff), bk, 0, st, a, b, d_runs,
                       d_work_diff, sub);
            });
            if (e != SL_OK) return e;
        }
        if (active_blocks_cell > 0) {
            e = timed(st, p, 3, [&](hipEvent_t a, hipEvent_t b) {
                launch(sl::k_grid<T>, dim3(active_blocks_cell), bk, 0, st, a, b, d_runs, d_work_cell);
            });
            if (e != SL_OK) return e;
        }
        if (fold_k >= 0 && fold_k < (chunk_len > 0 ? chunk_len : merge_g) - 1) return SL_OK;
        e = timed(st, p, 3, [&](hipEvent_t a, hipEvent_t b) {
            launch(sl::k_finalize<T>, dim3(active_runs), bk, 0, st, a, b, d_runs, d_run_list,
                   (int)sl::PHASE_STEP, defer_last ? 1 : 0, fold_k);
        });
        return e;
    }

    // The persistent kernel for the block size and exchange form in use.
    void launch_persist(hipStream_t st, hipEvent_t a, hipEvent_t b, int nsteps)
    {
        const dim3 g(persist_runs), bl(persist_block);
        if (persist_block > 512) {
            if (persist_radial)
                launch(sl::k_persist<T, 1024, true>, g, bl, persist_bytes, st, a, b, d_runs, d_persist_list, nsteps, lds_max);
            else
                launch(sl::k_persist<T, 1024>, g, bl, persist_bytes, st, a, b, d_runs, d_persist_list, nsteps, lds_max);
        } else {
            if (persist_radial)
                launch(sl::k_persist<T, 512, true>, g, bl, persist_bytes, st, a, b, d_runs, d_persist_list, nsteps, lds_max);
            else
                launch(sl::k_persist<T, 512>, g, bl, persist_bytes, st, a, b, d_runs, d_persist_list, nsteps, lds_max);
        }
    }

    // A colour pass with extra blocks (or a deferred half step) whose spin
    // blocks take the specialised site update of the engine's form.
    template <int LAT, bool MULTI>
    void spin_pass_as(dim3 g, dim3 bs, hipStream_t st, hipEvent_t a, hipEvent_t b, int pass, int nf, int merge,
                      int fold_k)
    {
        if (spin_spt == 2)
            launch(sl::k_spin_pass<T, 2, false, LAT, MULTI>, g, bs, 0, st, a, b, d_runs, d_work_spin, pass,
                   d_work_kick, active_blocks_spin, nf, merge, fold_k);
        else
            launch(sl::k_spin_pass<T, 1, false, LAT, MULTI>, g, bs, 0, st, a, b, d_runs, d_work_spin, pass,
                   d_work_kick, active_blocks_spin, nf, merge, fold_k);
    }
    void spin_pass_form(dim3 g, dim3 bs, hipStream_t st, hipEvent_t a, hipEvent_t b, int pass, int nf, int merge,
                        int fold_k)
    {
        if (lean_lat == SL_LATTICE_SC) {
            if (lean_multi) spin_pass_as<SL_LATTICE_SC, true>(g, bs, st, a, b, pass, nf, merge, fold_k);
            else spin_pass_as<SL_LATTICE_SC, false>(g, bs, st, a, b, pass, nf, merge, fold_k);
        } else if (lean_lat == SL_LATTICE_FCC) {
            if (lean_multi) spin_pass_as<SL_LATTICE_FCC, true>(g, bs, st, a, b, pass, nf, merge, fold_k);
            else spin_pass_as<SL_LATTICE_FCC, false>(g, bs, st, a, b, pass, nf, merge, fold_k);
        } else {
            if (lean_multi) spin_pass_as<SL_LATTICE_BCC, true>(g, bs, st, a, b, pass, nf, merge, fold_k);
            else spin_pass_as<SL_LATTICE_BCC, false>(g, bs, st, a, b, pass, nf, merge, fold_k);
        }
    }

    // Colour pass `pass` with the force kernel (k_spin_force) for the lanes
    // per atom and the site-update form in use.
    template <int LPA, int LAT, bool MULTI>
    void spin_force_as(hipStream_t st, hipEvent_t a, hipEvent_t b, int pass, int fold_k)
    {
        const dim3 g(force_spin_blocks + active_blocks_atom), bl(atom_block);
        if (spin_spt == 2)
            launch(sl::k_spin_force<T, LPA, LAT, MULTI, 2>, g, bl, 0, st, a, b, d_runs, d_work_spin,
                   active_blocks_spin, spin_eff, active_blocks_atom, d_work_atom, pass, bin_each_step ? 0 : 1,
                   fold_k, fold ? 1 : 0);
        else
            launch(sl::k_spin_force<T, LPA, LAT, MULTI>, g, bl, 0, st, a, b, d_runs, d_work_spin,
                   active_blocks_spin, spin_eff, active_blocks_atom, d_work_atom, pass, bin_each_step ? 0 : 1,
                   fold_k, fold ? 1 : 0);
    }
    template <int LPA> void spin_force_lanes(hipStream_t st, hipEvent_t a, hipEvent_t b, int pass, int fold_k)
    {
        if (lean_lat == SL_LATTICE_SC) {
            if (lean_multi) spin_force_as<LPA, SL_LATTICE_SC, true>(st, a, b, pass, fold_k);
            else spin_force_as<LPA, SL_LATTICE_SC, false>(st, a, b, pass, fold_k);
        } else if (lean_lat == SL_LATTICE_FCC) {
            if (lean_multi) spin_force_as<LPA, SL_LATTICE_FCC, true>(st, a, b, pass, fold_k);
            else spin_force_as<LPA, SL_LATTICE_FCC, false>(st, a, b, pass, fold_k);
        } else {
            if (lean_multi) spin_force_as<LPA, SL_LATTICE_BCC, true>(st, a, b, pass, fold_k);
            else spin_force_as<LPA, SL_LATTICE_BCC, false>(st, a, b, pass, fold_k);
        }
    }

    // The specialised colour pass for the engine's site-update form.
    void launch_lean(dim3 g, dim3 bs, hipStream_t st, hipEvent_t a, hipEvent_t b, int pass, int fold_k)
    {
        const bool two = spin_spt == 2;
        if (lean_lat == SL_LATTICE_SC) {
            if (lean_multi) {
                if (two) launch(sl::k_spin_pass_lean<T, 2, SL_LATTICE_SC, true>, g, bs, 0, st, a, b, d_runs, d_work_spin, pass, fold_k);
                else launch(sl::k_spin_pass_lean<T, 1, SL_LATTICE_SC, true>, g, bs, 0, st, a, b, d_runs, d_work_spin, pass, fold_k);
            } else {
                if (two) launch(sl::k_spin_pass_lean<T, 2, SL_LATTICE_SC, false>, g, bs, 0, st, a, b, d_runs, d_work_spin, pass, fold_k);
                else launch(sl::k_spin_pass_lean<T, 1, SL_LATTICE_SC, false>, g, bs, 0, st, a, b, d_runs, d_work_spin, pass, fold_k);
            }
        } else if (lean_lat == SL_LATTICE_FCC) {
            if (lean_multi) {
                if (two) launch(sl::k_spin_pass_lean<T, 2, SL_LATTICE_FCC, true>, g, bs, 0, st, a, b, d_runs, d_work_spin, pass, fold_k);
                else launch(sl::k_spin_pass_lean<T, 1, SL_LATTICE_FCC, true>, g, bs, 0, st, a, b, d_runs, d_work_spin, pass, fold_k);
            } else {
                if (two) launch(sl::k_spin_pass_lean<T, 2, SL_LATTICE_FCC, false>, g, bs, 0, st, a, b, d_runs, d_work_spin, pass, fold_k);
                else launch(sl::k_spin_pass_lean<T, 1, SL_LATTICE_FCC, false>, g, bs, 0, st, a, b, d_runs, d_work_spin, pass, fold_k);
            }
        } else {
            if (lean_multi) {
                if (two) launch(sl::k_spin_pass_lean<T, 2, SL_LATTICE_BCC, true>, g, bs, 0, st, a, b, d_runs, d_work_spin, pass, fold_k);
                else launch(sl::k_spin_pass_lean<T, 1, SL_LATTICE_BCC, true>, g, bs, 0, st, a, b, d_runs, d_work_spin, pass, fold_k);
            } else {
                if (two) launch(sl::k_spin_pass_lean<T, 2, SL_LATTICE_BCC, false>, g, bs, 0, st, a, b, d_runs, d_work_spin, pass, fold_k);
                else launch(sl::k_spin_pass_lean<T, 1, SL_LATTICE_BCC, false>, g, bs, 0, st, a, b, d_runs, d_work_spin, pass, fold_k);
            }
        }
    }

    // One chunk of merge_g steps (or len < merge_g steps, which end before
    // the next multiple of merge_g and so on no sample step): every step but
    // the last defers its last colour half step, every step but the first
    // applies the one deferred before it, so the chunk ends with complete
    // sweeps.
    sl_status enqueue_chunk(hipStream_t st, Prof* p, int len = 0, bool free_end = false)
    {
        if (len <= 0) len = merge_g;
        for (int k = 0; k < len; ++k) {
            sl_status e = enqueue_step(st, p, k > 0, k < len - 1, fold ? k : -1, len, free_end);
            if (e != SL_OK) return e;
        }
        return SL_OK;
    }

    // steps per graph replay
    int graph_len() const { return merge_g >= 2 ? merge_g : graph_steps; }

    // single steps before the next chunk boundary of the merged runs, from
    // one that still steps (all that step share the phase; one that reached
    // its target keeps its final count)
    int64_t chunk_head() const
    {
        for (int s : mk_runs)
            if (runs[s].steps < runs[s].target) return (merge_g - runs[s].steps % merge_g) % merge_g;
        return 0;
    }

    // The graph of a merged chunk of len < merge_g steps (captured on first use).
    sl_status chunk_graph(int len, bool free_end, hipGraphExec_t* out)
    {
        const int key = 2 * len + (free_end ? 1 : 0);
        for (auto& e : short_exec)
            if (e.first == key) {
                *out = e.second;
                return SL_OK;
            }
        hipGraph_t graph = nullptr;
        SL_HIP(hipStreamBeginCapture(cap_stream, hipStreamCaptureModeThreadLocal));
        enqueue_chunk(cap_stream, nullptr, len, free_end);
        hipError_t e = hipStreamEndCapture(cap_stream, &graph);
        if (e != hipSuccess) return fail(SL_EHIP, std::string("graph capture: ") + hipGetErrorString(e));
        hipGraphExec_t ex = nullptr;
        e = hipGraphInstantiate(&ex, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        if (e != hipSuccess) return fail(SL_EHIP, std::string("graph instantiate: ") + hipGetErrorString(e));
        short_exec.emplace_back(key, ex);
        *out = ex;
        return SL_OK;
    }

    sl_status capture()
    {
        drop_graph();
        hipGraph_t graph = nullptr;
        SL_HIP(hipStreamBeginCapture(cap_stream, hipStreamCaptureModeThreadLocal));
        if (merge_g >= 2)
            enqueue_chunk(cap_stream, nullptr);
        else
            for (int k = 0; k < graph_steps; ++k) enqueue_step(cap_stream, nullptr);
        hipError_t e = hipStreamEndCapture(cap_stream, &graph);
        if (e != hipSuccess) return fail(SL_EHIP, std::string("graph capture: ") + hipGetErrorString(e));
        e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        if (e != hipSuccess) return fail(SL_EHIP, std::string("graph instantiate: ") + hipGetErrorString(e));
        graph_ok = true;
        return SL_OK;
    }
};

Engine* make_engine_fp32(int max_runs);
Engine* make_engine_fp64(int max_runs);

}  // namespace slrt
