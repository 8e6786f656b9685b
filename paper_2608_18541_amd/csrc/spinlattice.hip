// spinlattice.hip -- C ABI of the gfx950 spin-lattice step (include/spinlattice.h)
// over the engines of sl_engine.hpp.
#include <hip/hip_runtime.h>

#include <memory>
#include <mutex>
#include <string>

#include "../../include/spinlattice.h"
#include "sl_engine.hpp"

namespace slrt {
thread_local std::string g_err;
}  // namespace slrt

using namespace slrt;

namespace {

Engine* make_engine(int precision, int max_runs)
{
    if (precision == SL_FP32) return make_engine_fp32(max_runs);
    return make_engine_fp64(max_runs);
}

sl_status setup_engine(Engine* e, int precision, void* stream, const sl_allocator* a, size_t budget,
                       int graph_steps)
{
    e->precision = precision;
    if (a) {
        if (!a->alloc || !a->free) return fail(SL_EINVAL, "allocator needs alloc and free");
        e->alloc.a = *a;
        e->alloc.custom = true;
    }
    if (stream) {
        e->stream = static_cast<hipStream_t>(stream);
    } else {
        SL_HIP(hipStreamCreateWithFlags(&e->stream, hipStreamNonBlocking));
        e->own_stream = true;
    }
    e->budget = budget;
    if (graph_steps > 0) e->graph_steps = graph_steps;
    return e->init_device();
}

}  // namespace

// ======================================================= static scratch
// The device buffer of sl_step_noalloc: the launch tables of a system
// stepped without allocation.  Every GPU the library runs on holds its own
// copy for the life of the process.  In host code `scratch` names a host-side
// stand-in, not device memory: the buffer's device address is taken once per
// device with hipGetSymbolAddress and only that address is used.
static __device__ __align__(256) unsigned char scratch[SL_NOALLOC_SCRATCH_BYTES];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
char* g_scratch_dev[kMaxDevices] = {};

// Device address of the current device's scratch buffer (looked up on the
// first call on that device).
sl_status scratch_address(char** out)
{
    int dev = 0;
    SL_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return fail(SL_EINVAL, "device ordinal out of range");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_dev[dev]) {
        void* p = nullptr;
        SL_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) return fail(SL_EHIP, "hipGetSymbolAddress returned no address for the scratch buffer");
        g_scratch_dev[dev] = static_cast<char*>(p);
    }
    *out = g_scratch_dev[dev];
    return SL_OK;
}

}  // namespace

// ==================================================================== C ABI
struct sl_system_s {
    std::unique_ptr<Engine> eng;
};

struct sl_batch_s {
    std::unique_ptr<Engine> eng;
};

extern "C" {

const char* sl_last_error(void) { return g_err.c_str(); }

sl_status sl_footprint_bytes(const sl_system_desc* desc, const sl_ttm_desc* ttm, size_t* bytes)
{
    if (!desc || !bytes) return fail(SL_EINVAL, "null argument");
    sl_ttm_desc t = ttm ? *ttm : default_ttm();
    std::string e = validate_desc(desc);
    if (!e.empty()) return fail(SL_EINVAL, e);
    Sizes z = run_sizes(desc, &t);
    *bytes = (desc->precision == SL_FP32 ? main_bytes<float>(desc, z) : main_bytes<double>(desc, z)) +
             grid_bytes(z);
    return SL_OK;
}

sl_status sl_init_system(const sl_system_desc* desc, sl_system* out)
{
    if (!desc || !out) return fail(SL_EINVAL, "null argument");
    std::string e = validate_desc(desc);
    if (!e.empty()) return fail(SL_EINVAL, e);
    auto h = std::make_unique<sl_system_s>();
    h->eng.reset(make_engine(desc->precision, 1));
    sl_status st = setup_engine(h->eng.get(), desc->precision, desc->stream, desc->alloc, 0, 0);
    if (st != SL_OK) return st;
    sl_ttm_desc t = default_ttm();
    int slot = -1;
    st = h->eng->add(desc, &t, INT64_MAX, &slot);
    if (st != SL_OK) return st;
    *out = h.release();
    return SL_OK;
}

sl_status sl_set_ttm_grid(sl_system h, const sl_ttm_desc* ttm)
{
    if (!h || !ttm) return fail(SL_EINVAL, "null argument");
    return h->eng->set_grid(0, ttm);
}

sl_status sl_step(sl_system h, int64_t n_steps)
{
    if (!h) return fail(SL_EINVAL, "null handle");
    return h->eng->advance(n_steps);
}

sl_status sl_step_noalloc(sl_system h, int64_t n_steps)
{
    if (!h) return fail(SL_EINVAL, "null handle");
    char* p = nullptr;
    sl_status st = scratch_address(&p);
    if (st != SL_OK) return st;
    return h->eng->advance_noalloc(n_steps, p, SL_NOALLOC_SCRATCH_BYTES);
}

sl_status sl_step_profiled(sl_system h, int64_t n_steps, double avg_ms[6], int64_t launches[6])
{
    if (!h || !avg_ms || !launches) return fail(SL_EINVAL, "null argument");
    return h->eng->profiled(n_steps, avg_ms, launches);
}

sl_status sl_synchronize(sl_system h)
{
    if (!h) return fail(SL_EINVAL, "null handle");
    return h->eng->sync();
}

sl_status sl_observables(sl_system h, sl_obs* out, int64_t max_samples, int64_t* n_out)
{
    if (!h || !out || !n_out) return fail(SL_EINVAL, "null argument");
    return h->eng->get(0, nullptr, nullptr, nullptr, nullptr, out, max_samples, n_out);
}

sl_status sl_get_state(sl_system h, double* x, double* v, double* s, double* Te)
{
    if (!h) return fail(SL_EINVAL, "null handle");
    return h->eng->get(0, x, v, s, Te, nullptr, 0, nullptr);
}

sl_status sl_set_state(sl_system h, const double* x, const double* v, const double* s,
                       const double* Te)
{
    if (!h) return fail(SL_EINVAL, "null handle");
    return h->eng->set_state(0, x, v, s, Te);
}

sl_status sl_stats(sl_system h, sl_run_stats* out)
{
    if (!h) return fail(SL_EINVAL, "null handle");
    return h->eng->stats(0, out);
}

sl_status sl_info(sl_system h, int64_t* n_sites, int64_t* n_cells, int64_t* steps)
{
    if (!h) return fail(SL_EINVAL, "null handle");
    const Run& r = h->eng->runs[0];
    if (n_sites) *n_sites = r.z.n;
    if (n_cells) *n_cells = r.z.ncell;
    if (steps) *steps = r.steps;
    return SL_OK;
}

static sl_status set_tuning(Engine* e, const sl_tuning* t)
{
    if (!t) return fail(SL_EINVAL, "null tuning");
    const bool blk_ok = [](int b) { return b == 0 || b == 64 || b == 128 || b == 256; }(t->spin_block) &&
                        [](int b) { return b == 64 || b == 128 || b == 256; }(t->atom_block);
    if (!blk_ok) return fail(SL_EINVAL, "block sizes must be 64, 128 or 256 (spin_block also 0)");
    if (t->spin_spt != 1 && t->spin_spt != 2 && t->spin_spt != 4) return fail(SL_EINVAL, "spin_spt must be 1, 2 or 4");
    if (t->graph_steps < 1 || t->graph_steps > 256) return fail(SL_EINVAL, "graph_steps must be 1..256");
    if (t->persist_block != 0 && t->persist_block != 256 && t->persist_block != 512 &&
        t->persist_block != 1024)
        return fail(SL_EINVAL, "persist_block must be 0, 256, 512 or 1024");
    if (t->xcd_order != 0 && t->xcd_order != 1) return fail(SL_EINVAL, "xcd_order must be 0 or 1");
    if (t->bin_mode < 0 || t->bin_mode > 2) return fail(SL_EINVAL, "bin_mode must be 0, 1 or 2");
    if (t->atom_lanes != 0 && t->atom_lanes != 1 && t->atom_lanes != 2 && t->atom_lanes != 4)
        return fail(SL_EINVAL, "atom_lanes must be 0, 1, 2 or 4");
    if (t->atom_lanes > 0 && t->atom_block / t->atom_lanes < 64)
        return fail(SL_EINVAL, "atom_block / atom_lanes must be at least 64");
    if (t->merge_sweeps != 0 && t->merge_sweeps != 1) return fail(SL_EINVAL, "merge_sweeps must be 0 or 1");
    if (t->spin_access != 0 && t->spin_access != 1) return fail(SL_EINVAL, "spin_access must be 0 or 1");
    if (t->fuse_force != 0 && t->fuse_force != 1) return fail(SL_EINVAL, "fuse_force must be 0 or 1");
    e->spin_block = t->spin_block;
    e->spin_spt = t->spin_spt;
    e->atom_block = t->atom_block;
    e->graph_steps = t->graph_steps;
    e->persist_block = t->persist_block;
    e->xcd_ord = t->xcd_order;
    e->bin_mode = t->bin_mode;
    e->atom_lanes = t->atom_lanes;
    e->merge_sweeps = t->merge_sweeps;
    e->spin_access = t->spin_access;
    e->fuse_force = t->fuse_force;
    return e->retune();
}

static void get_tuning(const Engine* e, sl_tuning* t)
{
    t->spin_block = e->spin_block;
    t->spin_spt = e->spin_spt;
    t->atom_block = e->atom_block;
    t->graph_steps = e->graph_steps;
    t->persist_block = e->persist_block;
    t->xcd_order = e->xcd_ord;
    t->bin_mode = e->bin_mode;
    t->atom_lanes = e->atom_lanes;
    t->merge_sweeps = e->merge_sweeps;
    t->spin_access = e->spin_access;
    t->fuse_force = e->fuse_force;
}

sl_status sl_set_tuning(sl_system h, const sl_tuning* t)
{
    if (!h) return fail(SL_EINVAL, "null handle");
    return set_tuning(h->eng.get(), t);
}

sl_status sl_get_tuning(sl_system h, sl_tuning* t)
{
    if (!h || !t) return fail(SL_EINVAL, "null argument");
    get_tuning(h->eng.get(), t);
    return SL_OK;
}

sl_status sl_batch_set_tuning(sl_batch b, const sl_tuning* t)
{
    if (!b) return fail(SL_EINVAL, "null handle");
    return set_tuning(b->eng.get(), t);
}

sl_status sl_batch_get_tuning(sl_batch b, sl_tuning* t)
{
    if (!b || !t) return fail(SL_EINVAL, "null argument");
    get_tuning(b->eng.get(), t);
    return SL_OK;
}

void sl_destroy(sl_system h) { delete h; }

sl_status sl_batch_create(const sl_batch_desc* desc, sl_batch* out)
{
    if (!desc || !out) return fail(SL_EINVAL, "null argument");
    if (desc->precision != SL_FP64 && desc->precision != SL_FP32) return fail(SL_EINVAL, "precision must be 0 or 1");
    if (desc->max_runs < 1 || desc->max_runs > (1 << 20)) return fail(SL_EINVAL, "max_runs out of range");
    if (desc->graph_steps < 0) return fail(SL_EINVAL, "graph_steps must be >= 0");
    auto b = std::make_unique<sl_batch_s>();
    b->eng.reset(make_engine(desc->precision, desc->max_runs));
    sl_status st = setup_engine(b->eng.get(), desc->precision, desc->stream, desc->alloc,
                                desc->mem_budget, desc->graph_steps);
    if (st != SL_OK) return st;
    b->eng->persist_block = desc->precision == SL_FP32 ? 1024 : 512;
    *out = b.release();
    return SL_OK;
}

sl_status sl_batch_add(sl_batch b, const sl_system_desc* desc, const sl_ttm_desc* ttm, int64_t n_steps,
                       int32_t* slot)
{
    if (!b || !desc || !slot) return fail(SL_EINVAL, "null argument");
    if (n_steps < 0) return fail(SL_EINVAL, "negative step count");
    sl_system_desc d = *desc;
    d.precision = b->eng->precision;
    sl_ttm_desc t = ttm ? *ttm : default_ttm();
    int s = -1;
    sl_status st = b->eng->add(&d, &t, n_steps, &s);
    if (st == SL_OK) *slot = s;
    return st;
}

sl_status sl_batch_advance(sl_batch b, int64_t n_steps)
{
    if (!b) return fail(SL_EINVAL, "null handle");
    return b->eng->advance(n_steps);
}

sl_status sl_batch_advance_profiled(sl_batch b, int64_t n_steps, double avg_ms[6], int64_t launches[6])
{
    if (!b || !avg_ms || !launches) return fail(SL_EINVAL, "null argument");
    return b->eng->profiled(n_steps, avg_ms, launches);
}

sl_status sl_batch_runs(sl_batch b, sl_run_info* info, int32_t cap, int32_t* n_out)
{
    if (!b || !n_out) return fail(SL_EINVAL, "null argument");
    int32_t k = 0;
    for (size_t s = 0; s < b->eng->runs.size(); ++s) {
        const Run& r = b->eng->runs[s];
        if (!r.used) continue;
        if (info && k < cap) {
            info[k].slot = (int32_t)s;
            info[k].status = SL_OK;
            info[k].steps_done = r.steps;
            info[k].steps_target = r.target;
            info[k].n_samples = r.d.obs_every > 0 ? 1 + r.steps / r.d.obs_every : 0;
        }
        ++k;
    }
    *n_out = k;
    return SL_OK;
}

sl_status sl_batch_get(sl_batch b, int32_t slot, double* x, double* v, double* s, double* Te,
                       sl_obs* obs, int64_t max_samples, int64_t* n_obs)
{
    if (!b) return fail(SL_EINVAL, "null handle");
    return b->eng->get(slot, x, v, s, Te, obs, max_samples, n_obs);
}

sl_status sl_batch_remove(sl_batch b, int32_t slot)
{
    if (!b) return fail(SL_EINVAL, "null handle");
    return b->eng->remove(slot);
}

sl_status sl_batch_stats(sl_batch b, int32_t slot, sl_run_stats* out)
{
    if (!b) return fail(SL_EINVAL, "null handle");
    return b->eng->stats(slot, out);
}

sl_status sl_batch_memory(sl_batch b, size_t* used, size_t* budget)
{
    if (!b) return fail(SL_EINVAL, "null handle");
    if (used) *used = b->eng->used_bytes;
    if (budget) *budget = b->eng->budget;
    return SL_OK;
}

sl_status sl_batch_synchronize(sl_batch b)
{
    if (!b) return fail(SL_EINVAL, "null handle");
    return b->eng->sync();
}

void sl_batch_destroy(sl_batch b) { delete b; }

}  // extern "C"
