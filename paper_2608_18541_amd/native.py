"""ctypes binding of ``libspinlattice.so`` (the C ABI in include/spinlattice.h).

Only argument marshalling lives here: every step of the dynamics runs in
the library's HIP kernels.  PyTorch supplies device memory (its caching
allocator, through the ABI's allocator callbacks) and the stream.  Importing
this module fails loudly when the library has not been built.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional, Sequence

import numpy as np

from . import inputs as I

_LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libspinlattice.so")

SL_OK, SL_EINVAL, SL_ENOMEM, SL_EHIP, SL_ENUMERIC, SL_EBUSY = 0, -1, -2, -3, -4, -5
SL_FP64, SL_FP32 = 0, 1


class SLError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__("%s (status %d)" % (msg, code))
        self.code = code


ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_void_p, C.c_size_t)
FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p)


class sl_allocator(C.Structure):
    _fields_ = [("ctx", C.c_void_p), ("alloc", ALLOC_FN), ("free", FREE_FN)]


class sl_system_desc(C.Structure):
    _fields_ = [
        ("lattice", C.c_int32), ("ncell", C.c_int32 * 3), ("a", C.c_double),
        ("n_species", C.c_int32), ("species", C.POINTER(C.c_int8)), ("mu", C.c_double * 4),
        ("mass", C.c_double * 4), ("n_shells", C.c_int32), ("J", ((C.c_double * 4) * 4) * 2),
        ("B", C.c_double * 3), ("K", C.c_double * 4), ("alpha", C.c_double),
        ("noise_mode", C.c_int32),
        ("mu_ref", C.c_double), ("lattice_mode", C.c_int32), ("morse", C.c_double * 4),
        ("skin", C.c_double), ("dt", C.c_double), ("seed", C.c_uint32), ("run_id", C.c_uint32),
        ("precision", C.c_int32), ("obs_every", C.c_int32), ("obs_capacity", C.c_int32),
        ("spin0", C.POINTER(C.c_double)), ("vel0", C.POINTER(C.c_double)),
        ("disp0", C.POINTER(C.c_double)), ("stream", C.c_void_p),
        ("alloc", C.POINTER(sl_allocator)),
        ("exch_radial", C.c_int32), ("exch_r", (C.c_double * 2) * 2),
    ]


class sl_ttm_desc(C.Structure):
    _fields_ = [
        ("n", C.c_int32 * 3), ("mode", C.c_int32), ("Te0", C.c_double),
        ("Te_init", C.POINTER(C.c_double)), ("gamma_e", C.c_double), ("G_el", C.c_double),
        ("kappa_e", C.c_double), ("n_sub", C.c_int32), ("S0", C.c_double), ("t0", C.c_double),
        ("fwhm", C.c_double), ("profile", C.c_int32), ("depth", C.c_double),
        ("step_T", C.c_double * 3), ("step_end", C.c_double * 2),
    ]


class sl_obs(C.Structure):
    _fields_ = [
        ("t", C.c_double), ("step", C.c_int64), ("M", (C.c_double * 3) * 4),
        ("m", C.c_double * 3), ("m_abs", C.c_double), ("E_ex", C.c_double),
        ("E_z", C.c_double), ("KE", C.c_double), ("PE", C.c_double), ("E_e", C.c_double),
        ("Te_mean", C.c_double), ("Te_max", C.c_double), ("Tl", C.c_double),
        ("Tspin", C.c_double * 4),
    ]


class sl_batch_desc(C.Structure):
    _fields_ = [
        ("precision", C.c_int32), ("max_runs", C.c_int32), ("mem_budget", C.c_size_t),
        ("graph_steps", C.c_int32), ("stream", C.c_void_p),
        ("alloc", C.POINTER(sl_allocator)),
    ]


class sl_tuning(C.Structure):
    _fields_ = [("spin_block", C.c_int32), ("spin_spt", C.c_int32), ("atom_block", C.c_int32),
                ("graph_steps", C.c_int32), ("persist_block", C.c_int32),
                ("xcd_order", C.c_int32), ("bin_mode", C.c_int32), ("atom_lanes", C.c_int32),
                ("merge_sweeps", C.c_int32), ("spin_access", C.c_int32),
                ("fuse_force", C.c_int32)]

    def to_dict(self) -> dict:
        return {k: getattr(self, k) for k, _ in self._fields_}


class sl_run_stats(C.Structure):
    _fields_ = [("steps", C.c_int64), ("samples", C.c_int64), ("list_rebuilds", C.c_int64),
                ("max_list", C.c_int32), ("list_capacity", C.c_int32),
                ("list_rescans", C.c_int32), ("error", C.c_int32)]

    def to_dict(self) -> dict:
        return {k: getattr(self, k) for k, _ in self._fields_}


class sl_run_info(C.Structure):
    _fields_ = [
        ("slot", C.c_int32), ("status", C.c_int32), ("steps_done", C.c_int64),
        ("steps_target", C.c_int64), ("n_samples", C.c_int64),
    ]


EXPORTS = {
    # name: (restype, argtypes)
    "sl_init_system": (C.c_int32, [C.POINTER(sl_system_desc), C.POINTER(C.c_void_p)]),
    "sl_set_ttm_grid": (C.c_int32, [C.c_void_p, C.POINTER(sl_ttm_desc)]),
    "sl_step": (C.c_int32, [C.c_void_p, C.c_int64]),
    "sl_step_noalloc": (C.c_int32, [C.c_void_p, C.c_int64]),
    "sl_synchronize": (C.c_int32, [C.c_void_p]),
    "sl_observables": (C.c_int32, [C.c_void_p, C.POINTER(sl_obs), C.c_int64,
                                   C.POINTER(C.c_int64)]),
    "sl_get_state": (C.c_int32, [C.c_void_p] + [C.POINTER(C.c_double)] * 4),
    "sl_set_state": (C.c_int32, [C.c_void_p] + [C.POINTER(C.c_double)] * 4),
    "sl_stats": (C.c_int32, [C.c_void_p, C.POINTER(sl_run_stats)]),
    "sl_batch_stats": (C.c_int32, [C.c_void_p, C.c_int32, C.POINTER(sl_run_stats)]),
    "sl_info": (C.c_int32, [C.c_void_p] + [C.POINTER(C.c_int64)] * 3),
    "sl_footprint_bytes": (C.c_int32, [C.POINTER(sl_system_desc), C.POINTER(sl_ttm_desc),
                                       C.POINTER(C.c_size_t)]),
    "sl_step_profiled": (C.c_int32, [C.c_void_p, C.c_int64, C.POINTER(C.c_double),
                                     C.POINTER(C.c_int64)]),
    "sl_set_tuning": (C.c_int32, [C.c_void_p, C.POINTER(sl_tuning)]),
    "sl_get_tuning": (C.c_int32, [C.c_void_p, C.POINTER(sl_tuning)]),
    "sl_batch_set_tuning": (C.c_int32, [C.c_void_p, C.POINTER(sl_tuning)]),
    "sl_batch_get_tuning": (C.c_int32, [C.c_void_p, C.POINTER(sl_tuning)]),
    "sl_destroy": (None, [C.c_void_p]),
    "sl_last_error": (C.c_char_p, []),
    "sl_batch_create": (C.c_int32, [C.POINTER(sl_batch_desc), C.POINTER(C.c_void_p)]),
    "sl_batch_add": (C.c_int32, [C.c_void_p, C.POINTER(sl_system_desc), C.POINTER(sl_ttm_desc),
                                 C.c_int64, C.POINTER(C.c_int32)]),
    "sl_batch_advance": (C.c_int32, [C.c_void_p, C.c_int64]),
    "sl_batch_advance_profiled": (C.c_int32, [C.c_void_p, C.c_int64, C.POINTER(C.c_double),
                                              C.POINTER(C.c_int64)]),
    "sl_batch_runs": (C.c_int32, [C.c_void_p, C.POINTER(sl_run_info), C.c_int32,
                                  C.POINTER(C.c_int32)]),
    "sl_batch_get": (C.c_int32, [C.c_void_p, C.c_int32] + [C.POINTER(C.c_double)] * 4 +
                     [C.POINTER(sl_obs), C.c_int64, C.POINTER(C.c_int64)]),
    "sl_batch_remove": (C.c_int32, [C.c_void_p, C.c_int32]),
    "sl_batch_memory": (C.c_int32, [C.c_void_p, C.POINTER(C.c_size_t), C.POINTER(C.c_size_t)]),
    "sl_batch_synchronize": (C.c_int32, [C.c_void_p]),
    "sl_batch_destroy": (None, [C.c_void_p]),
}

_lib = None


def lib():
    """The loaded library; raises ImportError when it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            raise ImportError("libspinlattice.so is not built: run __graft_entry__.build() "
                              "(hipcc --offload-arch=gfx950)")
        L = C.CDLL(_LIB_PATH)
        for name, (res, args) in EXPORTS.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def check(code: int) -> None:
    if code != SL_OK:
        raise SLError(code, lib().sl_last_error().decode())


def _dp(a: Optional[np.ndarray]):
    if a is None:
        return None
    return a.ctypes.data_as(C.POINTER(C.c_double))


# ------------------------------------------------------- torch plumbing

class TorchAllocator:
    """Device memory from PyTorch's caching allocator via the ABI callbacks."""

    def __init__(self):
        import torch
        self._torch = torch
        self._live = {}
        self.n_allocs = 0
        self.history = []          # (device address, bytes) of every allocation, in order
        self._alloc = ALLOC_FN(self._do_alloc)
        self._free = FREE_FN(self._do_free)
        self.struct = sl_allocator(None, self._alloc, self._free)

    def _do_alloc(self, ctx, nbytes):
        t = self._torch.empty(int(nbytes) + 256, dtype=self._torch.uint8, device="cuda")
        p = t.data_ptr()
        aligned = (p + 255) & ~255
        self._live[aligned] = t
        self.n_allocs += 1
        self.history.append((aligned, int(nbytes)))
        return aligned

    def _do_free(self, ctx, ptr):
        self._live.pop(ptr, None)


def torch_stream() -> int:
    import torch
    return int(torch.cuda.current_stream().cuda_stream)


# -------------------------------------------------- description builders

def system_desc(spec: I.SystemSpec, state: I.InitialState, precision: int = SL_FP64,
                obs_every: int = 0, obs_capacity: int = 1, stream=None, alloc=None):
    """Fills an sl_system_desc; returns (desc, keep) where keep holds the
    arrays that must outlive the call."""
    n = spec.n_sites
    keep = {}
    d = sl_system_desc()
    d.lattice = spec.lattice
    d.ncell = (C.c_int32 * 3)(*spec.ncell)
    d.a = spec.a
    d.n_species = spec.n_species
    sp = np.ascontiguousarray(np.asarray(state.species, dtype=np.int8).reshape(n))
    keep["species"] = sp
    d.species = sp.ctypes.data_as(C.POINTER(C.c_int8))
    d.mu = (C.c_double * 4)(*spec.mu)
    d.mass = (C.c_double * 4)(*spec.mass)
    d.n_shells = spec.n_shells
    J = np.asarray(spec.J, dtype=np.float64)
    for sh in range(2):
        for a in range(4):
            for b in range(4):
                d.J[sh][a][b] = float(J[sh, a, b])
    d.B = (C.c_double * 3)(*spec.B)
    d.K = (C.c_double * 4)(*spec.K)
    d.alpha = spec.alpha
    d.noise_mode = spec.noise_mode
    d.mu_ref = spec.mu_ref
    d.lattice_mode = spec.lattice_mode
    d.morse = (C.c_double * 4)(*spec.morse)
    d.skin = spec.skin
    d.dt = spec.dt
    d.seed = spec.seed & 0xFFFFFFFF
    d.run_id = spec.run_id & 0xFFFFFFFF
    d.precision = precision
    d.obs_every = obs_every
    d.obs_capacity = max(1, obs_capacity)
    s0 = np.ascontiguousarray(np.asarray(state.spins, dtype=np.float64).reshape(n, 3))
    keep["s0"] = s0
    d.spin0 = _dp(s0)
    if state.vel is not None:
        v0 = np.ascontiguousarray(np.asarray(state.vel, dtype=np.float64).reshape(n, 3))
        keep["v0"] = v0
        d.vel0 = _dp(v0)
    if state.disp is not None:
        u0 = np.ascontiguousarray(np.asarray(state.disp, dtype=np.float64).reshape(n, 3))
        keep["u0"] = u0
        d.disp0 = _dp(u0)
    d.exch_radial = int(getattr(spec, "exch_radial", 0))
    er = getattr(spec, "exch_r", ((0.0, 0.0), (0.0, 0.0)))
    for sh in range(2):
        for q in range(2):
            d.exch_r[sh][q] = float(er[sh][q])
    d.stream = stream
    if alloc is not None:
        d.alloc = C.pointer(alloc.struct)
        keep["alloc"] = alloc
    return d, keep


def ttm_desc(spec: I.SystemSpec, Te: Optional[np.ndarray] = None):
    t = sl_ttm_desc()
    t.n = (C.c_int32 * 3)(*spec.tn)
    t.mode = spec.ttm_mode
    t.Te0 = spec.Te0
    keep = {}
    if Te is not None:
        a = np.ascontiguousarray(np.asarray(Te, dtype=np.float64).reshape(spec.n_tcells))
        keep["Te"] = a
        t.Te_init = _dp(a)
    t.gamma_e = spec.gamma_e
    t.G_el = spec.G_el
    t.kappa_e = spec.kappa_e
    t.n_sub = max(1, spec.n_sub)
    t.S0 = spec.S0
    t.t0 = spec.t0
    t.fwhm = spec.fwhm
    t.profile = spec.profile
    t.depth = spec.depth
    t.step_T = (C.c_double * 3)(*spec.step_T)
    t.step_end = (C.c_double * 2)(*spec.step_end)
    return t, keep


def obs_to_dict(o: sl_obs) -> dict:
    return {
        "t": o.t, "step": o.step,
        "M": np.array([[o.M[s][k] for k in range(3)] for s in range(4)]),
        "m": np.array([o.m[k] for k in range(3)]), "m_abs": o.m_abs, "E_ex": o.E_ex,
        "E_z": o.E_z, "KE": o.KE, "PE": o.PE, "E_e": o.E_e, "Te_mean": o.Te_mean,
        "Te_max": o.Te_max, "Tl": o.Tl, "Tspin": np.array([o.Tspin[s] for s in range(4)]),
    }


# ------------------------------------------------------------ the plain run

class System:
    """One run on the GPU (the plain one-run-per-launch path)."""

    def __init__(self, spec: I.SystemSpec, state: I.InitialState, precision: int = SL_FP64,
                 obs_every: int = 0, obs_capacity: int = 4096, Te=None, use_torch: bool = True):
        self.spec = spec
        self.n = spec.n_sites
        self._alloc = TorchAllocator() if use_torch else None
        stream = torch_stream() if use_torch else None
        d, keep = system_desc(spec, state, precision, obs_every, obs_capacity, stream,
                              self._alloc)
        h = C.c_void_p()
        check(lib().sl_init_system(C.byref(d), C.byref(h)))
        self._h = h
        t, keep2 = ttm_desc(spec, Te)
        check(lib().sl_set_ttm_grid(self._h, C.byref(t)))

    def close(self):
        if getattr(self, "_h", None):
            lib().sl_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def step(self, n: int = 1) -> None:
        check(lib().sl_step(self._h, int(n)))

    def step_noalloc(self, n: int = 1) -> None:
        """As step, through the allocation-free entry point."""
        check(lib().sl_step_noalloc(self._h, int(n)))

    def synchronize(self) -> None:
        check(lib().sl_synchronize(self._h))

    def state(self) -> dict:
        n = self.n
        x = np.zeros((n, 3)); v = np.zeros((n, 3)); s = np.zeros((n, 3))
        Te = np.zeros(self.spec.n_tcells)
        check(lib().sl_get_state(self._h, _dp(x), _dp(v), _dp(s), _dp(Te)))
        return {"x": x, "v": v, "s": s, "Te": Te}

    def stats(self) -> dict:
        """Device-side counters: steps, samples, list rebuilds, longest list."""
        out = sl_run_stats()
        check(lib().sl_stats(self._h, C.byref(out)))
        return out.to_dict()

    def set_state(self, x=None, v=None, s=None, Te=None) -> None:
        """Replaces any of positions, velocities, spins and the electron grid
        (canonical order); the step counter and the noise stream continue."""
        def arr(a, shape):
            if a is None:
                return None
            a = np.ascontiguousarray(a, dtype=np.float64)
            if a.shape != shape:
                raise ValueError("expected shape %s, got %s" % (shape, a.shape))
            return a
        n = self.n
        bufs = [arr(x, (n, 3)), arr(v, (n, 3)), arr(s, (n, 3)), arr(Te, (self.spec.n_tcells,))]
        ptrs = [None if b is None else _dp(b) for b in bufs]
        check(lib().sl_set_state(self._h, *ptrs))

    def observables(self, max_samples: int = 1 << 20) -> list:
        buf = (sl_obs * max_samples)()
        n = C.c_int64()
        check(lib().sl_observables(self._h, buf, max_samples, C.byref(n)))
        return [obs_to_dict(buf[k]) for k in range(n.value)]

    def info(self) -> tuple:
        a, b, c = C.c_int64(), C.c_int64(), C.c_int64()
        check(lib().sl_info(self._h, C.byref(a), C.byref(b), C.byref(c)))
        return a.value, b.value, c.value

    def step_profiled(self, n: int):
        avg = (C.c_double * 6)()
        cnt = (C.c_int64 * 6)()
        check(lib().sl_step_profiled(self._h, int(n), avg, cnt))
        return list(avg), list(cnt)

    def set_tuning(self, **kw) -> None:
        t = sl_tuning()
        check(lib().sl_get_tuning(self._h, C.byref(t)))
        for k, v in kw.items():
            setattr(t, k, int(v))
        check(lib().sl_set_tuning(self._h, C.byref(t)))

    def tuning(self) -> dict:
        t = sl_tuning()
        check(lib().sl_get_tuning(self._h, C.byref(t)))
        return t.to_dict()

    # uniform interface used by the autotuner
    def advance(self, n: int) -> None:
        self.step(n)


# ------------------------------------------------------------ batches

class Batch:
    """Many independent runs advancing in shared launches."""

    def __init__(self, precision: int = SL_FP32, max_runs: int = 64, mem_budget: int = 0,
                 graph_steps: int = 0, use_torch: bool = True):
        self._alloc = TorchAllocator() if use_torch else None
        d = sl_batch_desc()
        d.precision = precision
        d.max_runs = max_runs
        d.mem_budget = mem_budget
        d.graph_steps = graph_steps
        d.stream = torch_stream() if use_torch else None
        if self._alloc is not None:
            d.alloc = C.pointer(self._alloc.struct)
        h = C.c_void_p()
        check(lib().sl_batch_create(C.byref(d), C.byref(h)))
        self._h = h
        self.precision = precision
        self.specs = {}
        self.caps = {}

    def close(self):
        if getattr(self, "_h", None):
            lib().sl_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def add(self, spec: I.SystemSpec, state: I.InitialState, n_steps: int, obs_every: int = 0,
            obs_capacity: int = 4096, Te=None) -> int:
        d, keep = system_desc(spec, state, self.precision, obs_every, obs_capacity)
        t, keep2 = ttm_desc(spec, Te)
        slot = C.c_int32()
        check(lib().sl_batch_add(self._h, C.byref(d), C.byref(t), int(n_steps), C.byref(slot)))
        self.specs[slot.value] = spec
        self.caps[slot.value] = max(1, int(obs_capacity))
        return slot.value

    def try_add(self, *a, **k) -> Optional[int]:
        """Like add, but returns None when the batch is full or out of memory."""
        try:
            return self.add(*a, **k)
        except SLError as e:
            if e.code in (SL_EBUSY, SL_ENOMEM):
                return None
            raise

    def advance(self, n: int) -> None:
        check(lib().sl_batch_advance(self._h, int(n)))

    def set_tuning(self, **kw) -> None:
        t = sl_tuning()
        check(lib().sl_batch_get_tuning(self._h, C.byref(t)))
        for k, v in kw.items():
            setattr(t, k, int(v))
        check(lib().sl_batch_set_tuning(self._h, C.byref(t)))

    def tuning(self) -> dict:
        t = sl_tuning()
        check(lib().sl_batch_get_tuning(self._h, C.byref(t)))
        return t.to_dict()

    def stats(self, slot: int) -> dict:
        out = sl_run_stats()
        check(lib().sl_batch_stats(self._h, int(slot), C.byref(out)))
        return out.to_dict()

    def advance_profiled(self, n: int):
        avg = (C.c_double * 6)()
        cnt = (C.c_int64 * 6)()
        check(lib().sl_batch_advance_profiled(self._h, int(n), avg, cnt))
        return list(avg), list(cnt)

    def runs(self) -> list:
        cap = 1 << 16
        buf = (sl_run_info * cap)()
        n = C.c_int32()
        check(lib().sl_batch_runs(self._h, buf, cap, C.byref(n)))
        return [{"slot": buf[k].slot, "steps_done": buf[k].steps_done,
                 "steps_target": buf[k].steps_target} for k in range(min(cap, n.value))]

    def get(self, slot: int, max_samples: Optional[int] = None, state: bool = True) -> dict:
        """The run's samples (up to its ring capacity unless max_samples is
        given) and, with state=True, its positions, velocities, spins and
        electron grid."""
        spec = self.specs[slot]
        n = spec.n_sites
        if max_samples is None:
            max_samples = self.caps.get(slot, 1 << 16)
        x = v = s = Te = None
        if state:
            x = np.zeros((n, 3)); v = np.zeros((n, 3)); s = np.zeros((n, 3))
            Te = np.zeros(spec.n_tcells)
        buf = (sl_obs * max_samples)()
        k = C.c_int64()
        check(lib().sl_batch_get(self._h, slot, _dp(x), _dp(v), _dp(s), _dp(Te), buf,
                                 max_samples, C.byref(k)))
        out = {"obs": [obs_to_dict(buf[q]) for q in range(k.value)]}
        if state:
            out.update({"x": x, "v": v, "s": s, "Te": Te})
        return out

    def remove(self, slot: int) -> None:
        check(lib().sl_batch_remove(self._h, slot))
        self.specs.pop(slot, None)
        self.caps.pop(slot, None)

    def memory(self) -> tuple:
        u, b = C.c_size_t(), C.c_size_t()
        check(lib().sl_batch_memory(self._h, C.byref(u), C.byref(b)))
        return u.value, b.value

    def synchronize(self) -> None:
        check(lib().sl_batch_synchronize(self._h))


def footprint_bytes(spec: I.SystemSpec, precision: int = SL_FP32, obs_capacity: int = 4096) -> int:
    n = spec.n_sites
    st = I.InitialState(species=np.zeros(n, dtype=np.int8), spins=np.tile([0, 0, 1.0], (n, 1)),
                        vel=None)
    d, keep = system_desc(spec, st, precision, 1, obs_capacity)
    t, keep2 = ttm_desc(spec)
    out = C.c_size_t()
    check(lib().sl_footprint_bytes(C.byref(d), C.byref(t), C.byref(out)))
    return out.value
