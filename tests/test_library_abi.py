"""CPU checks of the C ABI library and its host-side logic (no GPU needed).

* the shared library loads and exports every entry point the header
  declares;
* the ctypes mirrors have the C layout (sizes and offsets from gcc);
* the integer logic of the device header (division by run-time constants,
  site numbering, Philox) compiled for the host agrees with brute force
  and with the oracle's independent Philox.
"""
import ctypes as C
import os
import re
import shutil
import subprocess
import tempfile

import numpy as np
import pytest

from paper_2608_18541_amd import build as B

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "spinlattice.h")


@pytest.fixture(scope="module")
def libpath():
    if not os.path.exists(B.LIB):
        B.build(force=True)
    return B.LIB


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"\b(sl_[a-z_0-9]+)\s*\(", text)
    return sorted(set(n for n in names if not n.startswith("sl_allocator")))


def test_library_exports_every_declared_symbol(libpath):
    lib = C.CDLL(libpath)
    names = declared_functions()
    assert len(names) >= 20
    for n in names:
        assert hasattr(lib, n), n
    from paper_2608_18541_amd import native
    assert set(names) == set(native.EXPORTS), set(names) ^ set(native.EXPORTS)


def test_binding_loads_without_gpu(libpath):
    from paper_2608_18541_amd import native
    L = native.lib()
    assert L.sl_last_error() == b""
    # a call that needs no device: invalid arguments are rejected cleanly
    d = native.sl_system_desc()
    out = C.c_size_t()
    assert L.sl_footprint_bytes(C.byref(d), None, C.byref(out)) == native.SL_EINVAL
    assert b"lattice" in L.sl_last_error() or b"ncell" in L.sl_last_error()


LAYOUT_PROBE = r"""
#include <stdio.h>
#include <stddef.h>
#include "spinlattice.h"
#define P(T, f) printf("%s %s %zu\n", #T, #f, offsetof(T, f));
int main(void) {
  printf("sl_system_desc size %zu\n", sizeof(sl_system_desc));
  P(sl_system_desc, a) P(sl_system_desc, species) P(sl_system_desc, J) P(sl_system_desc, B)
  P(sl_system_desc, dt) P(sl_system_desc, seed) P(sl_system_desc, spin0) P(sl_system_desc, alloc)
  P(sl_system_desc, exch_radial) P(sl_system_desc, exch_r)
  printf("sl_ttm_desc size %zu\n", sizeof(sl_ttm_desc));
  P(sl_ttm_desc, Te_init) P(sl_ttm_desc, n_sub) P(sl_ttm_desc, depth)
  printf("sl_obs size %zu\n", sizeof(sl_obs));
  P(sl_obs, M) P(sl_obs, Tspin) P(sl_obs, Tl)
  printf("sl_batch_desc size %zu\n", sizeof(sl_batch_desc));
  P(sl_batch_desc, mem_budget) P(sl_batch_desc, alloc)
  printf("sl_tuning size %zu\n", sizeof(sl_tuning));
  P(sl_tuning, graph_steps) P(sl_tuning, persist_block) P(sl_tuning, xcd_order) P(sl_tuning, bin_mode) P(sl_tuning, atom_lanes) P(sl_tuning, merge_sweeps) P(sl_tuning, spin_access)
  P(sl_tuning, fuse_force)
  printf("sl_run_stats size %zu\n", sizeof(sl_run_stats));
  P(sl_run_stats, list_rebuilds) P(sl_run_stats, max_list) P(sl_run_stats, list_capacity)
  P(sl_run_stats, list_rescans) P(sl_run_stats, error)
  printf("sl_run_info size %zu\n", sizeof(sl_run_info));
  P(sl_run_info, steps_done) P(sl_run_info, n_samples)
  return 0;
}
"""


def test_ctypes_layout_matches_c():
    from paper_2608_18541_amd import native as N
    with tempfile.TemporaryDirectory() as td:
        src = os.path.join(td, "l.c")
        exe = os.path.join(td, "l")
        open(src, "w").write(LAYOUT_PROBE)
        subprocess.check_call(["gcc", "-std=c11", "-I", os.path.dirname(HEADER), src, "-o", exe])
        out = subprocess.run([exe], capture_output=True, text=True, check=True).stdout
    types = {"sl_system_desc": N.sl_system_desc, "sl_ttm_desc": N.sl_ttm_desc,
             "sl_obs": N.sl_obs, "sl_batch_desc": N.sl_batch_desc,
             "sl_run_info": N.sl_run_info, "sl_tuning": N.sl_tuning,
             "sl_run_stats": N.sl_run_stats}
    for line in out.strip().splitlines():
        t, f, v = line.split()
        if f == "size":
            assert C.sizeof(types[t]) == int(v), line
        else:
            assert getattr(types[t], f).offset == int(v), line


HOST_PROBE = r"""
#include "sl_device.hpp"
#include <cstdio>
#include <cstdlib>
int main() {
  // division by invariant integers: all divisors up to 4096 on a sweep of n
  for (uint32_t d = 1; d <= 4096; ++d) {
    sl::FastDiv f = sl::make_fastdiv(d);
    for (uint32_t n = 0; n < (1u << 31); n = n < 70000 ? n + 1 : n * 3 + 7) {
      if (sl::fdiv(n, f) != n / d) { printf("FAIL div %u %u\n", n, d); return 1; }
    }
    uint32_t top = (1u << 31) - 1;
    if (sl::fdiv(top, f) != top / d) { printf("FAIL div top %u\n", d); return 1; }
  }
  // site numbering: internal <-> (x, y, z, b) is a bijection and colours are proper
  int dims[][4] = {{2, 2, 2, 1}, {4, 6, 2, 1}, {6, 6, 6, 2}, {8, 4, 10, 2}, {2, 2, 2, 2},
                   {2, 2, 2, 4}, {3, 5, 4, 4}, {13, 13, 13, 4}};
  for (auto& dm : dims) {
    sl::Geom g;
    g.Lx = dm[0]; g.Ly = dm[1]; g.Lz = dm[2]; g.nb = dm[3];
    g.par = g.nb == 4 ? 0 : 1;
    g.Lxh = g.par ? g.Lx / 2 : g.Lx;
    g.H = g.par ? g.Lx * g.Ly * g.Lz / 2 : g.Lx * g.Ly * g.Lz;
    g.C = g.nb == 4 ? 4 : 2 * g.nb;
    g.divH = sl::make_fastdiv(g.H); g.divLxh = sl::make_fastdiv(g.Lxh);
    g.divLy = sl::make_fastdiv(g.Ly);
    int n = g.nb * g.Lx * g.Ly * g.Lz;
    char* seen = (char*)calloc(n, 1);
    for (int i = 0; i < n; ++i) {
      sl::Site s = sl::decode_site(g, i);
      if (sl::encode_site(g, s.x, s.y, s.z, s.b) != i) { printf("FAIL enc %d\n", i); return 1; }
      int c = sl::canonical_of(g, s);
      if (c < 0 || c >= n || seen[c]) { printf("FAIL canon %d\n", i); return 1; }
      seen[c] = 1;
      int par = (s.x + s.y + s.z) & 1;
      int want = g.nb == 4 ? s.b : (g.nb == 2 ? 2 * s.b + par : par);
      if (s.k != want || s.x >= g.Lx || s.y >= g.Ly || s.z >= g.Lz) { printf("FAIL colour %d\n", i); return 1; }
    }
    free(seen);
  }
  // launch tables: the closed-form entries of a single run's tables equal the
  // explicit deal of the tiles over the 8 XCDs (the order the multi-run
  // tables are built in), natural order below 16 tiles
  for (int m = 1; m < 3000; m += (m < 200 ? 1 : 7)) {
    sl::TableFill f{};
    f.m[2] = m; f.tile[2] = 3; f.xcd[2] = 1;
    int* deal = (int*)malloc(sizeof(int) * m);
    int k = 0;
    if (m < 16) {
      for (int q = 0; q < m; ++q) deal[k++] = q;
    } else {
      int per = (m + 7) / 8;
      for (int j = 0; j < per; ++j)
        for (int x = 0; x < 8; ++x)
          if (x * per + j < m) deal[k++] = x * per + j;
    }
    if (k != m) { printf("FAIL deal count %d\n", m); return 1; }
    for (int q = 0; q < m; ++q) {
      int2 e = sl::fill_entry(f, 2, q, 5);
      if (e.x != 5 || e.y != 3 * deal[q]) { printf("FAIL table %d %d\n", m, q); return 1; }
    }
    f.xcd[2] = 0;
    for (int q = 0; q < m; ++q)
      if (sl::fill_entry(f, 2, q, 5).y != 3 * q) { printf("FAIL natural %d\n", m); return 1; }
    free(deal);
  }
  // Philox words for a few counters (compared with the oracle by the test)
  unsigned v[6];
  while (scanf("%u %u %u %u %u %u", &v[0], &v[1], &v[2], &v[3], &v[4], &v[5]) == 6) {
    sl::U4 c{v[0], v[1], v[2], v[3]};
    sl::U4 r = sl::philox4x32_10(c, v[4], v[5]);
    printf("%u %u %u %u\n", r.x, r.y, r.z, r.w);
  }
  printf("OK\n");
  return 0;
}
"""


def test_device_integer_logic_on_host():
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available")
    from oracle import oracle as O
    rng = np.random.default_rng(3)
    cases = [tuple(int(x) for x in rng.integers(0, 2**32, size=6, dtype=np.uint64))
             for _ in range(50)]
    with tempfile.TemporaryDirectory() as td:
        src = os.path.join(td, "h.cpp")
        exe = os.path.join(td, "h")
        open(src, "w").write(HOST_PROBE)
        subprocess.check_call([hipcc, "-O1", "-std=c++17", "-I", os.path.join(B.PKG, "csrc"),
                               src, "-o", exe], stdout=subprocess.DEVNULL,
                              stderr=subprocess.DEVNULL)
        inp = "\n".join(" ".join(map(str, c)) for c in cases) + "\n"
        out = subprocess.run([exe], input=inp, capture_output=True, text=True).stdout
    lines = out.strip().splitlines()
    assert lines[-1] == "OK", lines[-3:]
    for c, line in zip(cases, lines[:-1]):
        assert list(map(int, line.split())) == list(O.philox(c[:4], c[4:])), c


def test_footprint_and_site_limit(libpath):
    """Host-only calls: the HBM footprint grows with the site count and is
    smaller in FP32; runs of 2^27 sites or more are rejected before any
    array is read (per-atom arrays use 32-bit byte offsets)."""
    from paper_2608_18541_amd import inputs as I
    from paper_2608_18541_amd import native
    L = native.lib()
    sizes = {}
    for Lc in (8, 16):
        spec = I.gdfeco_sc_spec(L=Lc, tn=2)
        st = I.initial_state(spec, "afm")
        for prec in (native.SL_FP64, native.SL_FP32):
            d, keep = native.system_desc(spec, st, prec)
            t, keep2 = native.ttm_desc(spec)
            out = C.c_size_t()
            assert L.sl_footprint_bytes(C.byref(d), C.byref(t), C.byref(out)) == native.SL_OK
            sizes[(Lc, prec)] = out.value
    for prec in (native.SL_FP64, native.SL_FP32):
        ratio = sizes[(16, prec)] / sizes[(8, prec)]
        assert 7.0 < ratio < 8.5, ratio                # per-site arrays dominate
    # FP32 halves the 15 real per-atom arrays (spins, displacements,
    # velocities, forces, reference displacements), the padded position
    # vector and the three electron-phonon normals drawn per atom:
    # 15 x 4 + 16 + 3 x 4 bytes per atom less; lists, bins, ids and samples
    # keep their size
    for Lc in (8, 16):
        n = Lc ** 3
        assert sizes[(Lc, native.SL_FP64)] - sizes[(Lc, native.SL_FP32)] == (15 * 4 + 16 + 12) * n
    # 2^27 sites: bcc 512 x 512 x 256 cells, with the small run's arrays
    spec = I.gdfeco_sc_spec(L=8, tn=2)
    st = I.initial_state(spec, "afm")
    d, keep = native.system_desc(spec, st, native.SL_FP32)
    t, keep2 = native.ttm_desc(spec)
    d.lattice = 1
    d.ncell = (C.c_int32 * 3)(512, 512, 256)
    out = C.c_size_t()
    assert L.sl_footprint_bytes(C.byref(d), C.byref(t), C.byref(out)) == native.SL_EINVAL
    assert b"too many sites" in L.sl_last_error()
