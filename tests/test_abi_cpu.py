"""C-ABI checks that need no GPU: the library loads, exports every function
include/acs.h declares, its structs have the layout the binding assumes, and
invalid calls fail with the documented codes and a message (no compute)."""
from __future__ import annotations

import ctypes as C
import os
import re
import subprocess
import tempfile

import numpy as np
import pytest

from paper_1605_02669_amd import acs, inputs

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "acs.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:int|void|const char \*)\s*\**\s*(acs_\w+)\s*\(", text, flags=re.M)
    return sorted(set(names))


def test_header_declares_the_boundary():
    names = declared_functions()
    for must in ("acs_create", "acs_iterate", "acs_best_tour", "acs_pheromone_snapshot",
                 "acs_spm_snapshot", "acs_stats", "acs_destroy", "acs_last_error"):
        assert must in names


def test_library_exports_every_declared_symbol():
    lib = acs.load()
    for name in declared_functions():
        assert hasattr(lib, name), name
    out = subprocess.run(["nm", "-D", "--defined-only", acs.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    exported = set(re.findall(r" T (acs_\w+)", out))
    assert set(declared_functions()) <= exported


def test_struct_layout_matches_c():
    src = r'''
#include <stdio.h>
#include <stddef.h>
#include "acs.h"
int main(void) {
  printf("%zu %zu %zu %zu %zu %zu\n", sizeof(acs_params), offsetof(acs_params, beta),
         offsetof(acs_params, stream), sizeof(acs_stats_t),
         offsetof(acs_stats_t, construct_ms), offsetof(acs_stats_t, iterate_ms));
  return 0;
}
'''
    d = tempfile.mkdtemp()
    c = os.path.join(d, "layout.c")
    exe = os.path.join(d, "layout")
    open(c, "w").write(src)
    subprocess.run(["gcc", "-std=c11", "-I", os.path.join(ROOT, "include"), c, "-o", exe], check=True)
    vals = [int(x) for x in subprocess.run([exe], capture_output=True, text=True, check=True).stdout.split()]
    assert vals == [C.sizeof(acs.acs_params), acs.acs_params.beta.offset, acs.acs_params.stream.offset,
                    C.sizeof(acs.acs_stats_t), acs.acs_stats_t.construct_ms.offset,
                    acs.acs_stats_t.iterate_ms.offset]


def _create_rc(xy, **kw):
    lib = acs.load()
    p = acs.acs_default_params()
    for k, v in kw.items():
        setattr(p, k, v)
    xy = np.ascontiguousarray(xy, dtype=np.float64)
    h = C.c_void_p()
    rc = lib.acs_create(xy.ctypes.data_as(C.c_void_p), xy.shape[0], C.byref(p), C.byref(h))
    return rc, lib.acs_last_error().decode(), h


def test_default_params():
    p = acs.acs_default_params()
    assert p.struct_size == C.sizeof(acs.acs_params)
    assert (p.cl, p.beta, p.q0, p.phi, p.rho, p.spm_s) == (32, 2.0, 0.9, 0.1, 0.1, 8)


@pytest.mark.parametrize("kw,n,code,needle", [
    ({}, 2, acs.ACS_E_INVALID, "n = 2"),
    ({"q0": 1.5}, 10, acs.ACS_E_INVALID, "q0"),
    ({"phi": 0.0}, 10, acs.ACS_E_INVALID, "phi"),
    ({"rho": 1.0}, 10, acs.ACS_E_INVALID, "rho"),
    ({"beta": -1.0}, 10, acs.ACS_E_INVALID, "beta"),
    ({"mode": 7}, 10, acs.ACS_E_INVALID, "mode"),
    ({"memory": 3}, 10, acs.ACS_E_INVALID, "memory"),
    ({"struct_size": 8}, 10, acs.ACS_E_INVALID, "struct_size"),
    ({"cl": 0}, 10, acs.ACS_E_INVALID, "cl"),
    ({"cl": 100}, 200, acs.ACS_E_UNSUPPORTED, "cl = 100"),
    ({"local_update_period": 0}, 10, acs.ACS_E_INVALID, "period"),
    ({"mode": acs.ACS_SEQUENTIAL, "memory": acs.ACS_SPM}, 10, acs.ACS_E_UNSUPPORTED,
     "sequential mode needs dense"),
    ({"mode": acs.ACS_SEQUENTIAL, "lanes_per_ant": 32}, 10, acs.ACS_E_UNSUPPORTED,
     "asynchronous mode"),
])
def test_invalid_parameters_rejected_before_any_device_work(kw, n, code, needle):
    rc, msg, h = _create_rc(inputs.uniform(max(n, 3))[:n], **kw)
    assert rc == code and needle in msg and not h.value


def test_non_finite_coordinates_rejected():
    xy = inputs.uniform(20)
    xy[4, 1] = np.inf
    rc, msg, _ = _create_rc(xy)
    assert rc == acs.ACS_E_INVALID and "not finite" in msg


def test_calls_on_null_handle():
    lib = acs.load()
    assert lib.acs_iterate(None, 1) == acs.ACS_E_STATE
    assert "invalid handle" in lib.acs_last_error().decode()
    L = C.c_int64()
    assert lib.acs_best_tour(None, None, C.byref(L)) == acs.ACS_E_STATE
    assert lib.acs_pheromone_snapshot(None, None, 0) == acs.ACS_E_STATE
    s = acs.acs_stats_t()
    s.struct_size = C.sizeof(acs.acs_stats_t)
    assert lib.acs_stats(None, C.byref(s)) == acs.ACS_E_STATE
    lib.acs_destroy(None)  # no-op


def test_workspace_size_grows_with_instance():
    p = acs.acs_default_params()
    a = acs.acs_workspace_bytes(100, p)
    b = acs.acs_workspace_bytes(2392, p)
    assert 0 < a < b
    # dense pheromone + distances dominate: at least n*n*(4+2) bytes
    assert b >= 2392 * 2392 * 6


def test_mode_specific_workspace():
    p = acs.acs_default_params()
    p.mode = acs.ACS_ASYNC_ATOMIC
    base = acs.acs_workspace_bytes(1000, p)
    p.mode = acs.ACS_SEQUENTIAL
    seq = acs.acs_workspace_bytes(1000, p)
    p.mode = acs.ACS_SYNC
    sync = acs.acs_workspace_bytes(1000, p)
    # sequential: m = n = 1000 visited bitmaps of ceil(1000 / 32) words
    assert seq - base == (1000 * 32 * 4 + 255) // 256 * 256
    # synchronous: the second buffer of the dense matrix (ldn = 1024) and the
    # barrier flags (one 128-byte line per block of 16 ants after a first,
    # unused one), each 256-byte aligned
    flags = 8 * 16 * ((1000 + 15) // 16 + 1)
    assert sync - base == 1000 * 1024 * 4 + (flags + 255) // 256 * 256


def test_fallback_prefix_workspace():
    """The dense fallback's prefix (128 cities after the cl candidates, 8 bytes
    each, plus three per-city words) exists only where n - 1 > cl + 128: at
    n = 190 for cl = 32 but not for cl = 64."""
    def al(x):
        return (x + 255) // 256 * 256

    n = 190
    p = acs.acs_default_params()
    p.mode = acs.ACS_ASYNC_ATOMIC
    sizes = {}
    for cl in (32, 64):
        p.cl = cl
        sizes[cl] = acs.acs_workspace_bytes(n, p)
    # per-candidate arrays: record (16 B), index (4 B), reverse position
    # (1 B), live pheromone (4 B)
    def per_cand(cl):
        return al(16 * n * cl) + al(4 * n * cl) + al(n * cl) + al(4 * n * cl)
    prefix = al(8 * n * 128) + 3 * al(4 * n)
    assert sizes[64] - sizes[32] == per_cand(64) - per_cand(32) - prefix


def test_without_gpu_create_reports_device_error():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    rc, msg, _ = _create_rc(inputs.uniform(50))
    assert rc == acs.ACS_E_DEVICE and "device" in msg


def test_static_entry_rejects_what_it_cannot_hold():
    """acs_solve_static checks its arguments and the static workspace's size
    before it touches a device (no compute here)."""
    lib = acs.load()
    xy = inputs.uniform(4000)
    t = np.empty(4000, dtype=np.int32)
    L = C.c_int64()
    p = acs.make_params(mode=acs.ACS_SYNC)
    need = acs.acs_workspace_bytes(4000, p)
    assert need > 128 << 20
    rc = lib.acs_solve_static(xy.ctypes.data_as(C.c_void_p), 4000, C.byref(p), 1,
                              t.ctypes.data_as(C.c_void_p), C.byref(L))
    assert rc == acs.ACS_E_BUFSIZE
    assert "static workspace" in lib.acs_last_error().decode()
    p.workspace, p.workspace_bytes = 4096, need
    rc = lib.acs_solve_static(xy.ctypes.data_as(C.c_void_p), 4000, C.byref(p), 1,
                              t.ctypes.data_as(C.c_void_p), C.byref(L))
    assert rc == acs.ACS_E_INVALID
    p = acs.make_params(mode=acs.ACS_SYNC, q0=2.0)
    rc = lib.acs_solve_static(xy.ctypes.data_as(C.c_void_p), 100, C.byref(p), 1,
                              t.ctypes.data_as(C.c_void_p), C.byref(L))
    assert rc == acs.ACS_E_INVALID
