"""Host-side checks of the C ABI that need no GPU: the library loads, exports
every function declared in include/colt.h, and rejects malformed input with
COLT_ERR_ARG before touching the device."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_1409_4480_amd import colt, inputs

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    with open(os.path.join(ROOT, "include", "colt.h")) as f:
        text = f.read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(colt_[a-z_]+)\s*\(", text)))


def test_library_exports_every_declared_function():
    names = declared_functions()
    assert len(names) >= 14
    L = colt.lib()
    for n in names:
        assert hasattr(L, n), n
    assert set(names) == set(colt.EXPORTS)


def _desc(grid):
    d = colt.GridDesc()
    d.kind = grid["kind"]
    d.nx, d.ny, d.nz = grid.get("shape", (0, 0, 0))
    d.box_min[:] = list(grid["box_min"])
    d.box_max[:] = list(grid["box_max"])
    d.n_cells = np.asarray(grid["n_HI"]).size
    return d


def _init(d, keep):
    h = ctypes.c_void_p()
    rc = colt.lib().colt_init_grid(ctypes.byref(d), None, None, ctypes.byref(h))
    return rc, h


def test_invalid_grids_are_rejected():
    w = inputs.static_sphere(n=4, n_photons=1)
    n = np.ascontiguousarray(w["grid"]["n_HI"])
    T = np.ascontiguousarray(w["grid"]["T"])
    dp = ctypes.POINTER(ctypes.c_double)
    cases = []
    d = _desc(w["grid"]); d.kind = 7; cases.append(d)                       # bad kind
    d = _desc(w["grid"]); cases.append(d)                                   # missing arrays
    d = _desc(w["grid"]); d.nx = 0                                          # zero dimension
    d.n_HI = n.ctypes.data_as(dp); d.T = T.ctypes.data_as(dp); cases.append(d)
    d = _desc(w["grid"]); d.n_cells = 63                                    # count mismatch
    d.n_HI = n.ctypes.data_as(dp); d.T = T.ctypes.data_as(dp); cases.append(d)
    d = _desc(w["grid"]); d.box_max[0] = 3 * d.box_max[0]                   # non-cubic cells
    d.n_HI = n.ctypes.data_as(dp); d.T = T.ctypes.data_as(dp); cases.append(d)
    d = _desc(w["grid"]); d.dust_albedo = 1.5                               # albedo out of range
    d.n_HI = n.ctypes.data_as(dp); d.T = T.ctypes.data_as(dp); cases.append(d)
    bad_T = T.copy(); bad_T[5] = -1.0                                       # negative temperature
    d = _desc(w["grid"]); d.n_HI = n.ctypes.data_as(dp); d.T = bad_T.ctypes.data_as(dp)
    cases.append(d)
    for i, d in enumerate(cases):
        rc, h = _init(d, None)
        assert rc == -1, (i, rc, colt.lib().colt_last_error())
        assert not h.value
        assert colt.lib().colt_last_error()


def test_malformed_octrees_are_rejected():
    dp = ctypes.POINTER(ctypes.c_double)
    ip = ctypes.POINTER(ctypes.c_int32)
    n = np.ones(9)
    T = np.full(9, 1e4)
    for child in ([1, -1, -1, -1, -1, -1, -1, -1, 3],    # index out of range
                  [1, 1, -1, -1, -1, -1, -1, -1, -1],    # a node reached twice / cycle
                  [2, -1, -1, -1, -1, -1, -1, -1, -1]):  # node 1 unreachable, 9 out of range
        c = np.asarray(child, np.int32)
        d = colt.GridDesc()
        d.kind = 1
        d.box_min[:] = [0, 0, 0]
        d.box_max[:] = [1, 1, 1]
        d.n_cells = 9
        d.child = c.ctypes.data_as(ip)
        d.n_HI = n.ctypes.data_as(dp)
        d.T = T.ctypes.data_as(dp)
        rc, h = _init(d, None)
        assert rc == -1, (child, rc)


def test_invalid_samplers_and_launches_are_rejected():
    L = colt.lib()
    out = np.zeros(4)
    dp = ctypes.POINTER(ctypes.c_double)
    assert L.colt_sample(9, 0, 0, 0, 0, 1, 4, out.ctypes.data_as(dp), None, None) == -1
    assert L.colt_sample(8, 0, 0, 0, 0, 1, 4, out.ctypes.data_as(dp), None, None) == -1
    # scattering draws: 0..4096 leading draws
    assert L.colt_sample(7, 1, -1.0, 0, 0, 1, 4, out.ctypes.data_as(dp), None, None) == -1
    assert L.colt_sample(7, 1, 5000.0, 0, 0, 1, 4, out.ctypes.data_as(dp), None, None) == -1
    assert L.colt_sample(2, 5, 0, 0, 0, 1, 4, out.ctypes.data_as(dp), None, None) == -1
    assert L.colt_eval_voigt(3, None, None, 4, None, None) == -1
    lc = colt.Launch(100, 0, 0, 0)                        # block not a multiple of 64
    arr = (ctypes.c_void_p * 1)(None)
    assert L.colt_transport(arr, 0, ctypes.byref(lc), None) == -1
    assert L.colt_transport(arr, 1, None, None) == -1     # null job handle
    for bad in (colt.Launch(0, 0, 0, 0, 0, 0, 65, 0),     # tail_live beyond a wave
                colt.Launch(0, 0, 0, 0, 0, 0, -1, 0),
                colt.Launch(0, 0, 0, 0, 0, 0, 0, -2),     # negative launch count
                colt.Launch(0, 0, 0, 0, 0, 64, 0, 0)):    # stop token beyond 63
        assert L.colt_transport(arr, 0, ctypes.byref(bad), None) == -1
        assert L.colt_transport_static(arr, 0, ctypes.byref(bad), None) == -1
    ok = colt.Launch(0, 0, 0, 0, 0, 0, 16, 4)             # an empty job list does nothing
    assert L.colt_transport(arr, 0, ctypes.byref(ok), None) == 0
    assert L.colt_release_grid(None) == 0
    assert L.colt_last_kernel_ms() < 0
