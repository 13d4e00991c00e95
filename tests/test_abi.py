"""The C-ABI library loads and exports every symbol include/acom.h declares, and
host-checkable argument errors come back as status codes (no GPU needed: these
calls return before any HIP work)."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "acom.h")
LIB = os.path.join(ROOT, "paper_2111_00171_amd", "libacom.so")


def declared_symbols():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(acom_[a-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        from paper_2111_00171_amd import build
        build.build()
    return ctypes.CDLL(LIB)


def test_header_declares_the_paths_entry_points():
    syms = declared_symbols()
    for s in ("acom_build_plan", "acom_match", "acom_refine", "acom_score", "acom_score_grad"):
        assert s in syms


def test_every_declared_symbol_is_exported(lib):
    for s in declared_symbols():
        assert hasattr(lib, s), s


def test_invalid_arguments_return_status_codes():
    from paper_2111_00171_amd import acom
    L = acom.lib()
    prm = acom._Params()
    prm.k_max = 1.2
    prm.delta = 0.08
    prm.gamma = prm.omega = 1.0
    prm.accel_kV = 300.0
    prm.zone_step_deg = 5.0
    prm.n_radial = 32
    prm.n_angular = 90
    h = ctypes.c_void_p()
    ph = (acom._Phase * 1)()
    frac = (ctypes.c_double * 3)(0, 0, 0)
    ph[0].n_atoms = 1
    ph[0].frac_xyz = ctypes.cast(frac, ctypes.POINTER(ctypes.c_double))
    ph[0].n_triangles = 1
    # odd angular length
    prm.n_angular = 91
    assert L.acom_build_plan(ph, 1, ctypes.byref(prm), None, ctypes.byref(h)) == 1
    assert b"n_angular" in L.acom_last_error()
    # prime factor 7
    prm.n_angular = 14
    assert L.acom_build_plan(ph, 1, ctypes.byref(prm), None, ctypes.byref(h)) == 1
    prm.n_angular = 90
    prm.k_max = -1.0
    assert L.acom_build_plan(ph, 1, ctypes.byref(prm), None, ctypes.byref(h)) == 1
    prm.k_max = 1.2
    assert L.acom_build_plan(ph, 0, ctypes.byref(prm), None, ctypes.byref(h)) == 1
    assert L.acom_build_plan(None, 1, ctypes.byref(prm), None, ctypes.byref(h)) == 1
    assert L.acom_build_plan(ph, 1, ctypes.byref(prm), None, None) == 1
    # null plan handles
    assert L.acom_match(None, None, 1, 0, 0, None, 0, None, None) == 1
    assert L.acom_refine(None, None, 1, None, None, 10, None, None, None, None, None) == 1
    assert L.acom_score(None, None, None, None, None, None, None) == 1
    assert L.acom_match_noalloc(None, None, 1, 0, None, None) == 1
    assert L.acom_plan_bound_split(None, 0, None, None) == 1
    assert L.acom_plan_destroy(None) == 0
    assert L.acom_status_string(5) == b"workspace too small"


@pytest.mark.parametrize("axis,tmax,step,phis", [([0, 0, 1], 10.0, 2.0, (0, 360)), ([1, 1, 1], 15.0, 1.0, (0, 60)),
                                                  ([0.3, -1, 2], 5.0, 0.5, (10, 370))])
def test_fiber_zones_host_call_matches_oracle(axis, tmax, step, phis):
    """acom_fiber_zones is a host-only call (no GPU): its zone list equals the
    oracle's fiber grid direction by direction (the same reading, written twice)."""
    from paper_2111_00171_amd import acom
    from oracle import zones
    w = acom.fiber_zones(axis, tmax, step, phis)
    o = zones.fiber_grid(axis, tmax, step, *phis)
    assert w.shape == o.shape
    np.testing.assert_allclose(w, o, atol=1e-12)
