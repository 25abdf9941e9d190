"""CPU checks of the C ABI library: it loads, exports every function that
include/pair.h declares, its struct layouts match the binding, host-only entry
points work, and null handles are rejected (no GPU work is started here)."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_1910_11463_amd import binding as B

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    txt = open(os.path.join(ROOT, "include", "pair.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(pair_[a-z0-9_]+)\s*\(", txt)))


def test_library_exports_every_declared_symbol():
    lib = B.load()
    names = _declared()
    assert len(names) >= 25
    for n in names:
        assert hasattr(lib, n), n
        assert n in B._SIGS, "binding lacks " + n


def test_struct_layout_matches():
    lib = B.load()
    o, s = ctypes.c_int64(), ctypes.c_int64()
    assert lib.pair_abi_sizes(ctypes.byref(o), ctypes.byref(s)) == 0
    assert o.value == ctypes.sizeof(B.pair_options)
    assert s.value == ctypes.sizeof(B.pair_stats)


def test_default_options():
    o = B.default_options()
    assert (o.lair_distance, o.theta, o.eps_r, o.omega) == (1, 0.25, 0.01, 1.0)
    assert (o.coarse_max, o.max_levels, o.kmax) == (64, 25, 64)
    assert o.tol_inner == 1e-8 and o.max_inner == 100
    assert o.streams == 1 and o.coarse_fp32 == 0 and o.fine_factored == 1
    assert o.tile_xy == 8 and o.tile_z == 0 and o.nair_degree == 0


def test_quadrature_matches_oracle():
    from oracle import quadrature as Q
    for order, M in ((2, 8), (4, 24), (8, 80)):
        m = ctypes.c_int()
        assert B.pair_quadrature_level_symmetric(order, ctypes.byref(m), None, None) == 0
        assert m.value == M
        om, w = np.zeros((M, 3)), np.zeros(M)
        assert B.pair_quadrature_level_symmetric(order, None, om, w) == 0
        o2, w2 = Q.level_symmetric(order)
        assert np.abs(om - o2).max() <= 1e-15
        assert np.abs(w - w2).max() <= 1e-14
    assert B.pair_quadrature_level_symmetric(6, None, None, None) == B.PAIR_E_INVALID


def test_null_handles_rejected():
    assert B.pair_set_mesh_hex(None, 2, 2, 2, None, None) == B.PAIR_E_INVALID
    assert B.pair_solve(None, 0, None, None, None, 0, None) == B.PAIR_E_INVALID
    assert B.pair_amg_solve(None, None, None, 0, None, None) == B.PAIR_E_INVALID
    assert B.pair_amg_num_levels(None) == 0


def test_pointer_marshalling():
    h = ctypes.c_void_p(12345)
    assert B._ptr(h) == 12345
    assert B._ptr(None) is None
    a = np.zeros(3)
    assert B._ptr(a) == a.ctypes.data
    with pytest.raises(ValueError):
        B._ptr(np.zeros((3, 3))[:, 0])
