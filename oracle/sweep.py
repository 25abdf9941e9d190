"""Python side of the exact sweep (oracle; test infrastructure only).

``build()`` compiles ``sweep.c`` with the host C compiler into
``oracle/_sweep.so``; ``sweep(blocks, rhs)`` solves one direction's block system
exactly (Sec. "Solution of the Transport Equation by Sweeping").  Pinned by the
dense LU of the same block matrix on tiny meshes, including a system whose
dependency graph has cycles (tests/test_oracle_dg.py).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "sweep.c")
_LIB = os.path.join(_HERE, "_sweep.so")
_lib = None


def build(force: bool = False) -> str:
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-shared", "-fPIC", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        build()
        lib = ctypes.CDLL(_LIB)
        lib.oracle_sweep.restype = ctypes.c_int
        lib.oracle_sweep.argtypes = [ctypes.c_int64, ctypes.c_int, ctypes.c_int,
                                     ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                     ctypes.c_void_p, ctypes.c_void_p]
        _lib = lib
    return _lib


def sweep_raw(D: np.ndarray, nbr: np.ndarray, Cpl: np.ndarray, rhs: np.ndarray):
    """Solve D_e psi_e + sum_f Cpl[e,f] psi_nbr[e,f] = rhs_e exactly.
    Returns (psi [E,k], number of multi-element cycles)."""
    lib = _load()
    E, k = rhs.shape[0], rhs.shape[1]
    F = nbr.shape[1]
    D = np.ascontiguousarray(D, dtype=np.float64)
    nbr = np.ascontiguousarray(nbr, dtype=np.int64)
    Cpl = np.ascontiguousarray(Cpl, dtype=np.float64)
    rhs = np.ascontiguousarray(rhs, dtype=np.float64)
    psi = np.zeros((E, k))
    rc = lib.oracle_sweep(E, k, F, D.ctypes.data, nbr.ctypes.data, Cpl.ctypes.data,
                          rhs.ctypes.data, psi.ctypes.data)
    if rc < 0:
        raise RuntimeError("oracle sweep: singular block")
    return psi, rc


def sweep(blocks, rhs: np.ndarray) -> np.ndarray:
    psi, _ = sweep_raw(blocks.D, blocks.nbr, blocks.Cpl, rhs)
    return psi
