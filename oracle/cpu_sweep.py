"""Python side of the compiled structured-hex sweep (oracle; test
infrastructure and the timed CPU baseline only).

``build()`` compiles ``cpu_sweep.c`` with gcc and OpenMP into
``oracle/_cpu_sweep.so``; ``sweep_all`` solves every direction's upwind DG
system exactly (Sec. "Solution of the Transport Equation by Sweeping") with the
closed-form Q1 element matrices, one direction per OpenMP thread at a time,
and forms phi = sum_m w_m psi_m (eq. angular_quad).

Pinned by the NumPy oracle (``dg.assemble`` + ``sweep``) to 1e-13 on
anisotropic meshes, random cross sections, a non-zero scattering source and
directions with zero components (tests/test_oracle_cpu_sweep.py).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "cpu_sweep.c")
_LIB = os.path.join(_HERE, "_cpu_sweep.so")
_lib = None
# x86-64-v3 (AVX2 + FMA): built here, run on the GPU host as well
CFLAGS = ["-O3", "-std=c99", "-march=x86-64-v3", "-fopenmp", "-shared", "-fPIC"]


def build(force: bool = False) -> str:
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc"] + CFLAGS + ["-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        build()
        lib = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        lib.cpu_sweep_hex.restype = ctypes.c_int
        lib.cpu_sweep_hex.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, P, P, P, P, P,
                                      ctypes.c_int, P, P, P, P, ctypes.c_int]
        lib.cpu_sweep_max_threads.restype = ctypes.c_int
        _lib = lib
    return _lib


def max_threads() -> int:
    return int(_load().cpu_sweep_max_threads())


def sweep_all(mesh, sigma_t, sigma_s, q, omega, w, phi=None, threads: int = 0, psi=None):
    """(psi [M,N], phi_out [N]) of one sweep over all directions of a
    structured hex workloads.Mesh.  psi may be passed in to reuse memory."""
    assert mesh.kind == 0, "structured hex meshes only"
    lib = _load()
    nx, ny, nz = mesh.nx, mesh.ny, mesh.nz
    h = np.array([(mesh.hi[d] - mesh.lo[d]) / n for d, n in enumerate((nx, ny, nz))])
    f64 = lambda a: np.ascontiguousarray(a, dtype=np.float64)
    st, ss, qq = f64(sigma_t), f64(sigma_s), f64(q)
    om, ww = f64(omega), f64(w)
    M, N = om.shape[0], 8 * nx * ny * nz
    if psi is None:
        psi = np.empty((M, N))
    out = np.empty(N)
    ph = None if phi is None else f64(phi)
    rc = lib.cpu_sweep_hex(nx, ny, nz, h.ctypes.data, st.ctypes.data, ss.ctypes.data, qq.ctypes.data,
                           None if ph is None else ph.ctypes.data, M, om.ctypes.data, ww.ctypes.data,
                           psi.ctypes.data, out.ctypes.data, int(threads))
    if rc != 0:
        raise RuntimeError("cpu sweep: singular element block")
    return psi, out
