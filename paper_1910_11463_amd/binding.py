"""ctypes binding of the C ABI in include/pair.h (argument marshalling only).

Every function of the header is exposed under its C name (``pair_create``,
``pair_solve``, ...).  Device pointers are passed as integers (for example
``tensor.data_ptr()`` of a torch CUDA tensor) together with ``where=PAIR_DEVICE``;
host arrays as NumPy arrays with ``where=PAIR_HOST``.  The library must have been
built (``python -m paper_1910_11463_amd.build``); there is no fallback.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpair.so")

PAIR_OK, PAIR_E_INVALID, PAIR_E_HIP, PAIR_E_OOM, PAIR_E_NOCONV, PAIR_E_STATE = 0, -1, -2, -3, -4, -5
PAIR_HOST, PAIR_DEVICE = 0, 1
PAIR_TET4 = 1
PAIR_PLAIN, PAIR_BATCHED = 0, 1
PAIR_MAX_LEVELS = 32

ERROR_NAMES = {0: "PAIR_OK", -1: "PAIR_E_INVALID", -2: "PAIR_E_HIP", -3: "PAIR_E_OOM",
               -4: "PAIR_E_NOCONV", -5: "PAIR_E_STATE"}

c_int, c_int64, c_double, c_void_p = ctypes.c_int, ctypes.c_int64, ctypes.c_double, ctypes.c_void_p


class pair_options(ctypes.Structure):
    _fields_ = [("lair_distance", c_int), ("theta", c_double), ("eps_r", c_double),
                ("omega", c_double), ("coarse_max", c_int), ("max_levels", c_int),
                ("max_coarse_ratio", c_double), ("kmax", c_int), ("pmis_seed", ctypes.c_uint64),
                ("tol_inner", c_double), ("max_inner", c_int), ("tol_outer", c_double),
                ("max_outer", c_int), ("outer_estimate", c_int), ("keep_psi", c_int),
                ("keep_hierarchy", c_int), ("warm_start", c_int), ("batch_size", c_int),
                ("use_graph", c_int), ("allow_any_weight_sum", c_int),
                ("relax_pre", ctypes.c_char * 16), ("relax_post", ctypes.c_char * 16),
                ("autotune", c_int),
                ("relax_pre_coarse", ctypes.c_char * 16), ("relax_post_coarse", ctypes.c_char * 16),
                ("streams", c_int), ("coarse_fp32", c_int), ("fixed_cycles", c_int),
                ("filter_r", c_double), ("fine_factored", c_int),
                ("tile_xy", c_int), ("tile_z", c_int), ("nair_degree", c_int),
                ("tet_tile_boxes", c_int)]


class pair_stats(ctypes.Structure):
    _fields_ = [("n_dir", c_int), ("outer_iters", c_int), ("outer_rel", c_double),
                ("vcycles_total", c_int64), ("vcycles_max", c_int), ("cf_mean", c_double),
                ("relres_max", c_double), ("levels_max", c_int), ("op_complexity", c_double),
                ("level_n", c_int64 * PAIR_MAX_LEVELS), ("level_nnz", c_int64 * PAIR_MAX_LEVELS),
                ("t_assemble_ms", c_double), ("t_setup_ms", c_double), ("t_solve_ms", c_double),
                ("t_other_ms", c_double), ("bytes_solve", c_double)]

    def as_dict(self) -> dict:
        d = {}
        for name, _ in self._fields_:
            v = getattr(self, name)
            if name in ("level_n", "level_nnz"):
                v = [int(x) for x in v]
            d[name] = v
        nl = max(1, self.levels_max)
        d["level_n"] = d["level_n"][:nl]
        d["level_nnz"] = d["level_nnz"][:nl]
        return d


P = c_void_p
_SIGS = {
    "pair_abi_sizes": (c_int, [P, P]),
    "pair_default_options": (None, [P]),
    "pair_create": (c_int, [P, P, P]),
    "pair_destroy": (None, [P]),
    "pair_last_error": (ctypes.c_char_p, [P]),
    "pair_set_options": (c_int, [P, P]),
    "pair_quadrature_level_symmetric": (c_int, [c_int, P, P, P]),
    "pair_set_mesh_hex": (c_int, [P, c_int, c_int, c_int, P, P]),
    "pair_set_mesh": (c_int, [P, c_int, c_int64, P, c_int64, P]),
    "pair_set_quadrature": (c_int, [P, c_int, P, P]),
    "pair_set_materials": (c_int, [P, P, P, P, c_int]),
    "pair_set_dual_source": (c_int, [P, P, c_int, c_int]),
    "pair_set_inflow": (c_int, [P, c_int, P, c_int]),
    "pair_solve": (c_int, [P, c_int, P, P, P, c_int, P]),
    "pair_transport_sweep": (c_int, [P, c_int, P, P, P, c_int, P]),
    "pair_prepare": (c_int, [P, c_int, P]),
    "pair_clear_cache": (c_int, [P]),
    "pair_adjoint": (c_int, [P, c_int, P, P, P, P, c_int, P]),
    "pair_direction_info": (c_int, [P, c_int, P, P, P]),
    "pair_export_fine_operator": (c_int, [P, c_int, P, P, P, P, P]),
    "pair_profile_enable": (c_int, [c_int]),
    "pair_profile_read": (c_int, [c_int, P, P, P]),
    "pair_amg_create": (c_int, [P, P, P]),
    "pair_amg_destroy": (None, [P]),
    "pair_amg_last_error": (ctypes.c_char_p, [P]),
    "pair_amg_setup": (c_int, [P, c_int, P, c_int64, P, P, P, c_int]),
    "pair_amg_num_levels": (c_int, [P]),
    "pair_amg_segment_levels": (c_int, [P, c_int]),
    "pair_amg_level_sizes": (c_int, [P, c_int, P, P, P]),
    "pair_amg_get_level": (c_int, [P, c_int, P, P, P, P, P, P, P, P]),
    "pair_amg_solve": (c_int, [P, P, P, c_int, P, P]),
    "pair_amg_solve_noalloc": (c_int, [P, P, P, P, P]),
}

_lib = None


def load() -> ctypes.CDLL:
    """Load libpair.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError("libpair.so is not built: run `python -m paper_1910_11463_amd.build`")
    lib = ctypes.CDLL(LIB_PATH)
    for name, (res, args) in _SIGS.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    osz, ssz = c_int64(), c_int64()
    lib.pair_abi_sizes(ctypes.byref(osz), ctypes.byref(ssz))
    if osz.value != ctypes.sizeof(pair_options) or ssz.value != ctypes.sizeof(pair_stats):
        raise RuntimeError("pair_options/pair_stats layout mismatch between library and binding")
    _lib = lib
    return lib


def _ptr(x):
    """Pointer argument: None, int (device address), NumPy array, torch tensor,
    a ctypes scalar such as a c_void_p handle (its value), a ctypes structure or
    array (its address) or a ctypes.byref() result (unchanged)."""
    if x is None or isinstance(x, (int, float)):
        return x
    if isinstance(x, np.ndarray):
        if not x.flags["C_CONTIGUOUS"]:
            raise ValueError("arrays passed to the library must be C-contiguous")
        return x.ctypes.data
    if hasattr(x, "data_ptr"):
        return x.data_ptr()
    if isinstance(x, ctypes._SimpleCData):
        return x.value          # e.g. a c_void_p handle: pass the pointer it holds
    if isinstance(x, (ctypes.Structure, ctypes.Array)):
        return ctypes.addressof(x)
    return x


class PairError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("%s: %s" % (ERROR_NAMES.get(code, code), msg))
        self.code = code


def check(code: int, handle=None, amg: bool = False):
    if code != PAIR_OK:
        lib = load()
        if handle is None:
            msg = ""
        else:
            msg = (lib.pair_amg_last_error if amg else lib.pair_last_error)(handle)
            msg = msg.decode() if msg else ""
        raise PairError(code, msg)
    return code


def _wrap(name):
    def f(*args):
        lib = load()
        return getattr(lib, name)(*[_ptr(a) for a in args])
    f.__name__ = name
    f.__doc__ = "C function %s from include/pair.h" % name
    return f


# Plain pass-through functions with the C names.
for _n in _SIGS:
    globals()[_n] = _wrap(_n)


def default_options(**overrides) -> pair_options:
    o = pair_options()
    load().pair_default_options(ctypes.byref(o))
    for k, v in overrides.items():
        if not hasattr(o, k):
            raise KeyError(k)
        if k.startswith("relax_") and isinstance(v, str):
            v = v.encode()
        setattr(o, k, v)
    return o
