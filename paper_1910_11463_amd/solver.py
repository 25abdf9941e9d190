"""Python conveniences over the C ABI: Solver (S_N transport), Amg (generic AIR)
and TransportSolve (torch.autograd.Function: phi(sigma_t, sigma_s) with the
adjoint in backward).  Marshalling only: all computation runs in libpair.so.

Device memory and the HIP stream come from PyTorch (ROCm build): tensors are
passed by ``data_ptr()`` with ``where=PAIR_DEVICE``; the context's stream is
``torch.cuda.current_stream().cuda_stream`` at creation time.
"""
from __future__ import annotations

import ctypes
from typing import Optional

import numpy as np

from . import binding as B


def _torch():
    import torch
    return torch


def _is_tensor(x):
    return hasattr(x, "data_ptr") and hasattr(x, "is_cuda")


def _where(x):
    return B.PAIR_DEVICE if _is_tensor(x) and x.is_cuda else B.PAIR_HOST


def _f64(x):
    if _is_tensor(x):
        torch = _torch()
        return x.detach().to(torch.float64).contiguous()
    return np.ascontiguousarray(x, dtype=np.float64)


class Solver:
    """One pAIR transport context (see include/pair.h for every call)."""

    def __init__(self, options: Optional[B.pair_options] = None, stream: Optional[int] = None,
                 **overrides):
        B.load()
        self.opt = options if options is not None else B.default_options(**overrides)
        if options is not None:
            for k, v in overrides.items():
                if k.startswith("relax_") and isinstance(v, str):
                    v = v.encode()
                setattr(self.opt, k, v)
        if stream is None:
            try:
                torch = _torch()
                stream = torch.cuda.current_stream().cuda_stream if torch.cuda.is_available() else None
            except Exception:
                stream = None
        h = ctypes.c_void_p()
        B.check(B.pair_create(ctypes.byref(h), ctypes.byref(self.opt), stream))
        self.h = h
        self.M = 0
        self.N = 0
        self.E = 0
        # incremented by every call that changes the problem or the solution
        # the adjoint would read (TransportSolve checks it in backward)
        self.state = 0

    def close(self):
        if getattr(self, "h", None) is not None and self.h.value:
            B.pair_destroy(self.h)
            self.h = None

    __del__ = close

    def _chk(self, rc, allow_noconv=False):
        if rc == B.PAIR_E_NOCONV and allow_noconv:
            return rc
        return B.check(rc, self.h)

    # ---------------------------------------------------------------- problem
    def set_options(self, **kw):
        for k, v in kw.items():
            if k.startswith("relax_") and isinstance(v, str):
                v = v.encode()
            setattr(self.opt, k, v)
        self.state += 1
        self._chk(B.pair_set_options(self.h, ctypes.byref(self.opt)))

    def set_mesh_hex(self, nx, ny=None, nz=None, lo=(0.0, 0.0, 0.0), hi=(1.0, 1.0, 1.0)):
        ny = nx if ny is None else ny
        nz = nx if nz is None else nz
        lo = np.asarray(lo, dtype=np.float64)
        hi = np.asarray(hi, dtype=np.float64)
        self.state += 1
        self._chk(B.pair_set_mesh_hex(self.h, nx, ny, nz, lo, hi))
        self.E = nx * ny * nz
        self.N = 8 * self.E

    def set_mesh_tet(self, xyz, elem_vert):
        xyz = np.ascontiguousarray(xyz, dtype=np.float64)
        ev = np.ascontiguousarray(elem_vert, dtype=np.int32)
        self.state += 1
        self._chk(B.pair_set_mesh(self.h, B.PAIR_TET4, xyz.shape[0], xyz, ev.shape[0], ev))
        self.E = ev.shape[0]
        self.N = 4 * self.E

    def set_mesh(self, mesh):
        """A workloads.Mesh (structured hex or tet)."""
        if mesh.kind == 0:
            self.set_mesh_hex(mesh.nx, mesh.ny, mesh.nz, mesh.lo, mesh.hi)
        else:
            self.set_mesh_tet(mesh.xyz, mesh.elem_vert)

    def set_quadrature(self, omega, w):
        omega = np.ascontiguousarray(omega, dtype=np.float64)
        w = np.ascontiguousarray(w, dtype=np.float64)
        self.state += 1
        self._chk(B.pair_set_quadrature(self.h, w.shape[0], omega, w))
        self.M = w.shape[0]

    @staticmethod
    def level_symmetric(order):
        M = ctypes.c_int()
        B.check(B.pair_quadrature_level_symmetric(order, ctypes.byref(M), None, None))
        om = np.zeros((M.value, 3))
        w = np.zeros(M.value)
        B.check(B.pair_quadrature_level_symmetric(order, None, om, w))
        return om, w

    def set_materials(self, sigma_t, sigma_s, q):
        st, ss, qq = _f64(sigma_t), _f64(sigma_s), _f64(q)
        if _where(st) != _where(ss) or _where(st) != _where(qq):
            raise ValueError("sigma_t, sigma_s and q must live in the same memory space")
        self.state += 1
        self._chk(B.pair_set_materials(self.h, st, ss, qq, _where(st)))
        self.q = qq

    def set_dual_source(self, src, per_direction=False):
        self.state += 1
        if src is None:
            self._chk(B.pair_set_dual_source(self.h, None, 0, B.PAIR_HOST))
            return
        s = _f64(src)
        self._chk(B.pair_set_dual_source(self.h, s, 1 if per_direction else 0, _where(s)))

    def set_inflow(self, g, m=-1):
        """Nodal inflow values g [N] (value of g at every DOF's node) for
        direction m (-1: every direction); g = None sets vacuum."""
        self.state += 1
        if g is None:
            self._chk(B.pair_set_inflow(self.h, m, None, B.PAIR_HOST))
            return
        gg = _f64(g)
        self._chk(B.pair_set_inflow(self.h, m, gg, _where(gg)))

    # ---------------------------------------------------------------- solves
    def _out(self, shape, device):
        if device:
            torch = _torch()
            return torch.empty(shape, dtype=torch.float64, device="cuda")
        return np.zeros(shape)

    def solve(self, mode=B.PAIR_PLAIN, phi0=None, want_psi=False, device=False):
        """Source iteration; returns (phi, psi or None, stats dict, return code)."""
        phi = self._out((self.N,), device)
        psi = self._out((self.M, self.N), device) if want_psi else None
        where = B.PAIR_DEVICE if device else B.PAIR_HOST
        if phi0 is not None:
            phi0 = _f64(phi0)
            if _where(phi0) != where:
                raise ValueError("phi0 must live where the outputs do")
        st = B.pair_stats()
        self.state += 1
        rc = self._chk(B.pair_solve(self.h, mode, phi0, phi, psi, where, ctypes.byref(st)),
                       allow_noconv=True)
        return phi, psi, st.as_dict(), rc

    def transport_sweep(self, mode=B.PAIR_PLAIN, phi_in=None, want_psi=True, device=False):
        """One sweep replacement; returns (psi or None, phi, stats dict, return code)."""
        phi = self._out((self.N,), device)
        psi = self._out((self.M, self.N), device) if want_psi else None
        where = B.PAIR_DEVICE if device else B.PAIR_HOST
        if phi_in is not None:
            phi_in = _f64(phi_in)
        st = B.pair_stats()
        self.state += 1
        rc = self._chk(B.pair_transport_sweep(self.h, mode, phi_in, psi, phi, where,
                                              ctypes.byref(st)), allow_noconv=True)
        return psi, phi, st.as_dict(), rc

    def adjoint(self, grad_phi, mode=B.PAIR_PLAIN):
        """Returns (dJ/dsigma_t, dJ/dsigma_s, phi_adj, stats, rc) in grad_phi's memory space."""
        g = _f64(grad_phi)
        device = _where(g) == B.PAIR_DEVICE
        gt = self._out((self.E,), device)
        gs = self._out((self.E,), device)
        pa = self._out((self.N,), device)
        st = B.pair_stats()
        rc = self._chk(B.pair_adjoint(self.h, mode, g, gt, gs, pa, _where(g), ctypes.byref(st)),
                       allow_noconv=True)
        return gt, gs, pa, st.as_dict(), rc

    def prepare(self, mode=B.PAIR_PLAIN):
        """Build every direction's fine operator and hierarchy without solving
        (needs keep_hierarchy=1); returns the setup statistics."""
        st = B.pair_stats()
        self._chk(B.pair_prepare(self.h, mode, ctypes.byref(st)))
        return st.as_dict()

    def clear_cache(self):
        self._chk(B.pair_clear_cache(self.h))

    def direction_info(self, m):
        it, cf, rr = ctypes.c_int(), ctypes.c_double(), ctypes.c_double()
        self._chk(B.pair_direction_info(self.h, m, ctypes.byref(it), ctypes.byref(cf),
                                        ctypes.byref(rr)))
        return it.value, cf.value, rr.value

    def export_fine_operator(self, m, with_rhs=True):
        """(rowptr, col, val, b) of D^{-1} A for direction m (host arrays)."""
        nnz = ctypes.c_int64()
        self._chk(B.pair_export_fine_operator(self.h, m, ctypes.byref(nnz), None, None, None, None))
        rp = np.zeros(self.N + 1, dtype=np.int64)
        col = np.zeros(nnz.value, dtype=np.int32)
        val = np.zeros(nnz.value)
        b = np.zeros(self.N) if with_rhs else None
        self._chk(B.pair_export_fine_operator(self.h, m, ctypes.byref(nnz), rp, col, val, b))
        return rp, col, val, b


class Amg:
    """Generic AIR hierarchy for a block-diagonal batch of CSR matrices."""

    def __init__(self, options: Optional[B.pair_options] = None, stream=None, **overrides):
        B.load()
        self.opt = options if options is not None else B.default_options(**overrides)
        h = ctypes.c_void_p()
        B.check(B.pair_amg_create(ctypes.byref(h), ctypes.byref(self.opt), stream))
        self.h = h
        self.n = 0
        self.n_seg = 0

    def close(self):
        if getattr(self, "h", None) is not None and self.h.value:
            B.pair_amg_destroy(self.h)
            self.h = None

    __del__ = close

    def _chk(self, rc, allow_noconv=False):
        if rc == B.PAIR_E_NOCONV and allow_noconv:
            return rc
        return B.check(rc, self.h, amg=True)

    def setup(self, rowptr, col, val, seg_rows=None):
        rowptr = np.ascontiguousarray(rowptr, dtype=np.int64)
        col = np.ascontiguousarray(col, dtype=np.int32)
        val = np.ascontiguousarray(val, dtype=np.float64)
        n = rowptr.shape[0] - 1
        seg = np.array([0, n] if seg_rows is None else seg_rows, dtype=np.int64)
        self._chk(B.pair_amg_setup(self.h, seg.shape[0] - 1, seg, n, rowptr, col, val, B.PAIR_HOST))
        self.n = n
        self.n_seg = seg.shape[0] - 1

    def num_levels(self):
        return B.pair_amg_num_levels(self.h)

    def segment_levels(self, s):
        return B.pair_amg_segment_levels(self.h, s)

    def level(self, l):
        n, nnz, nnzr = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
        self._chk(B.pair_amg_level_sizes(self.h, l, ctypes.byref(n), ctypes.byref(nnz),
                                         ctypes.byref(nnzr)))
        n, nnz, nnzr = n.value, nnz.value, nnzr.value
        rp = np.zeros(n + 1, dtype=np.int64)
        col = np.zeros(nnz, dtype=np.int32)
        val = np.zeros(nnz)
        cf = np.zeros(n, dtype=np.int8)
        p = np.zeros(n, dtype=np.int32)
        rr = rc = rv = None
        self._chk(B.pair_amg_get_level(self.h, l, rp, col, val, cf, p, None, None, None))
        if nnzr > 0:
            nc = int((cf > 0).sum())
            rr = np.zeros(nc + 1, dtype=np.int64)
            rc = np.zeros(nnzr, dtype=np.int32)
            rv = np.zeros(nnzr)
            self._chk(B.pair_amg_get_level(self.h, l, None, None, None, None, None, rr, rc, rv))
        return dict(rowptr=rp, col=col, val=val, cf=cf, p=p, r_rowptr=rr, r_col=rc, r_val=rv)

    def solve(self, b, x0=None, device=False):
        b = _f64(b)
        x = _f64(x0).copy() if x0 is not None else (np.zeros(self.n) if _where(b) == B.PAIR_HOST
                                                    else _torch().zeros_like(b))
        iters = np.zeros(self.n_seg, dtype=np.int32)
        rel = np.zeros(self.n_seg)
        rc = self._chk(B.pair_amg_solve(self.h, b, x, _where(b), iters, rel), allow_noconv=True)
        return x, iters, rel, rc


class TransportSolve:
    """phi = TransportSolve.apply(solver, sigma_t, sigma_s[, mode]).

    Forward: source iteration (pair_solve) with the given cross sections (the
    solver's mesh, quadrature and source q must be set; q is kept from the last
    set_materials call via ``solver.q``).  Backward: pair_adjoint with
    grad_phi as the dual-space derivative dJ/dphi, giving dJ/dsigma_t and
    dJ/dsigma_s.
    """

    @staticmethod
    def apply(solver: Solver, sigma_t, sigma_s, mode=B.PAIR_PLAIN):
        return _transport_fn().apply(solver, sigma_t, sigma_s, mode)


_FN = None


def _transport_fn():
    global _FN
    if _FN is not None:
        return _FN
    torch = _torch()

    class _Fn(torch.autograd.Function):
        @staticmethod
        def forward(ctx, solver, sigma_t, sigma_s, mode):
            q = solver.q
            solver.set_materials(sigma_t.detach(), sigma_s.detach(), q)
            device = sigma_t.is_cuda
            phi, _, st, rc = solver.solve(mode=mode, device=device)
            if rc != B.PAIR_OK:
                raise B.PairError(rc, "forward solve did not converge")
            ctx.solver = solver
            ctx.state = solver.state
            ctx.mode = mode
            out = phi if device else torch.from_numpy(phi)
            return out.to(sigma_t.dtype)

        @staticmethod
        def backward(ctx, grad_phi):
            # the adjoint reads the solver's last forward solution, operators
            # and cross sections: refuse if anything changed since this forward
            if ctx.solver.state != ctx.state:
                raise RuntimeError("TransportSolve.backward: the solver was used for another solve "
                                   "or its problem changed after this forward pass; the gradient "
                                   "would belong to that other state (use one solver per forward)")
            g = grad_phi.detach().to(torch.float64).contiguous()
            gt, gs, _, _, rc = ctx.solver.adjoint(g, mode=ctx.mode)
            if rc != B.PAIR_OK:
                raise B.PairError(rc, "adjoint solve did not converge")
            if not g.is_cuda:
                gt, gs = torch.from_numpy(gt), torch.from_numpy(gs)
            return None, gt, gs, None

    _FN = _Fn
    return _FN
