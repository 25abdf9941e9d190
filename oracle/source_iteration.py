"""Source iteration and the dense coupled system (oracle; test infrastructure only).

Source iteration (eq. sn_transport): with the scalar flux lagged, the M
direction problems are independent; each is solved exactly by a sweep, then
phi^{n+1} = sum_m w_m psi_m^{n+1} (eq. angular_quad).  Sec. "Accuracy of
Spatial Solves" writes the same problem as one block system in (psi_1..psi_M,
phi); on tiny meshes ``dense_coupled_solve`` solves that system directly, and
source iteration must converge to its solution (Richardson iteration on the
Schur complement S phi = b of that system).

Pinned by: the dense coupled solve (tests/test_oracle_si.py), particle balance,
the cube symmetries of a uniform problem, and the O(h^2) rates of the
pure-absorber closed form and of the manufactured solution.
"""
from __future__ import annotations

import dataclasses
from typing import Optional

import numpy as np

from . import dg
from .sweep import sweep
from concurrent.futures import ThreadPoolExecutor


@dataclasses.dataclass
class Problem:
    mesh: object
    sigma_t: np.ndarray
    sigma_s: np.ndarray
    q: np.ndarray
    omega: np.ndarray            # [M,3]
    w: np.ndarray                # [M]
    ext: Optional[np.ndarray] = None      # dual-space source [M,N] or [N] (added to each rhs)
    inflow: Optional[object] = None       # callable g(points, omega) for inflow boundary data
    inflow_nodal: Optional[np.ndarray] = None   # nodal inflow values [M,N] or [N] (face interpolant)
    cache_blocks: bool = True

    def __post_init__(self):
        self.topo = dg.topology(self.mesh)
        self._blocks = {}

    @property
    def M(self):
        return self.omega.shape[0]

    @property
    def N(self):
        return self.topo.E * self.topo.k

    def blocks(self, m: int):
        if m in self._blocks:
            return self._blocks[m]
        b = dg.assemble(self.topo, self.sigma_t, self.omega[m])
        if self.cache_blocks:
            self._blocks[m] = b
        return b

    def rhs(self, m: int, phi: Optional[np.ndarray]) -> np.ndarray:
        ext = None
        if self.ext is not None:
            ext = self.ext[m] if self.ext.ndim == 2 else self.ext
        f = dg.rhs(self.topo, self.sigma_s, self.q, phi, ext)
        if self.inflow is not None:
            om = self.omega[m]
            f = f + dg.inflow_rhs(self.topo, self.blocks(m), lambda p: self.inflow(p, om))
        if self.inflow_nodal is not None:
            g = self.inflow_nodal[m] if self.inflow_nodal.ndim == 2 else self.inflow_nodal
            f = f + dg.inflow_rhs_nodal(self.topo, self.blocks(m), g)
        return f


def transport_sweep(prob: Problem, phi: Optional[np.ndarray], threads: int = 1,
                    dirs=None) -> np.ndarray:
    """psi_m = L_m^{-1} b_m(phi) for every direction (one source iteration).
    Returns psi [M,N] (or [len(dirs),N])."""
    dirs = list(range(prob.M)) if dirs is None else list(dirs)

    def one(m):
        return sweep(prob.blocks(m), prob.rhs(m, phi)).ravel()

    if threads <= 1:
        out = [one(m) for m in dirs]
    else:
        with ThreadPoolExecutor(threads) as ex:
            out = list(ex.map(one, dirs))
    return np.stack(out)


def scalar_flux(prob: Problem, psi: np.ndarray) -> np.ndarray:
    """phi = sum_m w_m psi_m, summed in order m = 1..M (eq. angular_quad)."""
    phi = np.zeros(psi.shape[1])
    for m in range(psi.shape[0]):
        phi += prob.w[m] * psi[m]
    return phi


@dataclasses.dataclass
class SIResult:
    phi: np.ndarray
    psi: np.ndarray
    iterations: int
    history: list


def source_iteration(prob: Problem, tol: float = 1e-12, maxit: int = 100000,
                     estimate: bool = True, phi0=None, threads: int = 1) -> SIResult:
    """Iterate to convergence.  With ``estimate`` the stop test is the error
    estimate rho/(1-rho) * |dphi|/|phi| <= tol, rho = |dphi_n|/|dphi_{n-1}|;
    otherwise the plain difference |dphi|/|phi| <= tol."""
    phi = np.zeros(prob.N) if phi0 is None else np.array(phi0, dtype=np.float64)
    hist = []
    prev = None
    psi = None
    for it in range(1, maxit + 1):
        psi = transport_sweep(prob, phi, threads=threads)
        new = scalar_flux(prob, psi)
        d = np.linalg.norm(new - phi)
        nrm = np.linalg.norm(new)
        rel = d / nrm if nrm > 0 else d
        hist.append(rel)
        phi = new
        if estimate:
            if prev is not None and prev > 0:
                rho = min(d / prev, 0.999999)
                if rho / (1.0 - rho) * rel <= tol or rel == 0.0:
                    return SIResult(phi, psi, it, hist)
            elif rel == 0.0:
                return SIResult(phi, psi, it, hist)
        elif rel <= tol:
            return SIResult(phi, psi, it, hist)
        prev = d
    return SIResult(phi, psi, maxit, hist)


def dense_coupled_solve(prob: Problem):
    """Solve the (M+1)N block system of Sec. "Accuracy of Spatial Solves":
        L_m psi_m - M_sigma_s phi / (4 pi) = M q / (4 pi)   (m = 1..M)
        phi - sum_m w_m psi_m            = 0
    densely.  Returns (phi, psi[M,N])."""
    M, N = prob.M, prob.N
    topo = prob.topo
    K = np.zeros(((M + 1) * N, (M + 1) * N))
    b = np.zeros((M + 1) * N)
    Ms = np.zeros((N, N))
    k = topo.k
    for e in range(topo.E):
        Ms[k * e:k * e + k, k * e:k * e + k] = prob.sigma_s[e] * topo.mass[e]
    for m in range(M):
        A = dg.unscaled_csr(topo, prob.blocks(m)).toarray()
        K[m * N:(m + 1) * N, m * N:(m + 1) * N] = A
        K[m * N:(m + 1) * N, M * N:] = -Ms / dg.FOUR_PI
        b[m * N:(m + 1) * N] = prob.rhs(m, None).ravel()
        K[M * N:, m * N:(m + 1) * N] = -prob.w[m] * np.eye(N)
    K[M * N:, M * N:] = np.eye(N)
    x = np.linalg.solve(K, b)
    return x[M * N:], x[:M * N].reshape(M, N)
