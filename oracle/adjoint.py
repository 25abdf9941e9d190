"""Adjoint of the source-iteration fixed point (oracle; test infrastructure only).

Forward problem (the block system of Sec. "Accuracy of Spatial Solves"):
    L_m psi_m - M_s phi/(4 pi) - M q/(4 pi) = 0,   phi - sum_m w_m psi_m = 0,
with M_s the sigma_s-weighted mass matrix.  Functional J = c^T phi with
c_i = int_Det phi_i (the integral of phi over a detector region).

Lagrange multipliers lambda_m = w_m x_m give
    L_m^T x_m = nu,    nu = c + M_s phi_dag/(4 pi),    phi_dag = sum_m w_m x_m,
and L_m^T is the DG operator of the reflected direction -Omega_m (integration
by parts of the volume term; checked exactly as A(-Omega) = A(Omega)^T).  So
phi_dag is the forward source iteration with q = 0 and the dual-space source c,
and x_m is that problem's angular flux of direction -Omega_m.  Then
    dJ/dsigma_t,e = - sum_m w_m x_{m,e}^T M_e psi_{m,e}
    dJ/dsigma_s,e =   phi_dag_e^T M_e phi_e / (4 pi)
(partial derivatives: sigma_s is held fixed when sigma_t moves).

Pinned by central finite differences of J on small meshes and by the dense
adjoint (the transposed coupled system) in tests/test_oracle_adjoint.py.
"""
from __future__ import annotations

import numpy as np

from . import dg
from .quadrature import reflected_index
from .source_iteration import Problem, source_iteration, dense_coupled_solve


def detector_source(prob: Problem, detector: np.ndarray) -> np.ndarray:
    """c as an element-blocked dual vector [N]: c_e = M_e 1 for e in the detector."""
    E, k = prob.topo.E, prob.topo.k
    c = np.einsum("eab,b->ea", prob.topo.mass, np.ones(k))
    c[~detector] = 0.0
    return c.ravel()


def functional(phi: np.ndarray, c: np.ndarray) -> float:
    return float(np.dot(c, phi))


def adjoint_problem(prob: Problem, c: np.ndarray) -> Problem:
    return Problem(prob.mesh, prob.sigma_t, prob.sigma_s, np.zeros_like(prob.q),
                   prob.omega, prob.w, ext=c)


def gradients(prob: Problem, psi: np.ndarray, phi: np.ndarray, psi_dag: np.ndarray,
              phi_dag: np.ndarray, sn_order: int):
    """dJ/dsigma_t [E], dJ/dsigma_s [E] from forward (psi, phi) and the
    adjoint problem's (psi_dag, phi_dag); x_m = psi_dag[reflect(m)]."""
    topo = prob.topo
    E, k = topo.E, topo.k
    g_t = np.zeros(E)
    for m in range(prob.M):
        x = psi_dag[reflected_index(sn_order, m)].reshape(E, k)
        p = psi[m].reshape(E, k)
        g_t -= prob.w[m] * np.einsum("ea,eab,eb->e", x, topo.mass, p)
    g_s = np.einsum("ea,eab,eb->e", phi_dag.reshape(E, k), topo.mass, phi.reshape(E, k)) / dg.FOUR_PI
    return g_t, g_s


def adjoint_gradients(prob: Problem, detector: np.ndarray, sn_order: int, tol: float = 1e-14):
    fwd = source_iteration(prob, tol=tol)
    c = detector_source(prob, detector)
    adj = source_iteration(adjoint_problem(prob, c), tol=tol)
    g_t, g_s = gradients(prob, fwd.psi, fwd.phi, adj.psi, adj.phi, sn_order)
    return functional(fwd.phi, c), g_t, g_s


def dense_adjoint_gradients(prob: Problem, detector: np.ndarray):
    """Same gradients from the transposed dense coupled system (tiny meshes):
    K^T y = [0; c], then dJ/dp = -y^T (dK/dp) x."""
    M, N = prob.M, prob.N
    topo = prob.topo
    E, k = topo.E, topo.k
    phi, psi = dense_coupled_solve(prob)
    c = detector_source(prob, detector)
    # rebuild K (same layout as dense_coupled_solve)
    K = np.zeros(((M + 1) * N, (M + 1) * N))
    Ms = np.zeros((N, N))
    for e in range(E):
        Ms[k * e:k * e + k, k * e:k * e + k] = prob.sigma_s[e] * topo.mass[e]
    for m in range(M):
        K[m * N:(m + 1) * N, m * N:(m + 1) * N] = dg.unscaled_csr(topo, prob.blocks(m)).toarray()
        K[m * N:(m + 1) * N, M * N:] = -Ms / dg.FOUR_PI
        K[M * N:, m * N:(m + 1) * N] = -prob.w[m] * np.eye(N)
    K[M * N:, M * N:] = np.eye(N)
    g = np.zeros((M + 1) * N)
    g[M * N:] = c
    y = np.linalg.solve(K.T, g)
    x = np.concatenate([psi.ravel(), phi])
    g_t = np.zeros(E)
    g_s = np.zeros(E)
    for e in range(E):
        sl = slice(k * e, k * e + k)
        for m in range(M):
            # dK/dsigma_t,e : M_e in the (m,m) block at element e
            g_t[e] -= y[m * N:(m + 1) * N][sl] @ topo.mass[e] @ x[m * N:(m + 1) * N][sl]
            # dK/dsigma_s,e : -M_e/(4 pi) in the (m, phi) block
            g_s[e] += y[m * N:(m + 1) * N][sl] @ topo.mass[e] @ phi[sl] / dg.FOUR_PI
    return functional(phi, c), g_t, g_s
