"""Closed-form element matrices for the upwind DG transport form (oracle).

Test infrastructure only.  The weak form per direction (eq.
weak_form_transport) contributes, for test function phi_a and trial phi_b on
element T:

  volume   : -(psi, Omega.grad v)  ->  -C_ab,  C_ab = int_T phi_b Omega.grad(phi_a)
             (sigma_t psi, v)      ->  sigma_t M_ab,  M_ab = int_T phi_a phi_b
  faces    : <psi_upwind, v Omega.n>_F, the trace taken from the upwind element.

Q1 hex (axis-aligned box hx*hy*hz, local node a = ax + 2ay + 4az): the matrices
are Kronecker products of 1-D factors
  m(h) = h/6 [[2,1],[1,2]],   g_ab = int X_b X_a' dx = [[-1/2,-1/2],[1/2,1/2]],
  M = mz (x) my (x) mx,
  C = mu * mz(x)my(x)g + eta * mz(x)g(x)mx + xi * g(x)my(x)mx,
  face (axis d, side s): delta(a_d=s) delta(b_d=s) times the two other m's.

P1 tet (vertices x0..x3, volume |T|, barycentric lambda_a):
  M_ab = |T| (1 + delta_ab)/20,   C_ab = (Omega.grad lambda_a) |T|/4,
  face mass on the face's three nodes: A_f (1 + delta_ab)/12.

Pinned by: agreement with 3x3x3 / high-order Gauss quadrature computed
independently in the tests; sum_a C_ab = 0; 1^T M 1 = element volume.
"""
from __future__ import annotations

import numpy as np

G1 = np.array([[-0.5, -0.5], [0.5, 0.5]])


def m1(h: float) -> np.ndarray:
    return (h / 6.0) * np.array([[2.0, 1.0], [1.0, 2.0]])


def _k3(az, ay, ax):
    return np.kron(az, np.kron(ay, ax))


def hex_mass(hx, hy, hz) -> np.ndarray:
    return _k3(m1(hz), m1(hy), m1(hx))


def hex_advection(hx, hy, hz, omega) -> np.ndarray:
    """C_ab = int phi_b Omega.grad(phi_a) (row a = test function)."""
    mu, eta, xi = omega
    return (mu * _k3(m1(hz), m1(hy), G1)
            + eta * _k3(m1(hz), G1, m1(hx))
            + xi * _k3(G1, m1(hy), m1(hx)))


def _point(s: int) -> np.ndarray:
    e = np.zeros((2, 2))
    e[s, s] = 1.0
    return e


def _cross(s: int, t: int) -> np.ndarray:
    e = np.zeros((2, 2))
    e[s, t] = 1.0
    return e


def hex_face_mass(hx, hy, hz, axis: int, side: int) -> np.ndarray:
    """int_F phi_a phi_b over face (axis, side) of one element."""
    mats = [m1(hx), m1(hy), m1(hz)]
    mats[axis] = _point(side)
    return _k3(mats[2], mats[1], mats[0])


def hex_face_cross(hx, hy, hz, axis: int, side: int) -> np.ndarray:
    """int_F phi_a^e phi_b^U where F is face (axis, side) of e and U the element
    across it (U sees the same face as side 1 - side)."""
    mats = [m1(hx), m1(hy), m1(hz)]
    mats[axis] = _cross(side, 1 - side)
    return _k3(mats[2], mats[1], mats[0])


def hex_face_nodes(axis: int, side: int) -> list:
    return [a for a in range(8) if ((a >> axis) & 1) == side]


# --------------------------------------------------------------------------- tets

def tet_geometry(X: np.ndarray):
    """X [4,3] -> (volume, grad lambda [4,3])."""
    J = np.stack([X[1] - X[0], X[2] - X[0], X[3] - X[0]], axis=1)
    vol = abs(np.linalg.det(J)) / 6.0
    Ginv = np.linalg.inv(J)            # rows: grad lambda_1..3
    grads = np.empty((4, 3))
    grads[1:] = Ginv
    grads[0] = -Ginv.sum(axis=0)
    return vol, grads


def tet_mass(vol: float) -> np.ndarray:
    return vol * (np.ones((4, 4)) + np.eye(4)) / 20.0


def tet_advection(vol: float, grads: np.ndarray, omega) -> np.ndarray:
    og = grads @ np.asarray(omega, dtype=np.float64)   # Omega.grad lambda_a
    return np.outer(og, np.ones(4)) * (vol / 4.0)


def tri_face_mass(area: float) -> np.ndarray:
    return area * (np.ones((3, 3)) + np.eye(3)) / 12.0
