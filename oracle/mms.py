"""Manufactured solution of the Appendix (oracle; test infrastructure only).

psi_m(r) = Phi(r) Psi_m(r) with
    Phi   = sin(pi x/L) sin(pi y/L) sin(pi z/L),
    Psi_m = (1 + 2 mu (x - L/2)) (1 + 2 eta (y - L/2)) (1 + 2 xi (z - L/2)).
Phi vanishes on the boundary of the cube, so the boundary is vacuum.  With
sum w = 4 pi and a reflection-symmetric set, sum_m w_m Psi_m = 4 pi exactly
(the odd moments vanish), hence phi = 4 pi Phi and the angular source that makes
psi_m exact for the S_N equations is
    Q_m = Omega_m . grad(Phi Psi_m) + sigma_t Phi Psi_m - sigma_s Phi
(the Appendix's -sigma_s Phi/(4 pi) term corresponds to weights summing to 1;
here weights sum to 4 pi, so the scattering term is sigma_s phi/(4 pi) = sigma_s Phi).

Used for the O(h^2) discretisation-error pin of the Q1 DG solution.
"""
from __future__ import annotations

import math

import numpy as np

from . import dg

GL = np.polynomial.legendre.leggauss


def Phi(p, L=1.0):
    return np.sin(math.pi * p[..., 0] / L) * np.sin(math.pi * p[..., 1] / L) * np.sin(math.pi * p[..., 2] / L)


def gradPhi(p, L=1.0):
    s = [np.sin(math.pi * p[..., d] / L) for d in range(3)]
    c = [np.cos(math.pi * p[..., d] / L) * math.pi / L for d in range(3)]
    return np.stack([c[0] * s[1] * s[2], s[0] * c[1] * s[2], s[0] * s[1] * c[2]], axis=-1)


def Psi(p, om, L=1.0):
    return np.prod([1.0 + 2.0 * om[d] * (p[..., d] - L / 2) for d in range(3)], axis=0)


def gradPsi(p, om, L=1.0):
    f = [1.0 + 2.0 * om[d] * (p[..., d] - L / 2) for d in range(3)]
    return np.stack([2 * om[0] * f[1] * f[2], f[0] * 2 * om[1] * f[2], f[0] * f[1] * 2 * om[2]], axis=-1)


def source(p, om, sigma_t, sigma_s, L=1.0):
    ph, ps = Phi(p, L), Psi(p, om, L)
    grad = gradPhi(p, L) * ps[..., None] + ph[..., None] * gradPsi(p, om, L)
    return grad @ np.asarray(om) + sigma_t * ph * ps - sigma_s * ph


def hex_projected_source(topo: dg.Topology, omega: np.ndarray, sigma_t: float, sigma_s: float,
                         npts: int = 4) -> np.ndarray:
    """ext[m, 8e+a] = int_e Q_m phi_a (tensor Gauss, npts^3 points per element)."""
    x, w = GL(npts)
    x = 0.5 * (x + 1.0)
    w = 0.5 * w
    h = np.array(topo.h)
    E = topo.E
    M = omega.shape[0]
    out = np.zeros((M, E, 8))
    for i, (tx, wx) in enumerate(zip(x, w)):
        for j, (ty, wy) in enumerate(zip(x, w)):
            for k, (tz, wz) in enumerate(zip(x, w)):
                pts = topo.origin + np.array([tx, ty, tz]) * h
                wt = wx * wy * wz * h.prod()
                basis = np.array([(tx if a & 1 else 1 - tx) * (ty if a & 2 else 1 - ty) *
                                  (tz if a & 4 else 1 - tz) for a in range(8)])
                for m in range(M):
                    q = source(pts, omega[m], sigma_t, sigma_s)
                    out[m] += wt * q[:, None] * basis[None, :]
    return out.reshape(M, -1)


def hex_l2_error(topo: dg.Topology, u_nodal: np.ndarray, exact, npts: int = 4) -> float:
    """|| u_h - exact ||_{L2} with u_h the Q1 DG field [E*8]."""
    x, w = GL(npts)
    x = 0.5 * (x + 1.0)
    w = 0.5 * w
    h = np.array(topo.h)
    u = u_nodal.reshape(topo.E, 8)
    err = 0.0
    for tx, wx in zip(x, w):
        for ty, wy in zip(x, w):
            for tz, wz in zip(x, w):
                pts = topo.origin + np.array([tx, ty, tz]) * h
                basis = np.array([(tx if a & 1 else 1 - tx) * (ty if a & 2 else 1 - ty) *
                                  (tz if a & 4 else 1 - tz) for a in range(8)])
                uh = u @ basis
                err += wx * wy * wz * h.prod() * np.sum((uh - exact(pts)) ** 2)
    return math.sqrt(err)


def tet_l2_error(topo: dg.Topology, u_nodal: np.ndarray, exact, npts: int = 5) -> float:
    """|| u_h - exact ||_{L2} with u_h the P1 DG field [E*4], by the conical
    product (collapsed Gauss) rule on every tetrahedron: the unit cube mapped
    onto the tet with Jacobian 6 |T| (1-u)^2 (1-v)."""
    x, w = GL(npts)
    x = 0.5 * (x + 1.0)
    w = 0.5 * w
    X = topo.xyz[topo.elem_vert]                  # [E,4,3]
    u = u_nodal.reshape(topo.E, 4)
    err = 0.0
    for tu, wu in zip(x, w):
        for tv, wv in zip(x, w):
            for tw, ww in zip(x, w):
                l1 = tu
                l2 = tv * (1.0 - tu)
                l3 = tw * (1.0 - tu) * (1.0 - tv)
                lam = np.array([1.0 - l1 - l2 - l3, l1, l2, l3])
                jac = 6.0 * (1.0 - tu) ** 2 * (1.0 - tv)
                pts = np.einsum("a,ead->ed", lam, X)
                uh = u @ lam
                err += wu * wv * ww * jac * np.sum(topo.vol * (uh - exact(pts)) ** 2)
    return math.sqrt(err)
