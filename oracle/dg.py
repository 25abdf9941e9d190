"""Per-direction upwind DG operator in block form (oracle; test infrastructure only).

For a fixed direction Omega the upwind DG discretisation (eq.
weak_form_transport) couples element e only to its upwind neighbours, so the
global matrix A is block lower triangular in a topological element order
(Sec. "Solution of the Transport Equation by Sweeping").  Element-local form:

  D_e      = sigma_t,e M_e - C_e(Omega) + sum_{faces f of e with Omega.n_f > 0} (Omega.n_f) F_f
  A_{e,U}  = (Omega.n_f) int_f phi_a^e phi_b^U     for faces f with Omega.n_f < 0
             shared with the upwind element U
  f_e      = M_e (sigma_s,e phi_e + q_e) / (4 pi)  [+ external dual-space source]
             - sum_{inflow boundary faces} (Omega.n_f) int_f g phi_a

(q_total = (sigma_s phi + q)/(4 pi), eq. mono_transport / eq. sn_transport.)
Faces with |Omega.n| <= 1e-12 |n| carry no flux either way.  The face normal is
computed once per face from its vertices in ascending global-id order, so the
two sides see exactly opposite values of Omega.n.

Block scaling (Sec. "Sweeping with pAIR"): the left block-inverse scaling
D^{-1} A x = D^{-1} b gives a unit diagonal; within-block off-diagonals are
exactly zero.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Callable, Optional

import numpy as np
import scipy.sparse as sp

from . import elements as el

FOUR_PI = 4.0 * math.pi
ZERO_FLUX_TOL = 1e-12


@dataclasses.dataclass
class Topology:
    kind: int
    E: int
    k: int                 # nodes per element
    F: int                 # faces per element
    nbr: np.ndarray        # [E,F] neighbour element across face, -1 on the boundary
    enodes: np.ndarray     # [E,F,nf] local nodes of e on face f
    unodes: np.ndarray     # [E,F,nf] matching local nodes of the neighbour (or -1)
    # Omega.n for a direction is  dot(omega, nvec[e,f]) ; for tets nvec is the
    # un-normalised canonical normal oriented outward from e.
    nvec: np.ndarray       # [E,F,3]
    nlen: np.ndarray       # [E,F] |nvec|
    # element data
    vol: np.ndarray        # [E]
    mass: np.ndarray       # [E,k,k] (hex: broadcast view of one matrix)
    grads: Optional[np.ndarray] = None   # tets [E,4,3]
    h: Optional[tuple] = None            # hex (hx,hy,hz)
    origin: Optional[np.ndarray] = None  # hex element origins [E,3]
    xyz: Optional[np.ndarray] = None
    elem_vert: Optional[np.ndarray] = None


def hex_topology(mesh) -> Topology:
    nx, ny, nz = mesh.nx, mesh.ny, mesh.nz
    hx = (mesh.hi[0] - mesh.lo[0]) / nx
    hy = (mesh.hi[1] - mesh.lo[1]) / ny
    hz = (mesh.hi[2] - mesh.lo[2]) / nz
    E = nx * ny * nz
    e = np.arange(E)
    I = e % nx
    J = (e // nx) % ny
    K = e // (nx * ny)
    nbr = np.full((E, 6), -1, dtype=np.int64)
    strides = (1, nx, nx * ny)
    idx = (I, J, K)
    n = (nx, ny, nz)
    for ax in range(3):
        lo_ok = idx[ax] > 0
        hi_ok = idx[ax] < n[ax] - 1
        nbr[lo_ok, 2 * ax + 0] = e[lo_ok] - strides[ax]
        nbr[hi_ok, 2 * ax + 1] = e[hi_ok] + strides[ax]
    enodes = np.zeros((E, 6, 4), dtype=np.int64)
    unodes = np.zeros((E, 6, 4), dtype=np.int64)
    nvec = np.zeros((E, 6, 3))
    for ax in range(3):
        for s in range(2):
            f = 2 * ax + s
            en = el.hex_face_nodes(ax, s)
            un = [a ^ (1 << ax) for a in en]     # same position on the other side
            enodes[:, f] = en
            unodes[:, f] = un
            nvec[:, f, ax] = 2.0 * s - 1.0
    unodes[nbr < 0] = -1
    M = el.hex_mass(hx, hy, hz)
    return Topology(kind=0, E=E, k=8, F=6, nbr=nbr, enodes=enodes, unodes=unodes,
                    nvec=nvec, nlen=np.ones((E, 6)), vol=np.full(E, hx * hy * hz),
                    mass=np.broadcast_to(M, (E, 8, 8)), h=(hx, hy, hz),
                    origin=hex_origins(mesh))


def tet_topology(mesh) -> Topology:
    xyz = np.asarray(mesh.xyz, dtype=np.float64)
    ev = np.asarray(mesh.elem_vert, dtype=np.int64)
    E = ev.shape[0]
    # face f of a tet is opposite local vertex f
    loc = np.array([[1, 2, 3], [0, 2, 3], [0, 1, 3], [0, 1, 2]])
    fv = ev[:, loc]                                  # [E,4,3] global ids
    key = np.sort(fv, axis=2).reshape(-1, 3)
    order = np.lexsort((key[:, 2], key[:, 1], key[:, 0]))
    ks = key[order]
    same = np.all(ks[1:] == ks[:-1], axis=1)
    nbr = np.full(E * 4, -1, dtype=np.int64)
    a = order[:-1][same]
    b = order[1:][same]
    nbr[a] = b // 4
    nbr[b] = a // 4
    nbr = nbr.reshape(E, 4)
    # canonical normal from the sorted vertex triple, oriented outward from e
    sk = np.sort(fv, axis=2)
    p0, p1, p2 = xyz[sk[..., 0]], xyz[sk[..., 1]], xyz[sk[..., 2]]
    ncan = np.cross(p1 - p0, p2 - p0)                # [E,4,3]
    opp = xyz[ev]                                    # vertex f is opposite face f
    side = np.einsum("efk,efk->ef", opp - p0, ncan)
    sign = np.where(side > 0.0, -1.0, 1.0)
    nvec = ncan * sign[..., None]
    nlen = np.linalg.norm(ncan, axis=2)
    enodes = np.broadcast_to(loc, (E, 4, 3)).copy()
    unodes = np.full((E, 4, 3), -1, dtype=np.int64)
    for f in range(4):
        has = nbr[:, f] >= 0
        U = nbr[has, f]
        gv_e = fv[has, f]                            # [n,3] global ids on e's side
        gv_U = ev[U]                                 # [n,4]
        for t in range(3):
            m = gv_U == gv_e[:, t:t + 1]
            unodes[has, f, t] = np.argmax(m, axis=1)
    vols = np.empty(E)
    grads = np.empty((E, 4, 3))
    X = xyz[ev]                                      # [E,4,3]
    Jm = np.stack([X[:, 1] - X[:, 0], X[:, 2] - X[:, 0], X[:, 3] - X[:, 0]], axis=2)
    det = np.linalg.det(Jm)
    vols = np.abs(det) / 6.0
    Ginv = np.linalg.inv(Jm)
    grads[:, 1:] = Ginv
    grads[:, 0] = -Ginv.sum(axis=1)
    mass = vols[:, None, None] * (np.ones((4, 4)) + np.eye(4))[None] / 20.0
    return Topology(kind=1, E=E, k=4, F=4, nbr=nbr, enodes=enodes, unodes=unodes,
                    nvec=nvec, nlen=nlen, vol=vols, mass=mass, grads=grads,
                    xyz=xyz, elem_vert=ev)


def topology(mesh) -> Topology:
    return hex_topology(mesh) if mesh.kind == 0 else tet_topology(mesh)


@dataclasses.dataclass
class Blocks:
    """A(Omega) = blockdiag(D) + sum of coupling blocks, in element-local form."""
    D: np.ndarray       # [E,k,k]
    nbr: np.ndarray     # [E,F] upwind neighbour coupled through face f, else -1
    Cpl: np.ndarray     # [E,F,k,k]  A_{e,nbr[e,f]}
    odn: np.ndarray     # [E,F] Omega.n_f (unit normal), 0 on zero-flux faces


def _face_mass_e(topo: Topology, f: int, sel=slice(None)):
    """int_f phi_a phi_b over face f of the selected elements [n,k,k]."""
    if topo.kind == 0:
        hx, hy, hz = topo.h
        F = el.hex_face_mass(hx, hy, hz, f // 2, f % 2)
        n = topo.E if isinstance(sel, slice) else np.count_nonzero(sel) if sel.dtype == bool else len(sel)
        return np.broadcast_to(F, (n, 8, 8))
    area = 0.5 * topo.nlen[sel, f]
    out = np.zeros((area.shape[0], 4, 4))
    nodes = [a for a in range(4) if a != f]
    fm = (np.ones((3, 3)) + np.eye(3)) / 12.0
    for i, a in enumerate(nodes):
        for j, b in enumerate(nodes):
            out[:, a, b] = area * fm[i, j]
    return out


def assemble(topo: Topology, sigma_t: np.ndarray, omega) -> Blocks:
    omega = np.asarray(omega, dtype=np.float64)
    E, k, F = topo.E, topo.k, topo.F
    odn_raw = np.einsum("efk,k->ef", topo.nvec, omega)          # Omega . nvec
    zero = np.abs(odn_raw) <= ZERO_FLUX_TOL * topo.nlen
    odn = np.where(zero, 0.0, odn_raw / topo.nlen)              # Omega . n (unit)
    # volume terms
    if topo.kind == 0:
        hx, hy, hz = topo.h
        C = el.hex_advection(hx, hy, hz, omega)
        M = topo.mass[0]
        D = sigma_t[:, None, None] * M[None] - C[None]
    else:
        og = np.einsum("eak,k->ea", topo.grads, omega)           # Omega . grad lambda_a
        C = og[:, :, None] * (topo.vol / 4.0)[:, None, None] * np.ones((1, 1, 4))
        D = sigma_t[:, None, None] * topo.mass - C
    D = np.array(D)
    nbr = np.full((E, F), -1, dtype=np.int64)
    Cpl = np.zeros((E, F, k, k))
    for f in range(F):
        out = odn[:, f] > 0.0
        if np.any(out):
            D[out] += odn[out, f][:, None, None] * _face_mass_e(topo, f, out)
        inn = (odn[:, f] < 0.0) & (topo.nbr[:, f] >= 0)
        if np.any(inn):
            nbr[inn, f] = topo.nbr[inn, f]
            if topo.kind == 0:
                hx, hy, hz = topo.h
                X = el.hex_face_cross(hx, hy, hz, f // 2, f % 2)
                Cpl[inn, f] = odn[inn, f][:, None, None] * X[None]
            else:
                area = 0.5 * topo.nlen[inn, f]
                en = topo.enodes[inn, f]            # [n,3]
                un = topo.unodes[inn, f]            # [n,3]
                # global ids decide which trial node of U matches which test node of e
                for i in range(3):
                    for j in range(3):
                        val = area * (2.0 if i == j else 1.0) / 12.0
                        Cpl[np.flatnonzero(inn), f, en[:, i], un[:, j]] = odn[inn, f] * val
    return Blocks(D=D, nbr=nbr, Cpl=Cpl, odn=odn)


def rhs(topo: Topology, sigma_s, q, phi=None, ext=None) -> np.ndarray:
    """Unscaled right-hand side [E,k]: M (sigma_s phi + q)/(4 pi) (+ ext)."""
    E, k = topo.E, topo.k
    src = np.broadcast_to(q[:, None], (E, k)).astype(np.float64)
    if phi is not None:
        src = src + sigma_s[:, None] * phi.reshape(E, k)
    f = np.einsum("eab,eb->ea", topo.mass, src) / FOUR_PI
    if ext is not None:
        f = f + ext.reshape(E, k)
    return f


def _tri_rule(n: int = 5):
    """Collapsed (Duffy) Gauss rule on the reference triangle: barycentric
    coordinates [q,3] and weights [q] summing to 1 (the rule integrates a
    function's mean over the triangle; multiply by the area)."""
    x, w = np.polynomial.legendre.leggauss(n)
    x = 0.5 * (x + 1.0)
    w = 0.5 * w
    lam, wt = [], []
    for s, ws in zip(x, w):
        for t, wt_ in zip(x, w):
            l1 = s
            l2 = t * (1.0 - s)
            lam.append((1.0 - l1 - l2, l1, l2))
            wt.append(2.0 * ws * wt_ * (1.0 - s))
    return np.array(lam), np.array(wt)


def inflow_rhs(topo: Topology, blocks: Blocks, g: Callable) -> np.ndarray:
    """-sum_{inflow boundary faces} (Omega.n) int_f g phi_a  (eq.
    weak_form_transport, the inflow term on Gamma^-), integrated by quadrature:
    a 5x5 Gauss rule on each hex face, a 25-point collapsed Gauss rule on each
    tet face.  g maps points [n,3] -> values [n]."""
    if topo.kind == 1:
        return _tet_inflow_rhs(topo, blocks, g)
    xg, wg = np.polynomial.legendre.leggauss(5)
    xg = 0.5 * (xg + 1.0)
    wg = 0.5 * wg
    h = np.array(topo.h)
    out = np.zeros((topo.E, 8))
    for f in range(6):
        ax, s = f // 2, f % 2
        sel = (blocks.odn[:, f] < 0.0) & (topo.nbr[:, f] < 0)
        if not np.any(sel):
            continue
        ids = np.flatnonzero(sel)
        org = topo.origin[ids]
        o1, o2 = [d for d in range(3) if d != ax]
        for t1, w1 in zip(xg, wg):
            for t2, w2 in zip(xg, wg):
                pts = org.copy()
                pts[:, ax] += s * h[ax]
                pts[:, o1] += t1 * h[o1]
                pts[:, o2] += t2 * h[o2]
                gv = g(pts)
                wt = w1 * w2 * h[o1] * h[o2]
                for a in range(8):
                    if ((a >> ax) & 1) != s:
                        continue
                    c1 = t1 if (a >> o1) & 1 else 1.0 - t1
                    c2 = t2 if (a >> o2) & 1 else 1.0 - t2
                    out[ids, a] -= blocks.odn[ids, f] * wt * gv * c1 * c2
    return out


def _tet_inflow_rhs(topo: Topology, blocks: Blocks, g: Callable) -> np.ndarray:
    """Tet faces: the P1 basis of a face node is its barycentric coordinate on
    the face, and the face area is |nvec|/2."""
    lam, wq = _tri_rule(5)
    out = np.zeros((topo.E, 4))
    X = topo.xyz[topo.elem_vert]                      # [E,4,3]
    for f in range(4):
        sel = (blocks.odn[:, f] < 0.0) & (topo.nbr[:, f] < 0)
        if not np.any(sel):
            continue
        ids = np.flatnonzero(sel)
        nodes = [a for a in range(4) if a != f]
        P = X[ids][:, nodes]                          # [n,3,3] face vertices
        area = 0.5 * topo.nlen[ids, f]
        for lq, w in zip(lam, wq):
            pts = np.einsum("j,njd->nd", lq, P)
            gv = g(pts)
            for j, a in enumerate(nodes):
                out[ids, a] -= blocks.odn[ids, f] * area * w * gv * lq[j]
    return out


def inflow_rhs_nodal(topo: Topology, blocks: Blocks, g_nodal: np.ndarray) -> np.ndarray:
    """The inflow term with g replaced by its nodal interpolant on each face:
    -sum_{inflow boundary faces f} (Omega.n_f) F_f g_e, F_f the face mass
    matrix of the element's basis and g_e [k] the values of g at the element's
    nodes (only face nodes enter).  Equal to ``inflow_rhs`` whenever g is
    bilinear on hex faces / linear on tet faces."""
    g = np.asarray(g_nodal, dtype=np.float64).reshape(topo.E, topo.k)
    out = np.zeros((topo.E, topo.k))
    for f in range(topo.F):
        sel = (blocks.odn[:, f] < 0.0) & (topo.nbr[:, f] < 0)
        if not np.any(sel):
            continue
        Ff = _face_mass_e(topo, f, sel)               # [n,k,k]
        out[sel] -= blocks.odn[sel, f][:, None] * np.einsum("nab,nb->na", Ff, g[sel])
    return out


def node_coordinates(topo: Topology) -> np.ndarray:
    """Position of every DOF's node [E*k,3] (hex: origin + corner offsets;
    tets: the element's vertices)."""
    if topo.kind == 0:
        h = np.array(topo.h)
        off = np.array([[(a >> d) & 1 for d in range(3)] for a in range(8)], dtype=np.float64) * h
        return (topo.origin[:, None, :] + off[None]).reshape(-1, 3)
    return topo.xyz[topo.elem_vert].reshape(-1, 3)


def hex_origins(mesh) -> np.ndarray:
    nx, ny, nz = mesh.nx, mesh.ny, mesh.nz
    hx = (mesh.hi[0] - mesh.lo[0]) / nx
    hy = (mesh.hi[1] - mesh.lo[1]) / ny
    hz = (mesh.hi[2] - mesh.lo[2]) / nz
    e = np.arange(nx * ny * nz)
    return np.stack([mesh.lo[0] + (e % nx) * hx,
                     mesh.lo[1] + ((e // nx) % ny) * hy,
                     mesh.lo[2] + (e // (nx * ny)) * hz], axis=1)


def unscaled_csr(topo: Topology, blocks: Blocks) -> sp.csr_matrix:
    """Global A(Omega) as a sparse matrix, DOF = k*e + a."""
    E, k, F = topo.E, topo.k, topo.F
    rows, cols, vals = [], [], []
    ea = np.arange(E)
    r = (k * ea)[:, None, None] + np.arange(k)[None, :, None]
    c = (k * ea)[:, None, None] + np.arange(k)[None, None, :]
    rows.append(np.broadcast_to(r, (E, k, k)).ravel())
    cols.append(np.broadcast_to(c, (E, k, k)).ravel())
    vals.append(blocks.D.ravel())
    for f in range(F):
        sel = blocks.nbr[:, f] >= 0
        if not np.any(sel):
            continue
        ids = np.flatnonzero(sel)
        U = blocks.nbr[ids, f]
        r = (k * ids)[:, None, None] + np.arange(k)[None, :, None]
        c = (k * U)[:, None, None] + np.arange(k)[None, None, :]
        rows.append(np.broadcast_to(r, (ids.size, k, k)).ravel())
        cols.append(np.broadcast_to(c, (ids.size, k, k)).ravel())
        vals.append(blocks.Cpl[ids, f].ravel())
    A = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(E * k, E * k))
    A.eliminate_zeros()
    return A


def scaled_csr(topo: Topology, blocks: Blocks) -> sp.csr_matrix:
    """D^{-1} A with the exact unit diagonal and the structural pattern: each
    coupling through face f contributes k rows x (face nodes of U) columns."""
    E, k, F = topo.E, topo.k, topo.F
    Dinv = np.linalg.inv(blocks.D)
    rows = [np.arange(E * k)]
    cols = [np.arange(E * k)]
    vals = [np.ones(E * k)]
    for f in range(F):
        sel = blocks.nbr[:, f] >= 0
        if not np.any(sel):
            continue
        ids = np.flatnonzero(sel)
        U = blocks.nbr[ids, f]
        S = Dinv[ids] @ blocks.Cpl[ids, f]                  # [n,k,k]
        un = topo.unodes[ids, f]                            # [n,nf] face nodes of U
        nf = un.shape[1]
        r = (k * ids)[:, None, None] + np.arange(k)[None, :, None]
        c = (k * U)[:, None, None] + un[:, None, :]
        v = np.take_along_axis(S, np.broadcast_to(un[:, None, :], (ids.size, k, nf)), axis=2)
        rows.append(np.broadcast_to(r, (ids.size, k, nf)).ravel())
        cols.append(np.broadcast_to(c, (ids.size, k, nf)).ravel())
        vals.append(v.ravel())
    A = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(E * k, E * k)).tocsr()
    A.sort_indices()
    return A
