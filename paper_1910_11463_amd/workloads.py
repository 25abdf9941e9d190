"""Seeded synthetic inputs for the S_N transport workloads.

This module only *generates inputs*: meshes (vertex coordinates and element
connectivity), per-element material data (sigma_t, sigma_s, q) and the seeded
element picks used by the finite-difference gradient check.  It holds none of
the method's arithmetic (no quadrature, no element matrices, no solver), so both
the GPU path and the CPU oracle may use it.

The paper's own meshes (deal.II/p4est structured grids, Gmsh and zmesh
unstructured grids) are not available; these synthetic unit-cube meshes stand
in for them (Sec. "pAIR Performance for Transport" and the weak-scaling section
use structured and unstructured unit-cube style meshes with piecewise-constant
cross sections).

Conventions
-----------
Structured hex mesh: element e = i + nx*(j + ny*k); local node
a = ax + 2*ay + 4*az sits at (x_i + ax*hx, y_j + ay*hy, z_k + az*hz);
DOF = 8*e + a.

Tet mesh: each cube (i, j, k) of an n^3 grid is split into the 6 Kuhn tets;
tet t = 6*cube + p, where p enumerates the axis permutations pi in
lexicographic order; its vertices are v0 = cube corner (0,0,0),
v1 = v0 + e_pi0, v2 = v1 + e_pi1, v3 = corner (1,1,1).  Global vertices are
the (n+1)^3 grid points, lexicographic with x fastest.  DOF = 4*t + a where a
indexes the element's vertex list.
"""
from __future__ import annotations

import dataclasses
import itertools
import math
from typing import Optional

import numpy as np

HEX = 0
TET = 1

# axis permutations in lexicographic order (Kuhn split of a cube into 6 tets)
KUHN_PERMS = list(itertools.permutations(range(3)))


@dataclasses.dataclass
class Mesh:
    kind: int                      # HEX or TET
    n_elem: int
    nodes_per_elem: int            # 8 or 4
    # structured hex description (kind == HEX)
    nx: int = 0
    ny: int = 0
    nz: int = 0
    lo: tuple = (0.0, 0.0, 0.0)
    hi: tuple = (1.0, 1.0, 1.0)
    # unstructured tet description (kind == TET)
    xyz: Optional[np.ndarray] = None        # [n_vert, 3] float64
    elem_vert: Optional[np.ndarray] = None  # [n_elem, 4] int32

    @property
    def n_dof(self) -> int:
        return self.n_elem * self.nodes_per_elem

    def centroids(self) -> np.ndarray:
        """Element centroids [n_elem, 3] (used to place boxes of material/source)."""
        if self.kind == HEX:
            h = [(self.hi[d] - self.lo[d]) / n for d, n in enumerate((self.nx, self.ny, self.nz))]
            i = np.arange(self.nx)
            j = np.arange(self.ny)
            k = np.arange(self.nz)
            K, J, I = np.meshgrid(k, j, i, indexing="ij")
            c = np.stack([self.lo[0] + (I + 0.5) * h[0],
                          self.lo[1] + (J + 0.5) * h[1],
                          self.lo[2] + (K + 0.5) * h[2]], axis=-1)
            return c.reshape(-1, 3)
        return self.xyz[self.elem_vert].mean(axis=1)

    def hex_vertices(self) -> tuple[np.ndarray, np.ndarray]:
        """Explicit vertex list and [E,8] connectivity of a structured hex mesh
        (local node a = ax + 2ay + 4az)."""
        assert self.kind == HEX
        nx, ny, nz = self.nx, self.ny, self.nz
        xs = np.linspace(self.lo[0], self.hi[0], nx + 1)
        ys = np.linspace(self.lo[1], self.hi[1], ny + 1)
        zs = np.linspace(self.lo[2], self.hi[2], nz + 1)
        Z, Y, X = np.meshgrid(zs, ys, xs, indexing="ij")
        xyz = np.stack([X, Y, Z], axis=-1).reshape(-1, 3)
        vid = lambda i, j, k: i + (nx + 1) * (j + (ny + 1) * k)
        ev = np.empty((self.n_elem, 8), dtype=np.int32)
        K, J, I = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
        I, J, K = I.ravel(), J.ravel(), K.ravel()
        for a in range(8):
            ax, ay, az = a & 1, (a >> 1) & 1, (a >> 2) & 1
            ev[:, a] = vid(I + ax, J + ay, K + az)
        return xyz, ev


def hex_mesh(nx: int, ny: Optional[int] = None, nz: Optional[int] = None,
             lo=(0.0, 0.0, 0.0), hi=(1.0, 1.0, 1.0)) -> Mesh:
    ny = nx if ny is None else ny
    nz = nx if nz is None else nz
    return Mesh(kind=HEX, n_elem=nx * ny * nz, nodes_per_elem=8, nx=nx, ny=ny, nz=nz,
                lo=tuple(float(v) for v in lo), hi=tuple(float(v) for v in hi))


def kuhn_tet_mesh(n: int, jitter: float = 0.0, seed: Optional[int] = None) -> Mesh:
    """Unit cube split into n^3 cubes, 6 Kuhn tets each; interior vertices moved
    by U(-jitter*h, +jitter*h) per coordinate (one draw per interior vertex and
    coordinate, in vertex order, from numpy's PCG64 with ``seed``)."""
    h = 1.0 / n
    g = np.arange(n + 1) * h
    Z, Y, X = np.meshgrid(g, g, g, indexing="ij")
    xyz = np.stack([X, Y, Z], axis=-1).reshape(-1, 3).copy()
    if jitter > 0.0:
        rng = np.random.default_rng(seed)
        idx = np.stack(np.meshgrid(np.arange(n + 1), np.arange(n + 1), np.arange(n + 1),
                                   indexing="ij"), axis=-1).reshape(-1, 3)[:, ::-1]
        interior = np.all((idx > 0) & (idx < n), axis=1)
        nint = int(interior.sum())
        d = rng.uniform(-jitter * h, jitter * h, size=(nint, 3))
        xyz[interior] += d
    vid = lambda i, j, k: i + (n + 1) * (j + (n + 1) * k)
    K, J, I = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    I, J, K = I.ravel(), J.ravel(), K.ravel()
    ncube = n ** 3
    ev = np.empty((ncube, 6, 4), dtype=np.int32)
    for p, perm in enumerate(KUHN_PERMS):
        c = [np.zeros_like(I), np.zeros_like(I), np.zeros_like(I)]
        ev[:, p, 0] = vid(I, J, K)
        for s in range(2):
            c[perm[s]] = c[perm[s]] + 1
            ev[:, p, s + 1] = vid(I + c[0], J + c[1], K + c[2])
        ev[:, p, 3] = vid(I + 1, J + 1, K + 1)
    ev = ev.reshape(-1, 4)
    return Mesh(kind=TET, n_elem=ev.shape[0], nodes_per_elem=4, xyz=xyz, elem_vert=ev)


@dataclasses.dataclass
class Materials:
    sigma_t: np.ndarray  # [E]
    sigma_s: np.ndarray  # [E]
    q: np.ndarray        # [E]


def log_uniform(n: int, a: float, b: float, seed: int) -> np.ndarray:
    """One draw per element, in element order: exp(U(ln a, ln b)) (PCG64)."""
    rng = np.random.default_rng(seed)
    return np.exp(rng.uniform(math.log(a), math.log(b), size=n))


def in_box(c: np.ndarray, lo, hi) -> np.ndarray:
    lo = np.asarray(lo)
    hi = np.asarray(hi)
    return np.all((c >= lo) & (c <= hi), axis=1)


@dataclasses.dataclass
class Workload:
    name: str
    mesh: Mesh
    mats: Materials
    sn_order: int                 # level-symmetric S_N order (2, 4, 8)
    mode: str = "plain"           # "plain" (one direction at a time) or "batched"
    detector: Optional[np.ndarray] = None   # bool [E] (adjoint functional J)
    fd_elems: Optional[np.ndarray] = None   # int [16] (FD check elements)
    seeds: dict = dataclasses.field(default_factory=dict)

    @property
    def n_dir(self) -> int:
        n = self.sn_order
        return n * (n + 2)

    @property
    def dof_per_dir(self) -> int:
        return self.mesh.n_dof


# ---------------------------------------------------------------------------
# The five workloads (sizes, value distributions and seeds).  ``scale`` replaces
# the element count per axis to give a small version of the same recipe.
# ---------------------------------------------------------------------------

DEFAULT_N = {1: 8, 2: 64, 3: 48, 4: 32, 5: 32}


def make_config(i: int, scale: Optional[int] = None) -> Workload:
    n = DEFAULT_N[i] if scale is None else int(scale)
    if i == 1:
        mesh = hex_mesh(n)
        E = mesh.n_elem
        mats = Materials(np.full(E, 1.0), np.full(E, 0.5), np.full(E, 1.0))
        return Workload("hex%d^3-S2-uniform" % n, mesh, mats, 2)
    if i == 2:
        mesh = hex_mesh(n)
        E = mesh.n_elem
        st = log_uniform(E, 0.1, 10.0, seed=2)
        q = in_box(mesh.centroids(), (0.25,) * 3, (0.75,) * 3).astype(np.float64)
        return Workload("hex%d^3-S8-loguniform" % n, mesh, Materials(st, 0.9 * st, q), 8,
                        seeds={"sigma": 2})
    if i == 3:
        mesh = kuhn_tet_mesh(n, jitter=0.2, seed=303)
        E = mesh.n_elem
        st = log_uniform(E, 0.1, 10.0, seed=3)
        return Workload("tet%d^3x6-S4-loguniform" % n, mesh,
                        Materials(st, 0.5 * st, np.ones(E)), 4,
                        seeds={"jitter": 303, "sigma": 3})
    if i == 4:
        mesh = hex_mesh(n)
        E = mesh.n_elem
        b = max(1, n // 4)   # 8^3-element blocks at n = 32
        I = np.arange(E) % n
        J = (np.arange(E) // n) % n
        K = np.arange(E) // (n * n)
        even = ((I // b + J // b + K // b) % 2) == 0
        st = np.where(even, 1.0, 10.0)
        c = np.where(even, 0.99, 0.5)
        return Workload("hex%d^3-S8-checkerboard" % n, mesh,
                        Materials(st, c * st, np.ones(E)), 8, mode="batched")
    if i == 5:
        mesh = hex_mesh(n)
        E = mesh.n_elem
        st = log_uniform(E, 0.5, 5.0, seed=5)
        cen = mesh.centroids()
        q = in_box(cen, (0.0,) * 3, (0.25,) * 3).astype(np.float64)
        det = in_box(cen, (0.75,) * 3, (1.0,) * 3)
        fd = fd_elements(mesh, seed=505)
        return Workload("hex%d^3-S4-adjoint" % n, mesh, Materials(st, 0.8 * st, q), 4,
                        detector=det, fd_elems=fd, seeds={"sigma": 5, "fd": 505})
    raise ValueError("unknown workload %r" % (i,))


def fd_elements(mesh: Mesh, seed: int, count: int = 16) -> np.ndarray:
    """Seeded element picks for the gradient check: half drawn uniformly over all
    elements, half from the elements on the main diagonal between the source box
    and the detector box (where the gradient is well above roundoff)."""
    rng = np.random.default_rng(seed)
    E = mesh.n_elem
    half = count // 2
    uni = rng.choice(E, size=half, replace=False)
    n = mesh.nx
    diag = np.array([d + n * (d + n * d) for d in range(n)])
    c = mesh.centroids()[diag]
    mid = diag[np.all((c > 0.25) & (c < 0.75), axis=1)]
    pool = np.setdiff1d(mid, uni)
    pick = rng.choice(pool, size=min(half, pool.size), replace=False)
    return np.concatenate([uni, pick]).astype(np.int64)
