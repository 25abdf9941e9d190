"""Pins of the oracle's DG operator and exact sweep: brute-force dense LU, the
transpose identity A(-Omega) = A(Omega)^T, and block scaling."""
import numpy as np
import pytest

from paper_1910_11463_amd import workloads as wl
from oracle import dg, quadrature as Q, sweep as SW, source_iteration as si


def _meshes():
    return [wl.hex_mesh(1), wl.hex_mesh(2), wl.hex_mesh(3, 2, 2, hi=(1.0, 0.5, 2.0)),
            wl.kuhn_tet_mesh(2), wl.kuhn_tet_mesh(2, jitter=0.2, seed=11)]


@pytest.mark.parametrize("mi", range(5))
def test_sweep_equals_dense_lu(mi):
    mesh = _meshes()[mi]
    E = mesh.n_elem
    rng = np.random.default_rng(mi)
    st = rng.uniform(0.1, 3.0, E)
    om, w = Q.level_symmetric(4)
    prob = si.Problem(mesh, st, 0.5 * st, np.ones(E), om, w)
    for m in range(0, om.shape[0], 5):
        b = prob.blocks(m)
        f = prob.rhs(m, rng.uniform(0, 1, prob.N))
        A = dg.unscaled_csr(prob.topo, b).toarray()
        x = np.linalg.solve(A, f.ravel())
        psi = SW.sweep(b, f).ravel()
        assert np.abs(psi - x).max() <= 1e-13 * np.abs(x).max()


@pytest.mark.parametrize("mi", range(5))
def test_transpose_identity(mi):
    mesh = _meshes()[mi]
    E = mesh.n_elem
    st = np.random.default_rng(mi).uniform(0.1, 3.0, E)
    om, w = Q.level_symmetric(8)
    prob = si.Problem(mesh, st, st, st, om, w)
    for m in range(0, 80, 7):
        A = dg.unscaled_csr(prob.topo, prob.blocks(m)).toarray()
        B = dg.unscaled_csr(prob.topo, prob.blocks(Q.reflected_index(8, m))).toarray()
        assert np.abs(B - A.T).max() <= 1e-14 * np.abs(A).max()


def test_sweep_with_cycles_equals_dense():
    """A synthetic block system whose dependency graph has cycles (as can
    happen on unstructured meshes) is still solved exactly."""
    rng = np.random.default_rng(3)
    E, k, F = 9, 4, 3
    D = rng.normal(size=(E, k, k)) + 4 * np.eye(k)
    nbr = np.full((E, F), -1, dtype=np.int64)
    # 0->1->2->0 cycle, 3 depends on the cycle, 4<->5 two-cycle, 6..8 a chain
    edges = {0: [2], 1: [0], 2: [1], 3: [0, 2], 4: [5], 5: [4, 3], 6: [], 7: [6], 8: [7, 5]}
    for e, us in edges.items():
        for f, u in enumerate(us):
            nbr[e, f] = u
    Cpl = rng.normal(size=(E, F, k, k)) * (nbr[..., None, None] >= 0)
    rhs = rng.normal(size=(E, k))
    A = np.zeros((E * k, E * k))
    for e in range(E):
        A[e * k:e * k + k, e * k:e * k + k] = D[e]
        for f in range(F):
            if nbr[e, f] >= 0:
                u = nbr[e, f]
                A[e * k:e * k + k, u * k:u * k + k] += Cpl[e, f]
    x = np.linalg.solve(A, rhs.ravel())
    psi, ncyc = SW.sweep_raw(D, nbr, Cpl, rhs)
    assert ncyc == 2
    assert np.abs(psi.ravel() - x).max() <= 1e-12 * np.abs(x).max()


@pytest.mark.parametrize("mi", [1, 4])
def test_scaled_matrix(mi):
    """D^{-1} A: exact unit diagonal, structural pattern, and the same action as
    D^{-1} applied to A x."""
    mesh = _meshes()[mi]
    E = mesh.n_elem
    st = np.random.default_rng(5).uniform(0.1, 3.0, E)
    om, w = Q.level_symmetric(4)
    prob = si.Problem(mesh, st, st, st, om, w)
    b = prob.blocks(3)
    As = dg.scaled_csr(prob.topo, b)
    A = dg.unscaled_csr(prob.topo, b)
    assert np.all(As.diagonal() == 1.0)
    x = np.random.default_rng(1).normal(size=prob.N)
    k = prob.topo.k
    y = np.einsum("eab,eb->ea", np.linalg.inv(b.D), (A @ x).reshape(E, k)).ravel()
    assert np.abs(As @ x - y).max() <= 1e-13 * np.abs(y).max()
    # each row: unit diagonal + (#inflow interior faces) * (face nodes) entries
    nin = (b.nbr >= 0).sum(axis=1)
    nf = 4 if mesh.kind == 0 else 3
    assert np.array_equal(np.diff(As.indptr), np.repeat(1 + nf * nin, k))
