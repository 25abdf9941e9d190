"""Pins of the oracle's adjoint gradients: the transposed dense coupled system
and central finite differences of J on small meshes."""
import numpy as np
import pytest

from paper_1910_11463_amd import workloads as wl
from oracle import adjoint as ADJ, quadrature as Q, source_iteration as si


@pytest.mark.parametrize("kind,order", [("hex", 2), ("hex", 4), ("tet", 2)])
def test_adjoint_matches_dense_adjoint_and_fd(kind, order):
    mesh = wl.hex_mesh(2) if kind == "hex" else wl.kuhn_tet_mesh(1, jitter=0.0)
    E = mesh.n_elem
    rng = np.random.default_rng(order)
    st = rng.uniform(0.5, 2.0, E)
    ss = 0.8 * st
    q = np.zeros(E)
    q[0] = 1.0
    om, w = Q.level_symmetric(order)
    prob = si.Problem(mesh, st, ss, q, om, w)
    det = np.zeros(E, dtype=bool)
    det[-1] = True
    J, gt, gs = ADJ.adjoint_gradients(prob, det, order)
    J2, gt2, gs2 = ADJ.dense_adjoint_gradients(prob, det)
    assert abs(J - J2) <= 1e-12 * abs(J2)
    assert np.abs(gt - gt2).max() <= 1e-10 * np.abs(gt2).max()
    assert np.abs(gs - gs2).max() <= 1e-10 * np.abs(gs2).max()
    h = 1e-6
    fd_t, fd_s = [], []
    c = ADJ.detector_source(prob, det)
    for e in range(E):
        vals = []
        for which in ("t", "s"):
            for sgn in (1, -1):
                st2, ss2 = st.copy(), ss.copy()
                (st2 if which == "t" else ss2)[e] += sgn * h
                phi, _ = si.dense_coupled_solve(si.Problem(mesh, st2, ss2, q, om, w))
                vals.append(c @ phi)
        fd_t.append((vals[0] - vals[1]) / (2 * h))
        fd_s.append((vals[2] - vals[3]) / (2 * h))
    assert np.linalg.norm(np.array(fd_t) - gt) <= 1e-7 * np.linalg.norm(fd_t)
    assert np.linalg.norm(np.array(fd_s) - gs) <= 1e-7 * np.linalg.norm(fd_s)
