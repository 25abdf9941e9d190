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


def test_stored_central_differences_agree_with_the_oracle_adjoint():
    """The stored central differences of the 32^3 S4 workload (written by
    tests/golden/make_c5_fd.py with the compiled exact sweep) against the
    oracle's adjoint gradients computed here with the NumPy assembly and
    source iteration: two independent routes to dJ/dsigma on 16 elements."""
    import os
    from paper_1910_11463_amd import workloads as wl
    from oracle import adjoint as ADJ, quadrature as Q, source_iteration as si
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "c5_fd_gradients.txt")
    rows = [l.split() for l in open(path) if l.strip() and not l.startswith("#")]
    e = np.array([int(r[0]) for r in rows])
    fdt = np.array([float(r[1]) for r in rows])
    fds = np.array([float(r[2]) for r in rows])
    w = wl.make_config(5)
    assert np.array_equal(e, w.fd_elems)
    om, wt = Q.level_symmetric(w.sn_order)
    prob = si.Problem(w.mesh, w.mats.sigma_t, w.mats.sigma_s, w.mats.q, om, wt)
    threads = os.cpu_count() or 1
    fwd = si.source_iteration(prob, tol=1e-14, threads=threads)
    c = ADJ.detector_source(prob, w.detector)
    adj = si.source_iteration(ADJ.adjoint_problem(prob, c), tol=1e-14, threads=threads)
    gt, gs = ADJ.gradients(prob, fwd.psi, fwd.phi, adj.psi, adj.phi, w.sn_order)
    assert np.linalg.norm(gt[e] - fdt) <= 1e-5 * np.linalg.norm(fdt)
    assert np.linalg.norm(gs[e] - fds) <= 1e-5 * np.linalg.norm(fds)
