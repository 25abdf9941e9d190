"""Pins of the oracle's source iteration: the dense coupled block system of
Sec. "Accuracy of Spatial Solves", particle balance, cube symmetry, and the
O(h^2) rates of two closed-form solutions (pure absorber; the Appendix MMS)."""
import itertools
import math

import numpy as np
import pytest

from paper_1910_11463_amd import workloads as wl
from oracle import dg, mms, quadrature as Q, source_iteration as si


@pytest.mark.parametrize("mesh", [wl.hex_mesh(2), wl.kuhn_tet_mesh(1, jitter=0.0)])
def test_source_iteration_matches_dense_coupled_system(mesh):
    E = mesh.n_elem
    rng = np.random.default_rng(2)
    st = rng.uniform(0.5, 2.0, E)
    om, w = Q.level_symmetric(4)
    prob = si.Problem(mesh, st, 0.7 * st, rng.uniform(0, 1, E), om, w)
    phi_d, psi_d = si.dense_coupled_solve(prob)
    r = si.source_iteration(prob, tol=1e-14)
    assert np.abs(r.phi - phi_d).max() <= 1e-12 * np.abs(phi_d).max()
    assert np.abs(r.psi - psi_d).max() <= 1e-12 * np.abs(psi_d).max()


def _leakage(prob, psi):
    """sum_m w_m int_{outflow boundary} psi_m Omega.n."""
    topo = prob.topo
    tot = 0.0
    for m in range(prob.M):
        b = prob.blocks(m)
        p = psi[m].reshape(topo.E, topo.k)
        for f in range(topo.F):
            sel = (b.odn[:, f] > 0) & (topo.nbr[:, f] < 0)
            if not np.any(sel):
                continue
            Fm = dg._face_mass_e(topo, f, sel)
            tot += prob.w[m] * np.sum(b.odn[sel, f] * np.einsum("eab,eb->e", Fm, p[sel]))
    return tot


@pytest.mark.parametrize("mesh", [wl.hex_mesh(3), wl.kuhn_tet_mesh(2, jitter=0.2, seed=4)])
def test_particle_balance(mesh):
    E = mesh.n_elem
    rng = np.random.default_rng(9)
    st = rng.uniform(0.5, 2.0, E)
    ss = 0.6 * st
    q = rng.uniform(0, 1, E)
    om, w = Q.level_symmetric(4)
    prob = si.Problem(mesh, st, ss, q, om, w)
    r = si.source_iteration(prob, tol=1e-14)
    topo = prob.topo
    phi = r.phi.reshape(E, topo.k)
    absorb = np.sum((st - ss) * np.einsum("eab,eb->e", topo.mass, phi))
    src = np.sum(q * topo.vol)
    assert abs(_leakage(prob, r.psi) + absorb - src) <= 1e-12 * src


def test_cube_symmetry_of_uniform_problem():
    """Uniform material, S4: phi is invariant under the 48 symmetries of the cube."""
    n = 3
    mesh = wl.hex_mesh(n)
    E = mesh.n_elem
    om, w = Q.level_symmetric(4)
    prob = si.Problem(mesh, np.ones(E), 0.5 * np.ones(E), np.ones(E), om, w)
    phi = si.source_iteration(prob, tol=1e-14).phi
    e = np.arange(E)
    cell = np.stack([e % n, (e // n) % n, e // (n * n)], axis=1)
    for perm in itertools.permutations(range(3)):
        for flips in itertools.product((0, 1), repeat=3):
            mapped = np.empty_like(phi)
            for a in range(8):
                corner = np.array([(a >> d) & 1 for d in range(3)])
                c2 = cell[:, perm].copy()
                k2 = corner[list(perm)].copy()
                for d in range(3):
                    if flips[d]:
                        c2[:, d] = n - 1 - c2[:, d]
                        k2[d] = 1 - k2[d]
                e2 = c2[:, 0] + n * (c2[:, 1] + n * c2[:, 2])
                a2 = k2[0] + 2 * k2[1] + 4 * k2[2]
                mapped[8 * e + a] = phi[8 * e2 + a2]
            assert np.abs(mapped - phi).max() <= 1e-13 * np.abs(phi).max()


def test_pure_absorber_second_order():
    """sigma_s = q = 0 with inflow g = exp(-sigma Omega.r): exact psi = exp(-sigma Omega.r)."""
    sig = 2.0
    o = np.array([[0.3, 0.5, math.sqrt(1 - 0.34)]])
    errs = []
    for n in (4, 8, 16):
        mesh = wl.hex_mesh(n)
        E = mesh.n_elem
        prob = si.Problem(mesh, np.full(E, sig), np.zeros(E), np.zeros(E), o,
                          np.array([4 * math.pi]), inflow=lambda p, om: np.exp(-sig * (p @ om)))
        psi = si.transport_sweep(prob, None)[0]
        errs.append(mms.hex_l2_error(prob.topo, psi, lambda p: np.exp(-sig * (p @ o[0]))))
    rates = [math.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert min(rates) > 1.9, rates


def test_manufactured_solution_second_order():
    om, w = Q.level_symmetric(4)
    st, ss = 1.0, 0.5
    errs = []
    for n in (4, 8):
        mesh = wl.hex_mesh(n)
        E = mesh.n_elem
        prob = si.Problem(mesh, np.full(E, st), np.full(E, ss), np.zeros(E), om, w)
        prob.ext = mms.hex_projected_source(prob.topo, om, st, ss)
        phi = si.source_iteration(prob, tol=1e-12).phi
        errs.append(mms.hex_l2_error(prob.topo, phi, lambda p: 4 * math.pi * mms.Phi(p)))
    assert math.log2(errs[0] / errs[1]) > 1.9, errs


def _absorber(mesh, sig, o, nodal=False):
    E = mesh.n_elem
    g = lambda p, om: np.exp(-sig * (p @ om))
    prob = si.Problem(mesh, np.full(E, sig), np.zeros(E), np.zeros(E), o[None, :],
                      np.array([4 * math.pi]), inflow=None if nodal else g)
    if nodal:
        prob.inflow_nodal = g(dg.node_coordinates(prob.topo), o)
    return prob, si.transport_sweep(prob, None)[0]


@pytest.mark.parametrize("nodal", [False, True])
def test_pure_absorber_second_order_tets(nodal):
    """P1 tets (Kuhn split, jittered): the pure absorber with inflow
    g = exp(-sigma Omega.r) has exact psi = exp(-sigma Omega.r); the L2 error
    falls as h^2, with the inflow integrated exactly (5-point-per-axis rule)
    and with its nodal interpolant on each face."""
    sig = 1.5
    o = np.array([0.3, -0.5, math.sqrt(1 - 0.34)])
    errs = []
    for n in (4, 8, 16):
        mesh = wl.kuhn_tet_mesh(n, jitter=0.15, seed=7)
        prob, psi = _absorber(mesh, sig, o, nodal)
        errs.append(mms.tet_l2_error(prob.topo, psi, lambda p: np.exp(-sig * (p @ o))))
    rates = [math.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert min(rates) > 1.85, (rates, errs)


@pytest.mark.parametrize("kind", ["hex", "tet"])
def test_nodal_inflow_equals_exact_integration_for_face_polynomials(kind):
    """The nodal-interpolant inflow term equals the quadrature-integrated one
    when g is itself in the face space: multilinear on hex faces (any
    trilinear g), linear on tet faces (any affine g)."""
    mesh = wl.hex_mesh(3, 4, 2) if kind == "hex" else wl.kuhn_tet_mesh(3, jitter=0.2, seed=3)
    E = mesh.n_elem
    om, w = Q.level_symmetric(4)
    prob = si.Problem(mesh, np.ones(E), np.zeros(E), np.zeros(E), om, w)
    if kind == "hex":
        g = lambda p: 1.0 + 0.5 * p[:, 0] - 2.0 * p[:, 1] + 0.7 * p[:, 2] + 3.0 * p[:, 0] * p[:, 1] \
            - 1.1 * p[:, 1] * p[:, 2] + 0.4 * p[:, 0] * p[:, 2] + 2.5 * p[:, 0] * p[:, 1] * p[:, 2]
    else:
        g = lambda p: 1.0 + 0.5 * p[:, 0] - 2.0 * p[:, 1] + 0.7 * p[:, 2]
    gn = g(dg.node_coordinates(prob.topo))
    for m in range(prob.M):
        b = prob.blocks(m)
        exact = dg.inflow_rhs(prob.topo, b, g)
        nodal = dg.inflow_rhs_nodal(prob.topo, b, gn)
        assert np.abs(exact).max() > 0.0
        assert np.abs(nodal - exact).max() <= 1e-13 * np.abs(exact).max(), m


def test_inflow_term_is_the_boundary_flux():
    """Summed over the test functions (sum_a phi_a = 1), the inflow term is
    -int_{Gamma^-} (Omega.n) g: for g = 1 on a unit cube that is the
    projected area of the cube along Omega, sum_d |Omega_d| (hexes and tets)."""
    om, w = Q.level_symmetric(8)
    for mesh in (wl.hex_mesh(3), wl.kuhn_tet_mesh(3, jitter=0.2, seed=5)):
        E = mesh.n_elem
        prob = si.Problem(mesh, np.ones(E), np.zeros(E), np.zeros(E), om, w)
        for m in (0, 17, 43):
            f = dg.inflow_rhs(prob.topo, prob.blocks(m), lambda p: np.ones(p.shape[0]))
            assert abs(f.sum() - np.abs(om[m]).sum()) <= 1e-13
