"""Inflow boundary data (pair_set_inflow: the Gamma^- term of eq.
weak_form_transport) on the GPU against the oracle's nodal-interpolant inflow
term and against the pure absorber's closed form, plus the reported
per-level statistics and the autograd state check."""
import math

import numpy as np
import pytest

from paper_1910_11463_amd import binding as B
from paper_1910_11463_amd import workloads as wl
from tests.gpu_util import need_gpu, rel

pytestmark = pytest.mark.gpu

TIGHT = dict(tol_inner=1e-12, max_inner=200)


def _nodes(mesh):
    from oracle import dg
    return dg.node_coordinates(dg.topology(mesh))


def _solver(mesh, om, w, sig, **opts):
    from paper_1910_11463_amd.solver import Solver
    s = Solver(**opts)
    s.set_mesh(mesh)
    s.set_quadrature(om, w)
    E = mesh.n_elem
    s.set_materials(np.full(E, sig), np.zeros(E), np.zeros(E))
    return s


@pytest.mark.parametrize("kind,mode", [("hex", B.PAIR_BATCHED), ("hex", B.PAIR_PLAIN),
                                       ("tet", B.PAIR_BATCHED)])
def test_inflow_sweep_matches_oracle(kind, mode):
    """Every direction its own inflow g_m = exp(-sigma Omega_m.r) (set one
    direction at a time), sigma_s = q = 0: psi of one sweep replacement vs the
    oracle's exact sweep with the same nodal inflow data."""
    need_gpu()
    from oracle import quadrature as Q, source_iteration as si
    mesh = wl.hex_mesh(5, 4, 6) if kind == "hex" else wl.kuhn_tet_mesh(4, jitter=0.2, seed=11)
    print("inflow parity", kind, mode, flush=True)
    om, w = Q.level_symmetric(4)
    sig = 1.3
    X = _nodes(mesh)
    G = np.stack([np.exp(-sig * (X @ om[m])) for m in range(om.shape[0])])
    E = mesh.n_elem
    prob = si.Problem(mesh, np.full(E, sig), np.zeros(E), np.zeros(E), om, w, inflow_nodal=G)
    ref = si.transport_sweep(prob, None)
    s = _solver(mesh, om, w, sig, relax_pre="FC", relax_post="FC", **TIGHT)
    for m in range(om.shape[0]):
        s.set_inflow(G[m], m)
    psi, phi, st, rc = s.transport_sweep(mode=mode)
    assert rc == B.PAIR_OK
    for m in range(om.shape[0]):
        assert rel(psi[m], ref[m]) <= 1e-9, (m, rel(psi[m], ref[m]))
    s.close()


def test_inflow_broadcast_clear_and_errors():
    torch = need_gpu()
    from paper_1910_11463_amd.solver import Solver
    from oracle import quadrature as Q, source_iteration as si
    mesh = wl.hex_mesh(4)
    om, w = Q.level_symmetric(2)
    s = Solver(**TIGHT)
    s.set_mesh(mesh)
    with pytest.raises(B.PairError) as e:          # no quadrature yet
        s.set_inflow(np.ones(mesh.n_dof))
    assert e.value.code == B.PAIR_E_STATE
    s.set_quadrature(om, w)
    E = mesh.n_elem
    s.set_materials(np.full(E, 2.0), np.zeros(E), np.zeros(E))
    with pytest.raises(B.PairError) as e:
        s.set_inflow(np.ones(mesh.n_dof), m=8)
    assert e.value.code == B.PAIR_E_INVALID
    # the same g for every direction, from device memory
    g = 1.0 + _nodes(mesh)[:, 0]
    s.set_inflow(torch.tensor(g, device="cuda"), -1)
    psi, _, _, rc = s.transport_sweep()
    assert rc == B.PAIR_OK
    prob = si.Problem(mesh, np.full(E, 2.0), np.zeros(E), np.zeros(E), om, w, inflow_nodal=g)
    assert rel(psi, si.transport_sweep(prob, None)) <= 1e-9
    # vacuum again for direction 3 only, then for all
    s.set_inflow(None, 3)
    psi, _, _, _ = s.transport_sweep()
    assert np.abs(psi[3]).max() == 0.0 and np.abs(psi[2]).max() > 0.0
    s.set_inflow(None, -1)
    psi, _, _, _ = s.transport_sweep()
    assert np.abs(psi).max() == 0.0
    s.close()


def test_pure_absorber_second_order_on_the_gpu():
    """One direction with weight 4 pi: psi = exp(-sigma Omega.r) from the nodal
    inflow data; the L2 error against the closed form falls as h^2."""
    need_gpu()
    from oracle import dg, mms
    sig = 2.0
    o = np.array([[0.3, 0.5, math.sqrt(1 - 0.34)]])
    errs = []
    for n in (8, 16, 32):
        mesh = wl.hex_mesh(n)
        s = _solver(mesh, o, np.array([4 * math.pi]), sig, relax_pre="FC", relax_post="FC", **TIGHT)
        s.set_inflow(np.exp(-sig * (_nodes(mesh) @ o[0])), 0)
        psi, _, _, rc = s.transport_sweep()
        assert rc == B.PAIR_OK
        topo = dg.topology(mesh)
        errs.append(mms.hex_l2_error(topo, psi[0], lambda p: np.exp(-sig * (p @ o[0]))))
        s.close()
    rates = [math.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert min(rates) > 1.9, (rates, errs)


@pytest.mark.parametrize("mode", [B.PAIR_BATCHED, B.PAIR_PLAIN])
def test_level_statistics_are_direction_zeros(mode):
    """level_n / level_nnz report direction 0's hierarchy: on the finest level
    its rows N and the entries of its exported operator, whatever the batch."""
    need_gpu()
    from paper_1910_11463_amd.solver import Solver
    w = wl.make_config(2, scale=6)
    s = Solver(batch_size=8, relax_pre="FC", relax_post="FC", **TIGHT)
    s.set_mesh(w.mesh)
    om, wt = Solver.level_symmetric(4)
    s.set_quadrature(om, wt)
    s.set_materials(w.mats.sigma_t, w.mats.sigma_s, w.mats.q)
    _, _, st, rc = s.transport_sweep(mode=mode)
    assert rc == B.PAIR_OK
    rp, col, val, _ = s.export_fine_operator(0)
    assert st["level_n"][0] == w.mesh.n_dof
    assert st["level_nnz"][0] == col.shape[0]
    nl = sum(1 for x in st["level_n"] if x > 0)
    assert nl >= 2
    assert all(st["level_nnz"][l] >= st["level_n"][l] for l in range(nl))
    assert all(st["level_n"][l + 1] < st["level_n"][l] for l in range(nl - 1))
    s.close()


def test_autograd_refuses_a_changed_solver():
    """Backward of a first forward after a second forward on the same solver
    would use the second forward's state: it must raise, not return a wrong
    gradient."""
    torch = need_gpu()
    from paper_1910_11463_amd.solver import TransportSolve
    from tests.gpu_util import solver_for
    w = wl.make_config(5, scale=3)
    s = solver_for(w, tol_inner=1e-12, tol_outer=1e-12, outer_estimate=1, max_inner=200)
    s.q = torch.tensor(w.mats.q, device="cuda")
    st1 = torch.tensor(w.mats.sigma_t, device="cuda", requires_grad=True)
    ss1 = torch.tensor(w.mats.sigma_s, device="cuda", requires_grad=True)
    phi1 = TransportSolve.apply(s, st1, ss1)
    st2 = torch.tensor(1.1 * w.mats.sigma_t, device="cuda", requires_grad=True)
    phi2 = TransportSolve.apply(s, st2, ss1)
    with pytest.raises(RuntimeError, match="another solve"):
        phi1.sum().backward()
    phi2.sum().backward()            # the latest forward still differentiates
    assert torch.isfinite(st2.grad).all()
    s.close()
