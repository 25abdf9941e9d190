"""GPU adjoint gradients (transposed solves through the reflected directions'
pAIR hierarchies) against the oracle's adjoint, the dense transposed system and
central finite differences, and the autograd wrapper."""
import numpy as np
import pytest

from paper_1910_11463_amd import binding as B
from paper_1910_11463_amd import workloads as wl
from tests.gpu_util import need_gpu, oracle_problem, rel, solver_for

pytestmark = pytest.mark.gpu

TIGHT = dict(tol_inner=1e-12, tol_outer=1e-13, outer_estimate=1, max_inner=200)


def _detector_c(w, prob):
    from oracle import adjoint as ADJ
    return ADJ.detector_source(prob, w.detector)


@pytest.mark.parametrize("scale,mode", [(4, B.PAIR_PLAIN), (6, B.PAIR_BATCHED)])
def test_adjoint_matches_oracle(scale, mode):
    need_gpu()
    from oracle import adjoint as ADJ
    w = wl.make_config(5, scale=scale)
    print("adjoint", w.name, mode, flush=True)
    prob = oracle_problem(w)
    c = _detector_c(w, prob)
    J, gt_ref, gs_ref = ADJ.adjoint_gradients(prob, w.detector, w.sn_order, tol=1e-14)
    s = solver_for(w, **TIGHT)
    phi, _, st, rc = s.solve(mode=mode)
    assert rc == B.PAIR_OK
    assert abs(float(c @ phi) - J) <= 1e-10 * abs(J)
    gt, gs, phia, st2, rc2 = s.adjoint(c, mode=mode)
    assert rc2 == B.PAIR_OK
    assert rel(gt, gt_ref) <= 1e-8, rel(gt, gt_ref)
    assert rel(gs, gs_ref) <= 1e-8, rel(gs, gs_ref)
    s.close()


def test_adjoint_matches_dense_adjoint_tiny():
    need_gpu()
    from oracle import adjoint as ADJ
    w = wl.make_config(5, scale=2)
    prob = oracle_problem(w)
    J, gt_ref, gs_ref = ADJ.dense_adjoint_gradients(prob, w.detector)
    s = solver_for(w, **TIGHT)
    s.solve()
    gt, gs, _, _, rc = s.adjoint(_detector_c(w, prob))
    assert rc == B.PAIR_OK
    assert rel(gt, gt_ref) <= 1e-10
    assert rel(gs, gs_ref) <= 1e-10
    s.close()


def test_adjoint_central_differences():
    """Central differences (step 1e-6) of J computed with the oracle's exact
    sweep against the GPU gradient on seeded elements (the workload's
    gradient-check picks at a reduced mesh)."""
    need_gpu()
    from oracle import source_iteration as si
    w = wl.make_config(5, scale=6)
    prob = oracle_problem(w)
    c = _detector_c(w, prob)
    s = solver_for(w, **TIGHT)
    s.solve()
    gt, gs, _, _, rc = s.adjoint(c)
    assert rc == B.PAIR_OK
    h = 1e-6
    picks = w.fd_elems[:6]
    fdt, fds = [], []
    for e in picks:
        vals = []
        for which in ("t", "s"):
            for sg in (1, -1):
                st = w.mats.sigma_t.copy()
                ss = w.mats.sigma_s.copy()
                (st if which == "t" else ss)[e] += sg * h
                p2 = si.Problem(w.mesh, st, ss, w.mats.q, prob.omega, prob.w)
                vals.append(c @ si.source_iteration(p2, tol=1e-15).phi)
        fdt.append((vals[0] - vals[1]) / (2 * h))
        fds.append((vals[2] - vals[3]) / (2 * h))
    assert np.linalg.norm(gt[picks] - fdt) <= 1e-5 * np.linalg.norm(fdt)
    assert np.linalg.norm(gs[picks] - fds) <= 1e-5 * np.linalg.norm(fds)
    s.close()


def test_autograd_function():
    torch = need_gpu()
    from paper_1910_11463_amd.solver import TransportSolve
    from oracle import adjoint as ADJ
    w = wl.make_config(5, scale=4)
    prob = oracle_problem(w)
    c = torch.tensor(_detector_c(w, prob), device="cuda")
    s = solver_for(w, **TIGHT)
    st = torch.tensor(w.mats.sigma_t, device="cuda", requires_grad=True)
    ss = torch.tensor(w.mats.sigma_s, device="cuda", requires_grad=True)
    s.q = torch.tensor(w.mats.q, device="cuda")
    phi = TransportSolve.apply(s, st, ss)
    J = (phi * c).sum()
    J.backward()
    _, gt_ref, gs_ref = ADJ.adjoint_gradients(prob, w.detector, w.sn_order, tol=1e-14)
    assert rel(st.grad.cpu().numpy(), gt_ref) <= 1e-8
    assert rel(ss.grad.cpu().numpy(), gs_ref) <= 1e-8
    s.close()
