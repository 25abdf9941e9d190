"""Helpers shared by the GPU tests (not collected by pytest)."""
import numpy as np
import pytest


def need_gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def solver_for(workload, order=None, **opts):
    from paper_1910_11463_amd.solver import Solver
    s = Solver(**opts)
    s.set_mesh(workload.mesh)
    om, w = Solver.level_symmetric(order or workload.sn_order)
    s.set_quadrature(om, w)
    m = workload.mats
    s.set_materials(m.sigma_t, m.sigma_s, m.q)
    return s


def oracle_problem(workload, order=None):
    from oracle import quadrature as Q, source_iteration as si
    om, w = Q.level_symmetric(order or workload.sn_order)
    m = workload.mats
    return si.Problem(workload.mesh, m.sigma_t, m.sigma_s, m.q, om, w)


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b)))
