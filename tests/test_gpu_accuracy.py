"""Accuracy of spatial solves (Sec. "Accuracy of Spatial Solves"): source
iteration with a fixed number of pAIR V-cycles per direction solve converges to
the fixed point of the inexact inverses.  On the manufactured solution of the
Appendix (unit cube, S4, sigma_t = 1, sigma_s = 0.5) the L2 error of phi
approaches the exact-solve error after a handful of cycles, and finer meshes
need at least as many cycles."""
import math

import numpy as np
import pytest

from paper_1910_11463_amd import binding as B
from paper_1910_11463_amd import workloads as wl
from tests.gpu_util import need_gpu

pytestmark = pytest.mark.gpu

CYCLES = (1, 2, 3, 4, 6, 8)


def _errors(n):
    from oracle import dg, mms, quadrature as Q
    from paper_1910_11463_amd.solver import Solver
    mesh = wl.hex_mesh(n)
    E = mesh.n_elem
    om, w = Q.level_symmetric(4)
    st, ss = 1.0, 0.5
    topo = dg.topology(mesh)
    ext = mms.hex_projected_source(topo, om, st, ss)
    out = {}
    for ell in CYCLES + (0,):
        s = Solver(tol_inner=1e-12, max_inner=300, tol_outer=1e-11, outer_estimate=1, max_outer=500,
                   keep_hierarchy=1, fixed_cycles=ell, batch_size=24, relax_pre="FFCF",
                   relax_post="FFCF", relax_pre_coarse="F", relax_post_coarse="F")
        s.set_mesh(mesh)
        s.set_quadrature(om, w)
        s.set_materials(np.full(E, st), np.full(E, ss), np.zeros(E))
        s.set_dual_source(ext, per_direction=True)
        phi, _, stt, rc = s.solve(mode=B.PAIR_BATCHED)
        assert rc == B.PAIR_OK, (n, ell, rc)
        out[ell] = mms.hex_l2_error(topo, phi, lambda p: 4 * math.pi * mms.Phi(p))
        s.close()
    return out


def test_fixed_cycles_approach_discretization_error():
    need_gpu()
    table = {}
    for n in (8, 16, 32):
        print("accuracy study, %d^3" % n, flush=True)
        table[n] = _errors(n)
        print("  L2 error of phi by V-cycles per solve (0 = to 1e-12):",
              {k: "%.4e" % v for k, v in table[n].items()}, flush=True)
    # exact solves: second order (the Q1 discretisation error)
    assert math.log2(table[8][0] / table[16][0]) > 1.9
    assert math.log2(table[16][0] / table[32][0]) > 1.9
    first_ok = []
    for n in (8, 16, 32):
        e = table[n]
        # more cycles never make the answer worse than the exact solve's by more
        # than they did with fewer (up to 1e-3 relative slack for rounding)
        gaps = [abs(e[ell] - e[0]) / e[0] for ell in CYCLES]
        assert gaps[-1] <= 1e-3, (n, gaps)
        first_ok.append(next(ell for ell, g in zip(CYCLES, gaps) if g <= 1e-2))
        print("  %d^3: cycles for 1%% of the exact-solve error: %d" % (n, first_ok[-1]), flush=True)
    # a handful of cycles suffices, and finer meshes need at least as many
    assert max(first_ok) <= 6, first_ok
    assert first_ok == sorted(first_ok), first_ok
