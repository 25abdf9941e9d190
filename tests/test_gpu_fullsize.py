"""Parity at the workloads' full sizes, in the launch configuration the benchmark
times: sampled directions against the oracle's exact sweep, bitwise batched ==
plain, and properties that hold at any size (adjoint duality)."""
import numpy as np
import pytest

from paper_1910_11463_amd import binding as B
from paper_1910_11463_amd import workloads as wl
from tests.gpu_util import need_gpu, oracle_problem, rel, solver_for

pytestmark = pytest.mark.gpu


# the benchmark's launch configuration (structured hexes: three tile sweeps
# before and after the coarse-grid correction on the finest level)
BENCH_OPTS = dict(relax_pre="TTT", relax_post="TTT", relax_pre_coarse="F", relax_post_coarse="",
                  tile_xy=16, tile_z=0, autotune=1, streams=5, batch_size=16, filter_r=1.0)
# the same with F/C half-sweep ladders (tets have no tile sweeps)
FC_OPTS = dict(BENCH_OPTS, relax_pre="FCFCFCFCFCFCF", relax_post="FCFCFCFCFCFCF")


def _sampled(cfg, dirs, mode, tol=1e-12, opts=BENCH_OPTS):
    from oracle import source_iteration as si
    w = wl.make_config(cfg)
    print("full size", w.name, "mode", mode, flush=True)
    s = solver_for(w, tol_inner=tol, max_inner=300, **opts)
    psi, phi, st, rc = s.transport_sweep(mode=mode)
    assert rc == B.PAIR_OK
    assert st["relres_max"] <= tol
    print("  GPU done: levels %d, V-cycles %d" % (st["levels_max"], st["vcycles_total"]), flush=True)
    s.close()
    prob = oracle_problem(w)
    prob.cache_blocks = False
    ref = si.transport_sweep(prob, None, threads=4, dirs=dirs)
    errs = [rel(psi[m], ref[k]) for k, m in enumerate(dirs)]
    print("  sampled direction errors", errs, flush=True)
    return errs


@pytest.mark.parametrize("mode", [B.PAIR_BATCHED, B.PAIR_PLAIN])
def test_structured_64(mode):
    """64^3 hexes, S8 (the benchmark's workload), batches of 16 directions on
    5 streams and one direction at a time."""
    need_gpu()
    errs = _sampled(2, [0, 37, 79], mode)
    assert max(errs) <= 1e-9


def test_structured_64_fc_ladders():
    """The same with the F/C half-sweep schedules instead of tile sweeps."""
    need_gpu()
    errs = _sampled(2, [11, 62], B.PAIR_BATCHED, opts=FC_OPTS)
    assert max(errs) <= 1e-9


def test_unstructured_tets_48():
    """48^3 x 6 jittered tets (2.65M DOF per direction), S4."""
    need_gpu()
    errs = _sampled(3, [5, 18], B.PAIR_PLAIN, opts=FC_OPTS)
    assert max(errs) <= 1e-9


def test_batched_checkerboard_32():
    """32^3 checkerboard, S8, all 80 directions batched; sampled directions
    against the exact sweep and every direction bitwise equal to the
    one-direction-at-a-time solve."""
    need_gpu()
    errs = _sampled(4, [3, 50], B.PAIR_BATCHED)
    assert max(errs) <= 1e-9
    w = wl.make_config(4)
    a = solver_for(w)
    b = solver_for(w)
    pa, fa, _, ra = a.transport_sweep(mode=B.PAIR_PLAIN)
    pb, fb, _, rb = b.transport_sweep(mode=B.PAIR_BATCHED)
    assert ra == B.PAIR_OK and rb == B.PAIR_OK
    assert np.array_equal(pa, pb) and np.array_equal(fa, fb)
    a.close()
    b.close()


def test_adjoint_duality_full_size():
    """32^3 hexes, S4: J = c^T phi equals the adjoint-weighted source
    phi_adj^T M q / (4 pi) (both from GPU solves; the identity follows from the
    coupled system and its transpose), and the gradients are finite."""
    need_gpu()
    from oracle import adjoint as ADJ
    w = wl.make_config(5)
    prob = oracle_problem(w)
    c = ADJ.detector_source(prob, w.detector)
    s = solver_for(w, tol_inner=1e-12, tol_outer=1e-12, outer_estimate=1, max_inner=300, **BENCH_OPTS)
    phi, _, st, rc = s.solve(mode=B.PAIR_BATCHED)
    assert rc == B.PAIR_OK
    gt, gs, phia, _, rc2 = s.adjoint(c, mode=B.PAIR_BATCHED)
    assert rc2 == B.PAIR_OK
    E, k = prob.topo.E, prob.topo.k
    mq = np.einsum("eab,eb->ea", prob.topo.mass, np.broadcast_to(w.mats.q[:, None], (E, k))).ravel()
    J = float(c @ phi)
    Jd = float(phia @ mq) / (4 * np.pi)
    assert abs(J - Jd) <= 1e-9 * abs(J), (J, Jd)
    assert np.all(np.isfinite(gt)) and np.all(np.isfinite(gs))
    s.close()
