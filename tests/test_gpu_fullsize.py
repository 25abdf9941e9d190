"""Parity at the workloads' full sizes, in the launch configuration the benchmark
times: every direction against the oracle's exact sweep, bitwise batched ==
plain, the adjoint gradients of the 32^3 S4 workload against the oracle's
adjoint on every element and against central differences (stored, computed
by tests/golden/make_c5_fd.py from the oracle alone), and the adjoint
duality."""
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
# the same with F/C half-sweep ladders
FC_OPTS = dict(BENCH_OPTS, relax_pre="FCFCFCFCFCFCF", relax_post="FCFCFCFCFCFCF")
# tets: five tile sweeps over the default centroid-box tiles, as the
# benchmark's tet source iteration runs them
TET_OPTS = dict(relax_pre="TTTTT", relax_post="TTTTT", relax_pre_coarse="F", relax_post_coarse="F",
                streams=5, batch_size=16, filter_r=1.0)


def _reference(w, dirs):
    """The oracle's exact sweep of the given directions: the compiled
    structured-hex sweep (oracle/cpu_sweep.c, pinned to the NumPy oracle) on
    hexes, the NumPy assembly + C sweep on tets, on the host's threads."""
    import os
    from oracle import cpu_sweep as CS, source_iteration as si
    threads = min(16, os.cpu_count() or 1)
    if w.mesh.kind == 0:
        om, wt = _quadrature(w)
        psi, _ = CS.sweep_all(w.mesh, w.mats.sigma_t, w.mats.sigma_s, w.mats.q, om[dirs], wt[dirs],
                              threads=threads)
        return psi
    prob = oracle_problem(w)
    prob.cache_blocks = False
    return si.transport_sweep(prob, None, threads=min(8, threads), dirs=dirs)


def _quadrature(w):
    from oracle import quadrature as Q
    return Q.level_symmetric(w.sn_order)


def _checked(cfg, mode, tol=1e-12, opts=BENCH_OPTS, dirs=None):
    """One sweep replacement on the GPU; every direction (or `dirs`) against
    the oracle's exact sweep; returns the per-direction relative errors."""
    w = wl.make_config(cfg)
    print("full size", w.name, "mode", mode, flush=True)
    s = solver_for(w, tol_inner=tol, max_inner=300, **opts)
    psi, phi, st, rc = s.transport_sweep(mode=mode)
    assert rc == B.PAIR_OK
    assert st["relres_max"] <= tol
    print("  GPU done: levels %d, V-cycles %d" % (st["levels_max"], st["vcycles_total"]), flush=True)
    s.close()
    dirs = list(range(w.n_dir)) if dirs is None else dirs
    errs = []
    for k0 in range(0, len(dirs), 16):          # bounded host memory per chunk
        chunk = dirs[k0:k0 + 16]
        ref = _reference(w, chunk)
        errs += [rel(psi[m], ref[k]) for k, m in enumerate(chunk)]
    print("  worst direction error %.3e over %d directions" % (max(errs), len(errs)), flush=True)
    return errs


@pytest.mark.parametrize("mode", [B.PAIR_BATCHED, B.PAIR_PLAIN])
def test_structured_64(mode):
    """64^3 hexes, S8 (the benchmark's workload), batches of 16 directions on
    5 streams and one direction at a time."""
    need_gpu()
    errs = _checked(2, mode)
    assert max(errs) <= 1e-9


def test_structured_64_fc_ladders():
    """The same with the F/C half-sweep schedules instead of tile sweeps."""
    need_gpu()
    errs = _checked(2, B.PAIR_BATCHED, opts=FC_OPTS)
    assert max(errs) <= 1e-9


@pytest.mark.parametrize("sched", ["fc_plain", "tiles_batched"])
def test_unstructured_tets_48(sched):
    """48^3 x 6 jittered tets (2.65M DOF per direction), S4: F/C ladders one
    direction at a time, and tile sweeps in batches of 16 on 5 streams."""
    need_gpu()
    if sched == "fc_plain":
        errs = _checked(3, B.PAIR_PLAIN, opts=FC_OPTS)
    else:
        errs = _checked(3, B.PAIR_BATCHED, opts=TET_OPTS)
    assert max(errs) <= 1e-9


def test_batched_checkerboard_32():
    """32^3 checkerboard, S8, all 80 directions batched; every direction
    against the exact sweep and bitwise equal to the one-direction-at-a-time
    solve."""
    need_gpu()
    errs = _checked(4, B.PAIR_BATCHED)
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


def _fd_golden():
    import os
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "c5_fd_gradients.txt")
    J = None
    rows = []
    for line in open(path):
        if line.startswith("# J "):
            J = float(line.split()[2])
        elif not line.startswith("#") and line.strip():
            e, gt, gs = line.split()
            rows.append((int(e), float(gt), float(gs)))
    return J, rows


def test_adjoint_gradients_full_size():
    """32^3 hexes, S4, sigma_s = 0.8 sigma_t: dJ/dsigma_t and dJ/dsigma_s from
    the GPU adjoint (transposed pAIR solves) on all 32768 elements against the
    oracle's adjoint (forward and adjoint source iteration with the exact
    sweep, stop 1e-14) within 1e-8, and on the 16 seeded elements against the
    stored central differences (step 1e-6) within 1e-5."""
    need_gpu()
    import os
    from oracle import adjoint as ADJ, source_iteration as si
    w = wl.make_config(5)
    J_fd, rows = _fd_golden()
    picks = np.array([r[0] for r in rows])
    assert np.array_equal(picks, w.fd_elems)
    prob = oracle_problem(w)
    c = ADJ.detector_source(prob, w.detector)
    print("adjoint full size: GPU", flush=True)
    s = solver_for(w, tol_inner=1e-12, tol_outer=1e-14, outer_estimate=1, max_inner=300, **BENCH_OPTS)
    phi, _, st, rc = s.solve(mode=B.PAIR_BATCHED)
    assert rc == B.PAIR_OK
    gt, gs, _, _, rc2 = s.adjoint(c, mode=B.PAIR_BATCHED)
    assert rc2 == B.PAIR_OK
    s.close()
    J = float(c @ phi)
    assert abs(J - J_fd) <= 1e-10 * abs(J_fd), (J, J_fd)
    fdt = np.array([r[1] for r in rows])
    fds = np.array([r[2] for r in rows])
    et = np.linalg.norm(gt[picks] - fdt) / np.linalg.norm(fdt)
    es = np.linalg.norm(gs[picks] - fds) / np.linalg.norm(fds)
    print("  vs central differences: %.2e (sigma_t) %.2e (sigma_s)" % (et, es), flush=True)
    assert et <= 1e-5 and es <= 1e-5
    print("adjoint full size: oracle adjoint", flush=True)
    threads = min(16, os.cpu_count() or 1)
    fwd = si.source_iteration(prob, tol=1e-14, threads=threads)
    adj = si.source_iteration(ADJ.adjoint_problem(prob, c), tol=1e-14, threads=threads)
    gt_ref, gs_ref = ADJ.gradients(prob, fwd.psi, fwd.phi, adj.psi, adj.phi, w.sn_order)
    print("  vs oracle adjoint: %.2e (sigma_t) %.2e (sigma_s)" % (rel(gt, gt_ref), rel(gs, gs_ref)),
          flush=True)
    assert rel(gt, gt_ref) <= 1e-8
    assert rel(gs, gs_ref) <= 1e-8
