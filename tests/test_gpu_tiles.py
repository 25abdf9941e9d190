"""GPU parity of the tile sweeps (schedule letter T: block Jacobi over boxes of
elements with an exact forward solve inside each box) against the oracle's
TileSolver, through the C ABI."""
import numpy as np
import pytest
import scipy.sparse as sp

from paper_1910_11463_amd import binding as B
from paper_1910_11463_amd import workloads as wl
from tests.gpu_util import need_gpu, oracle_problem, rel, solver_for

pytestmark = pytest.mark.gpu


def _print(*a):
    print(*a, flush=True)


def _aniso():
    mesh = wl.hex_mesh(6, 5, 7, hi=(1.0, 2.0, 0.7))
    E = mesh.n_elem
    st = wl.log_uniform(E, 0.1, 10.0, seed=11)
    return wl.Workload("hex6x5x7-aniso-S8", mesh, wl.Materials(st, 0.9 * st, np.ones(E)), 8)


def _box(nx, ny, nz, seed):
    mesh = wl.hex_mesh(nx, ny, nz, hi=(1.0, ny / nx, nz / nx))
    E = mesh.n_elem
    st = wl.log_uniform(E, 0.1, 10.0, seed=seed)
    return wl.Workload("hex%dx%dx%d-S8" % (nx, ny, nz), mesh, wl.Materials(st, 0.9 * st, np.ones(E)), 8)


# (mesh, tile_xy, tile_z, pre, post, directions): ragged boxes on every axis,
# one box per axis, several, and T mixed with F/C half-sweeps.  Meshes small
# enough for a two-level hierarchy (coarse level <= 2048 rows, solved densely).
CASES = [
    ((6, 5, 7), 8, 3, "TF", "FT", (0, 17, 46, 79)),
    ((17, 10, 3), 8, 0, "T", "T", (0, 41, 79)),
    ((18, 17, 2), 16, 1, "TT", "CT", (9, 62)),
    ((9, 8, 8), 8, 1, "T", "", (30,)),
]


@pytest.mark.parametrize("case", range(len(CASES)))
def test_tile_cycles_match_oracle_two_level_cycles(case):
    """Two two-level V-cycles from x = 0 per direction with tile sweeps on the
    finest level, against the oracle's setup, TileSolver and V-cycle on the
    library's exported operator (see the factored-relaxation test for why the
    operator values are the library's)."""
    need_gpu()
    from oracle import air_ref as ar
    dims, txy, tz, pre, post, dirs = CASES[case]
    w = _aniso() if dims == (6, 5, 7) else _box(*dims, seed=case)
    mesh = w.mesh
    s = solver_for(w, fixed_cycles=2, filter_r=1.0, batch_size=16, max_levels=2, relax_pre=pre,
                   relax_post=post, relax_pre_coarse="F", relax_post_coarse="", tile_xy=txy, tile_z=tz)
    _print("tiles", w.name, "boxes", txy, txy, tz, "schedules", pre, post)
    psi, phi, st, rc = s.transport_sweep(mode=B.PAIR_BATCHED)
    assert rc == B.PAIR_OK
    tiles = ar.hex_tiles(mesh.nx, mesh.ny, mesh.nz, txy, txy, tz if tz > 0 else mesh.nz)
    opts = ar.Options(filter_r=1.0, max_levels=2)
    for m in dirs:
        rp, col, val, b = s.export_fine_operator(m)
        A = sp.csr_matrix((val, col, rp), shape=(b.shape[0], b.shape[0]))
        levels = ar.setup(A, opts)
        ts = ar.TileSolver(A, tiles)
        x = np.zeros_like(b)
        for _ in range(2):
            x = ar.vcycle(levels, b, x, pre=pre, post=post, pre_c="F", post_c="", tiles=ts)
        _print("  direction", m, "rel diff %.2e" % rel(psi[m], x))
        assert len(levels) == 2
        assert rel(psi[m], x) <= 1e-12, m
    s.close()


@pytest.mark.parametrize("mode,txy,tz", [(B.PAIR_PLAIN, 8, 0), (B.PAIR_BATCHED, 16, 5),
                                         (B.PAIR_BATCHED, 8, 4)])
def test_tile_solve_converges_to_exact_sweep(mode, txy, tz):
    """Full hierarchies with tile sweeps converge to the oracle's exact sweep."""
    need_gpu()
    from oracle import source_iteration as si
    w = wl.make_config(2, scale=12)
    s = solver_for(w, tol_inner=1e-12, max_inner=200, batch_size=16, filter_r=1.0,
                   relax_pre="TT", relax_post="TT", relax_pre_coarse="F", relax_post_coarse="",
                   tile_xy=txy, tile_z=tz)
    _print("tile solve", w.name, "mode", mode, "boxes", txy, tz)
    psi, phi, st, rc = s.transport_sweep(mode=mode)
    assert rc == B.PAIR_OK
    ref = si.transport_sweep(oracle_problem(w), None)
    for m in range(len(ref)):
        assert rel(psi[m], ref[m]) <= 1e-9, (m, rel(psi[m], ref[m]))
    assert st["relres_max"] <= 1e-12
    _print("  V-cycles max", st["vcycles_max"])
    s.close()


def test_one_box_is_the_exact_solve():
    """A box holding the whole mesh makes one tile sweep the exact solve: a
    single fixed V-cycle with one T pre-sweep and no post-smoothing returns
    the exact sweep (the coarse correction of an exact iterate is zero)."""
    need_gpu()
    from oracle import source_iteration as si
    w = wl.make_config(2, scale=8)
    s = solver_for(w, fixed_cycles=1, filter_r=1.0, batch_size=16, relax_pre="T", relax_post="",
                   relax_pre_coarse="F", relax_post_coarse="", tile_xy=8, tile_z=0)
    psi, phi, st, rc = s.transport_sweep(mode=B.PAIR_BATCHED)
    assert rc == B.PAIR_OK
    ref = si.transport_sweep(oracle_problem(w), None)
    for m in range(len(ref)):
        assert rel(psi[m], ref[m]) <= 1e-12, (m, rel(psi[m], ref[m]))
    s.close()


def test_tile_schedule_errors():
    need_gpu()
    from paper_1910_11463_amd.solver import Solver
    w = wl.make_config(2, scale=3)
    s = solver_for(w, relax_pre="T", relax_post="F", relax_pre_coarse="F", relax_post_coarse="F",
                   fine_factored=0)
    with pytest.raises(B.PairError) as e:
        s.transport_sweep(mode=B.PAIR_BATCHED)
    assert "tile sweeps" in str(e.value)
    s.close()
    # a tet tile holding more than 1024 elements
    w = wl.make_config(3, scale=6)
    s = solver_for(w, relax_pre="T", relax_post="T", relax_pre_coarse="F", relax_post_coarse="",
                   tet_tile_boxes=1)
    with pytest.raises(B.PairError) as e:
        s.transport_sweep(mode=B.PAIR_BATCHED)
    assert "more than 1024" in str(e.value)
    s.close()
    s = Solver()
    for bad in (dict(relax_pre="T"), dict(relax_pre="FT", relax_pre_coarse="T"),
                dict(tile_xy=4), dict(tile_z=-1), dict(tet_tile_boxes=-1)):
        with pytest.raises(B.PairError) as e:
            s.set_options(**bad)
        assert e.value.code == B.PAIR_E_INVALID
        s.opt = B.default_options()
    s.close()


TILE_OPTS = dict(relax_pre="TTT", relax_post="TTT", relax_pre_coarse="F", relax_post_coarse="",
                 tile_xy=16, tile_z=5, filter_r=1.0, tol_inner=1e-10, max_inner=50)


def test_tile_batched_equals_plain_bitwise():
    """With tile sweeps, batched launches (16 directions per hierarchy) give
    bit-identical psi and phi to one-direction-at-a-time solves (each box's
    solve depends only on its own direction's data)."""
    need_gpu()
    w = _box(20, 18, 11, seed=7)
    a = solver_for(w, **TILE_OPTS)
    b = solver_for(w, batch_size=16, **TILE_OPTS)
    _print("tiles batched vs plain", w.name)
    psi_p, phi_p, _, rc_p = a.transport_sweep(mode=B.PAIR_PLAIN)
    psi_b, phi_b, _, rc_b = b.transport_sweep(mode=B.PAIR_BATCHED)
    assert rc_p == B.PAIR_OK and rc_b == B.PAIR_OK
    assert np.array_equal(psi_p, psi_b)
    assert np.array_equal(phi_p, phi_b)
    a.close()
    b.close()


def test_tile_streams_bitwise():
    """With tile sweeps, batches on three worker streams give the same psi and
    phi as one stream, cold and then warm on the kept hierarchies."""
    need_gpu()
    w = _box(20, 18, 11, seed=8)
    out = []
    for streams in (1, 3):
        s = solver_for(w, batch_size=8, streams=streams, keep_hierarchy=1, **TILE_OPTS)
        _print("tiles streams", streams)
        psi, phi, _, rc = s.transport_sweep(mode=B.PAIR_BATCHED)
        assert rc == B.PAIR_OK
        psi2, phi2, _, rc2 = s.transport_sweep(mode=B.PAIR_BATCHED)
        assert rc2 == B.PAIR_OK
        out.append((psi, phi, psi2, phi2))
        s.close()
    for x, y in zip(out[0], out[1]):
        assert np.array_equal(x, y)


def _tets(n, seed, jitter=0.2):
    mesh = wl.kuhn_tet_mesh(n, jitter=jitter, seed=seed)
    E = mesh.n_elem
    st = wl.log_uniform(E, 0.1, 10.0, seed=seed + 1)
    return wl.Workload("tet%d^3x6-S4" % n, mesh, wl.Materials(st, 0.5 * st, np.ones(E)), 4)


# (mesh size, tet_tile_boxes, pre, post, directions); the last: 10^3 boxes over
# 384 tets, so most tiles are empty or hold one or two elements
TET_CASES = [(5, 2, "T", "T", (0, 7, 13, 23)), (5, 0, "TF", "FT", (2, 19)), (4, 3, "TT", "C", (5, 11)),
             (4, 10, "T", "T", (0, 9, 17))]


@pytest.mark.parametrize("case", range(len(TET_CASES)))
def test_tet_tile_cycles_match_oracle_two_level_cycles(case):
    """Jittered tets: two two-level V-cycles from x = 0 per direction with tile
    sweeps over the centroid-box tiles on the finest level, against the
    oracle's setup, TileSolver (sparse LU of the tile-diagonal part) and
    V-cycle on the library's exported operator."""
    need_gpu()
    from oracle import air_ref as ar
    n, nbox, pre, post, dirs = TET_CASES[case]
    w = _tets(n, seed=20 + case)
    s = solver_for(w, fixed_cycles=2, filter_r=1.0, batch_size=12, max_levels=2, relax_pre=pre,
                   relax_post=post, relax_pre_coarse="F", relax_post_coarse="", tet_tile_boxes=nbox)
    _print("tet tiles", w.name, "boxes", nbox, "schedules", pre, post)
    psi, phi, st, rc = s.transport_sweep(mode=B.PAIR_BATCHED)
    assert rc == B.PAIR_OK
    tiles = ar.tet_tiles(w.mesh.xyz, w.mesh.elem_vert, nbox)
    opts = ar.Options(filter_r=1.0, max_levels=2)
    for m in dirs:
        rp, col, val, b = s.export_fine_operator(m)
        A = sp.csr_matrix((val, col, rp), shape=(b.shape[0], b.shape[0]))
        levels = ar.setup(A, opts)
        ts = ar.TileSolver(A, tiles)
        x = np.zeros_like(b)
        for _ in range(2):
            x = ar.vcycle(levels, b, x, pre=pre, post=post, pre_c="F", post_c="", tiles=ts)
        _print("  direction", m, "rel diff %.2e" % rel(psi[m], x))
        assert len(levels) == 2
        assert rel(psi[m], x) <= 1e-12, m
    s.close()


@pytest.mark.parametrize("mode", [B.PAIR_PLAIN, B.PAIR_BATCHED])
def test_tet_tile_solve_converges_to_exact_sweep(mode):
    """Full hierarchies with tet tile sweeps reach the oracle's exact sweep."""
    need_gpu()
    from oracle import source_iteration as si
    w = wl.make_config(3, scale=8)
    s = solver_for(w, tol_inner=1e-12, max_inner=200, batch_size=12, filter_r=1.0,
                   relax_pre="TT", relax_post="TT", relax_pre_coarse="F", relax_post_coarse="")
    _print("tet tile solve", w.name, "mode", mode)
    psi, phi, st, rc = s.transport_sweep(mode=mode)
    assert rc == B.PAIR_OK
    ref = si.transport_sweep(oracle_problem(w), None)
    for m in range(len(ref)):
        assert rel(psi[m], ref[m]) <= 1e-9, (m, rel(psi[m], ref[m]))
    _print("  V-cycles max", st["vcycles_max"])
    s.close()


def test_tet_one_tile_is_the_exact_solve():
    """One tile holding the whole tet mesh: one tile sweep is the exact solve."""
    need_gpu()
    from oracle import source_iteration as si
    w = wl.make_config(3, scale=5)              # 750 tets, one tile
    s = solver_for(w, fixed_cycles=1, filter_r=1.0, batch_size=12, relax_pre="T", relax_post="",
                   relax_pre_coarse="F", relax_post_coarse="", tet_tile_boxes=1)
    psi, phi, st, rc = s.transport_sweep(mode=B.PAIR_BATCHED)
    assert rc == B.PAIR_OK
    ref = si.transport_sweep(oracle_problem(w), None)
    for m in range(len(ref)):
        assert rel(psi[m], ref[m]) <= 1e-12, (m, rel(psi[m], ref[m]))
    s.close()


def test_tet_tile_batched_equals_plain_and_streams_bitwise():
    """Tet tile sweeps: batched == plain, and three worker streams == one, bitwise."""
    need_gpu()
    w = _tets(7, seed=31)
    opts = dict(relax_pre="TT", relax_post="TT", relax_pre_coarse="F", relax_post_coarse="", filter_r=1.0,
                tol_inner=1e-10, max_inner=60)
    out = []
    for mode, bs, streams in ((B.PAIR_PLAIN, 0, 1), (B.PAIR_BATCHED, 8, 1), (B.PAIR_BATCHED, 8, 3)):
        s = solver_for(w, batch_size=bs, streams=streams, **opts)
        psi, phi, _, rc = s.transport_sweep(mode=mode)
        assert rc == B.PAIR_OK
        out.append((psi, phi))
        s.close()
    for k in (1, 2):
        assert np.array_equal(out[0][0], out[k][0]) and np.array_equal(out[0][1], out[k][1])


# Strongly jittered tets whose upwind graphs have cycles inside the tiles
# (strongly connected sets of up to 5-7 elements in every S4 direction, found
# with the oracle's topology): the tile solve condenses them and solves each
# set densely.
@pytest.mark.parametrize("nbox", [2, 1])
def test_tet_tiles_with_upwind_cycles_match_oracle(nbox):
    """Two two-level V-cycles with TT/TT on a mesh with in-tile cycles against
    the oracle's TileSolver (sparse LU of the tile-diagonal part) on the
    exported operator; one tile: a single T sweep is the oracle's exact sweep
    (dense solves of the cycles)."""
    need_gpu()
    from oracle import air_ref as ar, source_iteration as si
    # 2 x 2 x 2 tiles: sets of up to 7 elements; one tile: up to 5
    w = _tets(5, seed=50, jitter=0.42) if nbox == 2 else _tets(5, seed=44, jitter=0.4)
    _print("tet tiles with cycles, boxes", nbox)
    if nbox == 2:
        s = solver_for(w, fixed_cycles=2, filter_r=1.0, batch_size=12, max_levels=2, relax_pre="TT",
                       relax_post="TT", relax_pre_coarse="F", relax_post_coarse="", tet_tile_boxes=nbox)
        psi, phi, st, rc = s.transport_sweep(mode=B.PAIR_BATCHED)
        assert rc == B.PAIR_OK
        tiles = ar.tet_tiles(w.mesh.xyz, w.mesh.elem_vert, nbox)
        for m in (0, 9, 17):
            rp, col, val, b = s.export_fine_operator(m)
            A = sp.csr_matrix((val, col, rp), shape=(b.shape[0], b.shape[0]))
            levels = ar.setup(A, ar.Options(filter_r=1.0, max_levels=2))
            ts = ar.TileSolver(A, tiles)
            x = np.zeros_like(b)
            for _ in range(2):
                x = ar.vcycle(levels, b, x, pre="TT", post="TT", pre_c="F", post_c="", tiles=ts)
            _print("  direction", m, "rel diff %.2e" % rel(psi[m], x))
            assert rel(psi[m], x) <= 1e-12, m
    else:
        s = solver_for(w, fixed_cycles=1, filter_r=1.0, batch_size=12, relax_pre="T", relax_post="",
                       relax_pre_coarse="F", relax_post_coarse="", tet_tile_boxes=1)
        psi, phi, st, rc = s.transport_sweep(mode=B.PAIR_BATCHED)
        assert rc == B.PAIR_OK
        ref = si.transport_sweep(oracle_problem(w), None)
        for m in range(len(ref)):
            assert rel(psi[m], ref[m]) <= 1e-11, (m, rel(psi[m], ref[m]))
    s.close()


def test_tet_tiles_with_upwind_cycles_converge_and_agree_bitwise():
    """5^3 x 6 tets, jitter 0.42, 2 x 2 x 2 tiles (cycles of up to 7 elements
    inside the tiles): full hierarchies with TT/TT reach the oracle's exact
    sweep, and plain, batched and three-stream solves agree bitwise.  On so
    distorted a mesh the AIR hierarchy diverges for some directions (in the
    oracle too, with tile or F/C relaxation alike); the six S4 directions used
    here converge in the oracle in 14-28 V-cycles."""
    need_gpu()
    from paper_1910_11463_amd.solver import Solver
    from oracle import quadrature as Q, source_iteration as si
    w = _tets(5, seed=50, jitter=0.42)
    om, wt = Q.level_symmetric(4)
    dirs = [1, 4, 14, 18, 19, 20]
    om, wt = om[dirs], wt[dirs] * (4 * np.pi / wt[dirs].sum())    # a quadrature of its own
    opts = dict(relax_pre="TT", relax_post="TT", relax_pre_coarse="F", relax_post_coarse="", filter_r=1.0,
                tol_inner=1e-12, max_inner=200, tet_tile_boxes=2)
    out = []
    for mode, bs, streams in ((B.PAIR_BATCHED, 4, 1), (B.PAIR_PLAIN, 0, 1), (B.PAIR_BATCHED, 4, 3)):
        _print("cyclic tets, mode", mode, "streams", streams)
        s = Solver(batch_size=bs, streams=streams, **opts)
        s.set_mesh(w.mesh)
        s.set_quadrature(om, wt)
        s.set_materials(w.mats.sigma_t, w.mats.sigma_s, w.mats.q)
        psi, phi, st, rc = s.transport_sweep(mode=mode)
        assert rc == B.PAIR_OK
        out.append((psi, phi))
        s.close()
    m = w.mats
    ref = si.transport_sweep(si.Problem(w.mesh, m.sigma_t, m.sigma_s, m.q, om, wt), None)
    for k in range(len(dirs)):
        assert rel(out[0][0][k], ref[k]) <= 1e-9, (k, rel(out[0][0][k], ref[k]))
    for k in (1, 2):
        assert np.array_equal(out[0][0], out[k][0]) and np.array_equal(out[0][1], out[k][1])


def test_tet_tile_cycle_over_16_elements_is_rejected():
    """An in-tile cycle of 23 elements (jitter 0.48, one tile) exceeds the dense
    set solve: an error naming the limit, not a wrong answer."""
    need_gpu()
    w = _tets(5, seed=48, jitter=0.48)
    s = solver_for(w, relax_pre="T", relax_post="T", relax_pre_coarse="F", relax_post_coarse="",
                   tet_tile_boxes=1)
    with pytest.raises(B.PairError) as e:
        s.transport_sweep(mode=B.PAIR_BATCHED)
    assert "more than 16 elements" in str(e.value)
    s.close()
