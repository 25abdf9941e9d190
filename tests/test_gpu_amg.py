"""Component parity of the GPU AIR setup and V-cycle against the reference AIR
(oracle/air_ref.py) on the same input matrices, through the generic C ABI."""
import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from paper_1910_11463_amd import binding as B
from paper_1910_11463_amd import workloads as wl
from tests.gpu_util import need_gpu

pytestmark = pytest.mark.gpu


def _matrix(cfg, scale, m):
    from oracle import dg, quadrature as Q, source_iteration as si
    w = wl.make_config(cfg, scale=scale)
    om, wt = Q.level_symmetric(w.sn_order)
    prob = si.Problem(w.mesh, w.mats.sigma_t, w.mats.sigma_s, w.mats.q, om, wt)
    blk = prob.blocks(m)
    A = dg.scaled_csr(prob.topo, blk)
    b = np.einsum("eab,eb->ea", np.linalg.inv(blk.D), prob.rhs(m, None)).ravel()
    return A, b


CASES = [(2, 6, 5), (3, 2, 7), (5, 5, 13), (4, 6, 40)]


def _amg(A, coarse_max, seed=0, seg=None, kmax=64, pre="FC", post="FC", max_levels=25,
         pre_c="=", post_c="=", filter_r=0.0, **kw):
    from paper_1910_11463_amd.solver import Amg
    a = Amg(coarse_max=coarse_max, pmis_seed=seed, tol_inner=1e-10, max_inner=200, kmax=kmax,
            relax_pre=pre.encode(), relax_post=post.encode(), max_levels=max_levels,
            relax_pre_coarse=pre_c.encode(), relax_post_coarse=post_c.encode(), filter_r=filter_r,
            **kw)
    a.setup(A.indptr, A.indices, A.data, seg)
    return a


@pytest.mark.parametrize("cfg,scale,m,kmax", [c + (64,) for c in CASES] + [(2, 6, 5, 3), (3, 2, 7, 2)])
def test_hierarchy_matches_reference(cfg, scale, m, kmax):
    """Every coarsening step of the reference hierarchy, redone on the GPU from
    the same level matrix: same strength-based C/F split, interpolation and
    restriction pattern (bit-exact), restriction values and Galerkin operator
    within 1e-12 relative.  Each step starts from the reference's own level
    matrix, so rounding-order differences in earlier products cannot move a
    near-tie decision.  Small kmax exercises the truncation of long local
    systems to the strongest entries."""
    need_gpu()
    from oracle import air_ref as AR
    A, _ = _matrix(cfg, scale, m)
    print("hierarchy parity", cfg, scale, m, kmax, A.shape, flush=True)
    seed = 3
    ref = AR.setup(A, AR.Options(coarse_max=64, seed=seed, kmax=kmax))
    assert len(ref) >= 2
    for l, L in enumerate(ref[:-1]):
        if L.cf is None:
            break
        # one coarsening step of the reference on this level, measure hashed as level 0
        one = AR.setup(L.A, AR.Options(coarse_max=64, seed=seed, kmax=kmax, max_levels=2))
        g = _amg(L.A, 64, seed, kmax=kmax, max_levels=2)
        assert g.num_levels() == len(one)
        got, R0 = g.level(0), one[0]
        assert np.array_equal(got["cf"], R0.cf.astype(np.int8)), l
        assert np.array_equal(got["p"], R0.p.astype(np.int32)), l
        assert np.array_equal(got["r_rowptr"], R0.R.indptr), l
        assert np.array_equal(got["r_col"], R0.R.indices), l
        assert np.abs(got["r_val"] - R0.R.data).max() <= 1e-12 * np.abs(R0.R.data).max(), l
        nxt, R1 = g.level(1), one[1]
        assert np.array_equal(nxt["rowptr"], R1.A.indptr), l
        assert np.array_equal(nxt["col"], R1.A.indices), l
        assert np.abs(nxt["val"] - R1.A.data).max() <= 1e-12 * np.abs(R1.A.data).max(), l


def _ragged_matrix(n, lo, hi, diag, seed):
    """Random nonsymmetric matrix whose rows have their own fill fraction in
    [lo, hi): row lengths from a few entries to over a hundred."""
    rng = np.random.default_rng(seed)
    fill = rng.uniform(lo, hi, n)[:, None]
    M = (rng.random((n, n)) < fill) * rng.uniform(-1.0, 1.0, (n, n))
    np.fill_diagonal(M, rng.uniform(diag, 1.5 * diag, n))
    return sp.csr_matrix(M)


@pytest.mark.parametrize("n,seed", [(600, 5), (800, 7)])
def test_every_local_system_size_matches_reference(n, seed):
    """Distance-1 restriction rows whose local systems fall in every size class
    the GPU solves separately (K <= 8, 9-12, 13-14, 15-16, 17-32, 33-64, each
    class's upper edge included where the matrix reaches it), with rows of more
    than 64 strong F neighbours truncated to the 64 strongest: split and
    interpolation exact, R's pattern exact, R and the Galerkin coarse operator
    within 1e-12 of their largest entries."""
    need_gpu()
    from oracle import air_ref as AR
    A = _ragged_matrix(n, 0.004, 0.25, 40.0, seed)
    one = AR.setup(A, AR.Options(coarse_max=64, seed=3, max_levels=2, kmax=64))
    R = one[0].R.tocsr()
    K = np.diff(R.indptr) - 1
    cls = np.searchsorted([8, 12, 14, 16, 32], K, side="left")
    assert (np.bincount(cls, minlength=6) > 0).all() and K.max() == 64
    untrunc = AR.lair_restriction(A, one[0].cf, AR.Options(kmax=10 ** 6)).tocsr()
    assert (np.diff(untrunc.indptr) - 1 > 64).sum() >= 3
    print("local system classes", n, seed, np.bincount(cls, minlength=6).tolist(), flush=True)
    g = _amg(A, 64, 3, max_levels=2, kmax=64)
    got, coarse = g.level(0), g.level(1)
    g.close()
    assert np.array_equal(got["cf"], one[0].cf.astype(np.int8))
    assert np.array_equal(got["p"], one[0].p.astype(np.int32))
    assert np.array_equal(got["r_rowptr"], R.indptr) and np.array_equal(got["r_col"], R.indices)
    assert np.abs(got["r_val"] - R.data).max() <= 1e-12 * np.abs(R.data).max()
    Ac = one[1].A.toarray()
    n1 = Ac.shape[0]
    Cg = sp.csr_matrix((coarse["val"], coarse["col"], coarse["rowptr"]), shape=(n1, n1)).toarray()
    assert np.abs(Cg - Ac).max() <= 1e-12 * np.abs(Ac).max()


@pytest.mark.parametrize("distance", [1, 2])
def test_singular_local_system_is_reported(distance):
    """40 independent 3 x 3 blocks [[10, -3, -2], [-20, 4, 4], [-24, 4, 4]] (each
    scaled by its own power of two; the block itself is nonsingular): the first
    point is the C point (both others depend on it strongly), its two F
    neighbours form the local system [[4, 4], [4, 4]] times the scale.  With a
    power-of-two scale the elimination is exact, so the second pivot is exactly
    zero, the condition under which LAPACK's solve fails too; the setup reports
    every such row as an error instead of writing R.  (Under another scale the
    multiplier 4s * (1 / 4s) can round off 1 and leave a pivot of one unit in
    the last place: nearly singular systems are solved, not reported, on either
    side.)"""
    need_gpu()
    from oracle import air_ref as AR
    rng = np.random.default_rng(1)
    blk = np.array([[10.0, -3.0, -2.0], [-20.0, 4.0, 4.0], [-24.0, 4.0, 4.0]])
    A = sp.csr_matrix(sp.block_diag([2.0 ** rng.integers(-4, 5) * blk for _ in range(40)]))
    cf = AR.pmis(AR.strength(A, 0.25), 0, 3)
    assert np.array_equal(cf, np.tile([1, -1, -1], 40))
    with pytest.raises(np.linalg.LinAlgError):
        AR.lair_restriction(A, cf, AR.Options(distance=distance))
    with pytest.raises(B.PairError) as e:
        _amg(A, 8, 3, max_levels=2, lair_distance=distance)
    assert "singular local lAIR system in 40 rows" in str(e.value)


def test_singular_long_distance2_system_is_reported():
    """Distance-2 local systems of 70 unknowns (solved by the blocked LU of the
    long-row kernel, not by the one-wave kernel of at most 64): 10 independent
    blocks, each a C point whose 70 F neighbours all depend on it strongly, with
    A(R, R) = 4 I except [[4, 4], [4, 4]] for two of them, scaled by a power of
    two (the matrix itself is nonsingular).  The elimination is exact, the
    pivot of the second of the two is exactly zero as in LAPACK's solve, and the
    setup reports the 10 rows."""
    need_gpu()
    from oracle import air_ref as AR

    def block(nf, scale):
        M = np.zeros((nf + 1, nf + 1))
        M[0, 0] = 100.0
        M[0, 1:] = -1.0
        M[0, 2] = -0.5            # columns 1 and 2 differ in row 0
        for j in range(1, nf + 1):
            M[j, j] = 4.0
            M[j, 0] = -32.0
        M[2, 0] = -64.0           # rows 1 and 2 differ in column 0
        M[1, 2] = M[2, 1] = 4.0   # A(R, R) holds [[4, 4], [4, 4]] for F points 1 and 2
        return scale * M

    rng = np.random.default_rng(2)
    A = sp.csr_matrix(sp.block_diag([block(70, 2.0 ** rng.integers(-3, 4)) for _ in range(10)]))
    assert np.linalg.matrix_rank(A.toarray()) == A.shape[0]
    cf = AR.pmis(AR.strength(A, 0.25), 0, 3)
    assert np.array_equal(cf, np.tile([1] + [-1] * 70, 10))
    assert len(AR._r_pattern(A, AR.strength(A, 0.01), cf, 0, AR.Options(distance=2))) == 70
    with pytest.raises(np.linalg.LinAlgError):
        AR.lair_restriction(A, cf, AR.Options(distance=2))
    with pytest.raises(B.PairError) as e:
        _amg(A, 8, 3, max_levels=2, lair_distance=2)
    assert "singular local lAIR system in 10 rows" in str(e.value)


@pytest.mark.parametrize("cfg,scale,m", CASES[:3])
def test_filtered_restriction_matches_reference(cfg, scale, m):
    """R filtered with phi_R = 0.2 from the reference's level matrix: the kept
    pattern is the reference's except for entries within 1e-9 (relative) of the
    threshold, and the values agree to 1e-12."""
    need_gpu()
    from oracle import air_ref as AR
    A, _ = _matrix(cfg, scale, m)
    phi = 0.2
    one = AR.setup(A, AR.Options(coarse_max=64, seed=3, max_levels=2, filter_r=phi))
    full = AR.lair_restriction(A, one[0].cf, AR.Options()).tocsr()   # unfiltered values
    g = _amg(A, 64, 3, max_levels=2, filter_r=phi)
    got = g.level(0)
    assert np.array_equal(got["cf"], one[0].cf.astype(np.int8))
    cpts = np.flatnonzero(one[0].cf > 0)
    rp, rc, rv = got["r_rowptr"], got["r_col"], got["r_val"]
    Rr = one[0].R.tocsr()
    scale_v = np.abs(Rr.data).max()
    for I, i in enumerate(cpts):
        c0 = full.indices[full.indptr[I]:full.indptr[I + 1]]
        v0 = full.data[full.indptr[I]:full.indptr[I + 1]]
        off = c0 != i
        thr = phi * (np.abs(v0[off]).max() if off.any() else 0.0)
        want = set(Rr.indices[Rr.indptr[I]:Rr.indptr[I + 1]].tolist())
        have = dict(zip(rc[rp[I]:rp[I + 1]].tolist(), rv[rp[I]:rp[I + 1]].tolist()))
        for c, v in zip(c0, v0):
            if abs(abs(v) - thr) <= 1e-9 * max(thr, 1e-300):
                continue   # on the threshold: either side is right
            assert (c in have) == (c in want), (I, c)
            if c in have:
                assert abs(have[c] - v) <= 1e-12 * scale_v
    nxt, R1 = g.level(1), one[1]
    if np.array_equal(nxt["rowptr"], R1.A.indptr):
        assert np.abs(nxt["val"] - R1.A.data).max() <= 1e-12 * np.abs(R1.A.data).max()


@pytest.mark.parametrize("cfg,scale,m,pre,post,pre_c,post_c",
                         [c + ("FC", "FC", "=", "=") for c in CASES] +
                         [(2, 6, 5, "FFC", "FFC", "=", "="), (3, 2, 7, "", "FFC", "=", "="),
                          (5, 5, 13, "FC", "FFC", "=", "="), (2, 6, 5, "FFC", "FFC", "F", "FC"),
                          (2, 6, 5, "FFCF", "FFCF", "F", "F"), (3, 2, 7, "FFCF", "FFCF", "F", "F")])
@pytest.mark.parametrize("filter_r", [0.0, 0.2])
def test_vcycles_match_reference(cfg, scale, m, pre, post, pre_c, post_c, filter_r):
    """Same iteration count as the reference cycle for each relaxation schedule
    (within one: the two full hierarchies may settle a near-tie in a coarse
    level differently, since their Galerkin sums round in different orders)."""
    need_gpu()
    from oracle import air_ref as AR
    A, b = _matrix(cfg, scale, m)
    ref = AR.setup(A, AR.Options(coarse_max=64, filter_r=filter_r))
    xr, itr, hist = AR.solve(ref, b, tol=1e-10, maxit=200, pre=pre, post=post,
                             pre_c=None if pre_c == "=" else pre_c,
                             post_c=None if post_c == "=" else post_c)
    g = _amg(A, 64, pre=pre, post=post, pre_c=pre_c, post_c=post_c, filter_r=filter_r)
    x, iters, rel, rc = g.solve(b)
    assert rc == B.PAIR_OK
    assert abs(int(iters[0]) - itr) <= 1, (iters[0], itr)
    assert rel[0] <= 1e-10
    xe = spla.spsolve(A.tocsc(), b)
    assert np.linalg.norm(x - xe) <= 1e-8 * np.linalg.norm(xe)
    assert np.linalg.norm(x - xr) <= 1e-8 * np.linalg.norm(xe)


@pytest.mark.parametrize("cfg,scale,m", [(2, 6, 5), (3, 2, 7)])
def test_coarse_fp32_keeps_the_fp64_solution(cfg, scale, m):
    """FP32 operators below the finest level perturb only the coarse-grid
    correction: the cycle still converges to the FP64 solution, in about as many
    cycles."""
    need_gpu()
    from paper_1910_11463_amd.solver import Amg
    A, b = _matrix(cfg, scale, m)
    xe = spla.spsolve(A.tocsc(), b)
    its = []
    for f32 in (0, 1):
        g = Amg(coarse_max=64, tol_inner=1e-12, max_inner=200, relax_pre=b"FFCF", relax_post=b"FFCF",
                relax_pre_coarse=b"F", relax_post_coarse=b"F", coarse_fp32=f32)
        g.setup(A.indptr, A.indices, A.data)
        x, iters, rel, rc = g.solve(b)
        assert rc == B.PAIR_OK and rel[0] <= 1e-12
        assert np.linalg.norm(x - xe) <= 1e-10 * np.linalg.norm(xe)
        its.append(int(iters[0]))
    assert its[1] <= its[0] + 2, its


def test_segments_are_independent_and_bitwise_equal():
    """A block-diagonal batch of three matrices gives each segment exactly the
    hierarchy and iterates it gets alone."""
    need_gpu()
    mats = [_matrix(2, 5, 3), _matrix(3, 2, 1), _matrix(2, 5, 70)]
    blocks = sp.block_diag([a for a, _ in mats], format="csr")
    blocks.sort_indices()
    rhs = np.concatenate([b for _, b in mats])
    sizes = [a.shape[0] for a, _ in mats]
    seg = np.concatenate([[0], np.cumsum(sizes)])
    g = _amg(blocks, 32, seg=seg)
    xb, itb, relb, rc = g.solve(rhs)
    assert rc == B.PAIR_OK
    for k, (a, b) in enumerate(mats):
        s = _amg(a, 32)
        x, it, rel, rc1 = s.solve(b)
        assert rc1 == B.PAIR_OK
        assert itb[k] == it[0]
        assert np.array_equal(xb[seg[k]:seg[k + 1]], x)
        assert g.segment_levels(k) == s.num_levels()


def test_invalid_inputs_rejected():
    need_gpu()
    from paper_1910_11463_amd.solver import Amg
    a = Amg()
    A = sp.csr_matrix(np.array([[1.0, 0.5], [0.0, 0.0]]))   # row 1 lacks its diagonal entry
    A.eliminate_zeros()
    with pytest.raises(B.PairError):
        a.setup(A.indptr, A.indices, A.data)
    C = sp.csr_matrix(np.array([[1.0, 0.5], [0.5, 1.0]]))
    with pytest.raises(B.PairError):   # coupling across two one-row segments
        a.setup(C.indptr, C.indices, C.data, [0, 1, 2])


@pytest.mark.parametrize("cfg,scale,m,phi", [(2, 6, 5, 0.1), (3, 2, 7, 0.1), (5, 5, 13, 0.1),
                                             (4, 6, 40, 0.1), (3, 3, 5, 0.0), (1, 4, 0, 0.0)])
def test_nair_matches_reference(cfg, scale, m, phi):
    """Degree-1 nAIR, every coarsening step redone on the GPU from the oracle's
    level matrix: the C/F split exact, the restriction's kept pattern the
    oracle's except entries within 1e-9 (relative) of the phi_R threshold, its
    values within 1e-12 of the largest; with phi_R = 0 every computed entry
    is kept and the rows are compared densely."""
    need_gpu()
    from oracle import air_ref as AR
    A, _ = _matrix(cfg, scale, m)
    print("nAIR parity", cfg, scale, m, phi, A.shape, flush=True)
    ref = AR.setup(A, AR.Options(coarse_max=64, seed=3, nair_degree=1, filter_r=phi))
    assert len(ref) >= 2
    for l, L in enumerate(ref[:-1]):
        if L.cf is None:
            break
        one = AR.setup(L.A, AR.Options(coarse_max=64, seed=3, max_levels=2, nair_degree=1, filter_r=phi))
        full = AR.nair_restriction(L.A, one[0].cf, AR.Options(nair_degree=1)).tocsr()
        g = _amg(L.A, 64, 3, max_levels=2, filter_r=phi, nair_degree=1)
        got = g.level(0)
        g.close()
        assert np.array_equal(got["cf"], one[0].cf.astype(np.int8)), l
        rp, rc, rv = got["r_rowptr"], got["r_col"], got["r_val"]
        Rr = one[0].R.tocsr()
        scale_v = np.abs(full.data).max()
        cpts = np.flatnonzero(one[0].cf > 0)
        if phi == 0.0:
            dense_g = np.zeros((len(cpts), L.A.shape[0]))
            for I in range(len(cpts)):
                dense_g[I, rc[rp[I]:rp[I + 1]]] = rv[rp[I]:rp[I + 1]]
            assert np.abs(dense_g - full.toarray()).max() <= 1e-12 * scale_v, l
            continue
        for I, i in enumerate(cpts):
            c0 = full.indices[full.indptr[I]:full.indptr[I + 1]]
            v0 = full.data[full.indptr[I]:full.indptr[I + 1]]
            off = c0 != i
            thr = phi * (np.abs(v0[off]).max() if off.any() else 0.0)
            want = set(Rr.indices[Rr.indptr[I]:Rr.indptr[I + 1]].tolist())
            have = dict(zip(rc[rp[I]:rp[I + 1]].tolist(), rv[rp[I]:rp[I + 1]].tolist()))
            assert list(have) == sorted(have), (l, I)
            assert have.get(int(i)) == 1.0
            for c, v in zip(c0, v0):
                if c == i or abs(abs(v) - thr) <= 1e-9 * max(thr, 1e-300):
                    continue
                assert (c in have) == (c in want), (l, I, c)
                if c in have:
                    assert abs(have[c] - v) <= 1e-12 * scale_v, (l, I, c)


def _rowlen_matrix(n, lo, hi, diag, seed):
    """Random nonsymmetric matrix whose row i holds its diagonal and between
    lo - 1 and hi - 1 off-diagonal entries at random distinct columns."""
    rng = np.random.default_rng(seed)
    rows, cols, vals = [], [], []
    for i in range(n):
        k = int(rng.integers(lo, hi + 1))
        c = rng.choice(np.delete(np.arange(n), i), size=k - 1, replace=False)
        rows += [i] * k
        cols += [i] + c.tolist()
        vals += [rng.uniform(diag, 1.5 * diag)] + rng.uniform(-1.0, 1.0, k - 1).tolist()
    return sp.csr_matrix((vals, (rows, cols)), shape=(n, n))


@pytest.mark.parametrize("n,lo,hi,seed,diag,phi,over", [(3000, 12, 15, 3, 20.0, 0.5, (128,)),
                                                          (4000, 20, 34, 6, 20.0, 0.5, (256, 512)),
                                                          (3000, 12, 15, 3, 2.0, 0.2, (128,)),
                                                          (4000, 20, 34, 6, 3.0, 0.23, (256, 512))])
def test_nair_rows_deferred_to_larger_tables_match_reference(n, lo, hi, seed, diag, phi, over):
    """nAIR rows with more distinct columns than a table holds are finished by
    the next larger one: rows of at most 15 entries (first the 128-column
    table) of which some reach 129-151 distinct F columns, and rows of 20-34
    entries (first the 256-column table) that all reach more than 256 and some
    more than 512 (the 512-column table, then the 1024-column one).  With a
    weak diagonal and a low phi_R, deferred rows also keep more than 32
    entries (longer than their staging slot: computed again by the table that
    took them).  Split exact, kept pattern exact away from the phi_R threshold,
    values within 1e-12 of the largest."""
    need_gpu()
    from oracle import air_ref as AR
    A = _rowlen_matrix(n, lo, hi, diag, seed)
    one = AR.setup(A, AR.Options(coarse_max=64, seed=3, max_levels=2, nair_degree=1, filter_r=phi))
    full = AR.nair_restriction(A, one[0].cf, AR.Options(nair_degree=1)).tocsr()
    nf = np.diff(full.indptr) - 1          # distinct F columns of each row
    for c in over:
        assert (nf > c).any()
    kept = np.diff(one[0].R.indptr)
    if phi < 0.5:
        assert ((nf > over[0]) & (kept > 32)).any()
    print("nAIR deferral", n, lo, hi, "distinct F max", nf.max(), [(c, int((nf > c).sum())) for c in over],
          flush=True)
    g = _amg(A, 64, 3, max_levels=2, filter_r=phi, nair_degree=1)
    got = g.level(0)
    g.close()
    assert np.array_equal(got["cf"], one[0].cf.astype(np.int8))
    rp, rc, rv = got["r_rowptr"], got["r_col"], got["r_val"]
    Rr = one[0].R.tocsr()
    scale_v = np.abs(full.data).max()
    for I, i in enumerate(np.flatnonzero(one[0].cf > 0)):
        c0 = full.indices[full.indptr[I]:full.indptr[I + 1]]
        v0 = full.data[full.indptr[I]:full.indptr[I + 1]]
        off = c0 != i
        thr = phi * np.abs(v0[off]).max()
        want = set(Rr.indices[Rr.indptr[I]:Rr.indptr[I + 1]].tolist())
        have = dict(zip(rc[rp[I]:rp[I + 1]].tolist(), rv[rp[I]:rp[I + 1]].tolist()))
        assert list(have) == sorted(have) and have.get(int(i)) == 1.0, I
        for c, v in zip(c0, v0):
            if c == i or abs(abs(v) - thr) <= 1e-9 * thr:
                continue
            assert (c in have) == (c in want), (I, c)
            if c in have:
                assert abs(have[c] - v) <= 1e-12 * scale_v, (I, c)


def test_nair_transport_sweep_matches_exact_sweep():
    """A sweep replacement with nAIR hierarchies (degree 1, phi_R = 0.1) and
    F/C schedules converges to the oracle's exact sweep."""
    need_gpu()
    from oracle import source_iteration as si
    from tests.gpu_util import oracle_problem, rel, solver_for
    w = wl.make_config(2, scale=10)
    s = solver_for(w, tol_inner=1e-12, max_inner=300, batch_size=16, nair_degree=1, filter_r=0.1,
                   relax_pre="FCFCF", relax_post="FCFCF", relax_pre_coarse="F", relax_post_coarse="F")
    psi, phi, st, rc = s.transport_sweep(mode=B.PAIR_BATCHED)
    assert rc == B.PAIR_OK
    print("nAIR sweep: levels %d, V-cycles %d" % (st["levels_max"], st["vcycles_total"]), flush=True)
    ref = si.transport_sweep(oracle_problem(w), None)
    for k in range(len(ref)):
        assert rel(psi[k], ref[k]) <= 1e-9, (k, rel(psi[k], ref[k]))
    s.close()


def test_nair_rows_beyond_the_supported_length_are_rejected():
    """Unfiltered nAIR rows can keep more than 64 F entries (128 on the second
    level of this 6^3 S8 direction); the R A P kernels take at most 65 entries
    per row of R, so the setup reports an error instead of building them."""
    need_gpu()
    from oracle import air_ref as AR
    A, _ = _matrix(2, 6, 5)
    ref = AR.setup(A, AR.Options(coarse_max=64, seed=3, nair_degree=1))
    A1 = ref[1].A
    assert int(np.diff(AR.nair_restriction(A1, AR.setup(A1, AR.Options(
        coarse_max=64, seed=3, max_levels=2, nair_degree=1))[0].cf, AR.Options(nair_degree=1)).indptr).max()) > 65
    with pytest.raises(B.PairError) as e:
        _amg(A1, 64, 3, max_levels=2, nair_degree=1)
    assert "more than 64" in str(e.value)


def test_r_build_byte_count_matches_host_count():
    """The algorithmic bytes the lAIR row kernel adds up on the device (the
    figure behind the benchmark's roofline) equal the per-row formula evaluated
    on the host from the hierarchy it built (the row's pattern given, read from
    R): per C row 40 + 12 len_i + 4 (K + 1) + 16 K + 12 sum_{j in R_i} len_j +
    12 (K + 1)."""
    need_gpu()
    import ctypes
    A, _ = _matrix(2, 8, 5)
    B.check(B.pair_profile_enable(1))
    g = _amg(A, 64, 3)
    n, ms, by = ctypes.c_int64(), ctypes.c_double(), ctypes.c_double()
    B.check(B.pair_profile_read(5, ctypes.byref(n), ctypes.byref(ms), ctypes.byref(by)))
    B.check(B.pair_profile_enable(0))
    want = 0
    for l in range(g.num_levels() - 1):
        lv = g.level(l)
        rp, cf, rr, rc = lv["rowptr"], lv["cf"], lv["r_rowptr"], lv["r_col"]
        if rr is None:
            continue
        lens = np.diff(rp)
        for I, i in enumerate(np.flatnonzero(cf > 0)):
            cols = rc[rr[I]:rr[I + 1]]
            cols = cols[cols != i]
            K = len(cols)
            want += 40 + 12 * int(lens[i]) + 4 * (K + 1) + 16 * K + 12 * int(lens[cols].sum()) + 12 * (K + 1)
    print("r_build launches", n.value, "bytes", by.value, "host", want, flush=True)
    assert n.value > 0 and ms.value > 0.0
    assert int(by.value) == want
    g.close()


def test_rap_merge_byte_count_matches_host_count():
    """The algorithmic bytes the merging R (A P) kernel adds up on the device
    (a candidate for the benchmark's roofline kernel) equal the per-row formula
    evaluated on the host from the hierarchy it built: for every coarse row I
    whose row of R has rl <= 4 entries, 28 (list entry, two offsets in R, the
    output offset) + sum over its R entries k of (24 + 12 len_AP(k)) + 12 nnz of
    row I of the next level's operator, where len_AP(k) counts the distinct
    coarse points that the columns of row k of A interpolate from (one-point
    P)."""
    need_gpu()
    import ctypes
    A, _ = _matrix(2, 8, 5)
    B.check(B.pair_profile_enable(1))
    g = _amg(A, 64, 3)
    n, ms, by = ctypes.c_int64(), ctypes.c_double(), ctypes.c_double()
    B.check(B.pair_profile_read(8, ctypes.byref(n), ctypes.byref(ms), ctypes.byref(by)))
    B.check(B.pair_profile_enable(0))
    want = 0
    for l in range(g.num_levels() - 1):
        lv, nx = g.level(l), g.level(l + 1)
        rp, col, p, rr, rc = lv["rowptr"], lv["col"], lv["p"], lv["r_rowptr"], lv["r_col"]
        if rr is None:
            continue
        ap_len = {}
        clen = np.diff(nx["rowptr"])
        for I in range(len(rr) - 1):
            ks = rc[rr[I]:rr[I + 1]]
            if len(ks) > 4:
                continue
            row = 28 + 12 * int(clen[I])
            for k in ks:
                if k not in ap_len:
                    pk = p[col[rp[k]:rp[k + 1]]]
                    ap_len[k] = len(np.unique(pk[pk >= 0]))
                row += 24 + 12 * ap_len[k]
            want += row
    print("rap_merge launches", n.value, "bytes", by.value, "host", want, flush=True)
    assert n.value > 0 and ms.value > 0.0
    assert int(by.value) == want
    g.close()


def test_nair_rows_with_many_neighbours_match_reference():
    """nAIR rows with more F neighbours than the medium kernel holds (about 120
    per row here, above its 96) are finished by the large kernel: a random
    nonsymmetric matrix with 30% of entries filled, filtered with phi_R = 0.5,
    against the oracle on the same matrix (split exact, kept pattern exact away
    from the threshold, values within 1e-12)."""
    need_gpu()
    from oracle import air_ref as AR
    rng = np.random.default_rng(17)
    n = 400
    M = (rng.random((n, n)) < 0.3) * rng.uniform(-1.0, 1.0, (n, n))
    np.fill_diagonal(M, rng.uniform(40.0, 60.0, n))
    A = sp.csr_matrix(M)
    phi = 0.5
    one = AR.setup(A, AR.Options(coarse_max=64, seed=3, max_levels=2, nair_degree=1, filter_r=phi))
    full = AR.nair_restriction(A, one[0].cf, AR.Options(nair_degree=1)).tocsr()
    cpts = np.flatnonzero(one[0].cf > 0)
    fpts = one[0].cf < 0
    nn = [int(fpts[A.indices[A.indptr[i]:A.indptr[i + 1]]].sum()) for i in cpts]
    assert min(nn) > 96
    g = _amg(A, 64, 3, max_levels=2, filter_r=phi, nair_degree=1)
    got = g.level(0)
    g.close()
    assert np.array_equal(got["cf"], one[0].cf.astype(np.int8))
    rp, rc, rv = got["r_rowptr"], got["r_col"], got["r_val"]
    Rr = one[0].R.tocsr()
    scale_v = np.abs(full.data).max()
    for I, i in enumerate(cpts):
        c0 = full.indices[full.indptr[I]:full.indptr[I + 1]]
        v0 = full.data[full.indptr[I]:full.indptr[I + 1]]
        off = c0 != i
        thr = phi * np.abs(v0[off]).max()
        want = set(Rr.indices[Rr.indptr[I]:Rr.indptr[I + 1]].tolist())
        have = dict(zip(rc[rp[I]:rp[I + 1]].tolist(), rv[rp[I]:rp[I + 1]].tolist()))
        for c, v in zip(c0, v0):
            if c == i or abs(abs(v) - thr) <= 1e-9 * thr:
                continue
            assert (c in have) == (c in want), (I, c)
            if c in have:
                assert abs(have[c] - v) <= 1e-12 * scale_v


@pytest.mark.parametrize("cfg,scale,m,phi", [(2, 6, 5, 0.1), (3, 2, 7, 0.1), (5, 5, 13, 0.1), (4, 6, 40, 0.1),
                                             (2, 6, 5, 0.01), (1, 4, 0, 0.0), (3, 2, 7, 0.0), (2, 4, 17, 0.0),
                                             (2, 6, 5, 0.0), (5, 5, 13, 0.0), (4, 6, 40, 0.0)])
def test_distance2_matches_reference(cfg, scale, m, phi):
    """Distance-2 lAIR, every coarsening step redone on the GPU from the
    oracle's level matrix: the C/F split exact; the restriction's kept pattern
    the oracle's except entries within 1e-9 (relative) of the phi_R threshold;
    values within 1e-11 of the row set's largest (local systems of up to ~115
    unknowns here, eliminated in a different pivot order than LAPACK's); with
    phi_R = 0 the rows (up to 108 entries) are compared entry by entry."""
    need_gpu()
    from oracle import air_ref as AR
    A, _ = _matrix(cfg, scale, m)
    print("distance-2 parity", cfg, scale, m, phi, A.shape, flush=True)
    ref = AR.setup(A, AR.Options(coarse_max=64, seed=3, distance=2, filter_r=phi))
    assert len(ref) >= 2
    for l, L in enumerate(ref[:-1]):
        if L.cf is None:
            break
        one = AR.setup(L.A, AR.Options(coarse_max=64, seed=3, max_levels=2, distance=2, filter_r=phi))
        full = AR.lair_restriction(L.A, one[0].cf, AR.Options(distance=2)).tocsr()
        g = _amg(L.A, 64, 3, max_levels=2, filter_r=phi, lair_distance=2)
        got = g.level(0)
        g.close()
        assert np.array_equal(got["cf"], one[0].cf.astype(np.int8)), l
        rp, rc, rv = got["r_rowptr"], got["r_col"], got["r_val"]
        Rr = one[0].R.tocsr()
        scale_v = np.abs(full.data).max()
        cpts = np.flatnonzero(one[0].cf > 0)
        if phi == 0.0:
            assert np.array_equal(rp, full.indptr) and np.array_equal(rc, full.indices), l
            assert np.abs(rv - full.data).max() <= 1e-11 * scale_v, l
            continue
        for I, i in enumerate(cpts):
            c0 = full.indices[full.indptr[I]:full.indptr[I + 1]]
            v0 = full.data[full.indptr[I]:full.indptr[I + 1]]
            off = c0 != i
            thr = phi * (np.abs(v0[off]).max() if off.any() else 0.0)
            want = set(Rr.indices[Rr.indptr[I]:Rr.indptr[I + 1]].tolist())
            have = dict(zip(rc[rp[I]:rp[I + 1]].tolist(), rv[rp[I]:rp[I + 1]].tolist()))
            assert list(have) == sorted(have), (l, I)
            assert have.get(int(i)) == 1.0
            for c, v in zip(c0, v0):
                if c == i or abs(abs(v) - thr) <= 1e-9 * max(thr, 1e-300):
                    continue
                assert (c in have) == (c in want), (l, I, c)
                if c in have:
                    assert abs(have[c] - v) <= 1e-11 * scale_v, (l, I, c)


def test_distance2_transport_sweep_matches_exact_sweep():
    """A sweep replacement with distance-2 lAIR hierarchies (phi_R = 0.1) and
    tile-sweep schedules converges to the oracle's exact sweep."""
    need_gpu()
    from oracle import source_iteration as si
    from tests.gpu_util import oracle_problem, rel, solver_for
    w = wl.make_config(2, scale=10)
    s = solver_for(w, tol_inner=1e-12, max_inner=300, batch_size=16, lair_distance=2, filter_r=0.1,
                   relax_pre="TT", relax_post="TT", relax_pre_coarse="F", relax_post_coarse="F")
    psi, phi, st, rc = s.transport_sweep(mode=B.PAIR_BATCHED)
    assert rc == B.PAIR_OK
    print("distance-2 sweep: levels %d, V-cycles %d" % (st["levels_max"], st["vcycles_total"]), flush=True)
    ref = si.transport_sweep(oracle_problem(w), None)
    for k in range(len(ref)):
        assert rel(psi[k], ref[k]) <= 1e-9, (k, rel(psi[k], ref[k]))
    s.close()


def _random_matrix(n, fill, diag, seed):
    rng = np.random.default_rng(seed)
    M = (rng.random((n, n)) < fill) * rng.uniform(-1.0, 1.0, (n, n))
    np.fill_diagonal(M, rng.uniform(diag, 1.5 * diag, n))
    return sp.csr_matrix(M)


def test_distance2_long_rows_and_large_systems_match_reference():
    """Distance-2 rows of 90-291 entries (local systems of that size, rows of R
    staged in global memory by the R A P kernel): a random nonsymmetric 600 x 600
    matrix with 3% of entries filled, unfiltered, against the oracle: split
    exact, R's pattern exact and values within 1e-11 of the largest, and the
    Galerkin coarse operator within 1e-11 of its largest entry."""
    need_gpu()
    from oracle import air_ref as AR
    A = _random_matrix(600, 0.03, 10.0, 29)
    one = AR.setup(A, AR.Options(coarse_max=64, seed=3, max_levels=2, distance=2))
    R = one[0].R.tocsr()
    assert np.diff(R.indptr).min() > 65 and np.diff(R.indptr).max() > 256
    g = _amg(A, 64, 3, max_levels=2, lair_distance=2)
    got, coarse = g.level(0), g.level(1)
    g.close()
    assert np.array_equal(got["cf"], one[0].cf.astype(np.int8))
    assert np.array_equal(got["r_rowptr"], R.indptr) and np.array_equal(got["r_col"], R.indices)
    assert np.abs(got["r_val"] - R.data).max() <= 1e-11 * np.abs(R.data).max()
    Ac = one[1].A.toarray()
    n1 = Ac.shape[0]
    Cg = sp.csr_matrix((coarse["val"], coarse["col"], coarse["rowptr"]), shape=(n1, n1)).toarray()
    assert np.abs(Cg - Ac).max() <= 1e-11 * np.abs(Ac).max()


def test_distance2_limits_are_reported():
    """A local system of more than 512 F points (about 1430 here: a random
    1500 x 1500 matrix with 8% of entries filled reaches nearly every F point in
    two strong steps) is an error, and so is an unknown distance."""
    need_gpu()
    A = _random_matrix(1500, 0.08, 40.0, 23)
    with pytest.raises(B.PairError) as e:
        _amg(A, 64, 3, max_levels=2, lair_distance=2)
    assert "more than 512" in str(e.value)
    with pytest.raises(B.PairError) as e:
        _amg(A, 64, 3, max_levels=2, lair_distance=3)
    assert e.value.code == B.PAIR_E_INVALID
