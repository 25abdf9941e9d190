"""Reference AIR (approximate ideal restriction) AMG on small sparse matrices.

Oracle code: TEST INFRASTRUCTURE ONLY.  Plain NumPy/SciPy, one step at a time,
in the order the paper describes the method (Sec. "Use of Algebraic Multigrid",
Sec. "SOC Parameter for Building R"):

1. strength of connection for coarsening: j is strong for row i when
   |a_ij| >= theta * max_{k != i} |a_ik|   (absolute values, theta = 0.25);
2. C/F splitting of the strength graph (PMIS, a parallel maximal-independent-set
   split; the paper uses Falgout coarsening, which on one process reduces to a
   sequential first pass, so a parallel split is used here and on the GPU);
   as an option on the finest level, the Ruge-Stueben first pass inside given
   row groups (``Options.cf_groups``, ``rs_first_pass``), the per-processor
   pass of that coarsening, to study its effect on convergence;
3. restriction R by local approximate ideal restriction (lAIR): for each
   C-point i, the F-points strongly connected to i in the R-strength sense
   (eq. soc with epsilon_R = 0.01, absolute values) form R_i, and the row
   r_i = [z, 1] solves A(R_i, R_i)^T z = -A(i, R_i)^T, so that (r_i A)(R_i) = 0;
   the ideal restriction [-A_cf A_ff^{-1}, I] is the limit where R_i is all F;
4. interpolation "by value": each F-point takes the value of its strongest
   strongly-connected C-point (one-point interpolation), C-points by injection;
5. Petrov-Galerkin coarse operator A_c = R A P;
6. recursion until the level is small (<= 64 rows), coarsening stalls
   (n_c > 0.9 n) or 25 levels; a dense LU at the coarsest level;
7. V(1,1) cycles with FC-Jacobi relaxation: one Jacobi sweep over the
   F-points, then one over the C-points, before and after the coarse
   correction (omega = 1).

Readings where the paper is silent are the same as the GPU library's and are
listed in the design notes: absolute-value strength for both thresholds,
PMIS measure lambda_i + hash, smallest-column tie-break for one-point
interpolation, at most ``kmax`` entries per local solve (the strongest kept).

The PMIS measure uses SplitMix64 (Steele, Lea & Flood, "Fast splittable
pseudorandom number generators", OOPSLA 2014) on the key
seed*2^40 + level*2^32 + i; the GPU library implements the same published
generator on its own.

Pinned by (tests/test_oracle_strength.py): the strength test and the kmax
truncation on hand-written rows whose strong sets and truncated
neighbourhoods are written out by hand (diagonal outside the maximum, ">=" on
the threshold, absolute values, stored zeros, ties by smaller column).
Pinned by (tests/test_oracle_air.py): the ideal-restriction identities
(R A P equals the Schur complement A_cc - A_cf A_ff^{-1} A_fc for any
one-point P; a two-level cycle with ideal R, exact F-solve and exact coarse
solve is exact), the lAIR defining identity (R A)(i, R_i) = 0, PMIS validity
(independence and coverage), dense R @ A @ P, and convergence of the V-cycle to
the exact sweep answer; the Ruge-Stueben first pass by a chain whose split is
worked out by hand, by its invariants on random graphs (every C point's
dependents are F, no C point depends on another, an F point either has no
dependents or depends on a C point, the first C point has the largest
measure) and by its groups (links between groups dropped).  Convergence
*rates* are not pinned by the paper's numbers (parity unpinned; Table 5 only
gives a sanity range).
"""
from __future__ import annotations

import dataclasses
import heapq
from typing import List, Optional

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

MASK64 = (1 << 64) - 1


def splitmix64(x: int) -> int:
    z = (x + 0x9E3779B97F4A7C15) & MASK64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK64
    return z ^ (z >> 31)


def pmis_random(i: int, level: int, seed: int) -> int:
    """53-bit random integer of row i on a level."""
    key = ((seed << 40) + (level << 32) + i) & MASK64
    return splitmix64(key) >> 11


@dataclasses.dataclass
class Options:
    theta: float = 0.25
    eps_r: float = 0.01
    distance: Optional[int] = 1       # 1, 2, or None (= all F points: ideal R)
    kmax: int = 64
    omega: float = 1.0
    coarse_max: int = 64
    max_levels: int = 25
    max_coarse_ratio: float = 0.9
    seed: int = 0
    relax_pre: str = "FC"      # half-sweeps before the coarse correction
    relax_post: str = "FC"     # and after it ("FFC": F, F, then C)
    filter_r: float = 0.0      # phi_R: drop R entries below phi_R * row max (0: keep all)
    nair_degree: int = 0       # > 0: nAIR restriction of this Neumann degree instead of lAIR
    # finest level only: the Ruge-Stueben first pass inside these row groups
    # (one group id per row) instead of PMIS; coarser levels keep PMIS
    cf_groups: Optional[np.ndarray] = None


def _rows(A: sp.csr_matrix):
    for i in range(A.shape[0]):
        s, e = A.indptr[i], A.indptr[i + 1]
        yield i, A.indices[s:e], A.data[s:e]


def offdiag_rowmax(A: sp.csr_matrix) -> np.ndarray:
    out = np.zeros(A.shape[0])
    for i, cols, vals in _rows(A):
        m = 0.0
        for c, v in zip(cols, vals):
            if c != i and abs(v) > m:
                m = abs(v)
        out[i] = m
    return out


def strength(A: sp.csr_matrix, eps: float) -> sp.csr_matrix:
    """Boolean matrix S with S[i,j] = 1 when j != i and
    |a_ij| >= eps * max_{k != i} |a_ik| (a row with no off-diagonal, or whose
    off-diagonals are all zero, has no strong entries)."""
    mx = offdiag_rowmax(A)
    r, c = [], []
    for i, cols, vals in _rows(A):
        if mx[i] == 0.0:
            continue
        for j, v in zip(cols, vals):
            if j != i and abs(v) >= eps * mx[i]:
                r.append(i)
                c.append(j)
    n = A.shape[0]
    return sp.csr_matrix((np.ones(len(r), dtype=np.int8), (r, c)), shape=(n, n))


def pmis(S: sp.csr_matrix, level: int, seed: int) -> np.ndarray:
    """cf[i] = +1 (C) / -1 (F).

    measure(i) = (lambda_i, rand_i, i) compared lexicographically, with
    lambda_i = #{j : S[j,i]} (how many points strongly depend on i).
    Points with lambda_i = 0 start as F.  Each round, an undecided point whose
    measure exceeds that of every undecided neighbour in S + S^T becomes C;
    then every undecided point that strongly depends on a new C-point becomes F.
    """
    n = S.shape[0]
    ST = S.T.tocsr()
    lam = np.diff(ST.indptr)
    rnd = [pmis_random(i, level, seed) for i in range(n)]
    key = [(int(lam[i]), rnd[i], i) for i in range(n)]
    nbrs = []
    for i in range(n):
        a = set(S.indices[S.indptr[i]:S.indptr[i + 1]].tolist())
        b = set(ST.indices[ST.indptr[i]:ST.indptr[i + 1]].tolist())
        a |= b
        a.discard(i)
        nbrs.append(sorted(a))
    cf = np.zeros(n, dtype=np.int64)
    cf[lam == 0] = -1
    while np.any(cf == 0):
        und = np.flatnonzero(cf == 0)
        newc = [i for i in und if all(cf[j] != 0 or key[j] < key[i] for j in nbrs[i])]
        for i in newc:
            cf[i] = 1
        newc_set = set(newc)
        for i in und:
            if cf[i] != 0:
                continue
            deps = S.indices[S.indptr[i]:S.indptr[i + 1]]
            if any(j in newc_set for j in deps):
                cf[i] = -1
    return cf


def coarse_index(cf: np.ndarray) -> np.ndarray:
    ci = np.full(cf.shape[0], -1, dtype=np.int64)
    c = np.flatnonzero(cf > 0)
    ci[c] = np.arange(c.size)
    return ci


def _r_pattern(A: sp.csr_matrix, SR: sp.csr_matrix, cf, i: int, opts: Options):
    """F-points of the local ideal-restriction neighbourhood of C-point i."""
    row_cols = A.indices[A.indptr[i]:A.indptr[i + 1]]
    row_vals = A.data[A.indptr[i]:A.indptr[i + 1]]
    if opts.distance is None:
        cand = list(np.flatnonzero(cf < 0))
        return sorted(cand)
    strong = set(SR.indices[SR.indptr[i]:SR.indptr[i + 1]].tolist())
    d1 = [j for j in strong if cf[j] < 0]
    if opts.distance == 1:
        # keep at most kmax: largest |a_ij|, ties by smaller column
        if len(d1) > opts.kmax:
            mag = {int(c): abs(v) for c, v in zip(row_cols, row_vals)}
            d1 = sorted(d1, key=lambda j: (-mag[j], j))[:opts.kmax]
        return sorted(d1)
    out = set(d1)
    for j in d1:
        for k in SR.indices[SR.indptr[j]:SR.indptr[j + 1]]:
            if cf[k] < 0 and k != i:
                out.add(int(k))
    return sorted(out)


def lair_restriction(A: sp.csr_matrix, cf: np.ndarray, opts: Options) -> sp.csr_matrix:
    SR = strength(A, opts.eps_r)
    ci = coarse_index(cf)
    Ad = A.tocsc()
    rows, cols, vals = [], [], []
    Acsr = A.tocsr()
    for i in np.flatnonzero(cf > 0):
        Rset = _r_pattern(Acsr, SR, cf, int(i), opts)
        if Rset:
            sub = Acsr[Rset, :][:, Rset].toarray()             # A(R_i, R_i)
            rhs = -Acsr[int(i), Rset].toarray().ravel()        # -A(i, R_i)
            z = np.linalg.solve(sub.T, rhs)
        else:
            z = np.zeros(0)
        entries = list(zip(Rset, z))
        if opts.filter_r > 0.0 and len(z):
            # filtering of R after its construction (Sec. "SOC Parameter for
            # Building R"): the strength test of eq. (soc) with tolerance phi_R
            # applied to the computed row; the C point's own entry always stays
            zmax = float(np.abs(z).max())
            entries = [(j, v) for j, v in entries if abs(v) >= opts.filter_r * zmax]
        entries = entries + [(int(i), 1.0)]
        entries.sort()
        for j, v in entries:
            rows.append(ci[i])
            cols.append(j)
            vals.append(v)
    del Ad
    nc = int((cf > 0).sum())
    R = sp.csr_matrix((vals, (rows, cols)), shape=(nc, A.shape[0]))
    R.sort_indices()
    return R


def _filter_rows(R: sp.csr_matrix, ci_of_row: np.ndarray, phi: float) -> sp.csr_matrix:
    """Filtering of R after its construction (Sec. "SOC Parameter for Building
    R"): in row I an entry off the C point's own column ci_of_row[I] stays iff
    |r| >= phi * max over the row's other off-C entries; the C entry stays."""
    R = R.tocsr()
    rows, cols, vals = [], [], []
    for I in range(R.shape[0]):
        c = R.indices[R.indptr[I]:R.indptr[I + 1]]
        v = R.data[R.indptr[I]:R.indptr[I + 1]]
        off = c != ci_of_row[I]
        zmax = float(np.abs(v[off]).max()) if off.any() else 0.0
        keep = ~off | (np.abs(v) >= phi * zmax)
        rows += [I] * int(keep.sum())
        cols += c[keep].tolist()
        vals += v[keep].tolist()
    out = sp.csr_matrix((vals, (rows, cols)), shape=R.shape)
    out.sort_indices()
    return out


def nair_restriction(A: sp.csr_matrix, cf: np.ndarray, opts: Options) -> sp.csr_matrix:
    """Restriction by a truncated Neumann series (nAIR, Sec. "Use of Algebraic
    Multigrid"; the paper cites the method without a formula, so this follows
    the ideal restriction [-A_cf A_ff^{-1}, I] with A_ff^{-1} replaced by its
    Neumann series around the diagonal, truncated after degree d):

        R_cf = -A_cf  sum_{k=0..d} (I - D_ff^{-1} A_ff)^k  D_ff^{-1},   R = [R_cf, I],

    D_ff the diagonal of A_ff, all entries of A (no strength test), then the
    same filtering with phi_R as lAIR.  Rows are the C points in index order."""
    A = A.tocsr()
    F = np.flatnonzero(cf < 0)
    C = np.flatnonzero(cf > 0)
    n = A.shape[0]
    Aff = A[F, :][:, F]
    Acf = A[C, :][:, F]
    Dinv = sp.diags(1.0 / Aff.diagonal())
    M = sp.identity(len(F), format="csr") - Dinv @ Aff
    S = sp.identity(len(F), format="csr")
    term = sp.identity(len(F), format="csr")
    for _ in range(opts.nair_degree):
        term = term @ M
        S = S + term
    Rcf = -(Acf @ S @ Dinv)
    Rcf = Rcf.tocoo()
    rows = np.concatenate([Rcf.row, np.arange(len(C))])
    cols = np.concatenate([F[Rcf.col], C])
    vals = np.concatenate([Rcf.data, np.ones(len(C))])
    R = sp.csr_matrix((vals, (rows, cols)), shape=(len(C), n))
    R.sum_duplicates()
    R.sort_indices()
    if opts.filter_r > 0.0:
        R = _filter_rows(R, C, opts.filter_r)
    return R


def one_point_interp(A: sp.csr_matrix, S: sp.csr_matrix, cf: np.ndarray) -> np.ndarray:
    """p[i] = coarse column of row i of P (value 1), or -1 for an empty row."""
    ci = coarse_index(cf)
    p = np.full(A.shape[0], -1, dtype=np.int64)
    for i in range(A.shape[0]):
        if cf[i] > 0:
            p[i] = ci[i]
            continue
        strong = set(S.indices[S.indptr[i]:S.indptr[i + 1]].tolist())
        best, bj = -1.0, -1
        for j, v in zip(A.indices[A.indptr[i]:A.indptr[i + 1]], A.data[A.indptr[i]:A.indptr[i + 1]]):
            if j in strong and cf[j] > 0:
                if abs(v) > best or (abs(v) == best and j < bj):
                    best, bj = abs(v), int(j)
        if bj >= 0:
            p[i] = ci[bj]
    return p


def p_matrix(p: np.ndarray, nc: int) -> sp.csr_matrix:
    n = p.shape[0]
    has = p >= 0
    return sp.csr_matrix((np.ones(int(has.sum())), (np.flatnonzero(has), p[has])), shape=(n, nc))


def galerkin(R: sp.csr_matrix, A: sp.csr_matrix, P: sp.csr_matrix) -> sp.csr_matrix:
    """R A P with the structural pattern of the products (no cancellation drop):
    row I of the result gathers r_Ik * a_kj for every k in row I of R and every
    j in row k of A that P maps to a coarse column."""
    Pc = P.tocsr()
    pcol = np.full(P.shape[0], -1, dtype=np.int64)
    for i in range(P.shape[0]):
        if Pc.indptr[i + 1] > Pc.indptr[i]:
            pcol[i] = Pc.indices[Pc.indptr[i]]
    rows, cols, vals = [], [], []
    for I in range(R.shape[0]):
        acc = {}
        for k, rv in zip(R.indices[R.indptr[I]:R.indptr[I + 1]], R.data[R.indptr[I]:R.indptr[I + 1]]):
            for j, av in zip(A.indices[A.indptr[k]:A.indptr[k + 1]], A.data[A.indptr[k]:A.indptr[k + 1]]):
                J = pcol[j]
                if J >= 0:
                    acc[J] = acc.get(J, 0.0) + rv * av
        for J in sorted(acc):
            rows.append(I)
            cols.append(J)
            vals.append(acc[J])
    Ac = sp.csr_matrix((vals, (rows, cols)), shape=(R.shape[0], P.shape[1]))
    Ac.sort_indices()
    return Ac


@dataclasses.dataclass
class Level:
    A: sp.csr_matrix
    cf: Optional[np.ndarray] = None
    R: Optional[sp.csr_matrix] = None
    p: Optional[np.ndarray] = None
    P: Optional[sp.csr_matrix] = None


def rs_first_pass(S: sp.csr_matrix, groups: Optional[np.ndarray] = None) -> np.ndarray:
    """Ruge-Stueben first pass (the splitting the paper's Falgout coarsening runs
    inside each processor's rows, Sec. "Weak Scaling with Parallelism in Space"):
    cf[i] = +1 (C) / -1 (F).  With `groups`, strong links between rows of
    different groups are dropped first (a processor sees only its own rows).

    lambda_i = #{j : S[j,i]} (points strongly depending on i); points with
    lambda_i = 0 start as F.  Repeatedly the undecided point with the largest
    lambda (ties: the smaller index) becomes C; every undecided point that
    strongly depends on it becomes F, and each such new F point raises by one
    the lambda of every undecided point it strongly depends on (an F dependent
    counts twice); the new C point lowers by one the lambda of every undecided
    point it strongly depends on (a C point no longer counts)."""
    n = S.shape[0]
    S = sp.csr_matrix(S)
    if groups is not None:
        C = S.tocoo()
        keep = groups[C.row] == groups[C.col]
        S = sp.csr_matrix((np.ones(int(keep.sum()), dtype=np.int8), (C.row[keep], C.col[keep])), shape=(n, n))
    ST = S.T.tocsr()
    lam = np.diff(ST.indptr).astype(np.int64)
    cf = np.zeros(n, dtype=np.int64)
    cf[lam == 0] = -1
    heap = [(-int(lam[i]), i) for i in range(n) if cf[i] == 0]
    heapq.heapify(heap)
    while heap:
        negl, i = heapq.heappop(heap)
        if cf[i] != 0 or -negl != lam[i]:
            continue                       # decided, or a stale entry
        cf[i] = 1
        for j in ST.indices[ST.indptr[i]:ST.indptr[i + 1]]:      # j depends on i
            if cf[j] == 0:
                cf[j] = -1
                for k in S.indices[S.indptr[j]:S.indptr[j + 1]]:   # j depends on k
                    if cf[k] == 0:
                        lam[k] += 1
                        heapq.heappush(heap, (-int(lam[k]), int(k)))
        for k in S.indices[S.indptr[i]:S.indptr[i + 1]]:          # i depends on k
            if cf[k] == 0:
                lam[k] -= 1
                heapq.heappush(heap, (-int(lam[k]), int(k)))
    return cf


def setup(A: sp.csr_matrix, opts: Options = Options()) -> List[Level]:
    levels = []
    A = sp.csr_matrix(A)
    A.sort_indices()
    for lev in range(opts.max_levels):
        L = Level(A=A)
        levels.append(L)
        n = A.shape[0]
        if n <= opts.coarse_max or lev == opts.max_levels - 1:
            break
        S = strength(A, opts.theta)
        if lev == 0 and opts.cf_groups is not None:
            cf = rs_first_pass(S, opts.cf_groups)
        else:
            cf = pmis(S, lev, opts.seed)
        nc = int((cf > 0).sum())
        if nc == 0 or nc > opts.max_coarse_ratio * n:
            break
        L.cf = cf
        L.R = nair_restriction(A, cf, opts) if opts.nair_degree > 0 else lair_restriction(A, cf, opts)
        L.p = one_point_interp(A, S, cf)
        L.P = p_matrix(L.p, nc)
        A = galerkin(L.R, A, L.P)
    return levels


def _relax(A, d, b, x, mask, omega):
    r = b - A @ x
    x = x.copy()
    x[mask] += omega * r[mask] / d[mask]
    return x


def hex_tiles(nx: int, ny: int, nz: int, tx: int, ty: int, tz: int) -> np.ndarray:
    """Tile index of every row of a structured nx*ny*nz hex mesh (element
    e = i + nx (j + ny k), 8 rows per element): boxes of tx*ty*tz elements
    anchored at the origin, the last box along an axis cut by the mesh."""
    e = np.arange(nx * ny * nz)
    i, j, k = e % nx, (e // nx) % ny, e // (nx * ny)
    mx, my = -(-nx // tx), -(-ny // ty)
    t = (i // tx) + mx * ((j // ty) + my * (k // tz))
    return np.repeat(t, 8)


TET_TILE_TARGET = 384      # mean tets per tile when the box count is automatic


def tet_tile_boxes(E: int, nbox: int = 0) -> int:
    """Boxes per axis of the tet tiles: nbox if > 0, else the smallest count
    with E <= 384 nbox^3 (a box of about 4 x 4 x 4 Kuhn cubes)."""
    if nbox > 0:
        return nbox
    n = 1
    while E > TET_TILE_TARGET * n ** 3:
        n += 1
    return n


def tet_tiles(xyz: np.ndarray, elem_vert: np.ndarray, nbox: int = 0) -> np.ndarray:
    """Tile index of every row of a P1 tet mesh (4 rows per element, DOF 4 t + a):
    the mesh's bounding box cut into nbox^3 equal boxes, an element in the box of
    its centroid ((x0 + x1 + x2 + x3) / 4, summed in vertex order; a coordinate
    exactly on the far face goes to the last box)."""
    xyz = np.asarray(xyz, dtype=np.float64)
    ev = np.asarray(elem_vert, dtype=np.int64)
    nb = tet_tile_boxes(ev.shape[0], nbox)
    X = xyz[ev]                                   # [E,4,3]
    c = (((X[:, 0] + X[:, 1]) + X[:, 2]) + X[:, 3]) * 0.25
    lo = xyz.min(axis=0)
    hi = xyz.max(axis=0)
    q = np.floor((c - lo) / (hi - lo) * nb).astype(np.int64)
    q = np.clip(q, 0, nb - 1)
    t = q[:, 0] + nb * (q[:, 1] + nb * q[:, 2])
    return np.repeat(t, 4)


class TileSolver:
    """Block Jacobi over tiles with exact local solves (the paper's relaxation by
    an on-processor solve, Sec. "Use of Algebraic Multigrid": each processor
    inverts its principal submatrix exactly; here a "processor" is a tile of
    elements): x <- x + M^{-1} (b - A x), M the part of A that couples rows of
    one tile to rows of the same tile.  The local solve is a sparse LU of M."""

    def __init__(self, A: sp.csr_matrix, tiles: np.ndarray):
        C = A.tocoo()
        keep = tiles[C.row] == tiles[C.col]
        M = sp.csc_matrix((C.data[keep], (C.row[keep], C.col[keep])), shape=A.shape)
        self.lu = spla.splu(M)

    def relax(self, A, b, x):
        return x + self.lu.solve(b - A @ x)


def vcycle(levels: List[Level], b: np.ndarray, x: np.ndarray, lev: int = 0,
           omega: float = 1.0, pre: str = "FC", post: str = "FC", pre_c=None,
           post_c=None, tiles: Optional[TileSolver] = None) -> np.ndarray:
    """One V-cycle; each character of pre/post is one Jacobi half-sweep over the
    F-points ("F") or the C-points ("C"), or on the finest level one tile sweep
    ("T", undamped, needs `tiles`); pre_c/post_c (default: the same) apply on
    the coarser levels."""
    L = levels[lev]
    if lev > 0:
        pre = pre if pre_c is None else pre_c
        post = post if post_c is None else post_c
    if lev == len(levels) - 1:
        return np.linalg.solve(L.A.toarray(), b)
    d = L.A.diagonal()
    F = L.cf < 0
    C = ~F

    def smooth(x, ch):
        if ch == "T":
            if lev != 0 or tiles is None:
                raise ValueError("tile sweeps need the finest level and a TileSolver")
            return tiles.relax(L.A, b, x)
        return _relax(L.A, d, b, x, F if ch == "F" else C, omega)

    for ch in pre:
        x = smooth(x, ch)
    r = b - L.A @ x
    bc = L.R @ r
    pc = pre if pre_c is None else pre_c
    qc = post if post_c is None else post_c
    xc = vcycle(levels, bc, np.zeros(L.R.shape[0]), lev + 1, omega, pc, qc)
    x = x + L.P @ xc
    for ch in post:
        x = smooth(x, ch)
    return x


def solve(levels: List[Level], b: np.ndarray, tol: float = 1e-10, maxit: int = 200,
          x0=None, omega: float = 1.0, pre: str = "FC", post: str = "FC", pre_c=None,
          post_c=None, tiles: Optional[TileSolver] = None):
    A = levels[0].A
    x = np.zeros_like(b) if x0 is None else x0.copy()
    nb = np.linalg.norm(b)
    hist = []
    for it in range(maxit):
        rel = np.linalg.norm(b - A @ x) / nb if nb > 0 else 0.0
        hist.append(rel)
        if rel <= tol:
            return x, it, hist
        x = vcycle(levels, b, x, 0, omega, pre, post, pre_c, post_c, tiles)
    rel = np.linalg.norm(b - A @ x) / nb
    hist.append(rel)
    return x, maxit, hist
