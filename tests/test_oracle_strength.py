"""Pins of the oracle's strength of connection (eq. soc, Sec. "SOC Parameter for
Building R"; thresholds of Sec. "Weak Scaling with Parallelism in Space") and
of the kmax truncation of the distance-1 lAIR neighbourhood, on small
hand-written matrices whose strong sets are written out by hand.

The reading pinned here: j != i is strong for row i when
|a_ij| >= eps * max_{k != i} |a_ik| (absolute values, the diagonal outside the
maximum, ">=" so that an entry exactly at the threshold is strong); a row whose
off-diagonals are all zero has no strong entries.  Each row is built so that a
plausible misreading gives a different set:
  * the diagonal inside the maximum (rows 0, 3, 4),
  * ">" instead of ">=" (entries sitting exactly on the threshold: rows 0, 3, 4, 5),
  * signed values (negative-only couplings, or the signed maximum: rows 0, 1),
  * explicitly stored zeros counted as strong (row 2).
Thresholds are exact in binary: 0.25 * 2.0 = 0.5, 0.25 * 4.0 = 1.0,
0.01 * 1.0 = 0.01.
"""
import numpy as np
import pytest
import scipy.sparse as sp

from oracle import air_ref as AR


def _hand_matrix():
    rows = {
        # diag 10 > every off-diagonal; max_{k!=0} = 2, 0.25 * 2 = 0.5 exactly
        0: {0: 10.0, 1: 2.0, 2: -0.5, 3: 0.49, 4: -1.0},
        # a signed pair of equal magnitude
        1: {0: 0.75, 1: 1.0, 2: -0.75, 3: 0.1},
        # off-diagonals stored but zero
        2: {0: 0.0, 2: 3.0, 4: 0.0},
        # tiny diagonal, max 4 -> threshold 1.0 exactly (entry 4 sits on it)
        3: {0: 4.0, 2: 0.999, 3: 0.01, 4: 1.0},
        # negative diagonal larger than the off-diagonals; 0.25 exactly at threshold
        4: {1: -1.0, 3: 0.25, 4: -5.0},
        # eps_R-sized entries: 0.01 * 1.0 = 0.01 exactly
        5: {0: 1.0, 1: 0.01, 2: -0.0099, 5: 1.0},
    }
    n = 6
    r, c, v = [], [], []
    for i, row in rows.items():
        for j, a in row.items():
            r.append(i)
            c.append(j)
            v.append(a)
    # built from triplets, so the zeros of row 2 stay stored entries
    A = sp.csr_matrix((np.array(v), (np.array(r), np.array(c))), shape=(n, n))
    A.sum_duplicates()
    A.sort_indices()
    return A


def _sets(S):
    S = S.tocsr()
    return {i: sorted(S.indices[S.indptr[i]:S.indptr[i + 1]].tolist()) for i in range(S.shape[0])}


def test_stored_zeros_are_kept_by_the_fixture():
    A = _hand_matrix()
    cols2 = A.indices[A.indptr[2]:A.indptr[3]].tolist()
    assert cols2 == [0, 2, 4]          # the zeros of row 2 are stored entries


def test_strength_theta_quarter_hand_sets():
    got = _sets(AR.strength(_hand_matrix(), 0.25))
    want = {
        0: [1, 2, 4],      # 0.49 < 0.5 <= 0.5 (col 2), 1.0, 2.0
        1: [0, 2],         # both signs of 0.75; 0.1 < 0.1875
        2: [],             # all off-diagonals zero
        3: [0, 4],         # 0.999 < 1.0 <= 1.0 (col 4)
        4: [1, 3],         # max 1 (diagonal -5 outside), 0.25 on the threshold
        5: [0],            # 0.01 and 0.0099 below 0.25
    }
    assert got == want


def test_strength_eps_r_hand_sets():
    got = _sets(AR.strength(_hand_matrix(), 0.01))
    want = {
        0: [1, 2, 3, 4],   # threshold 0.02
        1: [0, 2, 3],      # threshold 0.0075
        2: [],
        3: [0, 2, 4],      # threshold 0.04: the diagonal 0.01 is never a candidate
        4: [1, 3],
        5: [0, 1],         # 0.01 exactly on the threshold, 0.0099 below
    }
    assert got == want


def test_offdiag_rowmax_excludes_the_diagonal():
    mx = AR.offdiag_rowmax(_hand_matrix())
    assert mx.tolist() == [2.0, 0.75, 0.0, 4.0, 1.0, 1.0]


def _kmax_matrix():
    # row 0 is a C point; its strong F neighbours have |a| = 3, 2, 2, 1 (a tie
    # between columns 2 and 3); column 5 is a C point (never in R_i) with the
    # largest entry; column 6 is a weak F neighbour (below eps_R * 5)
    A = np.eye(7)
    A[0, 1:7] = [3.0, -2.0, 2.0, 1.0, 5.0, 0.04]
    for i in range(1, 7):
        A[i, 0] = 0.1 * i          # something for the local systems to see
    A[2, 3] = 0.3
    A[3, 1] = -0.2
    return sp.csr_matrix(A)


@pytest.mark.parametrize("kmax,want", [(1, [1]), (2, [1, 2]), (3, [1, 2, 3]), (4, [1, 2, 3, 4]),
                                       (64, [1, 2, 3, 4])])
def test_kmax_truncation_keeps_largest_with_smaller_column_on_ties(kmax, want):
    A = _kmax_matrix()
    cf = np.array([1, -1, -1, -1, -1, 1, -1])
    opts = AR.Options(kmax=kmax)
    SR = AR.strength(A, opts.eps_r)
    got = AR._r_pattern(A.tocsr(), SR, cf, 0, opts)
    assert got == want


def test_kmax_truncated_row_satisfies_the_local_identity():
    """(R A)(0, R_0) = 0 on the truncated neighbourhood, and the row holds
    exactly R_0 plus the C point itself."""
    A = _kmax_matrix()
    cf = np.array([1, -1, -1, -1, -1, 1, -1])
    R = AR.lair_restriction(A, cf, AR.Options(kmax=2))
    r0 = R.getrow(0)
    assert sorted(r0.indices.tolist()) == [0, 1, 2]
    RA = (r0 @ A).toarray().ravel()
    assert np.abs(RA[[1, 2]]).max() <= 1e-14
    assert abs(r0[0, 0] - 1.0) == 0.0
