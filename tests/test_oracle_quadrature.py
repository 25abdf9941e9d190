"""Pins of the oracle's level-symmetric quadrature (phi = sum w psi, eq. angular_quad)."""
import math
import os

import numpy as np
import pytest

from oracle import quadrature as Q

GOLD = os.path.join(os.path.dirname(__file__), "golden", "ls_quadrature.txt")


def _golden():
    mu, w = {}, {}
    for line in open(GOLD):
        line = line.split("#")[0].split()
        if not line:
            continue
        order = int(line[0][1:])
        if line[1] == "mu":
            mu[order] = [float(v) for v in line[2:]]
        else:
            w.setdefault(order, {})[tuple(int(c) for c in line[2])] = float(line[3])
    return mu, w


@pytest.mark.parametrize("N,M", [(2, 8), (4, 24), (8, 80)])
def test_counts_and_weight_sum(N, M):
    om, w = Q.level_symmetric(N)
    assert om.shape == (M, 3) and w.shape == (M,)
    assert abs(w.sum() - 4 * math.pi) < 1e-13
    assert np.allclose(np.linalg.norm(om, axis=1), 1.0, atol=1e-15)


@pytest.mark.parametrize("N", [2, 4, 8])
def test_moments(N):
    om, w = Q.level_symmetric(N)
    for d in range(3):
        # odd moments vanish
        assert abs(np.dot(w, om[:, d])) < 1e-13
        assert abs(np.dot(w, om[:, d] ** 3)) < 1e-13
        assert abs(np.dot(w, om[:, d] ** 2) / (4 * math.pi) - 1.0 / 3.0) < 1e-14
        if N >= 4:
            assert abs(np.dot(w, om[:, d] ** 4) / (4 * math.pi) - 0.2) < 1e-14
    assert abs(np.dot(w, om[:, 0] * om[:, 1])) < 1e-13
    assert abs(np.dot(w, om[:, 0] * om[:, 1] * om[:, 2])) < 1e-13


@pytest.mark.parametrize("N", [2, 4, 8])
def test_reflection_pairs(N):
    om, w = Q.level_symmetric(N)
    for m in range(om.shape[0]):
        r = Q.reflected_index(N, m)
        assert np.array_equal(om[r], -om[m])
        assert w[r] == w[m]


@pytest.mark.parametrize("N", [2, 4, 8])
def test_tabulated_values(N):
    gmu, gw = _golden()
    om, w = Q.level_symmetric(N)
    levels = np.unique(np.round(np.abs(om), 12))
    assert np.allclose(levels, gmu[N], atol=6e-8)
    for m in range(om.shape[0]):
        cls = tuple(sorted(int(np.argmin(np.abs(np.array(gmu[N]) - abs(c)))) + 1 for c in om[m]))
        assert abs(w[m] * 8 / (4 * math.pi) - gw[N][cls]) < 6e-8
