"""Level-symmetric S_N angular quadrature (oracle; test infrastructure only).

The scalar flux is the weighted direction sum phi = sum_m w_m psi_m
(Introduction, eq. angular_quad).  The paper's weak-scaling runs use a square
Chebyshev-Legendre S4 set; the workloads here use level-symmetric S2/S4/S8 sets,
normalised so that sum w = 4*pi (phi is the integral over the unit sphere,
eq. mono_transport).

Construction (standard LQ_n): direction cosines mu_i^2 = mu_1^2 + (i-1)*D,
D = 2(1 - 3 mu_1^2)/(N - 2); the points of one octant are the triples
(mu_i, mu_j, mu_k) with i + j + k = N/2 + 2.  Weights are constant on each
permutation class and fixed by even moment conditions:
  S4: one class, mu_1 from <mu^4> = 1/5;
  S8: three classes, mu_1 = 0.2182179 (tabulated), weights from
      normalisation, <mu^4> = 1/5 and <mu^6> = 1/7.

Ordering: octant-major, octant o has sign bits (x: bit 0, y: bit 1, z: bit 2;
a set bit means a negative cosine); inside an octant the triples are
enumerated with i ascending, then j ascending.  The reflection -Omega of the
direction (o, triple) is the direction (o ^ 7, same triple).

Pinned by: sum w = 4 pi; odd moments vanish; <mu^2> = 1/3, <mu^4> = 1/5; the
tabulated 7-digit cosines and weights (tests/golden/ls_quadrature.txt).
"""
from __future__ import annotations

import math

import numpy as np

S8_MU1 = 0.2182179


def _mu_levels(N: int) -> np.ndarray:
    n = N // 2
    if N == 2:
        return np.array([1.0 / math.sqrt(3.0)])
    if N == 4:
        # 6 u^2 - 4 u + 2/5 = 0 (from 2 mu1^4 + mu2^4 = 3/5 with mu2^2 = 1 - 2 mu1^2)
        u = (4.0 - math.sqrt(16.0 - 9.6)) / 12.0
        mu1sq = u
    elif N == 8:
        mu1sq = S8_MU1 * S8_MU1
    else:
        raise ValueError("only S2, S4, S8 are provided")
    D = 2.0 * (1.0 - 3.0 * mu1sq) / (N - 2)
    return np.sqrt(np.array([mu1sq + i * D for i in range(n)]))


def _octant_triples(N: int):
    n = N // 2
    s = n + 2  # i + j + k, 1-based
    out = []
    for i in range(1, n + 1):
        for j in range(1, n + 1):
            k = s - i - j
            if 1 <= k <= n:
                out.append((i, j, k))
    return out


def _class_of(t):
    return tuple(sorted(t))


def level_symmetric(N: int):
    """Return (omega [M,3], w [M]) with sum(w) = 4*pi."""
    mu = _mu_levels(N)
    trip = _octant_triples(N)
    classes = sorted(set(_class_of(t) for t in trip))
    # weight per class from moment conditions on one octant (octant weights sum to 1)
    ncls = len(classes)
    if ncls == 1:
        wc = {classes[0]: 1.0 / len(trip)}
    else:
        rows = []
        rhs = []
        # normalisation
        rows.append([sum(1 for t in trip if _class_of(t) == c) for c in classes])
        rhs.append(1.0)
        for p, val in ((4, 1.0 / 5.0), (6, 1.0 / 7.0))[: ncls - 1]:
            rows.append([sum(mu[t[0] - 1] ** p for t in trip if _class_of(t) == c) for c in classes])
            rhs.append(val)
        sol = np.linalg.solve(np.array(rows, dtype=np.float64), np.array(rhs))
        wc = {c: sol[ic] for ic, c in enumerate(classes)}
    omega = []
    w = []
    for o in range(8):
        sx = -1.0 if (o & 1) else 1.0
        sy = -1.0 if (o & 2) else 1.0
        sz = -1.0 if (o & 4) else 1.0
        for t in trip:
            omega.append((sx * mu[t[0] - 1], sy * mu[t[1] - 1], sz * mu[t[2] - 1]))
            w.append(wc[_class_of(t)] * 4.0 * math.pi / 8.0)
    return np.array(omega, dtype=np.float64), np.array(w, dtype=np.float64)


def reflected_index(N: int, m: int) -> int:
    """Index of the direction -Omega_m."""
    per = len(_octant_triples(N))
    o, r = divmod(m, per)
    return (o ^ 7) * per + r
