"""Pins of the oracle's closed-form element matrices against quadrature
computed here, independently (Gauss rules on the reference element)."""
import numpy as np
import pytest

from oracle import elements as el

GL = np.polynomial.legendre.leggauss


def _hex_basis(t):
    """Q1 basis on [0,1]^3 and its reference gradient at point t (local node
    a = ax + 2ay + 4az)."""
    vals, grads = np.zeros(8), np.zeros((8, 3))
    for a in range(8):
        f = [t[d] if (a >> d) & 1 else 1 - t[d] for d in range(3)]
        df = [1.0 if (a >> d) & 1 else -1.0 for d in range(3)]
        vals[a] = f[0] * f[1] * f[2]
        grads[a] = [df[0] * f[1] * f[2], f[0] * df[1] * f[2], f[0] * f[1] * df[2]]
    return vals, grads


@pytest.mark.parametrize("h", [(1.0, 1.0, 1.0), (0.125, 0.25, 0.5)])
def test_hex_volume_terms_vs_gauss(h):
    om = np.array([0.3, -0.5, 0.81])
    om /= np.linalg.norm(om)
    x, w = GL(3)
    x, w = 0.5 * (x + 1), 0.5 * w
    M = np.zeros((8, 8))
    C = np.zeros((8, 8))
    J = np.prod(h)
    for i in range(3):
        for j in range(3):
            for k in range(3):
                v, g = _hex_basis((x[i], x[j], x[k]))
                g = g / np.array(h)
                wt = w[i] * w[j] * w[k] * J
                M += wt * np.outer(v, v)
                C += wt * np.outer(g @ om, v)   # row a: Omega.grad phi_a, col b: phi_b
    assert np.allclose(el.hex_mass(*h), M, rtol=0, atol=1e-15 * J * 10)
    assert np.allclose(el.hex_advection(*h, om), C, rtol=0, atol=1e-14)
    # column sums over the test index vanish, 1^T M 1 = volume
    assert np.allclose(el.hex_advection(*h, om).sum(axis=0), 0.0, atol=1e-15)
    assert abs(el.hex_mass(*h).sum() - J) < 1e-15


@pytest.mark.parametrize("axis,side", [(a, s) for a in range(3) for s in range(2)])
def test_hex_face_terms_vs_gauss(axis, side):
    h = (0.5, 0.25, 0.125)
    x, w = GL(3)
    x, w = 0.5 * (x + 1), 0.5 * w
    others = [d for d in range(3) if d != axis]
    F = np.zeros((8, 8))
    X = np.zeros((8, 8))
    area = h[others[0]] * h[others[1]]
    for i in range(3):
        for j in range(3):
            t = [0.0, 0.0, 0.0]
            t[axis] = float(side)
            t[others[0]], t[others[1]] = x[i], x[j]
            v, _ = _hex_basis(t)
            tu = list(t)
            tu[axis] = 1.0 - side            # same point seen from the neighbour
            vu, _ = _hex_basis(tu)
            F += w[i] * w[j] * area * np.outer(v, v)
            X += w[i] * w[j] * area * np.outer(v, vu)
    assert np.allclose(el.hex_face_mass(*h, axis, side), F, atol=1e-16)
    assert np.allclose(el.hex_face_cross(*h, axis, side), X, atol=1e-16)


def test_tet_terms_vs_quadrature():
    rng = np.random.default_rng(7)
    Xv = rng.uniform(-1, 1, size=(4, 3))
    om = np.array([0.2, 0.7, -0.3])
    om /= np.linalg.norm(om)
    vol, grads = el.tet_geometry(Xv)
    # independent: volume from the scalar triple product, gradients from the
    # face-area vectors grad(lambda_a) = -A_a n_a / (3 |T|)
    assert abs(vol - abs(np.dot(Xv[1] - Xv[0], np.cross(Xv[2] - Xv[0], Xv[3] - Xv[0]))) / 6) < 1e-15
    for a in range(4):
        o = [b for b in range(4) if b != a]
        nvec = 0.5 * np.cross(Xv[o[1]] - Xv[o[0]], Xv[o[2]] - Xv[o[0]])
        if np.dot(Xv[a] - Xv[o[0]], nvec) > 0:
            nvec = -nvec
        assert np.allclose(grads[a], -nvec / (3 * vol), atol=1e-13)
    # 4-point degree-2 rule (Keast): barycentric (a,b,b,b), weights 1/4
    A, B = 0.5854101966249685, 0.1381966011250105
    M = np.zeros((4, 4))
    C = np.zeros((4, 4))
    for p in range(4):
        lam = np.full(4, B)
        lam[p] = A
        M += 0.25 * vol * np.outer(lam, lam)
        C += 0.25 * vol * np.outer(grads @ om, lam)
    assert np.allclose(el.tet_mass(vol), M, atol=1e-15)
    assert np.allclose(el.tet_advection(vol, grads, om), C, atol=1e-14)
    # triangle face mass with the edge-midpoint rule (exact for degree 2)
    area = 0.37
    Fm = np.zeros((3, 3))
    for e in range(3):
        lam = np.full(3, 0.5)
        lam[e] = 0.0
        Fm += area / 3 * np.outer(lam, lam)
    assert np.allclose(el.tri_face_mass(area), Fm, atol=1e-16)
