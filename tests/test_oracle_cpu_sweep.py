"""The compiled structured-hex sweep (the timed CPU baseline) against the
NumPy oracle's assembly + exact sweep."""
import math

import numpy as np
import pytest

from paper_1910_11463_amd import workloads as wl
from oracle import cpu_sweep as CS, quadrature as Q, source_iteration as si


def _case(nx, ny, nz, order, seed):
    mesh = wl.hex_mesh(nx, ny, nz, lo=(0.0, -0.5, 0.25), hi=(1.0, 1.5, 0.75))
    rng = np.random.default_rng(seed)
    E = mesh.n_elem
    st = rng.uniform(0.1, 5.0, E)
    ss = st * rng.uniform(0.0, 0.9, E)
    q = rng.uniform(0.0, 2.0, E)
    om, w = Q.level_symmetric(order)
    return mesh, st, ss, q, om, w


@pytest.mark.parametrize("dims,order", [((3, 4, 5), 4), ((4, 2, 3), 8), ((1, 1, 1), 2)])
def test_cpu_sweep_matches_numpy_oracle(dims, order):
    mesh, st, ss, q, om, w = _case(*dims, order, seed=sum(dims))
    phi = np.random.default_rng(1).uniform(0.0, 1.0, mesh.n_dof)
    prob = si.Problem(mesh, st, ss, q, om, w)
    ref = si.transport_sweep(prob, phi)
    psi, phi_out = CS.sweep_all(mesh, st, ss, q, om, w, phi=phi, threads=3)
    assert np.abs(psi - ref).max() <= 1e-13 * np.abs(ref).max()
    assert np.abs(phi_out - si.scalar_flux(prob, ref)).max() <= 1e-13 * np.abs(phi_out).max()


def test_cpu_sweep_zero_components_and_thread_invariance():
    """Directions on the coordinate planes and axes (no flux through the
    parallel faces), and bitwise equal results for any thread count."""
    mesh, st, ss, q, _, _ = _case(3, 3, 4, 4, seed=9)
    s2 = math.sqrt(0.5)
    om = np.array([[1.0, 0.0, 0.0], [0.0, -1.0, 0.0], [s2, 0.0, -s2], [0.0, s2, s2],
                   [-0.6, 0.0, 0.8]])
    w = np.full(5, 4 * math.pi / 5)
    prob = si.Problem(mesh, st, ss, q, om, w)
    ref = si.transport_sweep(prob, None)
    psi1, phi1 = CS.sweep_all(mesh, st, ss, q, om, w, threads=1)
    psi4, phi4 = CS.sweep_all(mesh, st, ss, q, om, w, threads=4)
    assert np.abs(psi1 - ref).max() <= 1e-13 * np.abs(ref).max()
    assert np.array_equal(psi1, psi4) and np.array_equal(phi1, phi4)
