"""Writes c5_fd_gradients.txt: central finite differences (step 1e-6) of the
detector functional J = int_Det phi on the 32^3 S4 adjoint workload, at the
workload's 16 seeded elements, for sigma_t (sigma_s held fixed) and sigma_s
(sigma_t held fixed).  Calls only the oracle: the compiled exact sweep
(oracle/cpu_sweep.c, pinned to the NumPy oracle) inside source iteration
(eq. sn_transport), and the oracle's detector vector.

Each perturbed J starts source iteration from the unperturbed fixed point and
runs a fixed number of sweeps (with the spectral radius ~0.44 of this
workload the perturbation's own error contracts far below rounding), so the
difference quotient is limited by rounding in J (~1e-16 relative), not by the
iteration.  Run: python tests/golden/make_c5_fd.py [threads]
"""
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from paper_1910_11463_amd import workloads as wl          # noqa: E402
from oracle import adjoint as ADJ, cpu_sweep as CS, quadrature as Q, source_iteration as si  # noqa: E402

STEP = 1e-6
BASE_SWEEPS = 90
PERTURBED_SWEEPS = 50


def fixed_point(w, st, ss, om, wt, phi0, sweeps, threads):
    phi = np.zeros(w.mesh.n_dof) if phi0 is None else phi0.copy()
    psi = np.empty((om.shape[0], w.mesh.n_dof))
    rel = None
    for _ in range(sweeps):
        _, new = CS.sweep_all(w.mesh, st, ss, w.mats.q, om, wt, phi=phi, threads=threads, psi=psi)
        rel = np.linalg.norm(new - phi) / np.linalg.norm(new)
        phi = new
    return phi, rel


def main():
    threads = int(sys.argv[1]) if len(sys.argv) > 1 else 0
    w = wl.make_config(5)
    om, wt = Q.level_symmetric(w.sn_order)
    prob = si.Problem(w.mesh, w.mats.sigma_t, w.mats.sigma_s, w.mats.q, om, wt)
    c = ADJ.detector_source(prob, w.detector)
    st0, ss0 = w.mats.sigma_t, w.mats.sigma_s
    phi0, rel0 = fixed_point(w, st0, ss0, om, wt, None, BASE_SWEEPS, threads)
    J0 = float(c @ phi0)
    print("base J %.17e, last update %.2e" % (J0, rel0), flush=True)
    lines = []
    for e in w.fd_elems:
        g = []
        for which in ("t", "s"):
            vals = []
            for sg in (1.0, -1.0):
                st, ss = st0.copy(), ss0.copy()
                (st if which == "t" else ss)[e] += sg * STEP
                phi, rel = fixed_point(w, st, ss, om, wt, phi0, PERTURBED_SWEEPS, threads)
                vals.append(float(c @ phi))
            g.append((vals[0] - vals[1]) / (2.0 * STEP))
        print("element %d: dJ/dsigma_t %.10e dJ/dsigma_s %.10e (last update %.1e)" % (e, g[0], g[1], rel),
              flush=True)
        lines.append("%d %.17e %.17e" % (e, g[0], g[1]))
    out = os.path.join(os.path.dirname(os.path.abspath(__file__)), "c5_fd_gradients.txt")
    with open(out, "w") as f:
        f.write("# Central finite differences (step %.0e) of J = int_Det phi on the 32^3 Q1 hex,\n"
                "# S4 adjoint workload (sigma_t log-uniform [0.5, 5] seed 5, sigma_s = 0.8 sigma_t,\n"
                "# q = 1 in [0,0.25]^3, detector [0.75,1]^3), source iteration with the oracle's\n"
                "# exact sweep (eq. sn_transport).  Written by tests/golden/make_c5_fd.py.\n"
                "# J %.17e\n"
                "# element  dJ/dsigma_t  dJ/dsigma_s\n" % (STEP, J0))
        f.write("\n".join(lines) + "\n")
    print("wrote", out)


if __name__ == "__main__":
    main()
