"""CPU FP64 oracle for the pAIR S_N transport hot path.

TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the CPU
baseline leg of the benchmark may import, call, link or execute anything in
this package.  The product path (the HIP library and its Python binding) never
uses it and shares no code with it: the only common module is the seeded input
generator, which holds none of the method's arithmetic.

What it computes, and from which passage of the paper:

* ``quadrature``  -- level-symmetric S_N sets, phi = sum_m w_m psi_m
  (Introduction, eq. angular_quad).
* ``elements``    -- closed-form Q1 hex / P1 tet element matrices
  (upwind DG weak form, eq. weak_form_transport; isoparametric multilinear
  elements).
* ``dg``          -- per-direction block operator (diagonal blocks D_e,
  upwind coupling blocks), left block-inverse scaling (Sec. "Sweeping with
  pAIR": scaling by the block inverse gives a unit diagonal), right-hand
  sides (eq. sn_transport).
* ``sweep``       -- exact block forward solve in topological order ("sweep",
  Sec. "Solution of the Transport Equation by Sweeping"); strongly connected
  components solved densely.  The loop is in plain C (``sweep.c``).
* ``source_iteration`` -- lagged-scalar-flux iteration (eq. sn_transport) and
  the dense block system of Sec. "Accuracy of Spatial Solves" on tiny meshes.
* ``air_ref``     -- AIR setup and V-cycle on small sparse matrices, in the
  order the paper describes it (Sec. "Use of Algebraic Multigrid",
  "SOC Parameter for Building R"): strength, C/F split, local ideal
  restriction, one-point interpolation by value, R A P.
* ``adjoint``     -- adjoint source iteration and dJ/dsigma_t, dJ/dsigma_s.
* ``mms``         -- manufactured solution of the Appendix.

Parity status of each function is stated in its docstring ("pinned by ..." or
"parity unpinned").
"""
