"""pAIR S_N transport on MI355X (gfx950): hand-written HIP kernels behind a C ABI.

Modules (imported on demand; importing the package loads nothing):
  binding   -- ctypes binding of include/pair.h under the C names
  solver    -- Solver / Amg convenience wrappers and the TransportSolve autograd op
  workloads -- seeded synthetic meshes and materials
  build     -- builds libpair.so in-tree with hipcc
"""
__all__ = ["binding", "solver", "workloads", "build"]
