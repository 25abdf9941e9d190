// Optional per-kernel timing with HIP events recorded on the launching stream.
// When enabled (pair_profile_enable), selected launch sites record an event pair
// around the launch and the algorithmic bytes that launch must move; reads
// synchronise the events and sum durations per kernel kind.  Timing is skipped
// while a stream is being captured into a graph.
#pragma once

#include <hip/hip_runtime.h>

namespace pair {

enum ProfKind : int {
    PROF_RELAX_FINE = 0,     // FC-Jacobi half-sweeps on the finest level
    PROF_RESIDUAL_FINE = 1,  // r = b - A x on the finest level
    PROF_RESTRICT_FINE = 2,  // b_c = R r from the finest level
    PROF_RELAX_COARSE = 3,   // half-sweeps on all coarser levels
    PROF_NORM_FINE = 4,      // convergence test on the finest level
    PROF_NKINDS = 5
};

bool prof_enabled();
// Returns a handle for prof_end (or -1 when disabled / capturing).
int prof_begin(hipStream_t s, int kind);
void prof_end(hipStream_t s, int handle, double bytes);

}  // namespace pair
