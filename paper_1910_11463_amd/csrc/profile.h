// Optional per-kernel timing with HIP events recorded on the launching stream.
// When enabled (pair_profile_enable), selected launch sites record an event pair
// around the launch and the algorithmic bytes that launch must move; reads
// synchronise the events and sum durations per kernel kind.  Timing is skipped
// while a stream is being captured into a graph.
#pragma once

#include <hip/hip_runtime.h>

namespace pair {

// A named range for tracing tools (roctx push/pop on the calling thread):
// rocprofv3 --marker-trace shows it beside the kernels it encloses.
struct TraceRange {
    explicit TraceRange(const char* name);
    ~TraceRange();
    TraceRange(const TraceRange&) = delete;
    TraceRange& operator=(const TraceRange&) = delete;
};

enum ProfKind : int {
    PROF_RELAX_FINE = 0,     // finest-level relaxation (F/C half-sweeps, tile sweeps)
    PROF_RESIDUAL_FINE = 1,  // r = b - A x on the finest level
    PROF_RESTRICT_FINE = 2,  // b_c = R r from the finest level
    PROF_RELAX_COARSE = 3,   // half-sweeps on all coarser levels
    PROF_NORM_FINE = 4,      // convergence test on the finest level
    PROF_RBUILD = 5,         // lAIR rows with dense local systems (coarser levels' setup)
    PROF_RBUILD_ONCE = 6,    // the same launches, a gathered row of A counted once per launch
    PROF_RPATTERN = 7,       // the lAIR rows' patterns selected before their local systems
    PROF_RAP_MERGE = 8,      // R (A P) rows of at most four R entries, by merging (numeric pass)
    PROF_NKINDS = 9
};

bool prof_enabled();
// While alive, the calling thread records nothing (no events are created and
// no records grow): used where a call must not allocate.
struct ProfSuspend {
    ProfSuspend();
    ~ProfSuspend();
    ProfSuspend(const ProfSuspend&) = delete;
    ProfSuspend& operator=(const ProfSuspend&) = delete;
    bool prev;
};
// Returns a handle for prof_end (or -1 when disabled / capturing).
int prof_begin(hipStream_t s, int kind);
void prof_end(hipStream_t s, int handle, double bytes);
// For kernels whose algorithmic bytes depend on data only the device sees: a
// zeroed device array of kProfSubSlots counters the launch adds its bytes to
// (any entry; they are summed when read), or nullptr when the handle is -1.
// Close such a launch with prof_end_dev instead of prof_end.
constexpr int kProfSubSlots = 64;
unsigned long long* prof_dev_bytes(int handle);
void prof_end_dev(hipStream_t s, int handle);

}  // namespace pair
