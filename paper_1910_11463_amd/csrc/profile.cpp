// Event-pair kernel timing (see profile.h).
#include "profile.h"

#include <mutex>
#include <vector>

#include <rocprofiler-sdk-roctx/roctx.h>

#include "common.h"

namespace pair {
namespace {
struct Rec {
    hipEvent_t a, b;
    int kind;
    double bytes;
    int slot;     // >= 0: bytes are in the device counters of this slot
};
std::mutex g_mu;
bool g_on = false;
bool g_extra = false;    // also the profiling-only passes (PROF_RBUILD_ONCE)
std::vector<Rec> g_recs;
std::vector<hipEvent_t> g_pool;
constexpr int kMaxSlots = 4096;
unsigned long long* g_slots = nullptr;   // kMaxSlots x kProfSubSlots, zeroed when enabled
int g_next_slot = 0;

hipEvent_t take_event() {
    if (!g_pool.empty()) {
        hipEvent_t e = g_pool.back();
        g_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    PAIR_HIP(hipEventCreate(&e));
    return e;
}
}  // namespace

thread_local bool t_suspended = false;

TraceRange::TraceRange(const char* name) { roctxRangePushA(name); }
TraceRange::~TraceRange() { roctxRangePop(); }

bool prof_enabled() { return g_on; }

ProfSuspend::ProfSuspend() : prev(t_suspended) { t_suspended = true; }
ProfSuspend::~ProfSuspend() { t_suspended = prev; }

int prof_begin(hipStream_t s, int kind) {
    if (!g_on || t_suspended || kind < 0 || kind >= PROF_NKINDS) return -1;
    if (kind == PROF_RBUILD_ONCE && !g_extra) return -1;
    hipStreamCaptureStatus st = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(s, &st) != hipSuccess || st != hipStreamCaptureStatusNone) {
        (void)hipGetLastError();
        return -1;
    }
    std::lock_guard<std::mutex> g(g_mu);
    Rec r{take_event(), take_event(), kind, 0.0, -1};
    PAIR_HIP(hipEventRecord(r.a, s));
    g_recs.push_back(r);
    return static_cast<int>(g_recs.size()) - 1;
}

void prof_end(hipStream_t s, int h, double bytes) {
    if (h < 0) return;
    std::lock_guard<std::mutex> g(g_mu);
    PAIR_HIP(hipEventRecord(g_recs[h].b, s));
    g_recs[h].bytes = bytes;
}

unsigned long long* prof_dev_bytes(int h) {
    if (h < 0) return nullptr;
    std::lock_guard<std::mutex> g(g_mu);
    if (!g_slots || g_next_slot >= kMaxSlots) return nullptr;
    g_recs[h].slot = g_next_slot++;
    return g_slots + static_cast<size_t>(g_recs[h].slot) * kProfSubSlots;
}

void prof_end_dev(hipStream_t s, int h) {
    if (h < 0) return;
    std::lock_guard<std::mutex> g(g_mu);
    PAIR_HIP(hipEventRecord(g_recs[h].b, s));
}

void prof_enable(int on) {
    std::lock_guard<std::mutex> g(g_mu);
    g_extra = on >= 2;
    if (on) {
        for (auto& r : g_recs) {
            (void)hipEventSynchronize(r.b);
            g_pool.push_back(r.a);
            g_pool.push_back(r.b);
        }
        g_recs.clear();
        const size_t bytes = sizeof(unsigned long long) * kMaxSlots * kProfSubSlots;
        if (!g_slots) PAIR_HIP(hipMalloc(&g_slots, bytes));
        PAIR_HIP(hipDeviceSynchronize());
        PAIR_HIP(hipMemset(g_slots, 0, bytes));
        PAIR_HIP(hipDeviceSynchronize());
        g_next_slot = 0;
    }
    g_on = on != 0;
}

void prof_read(int kind, int64_t* launches, double* total_ms, double* total_bytes) {
    std::lock_guard<std::mutex> g(g_mu);
    int64_t n = 0;
    double ms = 0.0, by = 0.0;
    std::vector<unsigned long long> slots;
    for (auto& r : g_recs) {
        if (r.kind != kind) continue;
        PAIR_HIP(hipEventSynchronize(r.b));
        float t = 0.f;
        PAIR_HIP(hipEventElapsedTime(&t, r.a, r.b));
        ms += t;
        if (r.slot >= 0) {
            if (slots.empty()) {
                slots.resize(static_cast<size_t>(g_next_slot) * kProfSubSlots);
                PAIR_HIP(hipMemcpy(slots.data(), g_slots, slots.size() * sizeof(unsigned long long),
                                   hipMemcpyDeviceToHost));
            }
            for (int k = 0; k < kProfSubSlots; ++k)
                by += static_cast<double>(slots[static_cast<size_t>(r.slot) * kProfSubSlots + k]);
        } else {
            by += r.bytes;
        }
        ++n;
    }
    if (launches) *launches = n;
    if (total_ms) *total_ms = ms;
    if (total_bytes) *total_bytes = by;
}

}  // namespace pair
