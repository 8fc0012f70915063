// pd_internal.h -- host-side helpers shared by the C ABI sources of libpd:
// the per-launch event timing registry (pd_timing_enable / pd_timing_read)
// and the HIP error-to-status macro.
#pragma once
#include <hip/hip_runtime.h>

#include <vector>

namespace pd {

struct TimedLaunch {
    int kclass, level;
    hipEvent_t a, b;
};
inline bool g_timing = false;
inline std::vector<TimedLaunch> g_launches;

// Runs launch(); with timing on, brackets it with events on stream st.
template <typename F>
hipError_t timed(int kclass, int level, hipStream_t st, F &&launch)
{
    if (!g_timing) return launch();
    TimedLaunch t{kclass, level, nullptr, nullptr};
    hipError_t e;
    if ((e = hipEventCreate(&t.a)) != hipSuccess) return e;
    if ((e = hipEventCreate(&t.b)) != hipSuccess) return e;
    if ((e = hipEventRecord(t.a, st)) != hipSuccess) return e;
    e = launch();
    if (e != hipSuccess) return e;
    if ((e = hipEventRecord(t.b, st)) != hipSuccess) return e;
    g_launches.push_back(t);
    return hipSuccess;
}

inline void clear_timing()
{
    for (auto &t : g_launches) {
        (void)hipEventDestroy(t.a);
        (void)hipEventDestroy(t.b);
    }
    g_launches.clear();
}

inline size_t align_up(size_t v) { return (v + 255) & ~size_t(255); }

}  // namespace pd

#define PD_TRY_HIP(expr)                             \
    do {                                             \
        if ((expr) != hipSuccess) return PD_ERR_HIP; \
    } while (0)
