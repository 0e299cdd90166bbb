// host_common.hpp -- host-side helpers shared by the translation units of
// libpald: size arithmetic, launch status, and the device-time records that
// PALD_FLAG_TIMING calls leave for pald_timings_collect.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <mutex>
#include <vector>

#include "pald.h"

namespace pald_host {

constexpr size_t ALIGN = 256;

inline size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }
inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

// rows of an elementwise n x n kernel are grid-strided over gridDim.y <= 65535
inline unsigned rows_grid(int64_t n) { return (unsigned)std::min<int64_t>(n, 65535); }

inline bool aligned16(const void *p) { return (reinterpret_cast<uintptr_t>(p) & 15u) == 0; }

inline pald_status launch_status() {
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? PALD_OK : PALD_ERR_DEVICE;
}

// ---- timing records -------------------------------------------------------
// Kinds: 0 pass-1 focus sizes, 1 weights, 2 pass-2 cohesion, 3 finalize,
// 4 batched persistent kernel, 5-7 triplet pass 1 / pass 2 / finalize,
// 8 distances, 9 local depths, 10 strong-tie count + scan, 11 strong-tie fill,
// 12 graph distances, 13 row-block pass 1, 14 row-block pass 2, 15 host <->
// device copies of the out-of-core mode.
constexpr int NUM_KINDS = 16;

struct TimingRec {
    int kind;
    hipEvent_t start, stop;
};

inline std::mutex &timing_mutex() {
    static std::mutex m;
    return m;
}

inline std::vector<TimingRec> &timing_records() {
    static std::vector<TimingRec> v;
    return v;
}

// Records a start event now and a stop event when the scope ends, on stream s.
struct ScopedTiming {
    bool on;
    int kind;
    hipStream_t s;
    hipEvent_t a = nullptr, b = nullptr;
    ScopedTiming(bool on_, int kind_, hipStream_t s_) : on(on_), kind(kind_), s(s_) {
        if (on) {
            if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess) {
                on = false;
                return;
            }
            (void)hipEventRecord(a, s);
        }
    }
    ~ScopedTiming() {
        if (!on) return;
        (void)hipEventRecord(b, s);
        std::lock_guard<std::mutex> g(timing_mutex());
        timing_records().push_back({kind, a, b});
    }
    ScopedTiming(const ScopedTiming &) = delete;
    ScopedTiming &operator=(const ScopedTiming &) = delete;
};

}  // namespace pald_host
