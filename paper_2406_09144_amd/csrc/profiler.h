// Optional per-kernel timing: when enabled, every instrumented launch is
// bracketed by a pair of hipEvents recorded on its own stream; fr_profile_query
// sums the elapsed times per name.  Disabled (the default) it costs one branch.
#pragma once

#include "common.h"

namespace frmi {

constexpr size_t kProfilerPoolEvents = 8192;

struct ProfRec {
    hipEvent_t a, b;
};

struct Profiler {
    std::mutex mu;
    bool on = false;
    std::map<std::string, std::vector<ProfRec>> recs;
    std::vector<hipEvent_t> pool;
    hipEvent_t get_event() {
        if (!pool.empty()) {
            hipEvent_t e = pool.back();
            pool.pop_back();
            return e;
        }
        hipEvent_t e;
        HIP_CHECK(hipEventCreate(&e));
        return e;
    }
};

Profiler &profiler();

struct ProfScope {
    const char *name = nullptr;
    hipStream_t st = nullptr;
    hipEvent_t a = nullptr;
    ProfScope(const char *n, hipStream_t s) {
        Profiler &P = profiler();
        if (!P.on) return;
        std::lock_guard<std::mutex> g(P.mu);
        name = n;
        st = s;
        a = P.get_event();
        HIP_CHECK(hipEventRecord(a, st));
    }
    ~ProfScope() {
        if (!name) return;
        Profiler &P = profiler();
        std::lock_guard<std::mutex> g(P.mu);
        hipEvent_t b = P.get_event();
        if (hipEventRecord(b, st) == hipSuccess) P.recs[name].push_back({a, b});
    }
};

}  // namespace frmi
