// Host-layer environment switches.
//
// GHN_FAULT=alloc[:N] | launch[:N]   fault injection for the error paths: the N-th
//     (default: first) device allocation, or launch check, made after the variable
//     took its current value fails (hipErrorOutOfMemory, hipErrorLaunchFailure);
//     the others succeed.  Counting restarts whenever the value changes.  The kernels
//     themselves are untouched: an injected launch failure only changes the status
//     the host layer sees.
// GHN_LOG=1   one line on stderr per entry-point call, per failure, and per device
//     allocation and release of the library (so a test can check that nothing leaks).
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>

#include "ghn_internal.h"

namespace ghn {

namespace {

struct FaultPlan {
    std::mutex mu;
    std::string seen;     // the value the counters belong to
    long alloc_at = 0;    // fail this allocation (1-based), 0 = never
    long launch_at = 0;   // fail this launch check (1-based), 0 = never
    long allocs = 0, launches = 0;
};
FaultPlan g_plan;

// Parse "alloc", "alloc:N", "launch", "launch:N"; anything else injects nothing.
void parse_plan(const std::string& v, long* alloc_at, long* launch_at) {
    *alloc_at = *launch_at = 0;
    const size_t colon = v.find(':');
    const std::string what = v.substr(0, colon);
    long n = 1;
    if (colon != std::string::npos) {
        char* end = nullptr;
        n = std::strtol(v.c_str() + colon + 1, &end, 10);
        if (!end || *end != '\0' || n < 1) return;
    }
    if (what == "alloc") *alloc_at = n;
    else if (what == "launch") *launch_at = n;
}

// Count one event of the given kind; true if it is the one to fail.
bool injected(bool alloc) {
    const char* env = std::getenv("GHN_FAULT");
    std::lock_guard<std::mutex> lock(g_plan.mu);
    const std::string v = env ? env : "";
    if (v != g_plan.seen) {
        g_plan.seen = v;
        parse_plan(v, &g_plan.alloc_at, &g_plan.launch_at);
        g_plan.allocs = g_plan.launches = 0;
    }
    if (alloc) return g_plan.alloc_at > 0 && ++g_plan.allocs == g_plan.alloc_at;
    return g_plan.launch_at > 0 && ++g_plan.launches == g_plan.launch_at;
}

}  // namespace

hipError_t device_alloc(void** p, size_t bytes) {
    *p = nullptr;
    if (injected(true)) {
        log_line("GHN_FAULT: device allocation of %zu bytes fails", bytes);
        return hipErrorOutOfMemory;
    }
    const hipError_t e = hipMalloc(p, bytes ? bytes : 1);
    if (e == hipSuccess) log_line("alloc %p %zu", *p, bytes);
    return e;
}

void device_free(void* p) {
    if (!p) return;
    log_line("free %p", p);
    (void)hipFree(p);
}

hipError_t launch_status() {
    const hipError_t e = hipGetLastError();
    if (e == hipSuccess && injected(false)) {
        // the kernels did launch: let them finish before the caller's error path frees
        // memory they use
        (void)hipDeviceSynchronize();
        log_line("GHN_FAULT: launch check fails");
        return hipErrorLaunchFailure;
    }
    return e;
}

bool log_enabled() {
    const char* v = std::getenv("GHN_LOG");
    return v && *v && std::strcmp(v, "0") != 0;
}

void log_line(const char* fmt, ...) {
    if (!log_enabled()) return;
    char buf[768];
    va_list ap;
    va_start(ap, fmt);
    std::vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    std::fprintf(stderr, "ghn: %s\n", buf);
}

}  // namespace ghn
