// End-of-walk check (Section III-B: a walk returns the k nearest points, so every
// buffer entry it ends with is a row of the index).  A walk ends with k entries by
// construction: k <= n, and the stop bound is only met once the explored box holds
// every point.  If that invariant is ever broken the query's row is written as a
// "no answer" row and a fault bit is raised for ghn_walk_faults to report, instead
// of reading targets at a row id that is not one.
//
// Plain C++ with a host/device qualifier so that a CPU test compiles the same
// functions the kernels call.
#pragma once

#include <stdint.h>

#ifndef GHN_HD
#define GHN_HD __host__ __device__
#endif

namespace ghn {

constexpr int32_t STOP_NONFINITE = -1;  // stop layer of a query with a non-finite coordinate
constexpr int32_t STOP_SHORT = -2;      // stop layer of a walk that ended without k neighbours

// Is a buffer entry holding row id `id` a row of an index of n points?  Empty slots
// hold INT32_MAX, which is never below n (n < 2^31).
GHN_HD inline bool entry_ok(int32_t id, int64_t n) { return (uint32_t)id < (uint64_t)n; }

// A query's "no answer" row: ids -1, FP64 distances NaN, prediction -1 (classification)
// or NaN (regression), the given stop layer and zero diagnostics.  The calling thread
// writes the entries e = first, first + step, ... below k; the one with first == 0 also
// writes the per-query values.
GHN_HD inline void write_no_answer_row(int64_t* out_idx, double* out_d2, void* out_pred, int32_t* out_stop_layer,
                                       int64_t* out_cands, int64_t* out_probes, int64_t* out_rerank, bool classify,
                                       int32_t k, int64_t qi, int first, int step, int32_t stop_layer) {
    union { uint64_t u; double d; } nan64 = {0x7ff8000000000000ull};
    union { uint32_t u; float f; } nan32 = {0x7fc00000u};
    for (int e = first; e < k; e += step) {
        out_idx[qi * k + e] = -1;
        if (out_d2) out_d2[qi * k + e] = nan64.d;
    }
    if (first == 0) {
        if (classify) ((int32_t*)out_pred)[qi] = -1;
        else ((float*)out_pred)[qi] = nan32.f;
        if (out_stop_layer) out_stop_layer[qi] = stop_layer;
        if (out_cands) out_cands[qi] = 0;
        if (out_probes) out_probes[qi] = 0;
        if (out_rerank) out_rerank[qi] = 0;
    }
}

}  // namespace ghn
