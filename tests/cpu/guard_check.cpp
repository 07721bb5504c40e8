// CPU check of the end-of-walk guard the walk kernels call (ghn_guard.h), compiled
// with g++ by tests/test_guard_cpu.py: the entry test, and the "no answer" row written
// by 64 lanes (one wave per query) and by 16-lane rows (the grouped kernel).
#include <cmath>
#include <cstdio>
#include <cstring>
#include <vector>

#include "ghn_guard.h"

static int failures = 0;
#define CHECK(c)                                                        \
    do {                                                                \
        if (!(c)) {                                                     \
            std::printf("FAIL %s:%d: %s\n", __FILE__, __LINE__, #c);    \
            ++failures;                                                 \
        }                                                               \
    } while (0)

static bool is_nan_bits64(double d) { uint64_t u; std::memcpy(&u, &d, 8); return u == 0x7ff8000000000000ull; }
static bool is_nan_bits32(float f) { uint32_t u; std::memcpy(&u, &f, 4); return u == 0x7fc00000u; }

// Rows qi-1 and qi+1 keep their values; row qi is the no-answer row.
static void row_case(bool classify, int k, int lanes_per_row, bool with_optional) {
    const int m = 3, qi = 1;
    std::vector<int64_t> idx((size_t)m * k, 7);
    std::vector<double> d2((size_t)m * k, 0.5);
    std::vector<int32_t> lab(m, 3), stop(m, 9);
    std::vector<float> val(m, 2.5f);
    std::vector<int64_t> cands(m, 11), probes(m, 12), rerank(m, 13);
    void* pred = classify ? (void*)lab.data() : (void*)val.data();
    for (int lane = 0; lane < lanes_per_row; ++lane)
        ghn::write_no_answer_row(idx.data(), with_optional ? d2.data() : nullptr, pred,
                                 with_optional ? stop.data() : nullptr, with_optional ? cands.data() : nullptr,
                                 with_optional ? probes.data() : nullptr, with_optional ? rerank.data() : nullptr,
                                 classify, k, qi, lane, lanes_per_row, ghn::STOP_SHORT);
    for (int r = 0; r < m; ++r) {
        for (int e = 0; e < k; ++e) {
            const size_t at = (size_t)r * k + e;
            if (r == qi) {
                CHECK(idx[at] == -1);
                CHECK(with_optional ? is_nan_bits64(d2[at]) : d2[at] == 0.5);
            } else {
                CHECK(idx[at] == 7);
                CHECK(d2[at] == 0.5);
            }
        }
        const bool me = r == qi;
        if (classify) CHECK(lab[r] == (me ? -1 : 3));
        else CHECK(me ? is_nan_bits32(val[r]) : val[r] == 2.5f);
        CHECK(stop[r] == (me && with_optional ? ghn::STOP_SHORT : 9));
        CHECK(cands[r] == (me && with_optional ? 0 : 11));
        CHECK(probes[r] == (me && with_optional ? 0 : 12));
        CHECK(rerank[r] == (me && with_optional ? 0 : 13));
    }
}

int main() {
    // entries: row ids 0..n-1 only; empty slots hold INT32_MAX
    CHECK(ghn::entry_ok(0, 5) && ghn::entry_ok(4, 5));
    CHECK(!ghn::entry_ok(5, 5) && !ghn::entry_ok(-1, 5) && !ghn::entry_ok(INT32_MAX, 5));
    CHECK(!ghn::entry_ok(INT32_MAX, INT32_MAX) && ghn::entry_ok(INT32_MAX - 1, INT32_MAX));
    CHECK(!ghn::entry_ok(INT32_MIN, INT32_MAX) && !ghn::entry_ok(0, 0));
    // a wave's decision: any of the k buffer slots not a row (a short walk leaves
    // INT32_MAX in the slots past its count)
    {
        const int k = 6;
        int32_t slots[64];
        for (int l = 0; l < 64; ++l) slots[l] = INT32_MAX;
        for (int l = 0; l < 5; ++l) slots[l] = l;
        bool any = false;
        for (int l = 0; l < 64; ++l) any = any || (l < k && !ghn::entry_ok(slots[l], 100));
        CHECK(any);
        slots[5] = 99;
        any = false;
        for (int l = 0; l < 64; ++l) any = any || (l < k && !ghn::entry_ok(slots[l], 100));
        CHECK(!any);
    }
    for (int classify = 0; classify < 2; ++classify)
        for (int opt = 0; opt < 2; ++opt) {
            for (int k : {1, 10, 63, 64}) row_case(classify, k, 64, opt);
            for (int k : {1, 16, 17, 40, 64}) row_case(classify, k, 16, opt);
        }
    CHECK(ghn::STOP_SHORT != ghn::STOP_NONFINITE && ghn::STOP_SHORT < 0 && ghn::STOP_NONFINITE < 0);
    if (failures) return 1;
    std::printf("guard ok\n");
    return 0;
}
