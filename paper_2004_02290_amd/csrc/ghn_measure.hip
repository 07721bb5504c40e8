// The paper's cell measurement rule (Section III-A, Fig. 3).
//
// For each dimension the range [mn, mx] covered by the training points is cut
// into s equal splits of width w = fl32((mx - mn) / s); point x lies in split
// min(floor((x - mn) / w), s - 1) (exact floor; the last split is closed at mx).
// The cell measurement is the width of the largest s that leaves no split
// empty, and the grid origin is mn, so the cells of Eq. 1 are the splits.
//
// The column is sorted on the GPU (order-preserving integer keys, radix sort);
// the search runs on the host over the sorted distinct values v_0 < ... < v_{u-1}:
//   * the split index is non-decreasing along the sorted values, starts at 0 and
//     (checked) ends at s - 1, so no split is empty iff no two consecutive values
//     are two or more splits apart;
//   * that can only happen across a gap wider than w (up to rounding of the
//     FP64 differences, covered by a 2^-19 relative slack), so only the widest
//     gaps are checked for each s;
//   * a gap wider than 2w always contains a whole split, so s <= 2 (mx - mn) / G
//     for the widest gap G: the search starts there (or at u) and walks down,
//     since the property is not monotone in s.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "ghn_internal.h"

namespace ghn {
namespace {

constexpr int MT = 256;

__device__ __forceinline__ float column_value(const void* pts, int64_t idx, int32_t dtype) {
    if (dtype == GHN_BF16) return __uint_as_float((uint32_t)((const uint16_t*)pts)[idx] << 16);
    return ((const float*)pts)[idx];
}

// Order-preserving key of dimension j of every point (the sort's values are unused).
__global__ __launch_bounds__(MT) void k_column_keys(const void* pts, int64_t n, int32_t f, int32_t j, int32_t dtype,
                                                    uint64_t* __restrict__ keys, uint32_t* __restrict__ vals,
                                                    int* __restrict__ bad) {
    for (int64_t r = blockIdx.x * (int64_t)MT + threadIdx.x; r < n; r += (int64_t)gridDim.x * MT) {
        const float x = column_value(pts, r * f + j, dtype);
        if (!isfinite(x)) atomicOr(bad, 1);
        const uint32_t u = __float_as_uint(x);
        keys[r] = (u & 0x80000000u) ? ~u : (u | 0x80000000u);
        vals[r] = (uint32_t)r;
    }
}

float key_value(uint64_t key) {
    const uint32_t k = (uint32_t)key;
    const uint32_t u = (k & 0x80000000u) ? (k & 0x7fffffffu) : ~k;
    float x;
    std::memcpy(&x, &u, 4);
    return x;
}

// Exact floor of v / a (a > 0): the quotient's floor, corrected with the sign of
// the fused t * a - v (one rounding, so the sign is exact).
int64_t floor_quotient(double v, double a) {
    double t = std::floor(v / a);
    if (std::fma(t, a, -v) > 0.0) t -= 1.0;
    else if (std::fma(t + 1.0, a, -v) <= 0.0) t += 1.0;
    return (int64_t)t;
}

// The rule on one dimension's sorted distinct values.
void measure_sorted(const std::vector<double>& v, float* width, int64_t* splits) {
    const size_t u = v.size();
    *splits = 1;
    *width = 1.0f;
    if (u < 2) return;
    const double mn = v.front(), mx = v.back(), range = mx - mn;
    double gmax = 0.0;
    for (size_t k = 0; k + 1 < u; ++k) gmax = std::max(gmax, v[k + 1] - v[k]);
    double bound = std::floor(2.0 * range / gmax * (1.0 + 0x1p-20)) + 1.0;
    const int64_t s_hi = (int64_t)std::min((double)u, bound);
    const double w_lo = (double)(float)(range / (double)s_hi);
    std::vector<std::pair<double, size_t>> cand;  // gaps that some s in [1, s_hi] may need checked
    for (size_t k = 0; k + 1 < u; ++k) {
        const double g = v[k + 1] - v[k];
        if (g >= w_lo * (1.0 - 0x1p-19)) cand.emplace_back(g, k);
    }
    std::sort(cand.begin(), cand.end(), [](const std::pair<double, size_t>& a, const std::pair<double, size_t>& b) {
        return a.first > b.first;
    });
    for (int64_t s = s_hi; s >= 1; --s) {
        const float w = (float)(range / (double)s);
        if (!(w > 0.0f)) continue;
        const double wd = w;
        auto split_of = [&](double x) { return std::min(floor_quotient(x - mn, wd), s - 1); };
        bool ok = split_of(mx) == s - 1;
        for (size_t c = 0; ok && c < cand.size() && cand[c].first >= wd * (1.0 - 0x1p-19); ++c) {
            const size_t k = cand[c].second;
            if (split_of(v[k + 1]) - split_of(v[k]) >= 2) ok = false;
        }
        if (ok) {
            *splits = s;
            *width = w;
            return;
        }
    }
}

}  // namespace

hipError_t measure_cells(const void* pts, int64_t n, int32_t f, int32_t dtype, float* width, float* origin,
                         int64_t* splits, bool* nonfinite, hipStream_t s) {
    *nonfinite = false;
    uint64_t *k0 = nullptr, *k1 = nullptr;
    uint32_t *v0 = nullptr, *v1 = nullptr;
    void* temp = nullptr;
    int* bad = nullptr;
    hipError_t e = hipSuccess;
    auto release = [&]() {
        ghn::device_free(k0); ghn::device_free(k1); ghn::device_free(v0); ghn::device_free(v1); ghn::device_free(temp);
        ghn::device_free(bad);
    };
    if ((e = device_alloc((void**)&k0, n * 8)) != hipSuccess || (e = device_alloc((void**)&k1, n * 8)) != hipSuccess ||
        (e = device_alloc((void**)&v0, n * 4)) != hipSuccess || (e = device_alloc((void**)&v1, n * 4)) != hipSuccess ||
        (e = device_alloc(&temp, radix_sort_temp_bytes(n))) != hipSuccess || (e = device_alloc((void**)&bad, 4)) != hipSuccess) {
        release();
        return e;
    }
    std::vector<uint64_t> keys((size_t)n);
    int hbad = 0;
    for (int j = 0; j < f && e == hipSuccess; ++j) {
        int64_t g = (n + MT - 1) / MT;
        if (g > 4096) g = 4096;
        if ((e = hipMemsetAsync(bad, 0, 4, s)) != hipSuccess) break;
        hipLaunchKernelGGL(k_column_keys, dim3((unsigned)g), dim3(MT), 0, s, pts, n, f, j, dtype, k0, v0, bad);
        if ((e = launch_status()) != hipSuccess) break;
        bool alt = false;
        if ((e = radix_sort_pairs(k0, v0, k1, v1, n, 32, temp, &alt, s)) != hipSuccess) break;
        if ((e = hipMemcpyAsync(keys.data(), alt ? k1 : k0, n * 8, hipMemcpyDeviceToHost, s)) != hipSuccess ||
            (e = hipMemcpyAsync(&hbad, bad, 4, hipMemcpyDeviceToHost, s)) != hipSuccess ||
            (e = hipStreamSynchronize(s)) != hipSuccess)
            break;
        if (hbad) {
            *nonfinite = true;
            break;
        }
        std::vector<double> v;
        v.reserve((size_t)n);
        for (int64_t i = 0; i < n; ++i) {
            const double x = (double)key_value(keys[(size_t)i]);
            if (v.empty() || x != v.back()) v.push_back(x);
        }
        origin[j] = (float)v.front();
        measure_sorted(v, &width[j], &splits[j]);
    }
    release();
    return e;
}

}  // namespace ghn
