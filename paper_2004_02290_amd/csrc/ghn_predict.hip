// Exploration (Section III-B) over the dense cell table: one wave64 per query
// (the walk itself is in ghn_walk_dense.h), and the spatial sort key of queries.
#include "ghn_walk_dense.h"

namespace ghn {
namespace {

constexpr int PT = 256;  // threads per block = 4 waves = 4 queries
constexpr int WPB = PT / WAVE;

// Up to 4 dimensions the walk fits 64 VGPRs without scratch spills, which lets 8
// waves share a SIMD instead of 6; the extra waves hide more of the walk's latency
// (measured: 8 % faster on the 4-D clusters).  The other instances are held to the
// occupancy their walk loop reaches on its own, so that the rare set-up of a query
// far outside the box (setup_far) cannot lower it.
template <int FT, bool HASH> constexpr int dense_waves_per_eu() {
    return FT < 1 ? 1 : (!HASH ? (FT <= 4 ? 8 : (FT == 5 ? 6 : (FT == 6 ? 5 : 4)))
                                : (FT <= 2 ? 7 : (FT <= 4 ? 6 : (FT <= 6 ? 5 : 4))));
}

// The query set-up (central cell, FP64 coordinates, first and covering layers) is
// the same on every lane of a wave, so the block's first wave does it for all the
// block's queries at once, one lane each, and hands it over through LDS: one set-up
// pass per block instead of one per wave.
template <int FT, int STOP, bool HASH>
__global__ __launch_bounds__(PT) __attribute__((amdgpu_waves_per_eu(dense_waves_per_eu<FT, HASH>())))
void k_predict_dense(PredictArgs A) {
    __shared__ uint32_t s_begin[WPB][RUN_CAP];
    __shared__ uint32_t s_pre[WPB][RUN_CAP];
    __shared__ uint32_t s_key[WPB][RUN_CAP];
    constexpr bool SHARED_SETUP = FT > 0 && !HASH;  // (the hash instances keep their registers for the lookups)
    __shared__ Query<FT> s_query[SHARED_SETUP ? WPB : 1];
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x / WAVE);
    const int64_t slot = wave_slot(A, WPB);
    if constexpr (SHARED_SETUP) {
        const int lane = lane_id();
        if (wv == 0 && lane < WPB) {
            const int64_t s_l = slot - wv + lane;  // the slot of wave `lane` of this block
            if (s_l < A.m) {
                const int64_t q_l = A.order ? (int64_t)A.order[s_l] : s_l;
                Query<FT> Q;
                setup_query<FT>(A.ix, A.io.queries, q_l, FT, Q);
                s_query[lane] = Q;
            }
        }
        __syncthreads();
    }
    if (slot >= A.m) return;
    const int64_t qi = A.order ? (int64_t)A.order[slot] : slot;
    walk_dense<FT, STOP, HASH>(A.ix, A.io, qi, s_begin[wv], s_pre[wv], s_key[wv],
                               SHARED_SETUP ? &s_query[wv] : nullptr);
}

// Sort key of a query: Morton interleave of its central cell id clamped to the
// occupied box, keeping the `keep_bits` most significant bits.  Only the order of
// processing depends on it; every query's result is independent of the order.
__global__ __launch_bounds__(256) void k_query_keys(const float* __restrict__ qs, int64_t m, IndexView ix,
                                                    int keep_bits, uint64_t* __restrict__ keys,
                                                    uint32_t* __restrict__ vals) {
    const int f = ix.f;
    int bits[F_MAX];
    int total = 0, maxb = 0;
    for (int j = 0; j < f; ++j) {
        const uint32_t span = (uint32_t)(ix.cmax[j] - ix.cmin[j]);
        bits[j] = span ? 32 - __clz(span) : 0;
        total += bits[j];
        maxb = max(maxb, bits[j]);
    }
    const int drop = total > keep_bits ? total - keep_bits : 0;
    for (int64_t i = blockIdx.x * 256ll + threadIdx.x; i < m; i += (int64_t)gridDim.x * 256) {
        uint64_t code = 0;
        uint32_t u[F_MAX];
        for (int j = 0; j < f; ++j) {
            const float x = qs[i * f + j];
            int64_t c = isfinite(x) ? exact_floor_div(__dadd_rn((double)x, -(double)ix.o[j]), (double)ix.a[j]) : 0;
            c = min(max(c, (int64_t)ix.cmin[j]), (int64_t)ix.cmax[j]);
            u[j] = (uint32_t)(c - ix.cmin[j]);
        }
        int pos = total;  // only the top keep_bits bits of the code are formed
        for (int b = maxb - 1; b >= 0; --b)
            for (int j = 0; j < f; ++j)
                if (b < bits[j]) {
                    --pos;
                    if (pos >= drop) code = (code << 1) | ((u[j] >> b) & 1u);
                }
        keys[i] = code;
        vals[i] = (uint32_t)i;
    }
}

template <int FT, bool HASH>
void launch_stop(const PredictArgs& a, dim3 grid, dim3 block, hipStream_t s) {
    if (a.stop == GHN_STOP_PAPER)
        hipLaunchKernelGGL((k_predict_dense<FT, GHN_STOP_PAPER, HASH>), grid, block, 0, s, a);
    else
        hipLaunchKernelGGL((k_predict_dense<FT, GHN_STOP_EXACT, HASH>), grid, block, 0, s, a);
}

template <int FT>
hipError_t launch_ft(const PredictArgs& a, hipStream_t s) {
    const dim3 grid((unsigned)((a.m + WPB - 1) / WPB)), block(PT);
    if (a.ix.lookup == LOOKUP_HASH) launch_stop<FT, true>(a, grid, block, s);
    else launch_stop<FT, false>(a, grid, block, s);
    return launch_status();
}

}  // namespace

hipError_t launch_query_keys(const float* qs, int64_t m, const IndexView& ix, int keep_bits, uint64_t* keys,
                             uint32_t* vals, hipStream_t s) {
    int64_t g = (m + 255) / 256;
    if (g > 65536) g = 65536;
    hipLaunchKernelGGL(k_query_keys, dim3((unsigned)g), dim3(256), 0, s, qs, m, ix, keep_bits, keys, vals);
    return launch_status();
}

hipError_t launch_predict_dense(const PredictArgs& a, hipStream_t s) {
    switch (a.ix.f) {
        case 1: return launch_ft<1>(a, s);
        case 2: return launch_ft<2>(a, s);
        case 3: return launch_ft<3>(a, s);
        case 4: return launch_ft<4>(a, s);
        case 5: return launch_ft<5>(a, s);
        case 6: return launch_ft<6>(a, s);
        case 8: return launch_ft<8>(a, s);
        default: return launch_ft<0>(a, s);
    }
}

}  // namespace ghn
