// Exploration (Section III-B) on the GPU with the dense cell table.
//
// One wave64 walks one query.  For layer l (cells whose id differs from the
// central cell's by at most l in every dimension and by exactly l in one) the
// cells are enumerated as "rows": a choice of ids for dimensions 0..f-2 plus a
// run of ids along the last dimension.  Points are stored in cell order and
// the dense table is indexed row-major over the occupied box, so a run of
// cells along the last dimension is one contiguous run of points: a row costs
// two table reads.  Shell rows (some leading dimension at offset +-l) cover the
// whole run [c-l, c+l]; interior rows only its two end cells.
//
// Cells whose distance lower bound exceeds the current k-th distance are
// skipped: none of their points could enter the buffer, so neither the result
// nor the PAPER rule's "buffer changed in this layer" signal can change.
#include "ghn_walk.h"

namespace ghn {
namespace {

constexpr int PT = 256;  // threads per block = 4 waves = 4 queries
constexpr int WPB = PT / WAVE;

template <int FT, int STOP>
__global__ __launch_bounds__(PT) void k_predict_dense(PredictArgs A) {
    __shared__ uint32_t s_begin[WPB][RUN_CAP];
    __shared__ uint32_t s_pre[WPB][RUN_CAP];
    const IndexView& ix = A.ix;
    const int lane = lane_id();
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x / WAVE);
    const int64_t slot = wave_slot(A, WPB);
    if (slot >= A.m) return;
    const int64_t qi = A.order ? (int64_t)A.order[slot] : slot;
    const int f = FT > 0 ? FT : ix.f;
    const int k = A.k;
    const bool prune = !(A.flags & GHN_FLAG_NO_PRUNE);

    Query<FT> Q;
    setup_query<FT>(ix, A.queries, qi, f, Q);
    if (!Q.finite) {
        write_invalid(A, qi);
        return;
    }
    WaveState st;
    init_state(st);

    const int L = f - 1;  // the run dimension
    const double aL = ix.a[L];
    int64_t l = Q.l0;
    for (;; ++l) {
        st.updated = false;
        // Range of ids per dimension: layer box c +- l clipped to the occupied box.
        int64_t lo[FT > 0 ? FT : F_MAX], w[FT > 0 ? FT : F_MAX];
        int64_t rows = 1;
        bool empty = false;
#pragma unroll
        for (int j = 0; j < (FT > 0 ? FT : F_MAX); ++j) {
            if (FT == 0 && j >= f) break;
            const int64_t a0 = max(Q.c[j] - l, (int64_t)ix.cmin[j]);
            const int64_t b0 = min(Q.c[j] + l, (int64_t)ix.cmax[j]);
            lo[j] = a0;
            w[j] = b0 - a0 + 1;
            if (b0 < a0) empty = true;
            if (j < L) rows *= (b0 >= a0 ? (b0 - a0 + 1) : 0);
        }
        if (!empty) {
            const bool small = rows < (int64_t(1) << 32);
            for (int64_t rb = 0; rb < rows; rb += WAVE) {
                const int64_t r = rb + lane;
                uint32_t b0 = 0, n0 = 0, b1 = 0, n1 = 0, probes_l = 0;
                if (r < rows) {
                    // decode row r: ids of dimensions 0..L-1, the last of them fastest
                    int64_t maxoff = 0, lin = 0;
                    double lb = 0.0;
                    uint64_t rem64 = (uint64_t)r;
                    uint32_t rem32 = (uint32_t)r;
#pragma unroll
                    for (int j = (FT > 0 ? FT - 2 : F_MAX - 2); j >= 0; --j) {
                        if (FT == 0 && j > L - 1) continue;
                        int64_t digit;
                        if (small) {
                            const uint32_t wj = (uint32_t)w[j];
                            digit = rem32 % wj;
                            rem32 /= wj;
                        } else {
                            digit = (int64_t)(rem64 % (uint64_t)w[j]);
                            rem64 /= (uint64_t)w[j];
                        }
                        const int64_t oj = lo[j] + digit;
                        maxoff = max(maxoff, oj > Q.c[j] ? oj - Q.c[j] : Q.c[j] - oj);
                        lin += (oj - ix.cmin[j]) * ix.stride[j];
                        const double g = gap_to_cells(Q.v[j], oj, oj, (double)ix.a[j]);
                        lb = __dadd_rn(lb, __dmul_rn(g, g));
                    }
                    const bool pass_row = !prune || !(lb * LB_SHRINK > st.tau);
                    if (pass_row) {
                        const int64_t cL = Q.c[L];
                        const int64_t lo_l = lo[L], hi_l = lo[L] + w[L] - 1;
                        if (maxoff == l) {
                            // shell row: every cell of the run [c-l, c+l] inside the box
                            int64_t ta = lo_l, tb = hi_l;
                            if (prune && st.tau < 1.0e300) {
                                const double room = st.tau / LB_SHRINK - lb;
                                const double G = sqrt(room > 0.0 ? room : 0.0);
                                const double ub = floor((Q.v[L] + G) / aL) + 1.0;
                                const double lb_t = ceil((Q.v[L] - G) / aL) - 2.0;
                                if (ub < (double)tb) tb = (int64_t)ub;
                                if (lb_t > (double)ta) ta = (int64_t)lb_t;
                            }
                            if (ta <= tb) {
                                const uint32_t s0 = ix.cell_start[lin + (ta - ix.cmin[L])];
                                const uint32_t s1 = ix.cell_start[lin + (tb - ix.cmin[L]) + 1];
                                b0 = s0;
                                n0 = s1 - s0;
                                probes_l += 2;
                            }
                        } else {
                            // interior row: only the end cells c-l and c+l belong to layer l
                            for (int e = 0; e < 2; ++e) {
                                const int64_t t = e == 0 ? cL - l : cL + l;
                                if (t < lo_l || t > hi_l) continue;
                                if (prune) {
                                    const double g = gap_to_cells(Q.v[L], t, t, aL);
                                    if (__dadd_rn(lb, __dmul_rn(g, g)) * LB_SHRINK > st.tau) continue;
                                }
                                const uint32_t s0 = ix.cell_start[lin + (t - ix.cmin[L])];
                                const uint32_t s1 = ix.cell_start[lin + (t - ix.cmin[L]) + 1];
                                probes_l += 2;
                                if (e == 0) { b0 = s0; n0 = s1 - s0; }
                                else { b1 = s0; n1 = s1 - s0; }
                            }
                        }
                    }
                }
                st.probes += wave_sum_u32(probes_l);
                score_runs<FT>(ix, Q.q, f, k, b0, n0, b1, n1, s_begin[wv], s_pre[wv], st);
            }
        }
        if (stop_after_layer<FT, STOP>(ix, Q, f, k, l, st)) break;
    }
    finish_query(A, qi, l, st);
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
        for (int b = maxb - 1; b >= 0; --b)
            for (int j = 0; j < f; ++j)
                if (b < bits[j]) code = (code << 1) | ((u[j] >> b) & 1u);
        keys[i] = code >> drop;
        vals[i] = (uint32_t)i;
    }
}

template <int FT>
hipError_t launch_ft(const PredictArgs& a, hipStream_t s) {
    const dim3 grid((unsigned)((a.m + WPB - 1) / WPB)), block(PT);
    if (a.stop == GHN_STOP_PAPER)
        hipLaunchKernelGGL((k_predict_dense<FT, GHN_STOP_PAPER>), grid, block, 0, s, a);
    else
        hipLaunchKernelGGL((k_predict_dense<FT, GHN_STOP_EXACT>), grid, block, 0, s, a);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_query_keys(const float* qs, int64_t m, const IndexView& ix, int keep_bits, uint64_t* keys,
                             uint32_t* vals, hipStream_t s) {
    int64_t g = (m + 255) / 256;
    if (g > 65536) g = 65536;
    hipLaunchKernelGGL(k_query_keys, dim3((unsigned)g), dim3(256), 0, s, qs, m, ix, keep_bits, keys, vals);
    return hipGetLastError();
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
