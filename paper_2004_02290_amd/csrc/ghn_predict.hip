// Exploration (Section III-B) on the GPU, dense-box lookup, FP32 screen.
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
// The lanes of the wave gather candidates from the layer's runs in 64-wide
// chunks (load balanced through a per-wave LDS list of runs), screen them with
// an FP32 distance, and only candidates that can still enter the buffer get
// their FP64 distance.  The size-k buffer (Section III-B's heap) lives in
// lanes 0..k-1 sorted by (FP64 distance, row id); insertions shift it by one
// lane.  The buffer therefore always holds exactly the k best of everything
// scored so far, in the FP64 order the result is defined by.
//
// Cells whose distance lower bound exceeds the current k-th distance are
// skipped: none of their points could enter the buffer, so neither the result
// nor the PAPER rule's "buffer changed in this layer" signal can change.
#include "ghn_internal.h"

namespace ghn {
namespace {

constexpr int PT = 256;                 // threads per block = 4 waves = 4 queries
constexpr int WPB = PT / WAVE;
constexpr int SEG_CAP = 2 * WAVE;       // runs per 64-row batch (interior rows give 2)
constexpr int NUM_XCD = 8;
constexpr double LB_SHRINK = 1.0 - 0x1p-40;   // lower bounds are shrunk by this before pruning
constexpr double EXACT_SHRINK = 1.0 - 0x1p-44; // squared ring distance is shrunk by this (EXACT rule)

// Smallest float >= x (x >= 0, finite or inf).
__device__ __forceinline__ float f32_round_up(double x) {
    float r = (float)x;
    if ((double)r < x) r = __int_as_float(__float_as_int(r) + 1);
    return r;
}

// FP32 admission threshold for a k-th FP64 distance tau: any point with FP64
// distance <= tau has an FP32 screen distance <= the returned value.  The FP32
// screen (f rounded differences, squares and fused adds) and the FP64 value
// both lie within a relative (f + 2) * 2^-24 of the exact distance; 2^-16 covers
// that for f <= 32, and 2^-125 covers FP32 underflow.
__device__ __forceinline__ float admit_threshold(double tau) {
    if (!(tau < 1.0e300)) return __int_as_float(0x7f800000);
    return f32_round_up(tau * (1.0 + 0x1p-16)) + 0x1p-125f;
}

template <int FT>
struct Dims {
    static constexpr int value = FT;
};

template <int FT>
__device__ __forceinline__ void load_point(const float* __restrict__ p, float* x, int f) {
    if constexpr (FT == 2) {
        float2 v = *(const float2*)p;
        x[0] = v.x; x[1] = v.y;
    } else if constexpr (FT > 0 && FT % 4 == 0) {
#pragma unroll
        for (int j = 0; j < FT; j += 4) {
            float4 v = *(const float4*)(p + j);
            x[j] = v.x; x[j + 1] = v.y; x[j + 2] = v.z; x[j + 3] = v.w;
        }
    } else if constexpr (FT > 0) {
#pragma unroll
        for (int j = 0; j < FT; ++j) x[j] = p[j];
    } else {
        for (int j = 0; j < f; ++j) x[j] = p[j];
    }
}

// FP64 squared distance in the defined order: ((q0-x0)^2 + (q1-x1)^2) + ..., no FMA.
template <int FT>
__device__ __forceinline__ double dist64(const float* q, const float* x, int f) {
    double s = 0.0;
    const int F = FT > 0 ? FT : f;
#pragma unroll
    for (int j = 0; j < (FT > 0 ? FT : F_MAX); ++j) {
        if (FT == 0 && j >= F) break;
        double d = __dadd_rn((double)q[j], -(double)x[j]);
        s = __dadd_rn(s, __dmul_rn(d, d));
    }
    return s;
}

template <int FT>
__device__ __forceinline__ float dist32(const float* q, const float* x, int f) {
    float s = 0.0f;
#pragma unroll
    for (int j = 0; j < (FT > 0 ? FT : F_MAX); ++j) {
        if (FT == 0 && j >= f) break;
        float d = q[j] - x[j];
        s = __builtin_fmaf(d, d, s);
    }
    return s;
}

// Distance from v to the interval [o*a, (o+1)*a) in FP64 (0 inside).
__device__ __forceinline__ double gap_to_cell(double v, int64_t o, double a) {
    double lo = __dadd_rn(__dmul_rn((double)o, a), -v);
    double hi = __dadd_rn(v, -__dmul_rn((double)(o + 1), a));
    double g = lo > hi ? lo : hi;
    return g > 0.0 ? g : 0.0;
}

struct WaveState {
    double bd;      // this lane's buffer slot: distance (lanes < k)
    int bi;         // this lane's buffer slot: row id
    double tau;     // k-th distance (+inf while the buffer is not full)
    int tau_i;      // k-th row id
    float t32;      // FP32 admission threshold derived from tau
    int count;      // entries in the buffer (<= k)
    bool updated;   // an insertion happened in the current layer
    int64_t cands;  // candidates scored
    int64_t probes; // cell-table entries read
};

// One 64-wide chunk of candidates, gathered ahead of its scoring.
template <int FT>
struct Chunk {
    float x[FT > 0 ? FT : F_MAX];
    int id;
    bool valid;
};

template <int FT>
__device__ __forceinline__ void fetch_chunk(const IndexView& ix, int f, bool valid, uint32_t pidx, Chunk<FT>& c) {
    c.valid = valid;
    c.id = 0;
    if (valid) {
        load_point<FT>(ix.spts + (size_t)pidx * (FT > 0 ? FT : f), c.x, f);
        c.id = ix.sid[pidx];
    }
}

// Screen a chunk in FP32; candidates that may enter the buffer get their FP64
// distance and are inserted one at a time (exact (distance, id) comparison).
template <int FT>
__device__ __forceinline__ void score_chunk(const float* q, int f, int k, const Chunk<FT>& c, WaveState& st) {
    const int lane = lane_id();
    float d32 = __int_as_float(0x7f800000);
    if (c.valid) d32 = dist32<FT>(q, c.x, f);
    const bool adm = c.valid && d32 <= st.t32;
    uint64_t mask = ballot(adm);
    if (mask == 0) return;
    double d64 = 0.0;
    if (adm) d64 = dist64<FT>(q, c.x, f);
    while (mask) {
        const int src = __ffsll((unsigned long long)mask) - 1;
        mask &= mask - 1;
        const double cd = readlane_f64(d64, src);
        const int ci = readlane_i32(c.id, src);
        if (!(cd < st.tau || (cd == st.tau && ci < st.tau_i))) continue;
        // The new k-th entry is the old (k-1)-th unless the candidate lands last.
        double kd = cd;
        int ki = ci;
        if (k > 1) { kd = readlane_f64(st.bd, k - 2); ki = readlane_i32(st.bi, k - 2); }
        // Insert (cd, ci): slots holding a larger entry shift up by one lane.
        const uint64_t cb = (uint64_t)__double_as_longlong(cd);
        const uint64_t bb = (uint64_t)__double_as_longlong(st.bd);
        const bool gt = lane < k && (bb > cb || (bb == cb && st.bi > ci));
        const int pos = k - __popcll(ballot(gt));
        const double ud = shfl_up1_f64(st.bd);
        const int ui = shfl_up1_i32(st.bi);
        if (gt) {
            st.bd = lane == pos ? cd : ud;
            st.bi = lane == pos ? ci : ui;
        }
        st.updated = true;
        if (st.count < k) st.count += 1;
        if (st.count == k) {
            const bool last = pos == k - 1;
            st.tau = last ? cd : kd;
            st.tau_i = last ? ci : ki;
            st.t32 = admit_threshold(st.tau);
            mask &= ballot(c.valid && d32 <= st.t32);
        }
    }
}

template <int FT, int STOP>
__global__ __launch_bounds__(PT) void k_predict_dense(PredictArgs A) {
    __shared__ uint32_t s_begin[WPB][SEG_CAP];
    __shared__ uint32_t s_pre[WPB][SEG_CAP];
    const IndexView& ix = A.ix;
    const int lane = lane_id();
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x / WAVE);
    // With a spatial query order, give each XCD (blocks are dealt round-robin over the
    // 8 XCDs) one contiguous range of blocks, so each XCD's L2 serves one region.
    int64_t blk = blockIdx.x;
    if (A.order) {
        const int64_t nb = gridDim.x, x = blk % NUM_XCD, t = blk / NUM_XCD;
        blk = x * (nb / NUM_XCD) + min(x, nb % NUM_XCD) + t;
    }
    const int64_t slot = blk * WPB + wv;
    if (slot >= A.m) return;
    const int64_t qi = A.order ? (int64_t)A.order[slot] : slot;
    const int f = FT > 0 ? FT : ix.f;
    const int k = A.k;
    const bool prune = !(A.flags & GHN_FLAG_NO_PRUNE);

    float q[FT > 0 ? FT : F_MAX];
    double v[FT > 0 ? FT : F_MAX];
    int64_t c[FT > 0 ? FT : F_MAX];
    bool finite = true;
    int64_t l0 = 0, lcover = 0;
#pragma unroll
    for (int j = 0; j < (FT > 0 ? FT : F_MAX); ++j) {
        if (FT == 0 && j >= f) break;
        q[j] = A.queries[qi * f + j];
        finite = finite && isfinite(q[j]);
        v[j] = __dadd_rn((double)q[j], -(double)ix.o[j]);
        int64_t cj = finite ? exact_floor_div(v[j], (double)ix.a[j]) : 0;
        cj = max(cj, (int64_t)ix.cmin[j] - CLAMP);
        cj = min(cj, (int64_t)ix.cmax[j] + CLAMP);
        c[j] = cj;
        l0 = max(l0, max((int64_t)ix.cmin[j] - cj, cj - (int64_t)ix.cmax[j]));
        lcover = max(lcover, max(cj - (int64_t)ix.cmin[j], (int64_t)ix.cmax[j] - cj));
    }
    if (!finite) {
        if (lane < k) {
            A.out_idx[qi * k + lane] = -1;
            if (A.out_d2) A.out_d2[qi * k + lane] = __longlong_as_double(0x7ff8000000000000LL);
        }
        if (lane == 0) {
            if (ix.task == GHN_CLASSIFY) ((int32_t*)A.out_pred)[qi] = -1;
            else ((float*)A.out_pred)[qi] = __int_as_float(0x7fc00000);
            if (A.out_stop_layer) A.out_stop_layer[qi] = -1;
            if (A.out_cands) A.out_cands[qi] = 0;
            if (A.out_probes) A.out_probes[qi] = 0;
        }
        return;
    }

    WaveState st;
    st.bd = __longlong_as_double(0x7ff0000000000000LL);
    st.bi = INT32_MAX;
    st.tau = st.bd;
    st.tau_i = INT32_MAX;
    st.t32 = __int_as_float(0x7f800000);
    st.count = 0;
    st.cands = 0;
    st.probes = 0;

    const int L = f - 1;  // the run dimension
    int64_t l = l0;
    for (;; ++l) {
        st.updated = false;
        // Range of ids per dimension: layer box c +- l clipped to the occupied box.
        int64_t lo[FT > 0 ? FT : F_MAX], w[FT > 0 ? FT : F_MAX];
        int64_t rows = 1;
        bool empty = false;
#pragma unroll
        for (int j = 0; j < (FT > 0 ? FT : F_MAX); ++j) {
            if (FT == 0 && j >= f) break;
            int64_t a0 = max(c[j] - l, (int64_t)ix.cmin[j]);
            int64_t b0 = min(c[j] + l, (int64_t)ix.cmax[j]);
            lo[j] = a0;
            w[j] = b0 - a0 + 1;
            if (b0 < a0) empty = true;
            if (j < L) rows *= (b0 >= a0 ? (b0 - a0 + 1) : 0);
        }
        if (!empty) {
            const double aL = ix.a[L];
            for (int64_t rb = 0; rb < rows; rb += WAVE) {
                const int64_t r = rb + lane;
                uint32_t b0 = 0, n0 = 0, b1 = 0, n1 = 0, probes_l = 0;
                if (r < rows) {
                    // decode row r: offsets of dimensions 0..L-1, last of them fastest
                    int64_t maxoff = 0, lin = 0;
                    double lb = 0.0;
                    uint64_t rem64 = (uint64_t)r;
                    uint32_t rem32 = (uint32_t)r;
                    const bool small = rows < (int64_t(1) << 32);
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
                        maxoff = max(maxoff, oj > c[j] ? oj - c[j] : c[j] - oj);
                        lin += (oj - ix.cmin[j]) * ix.stride[j];
                        const double g = gap_to_cell(v[j], oj, (double)ix.a[j]);
                        lb = __dadd_rn(lb, __dmul_rn(g, g));
                    }
                    const bool pass_row = !prune || !(lb * LB_SHRINK > st.tau);
                    if (pass_row) {
                        const int64_t cL = c[L];
                        const int64_t lo_l = lo[L], hi_l = lo[L] + w[L] - 1;
                        if (maxoff == l) {
                            // shell row: every cell of the run [c-l, c+l] inside the box
                            int64_t ta = lo_l, tb = hi_l;
                            if (prune && st.tau < 1.0e300) {
                                const double room = st.tau / LB_SHRINK - lb;
                                const double G = sqrt(room > 0.0 ? room : 0.0);
                                const double ub = floor((v[L] + G) / aL) + 1.0;
                                const double lb_t = ceil((v[L] - G) / aL) - 2.0;
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
                                    const double g = gap_to_cell(v[L], t, aL);
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
                // Compact the non-empty runs of this batch into the wave's LDS list.
                const uint32_t nseg_l = (n0 > 0) + (n1 > 0);
                const uint32_t npts_l = n0 + n1;
                const uint32_t seg_incl = wave_incl_scan(nseg_l);
                const uint32_t pts_incl = wave_incl_scan(npts_l);
                const uint32_t nseg = readlane_i32((int)seg_incl, WAVE - 1);
                const uint32_t npts = readlane_i32((int)pts_incl, WAVE - 1);
                if (npts == 0) continue;
                uint32_t sidx = seg_incl - nseg_l, pofs = pts_incl - npts_l;
                if (n0 > 0) { s_begin[wv][sidx] = b0; s_pre[wv][sidx] = pofs; ++sidx; pofs += n0; }
                if (n1 > 0) { s_begin[wv][sidx] = b1; s_pre[wv][sidx] = pofs; }
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                __builtin_amdgcn_wave_barrier();
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
                // Position p of the batch -> point index (last run whose prefix is <= p).
                auto locate = [&](uint32_t p) -> uint32_t {
                    uint32_t a0 = 0, a1 = nseg;
                    while (a1 - a0 > 1) {
                        const uint32_t mid = (a0 + a1) >> 1;
                        if (s_pre[wv][mid] <= p) a0 = mid;
                        else a1 = mid;
                    }
                    return s_begin[wv][a0] + (p - s_pre[wv][a0]);
                };
                for (uint32_t base = 0; base < npts; base += WAVE) {
                    const uint32_t p = base + lane;
                    Chunk<FT> cur;
                    fetch_chunk<FT>(ix, f, p < npts, p < npts ? locate(p) : 0u, cur);
                    st.cands += __popcll(ballot(cur.valid));
                    score_chunk<FT>(q, f, k, cur, st);
                }
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                __builtin_amdgcn_wave_barrier();
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            }
        }
        // Stop rules, checked after every complete layer.
        if (l >= lcover) break;  // every occupied cell has been visited
        const bool full = st.count == k;
        if (STOP == GHN_STOP_PAPER) {
            if (full && !st.updated) break;
        } else if (full) {
            double r2 = __longlong_as_double(0x7ff0000000000000LL);
#pragma unroll
            for (int j = 0; j < (FT > 0 ? FT : F_MAX); ++j) {
                if (FT == 0 && j >= f) break;
                const double a = ix.a[j];
                const double glo = __dadd_rn(v[j], -__dmul_rn((double)(c[j] - l), a));
                const double ghi = __dadd_rn(__dmul_rn((double)(c[j] + l + 1), a), -v[j]);
                double g = glo < ghi ? glo : ghi;
                if (g < 0.0) g = 0.0;
                const double g2 = __dmul_rn(g, g);
                if (g2 < r2) r2 = g2;
            }
            if (st.tau < __dmul_rn(r2, EXACT_SHRINK)) break;
        }
    }

    // Results: neighbours in (distance, id) order, then the vote or the mean.
    if (lane < k) {
        A.out_idx[qi * k + lane] = st.bi;
        if (A.out_d2) A.out_d2[qi * k + lane] = st.bd;
    }
    if (ix.task == GHN_CLASSIFY) {
        const int32_t* lab = (const int32_t*)ix.targets;
        const int my = lane < k ? lab[st.bi] : INT32_MAX;
        uint64_t todo = ballot(lane < k);
        int best = INT32_MAX, best_n = -1;
        while (todo) {
            const int src = __ffsll((unsigned long long)todo) - 1;
            const int label = readlane_i32(my, src);
            const uint64_t same = ballot(lane < k && my == label);
            const int cnt = __popcll(same);
            if (cnt > best_n || (cnt == best_n && label < best)) { best = label; best_n = cnt; }
            todo &= ~same;
        }
        if (lane == 0) ((int32_t*)A.out_pred)[qi] = best;
    } else {
        const float* y = (const float*)ix.targets;
        const float my = lane < k ? y[st.bi] : 0.0f;
        double s = 0.0;
        for (int t = 0; t < k; ++t) s = __dadd_rn(s, (double)readlane_f32(my, t));
        if (lane == 0) ((float*)A.out_pred)[qi] = (float)(s / (double)k);
    }
    if (lane == 0) {
        if (A.out_stop_layer) A.out_stop_layer[qi] = (int32_t)l;
        if (A.out_cands) A.out_cands[qi] = st.cands;
        if (A.out_probes) A.out_probes[qi] = st.probes;
    }
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
