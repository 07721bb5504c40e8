// Per-query layer walk over the dense cell table (Section III-B), shared by the
// single-index and the batched kernels.
//
// For layer l (cells whose id differs from the central cell's by at most l in
// every dimension and by exactly l in one) the cells are enumerated as "rows": a
// choice of ids for dimensions 0..f-2 plus a run of ids along the last
// dimension.  Points are stored in cell order and the dense table is indexed
// row-major over the occupied box, so a run of cells along the last dimension
// is one contiguous run of points: a row costs two table reads.  Shell rows
// (some leading dimension at offset +-l) cover the whole run [c-l, c+l];
// interior rows only its two end cells.
//
// Cells whose distance lower bound exceeds the current k-th distance are
// skipped: none of their points could enter the buffer, so neither the result
// nor the PAPER rule's "buffer changed in this layer" signal can change.
#pragma once

#include <type_traits>

#include "ghn_walk.h"

namespace ghn {

// ceil(2^32 / w) for 2 <= w <= 64, the multiplier of the row decode (layer boxes up
// to 64 cells wide take it from this table instead of dividing).
struct RowMagic {
    uint32_t m[WAVE + 1];
};
constexpr RowMagic make_row_magic() {
    RowMagic t{};
    for (uint32_t w = 2; w <= WAVE; ++w) t.m[w] = 0xffffffffu / w + 1u;
    return t;
}
static __constant__ RowMagic kRowMagic = make_row_magic();

// Hash lookup: the points of the occupied cells t0..t1 (ids along the last
// dimension) of the row whose key without the last dimension is `lin`.  Keys are
// row-major with the last dimension fastest, so these cells' points are one
// contiguous run, from the first occupied cell of the range to the last.
__device__ __forceinline__ void hash_run(const IndexView& ix, uint64_t lin, int32_t t0, int32_t t1, int32_t cmin_l,
                                         uint32_t& b, uint32_t& n, uint32_t& reads) {
    b = 0;
    n = 0;
    int64_t first = -1;
    int32_t t = t0;
    for (; t <= t1; ++t) {
        first = hash_find(ix, lin + (uint64_t)(t - cmin_l), reads);
        if (first >= 0) break;
    }
    if (first < 0) return;
    int64_t last = first;
    for (int32_t u = t1; u > t; --u) {
        const int64_t c = hash_find(ix, lin + (uint64_t)(u - cmin_l), reads);
        if (c >= 0) {
            last = c;
            break;
        }
    }
    b = ix.cell_first[first];
    n = ix.cell_first[last + 1] - b;
}

// HASH: the cells come from the hash table (GHN_LOOKUP_HASH) instead of the dense
// offset table; the enumeration, bounds and scoring are the same.
template <int FT, int STOP, bool HASH>
__device__ __forceinline__ void walk_dense_layers(const IndexView& ix, const QueryIO& io, int64_t qi,
                                                  uint32_t* s_begin, uint32_t* s_pre, uint32_t* s_key,
                                                  const Query<FT>& Q) {
    using Lin = typename std::conditional<HASH, uint64_t, uint32_t>::type;  // row key without the last dimension
    const int lane = lane_id();
    const int f = FT > 0 ? FT : ix.f;
    const int k = io.k;
    const bool prune = !(io.flags & GHN_FLAG_NO_PRUNE);
    WaveState st;
    init_state(st);

    const int L = f - 1;  // the run dimension
    const double aL = ix.a[L];
    const double aLinv = ix.ainv[L];
    // ring schedule (EXACT rule only): each step walks the layers l .. lh at once
    RingStep ring(io);
    int32_t l = Q.l0, lh = Q.l0;
    for (;; l = lh + 1) {
        lh = STOP == GHN_STOP_PAPER ? l : ring.last_layer(l, st.count == k, Q.lcover);
        st.updated = false;
        // Range of ids per dimension: box c +- lh clipped to the occupied box.
        int32_t lo[FT > 0 ? FT : F_MAX], w[FT > 0 ? FT : F_MAX];
        int64_t rows = 1;
        bool empty = false;
#pragma unroll
        for (int j = 0; j < (FT > 0 ? FT : F_MAX); ++j) {
            if (FT == 0 && j >= f) break;
            const int32_t a0 = max(Q.c[j] - lh, ix.cmin[j]);
            const int32_t b0 = min(Q.c[j] + lh, ix.cmax[j]);
            lo[j] = a0;
            w[j] = b0 - a0 + 1;
            if (b0 < a0) empty = true;
            if (j < L) rows *= (b0 >= a0 ? (int64_t)(b0 - a0 + 1) : 0);
        }
        if (!empty) {
            // row decode by multiply-high with ceil(2^32 / w): exact while rem * w < 2^32
            int32_t wmax = 1;
            uint32_t mag[FT > 1 ? FT - 1 : 1];
#pragma unroll
            for (int j = 0; j < (FT > 1 ? FT - 1 : (FT == 1 ? 0 : F_MAX - 1)); ++j) {
                if (FT == 0 && j >= L) break;
                wmax = max(wmax, w[j]);
                const uint32_t wj = (uint32_t)w[j];
                mag[FT > 1 ? j : 0] = wj <= 1 ? 0u : (wj <= WAVE ? kRowMagic.m[wj] : 0xffffffffu / wj + 1u);
            }
            const bool small = FT > 0 && rows * (int64_t)wmax < (int64_t(1) << 32);
            for (int64_t rb = 0; rb < rows; rb += WAVE) {
                const int64_t r = rb + lane;
                uint32_t b0 = 0, n0 = 0, b1 = 0, n1 = 0, key0 = 0, key1 = 0, probes_l = 0;
                if (lh == 0) {
                    // layer 0 is the central cell alone (l0 = 0: it lies inside the box)
                    if (lane == 0) {
                        Lin lin = 0;
#pragma unroll
                        for (int j = 0; j < (FT > 0 ? FT : F_MAX); ++j) {
                            if (FT == 0 && j >= f) break;
                            lin += (Lin)(Q.c[j] - ix.cmin[j]) * (HASH ? (Lin)ix.hstride[j] : (Lin)ix.stride[j]);
                        }
                        if constexpr (HASH) {
                            const int64_t c = hash_find(ix, lin, probes_l);
                            if (c >= 0) {
                                b0 = ix.cell_first[c];
                                n0 = ix.cell_first[c + 1] - b0;
                            }
                        } else {
                            b0 = ix.cell_start[lin];
                            n0 = ix.cell_start[lin + 1] - b0;
                            probes_l = 2;
                        }
                    }
                } else if (r < rows) {
                    // decode row r: ids of dimensions 0..L-1, the last of them fastest
                    int32_t maxoff = 0;
                    Lin lin = 0;
                    double lb = 0.0;
                    uint64_t rem64 = (uint64_t)r;
                    uint32_t rem32 = (uint32_t)r;
#pragma unroll
                    for (int j = (FT > 0 ? FT - 2 : F_MAX - 2); j >= 0; --j) {
                        if (FT == 0 && j > L - 1) continue;
                        int32_t digit;
                        if (small) {
                            const uint32_t wj = (uint32_t)w[j];
                            const uint32_t qd = wj > 1 ? __umulhi(rem32, mag[FT > 1 ? j : 0]) : rem32;
                            digit = (int32_t)(rem32 - qd * wj);
                            rem32 = qd;
                        } else {
                            digit = (int32_t)(rem64 % (uint64_t)w[j]);
                            rem64 /= (uint64_t)w[j];
                        }
                        const int32_t oj = lo[j] + digit;
                        maxoff = max(maxoff, oj > Q.c[j] ? oj - Q.c[j] : Q.c[j] - oj);
                        lin += (Lin)(oj - ix.cmin[j]) * (HASH ? (Lin)ix.hstride[j] : (Lin)ix.stride[j]);
                        const double g = gap_to_cells(Q.v[j], oj, oj, (double)ix.a[j]);
                        lb = __dadd_rn(lb, __dmul_rn(g, g));
                    }
                    const bool pass_row = !prune || !(lb * LB_SHRINK > st.tau);
                    if (pass_row) {
                        const int32_t cL = Q.c[L];
                        const int32_t lo_l = lo[L], hi_l = lo[L] + w[L] - 1;
                        if (maxoff >= l) {
                            // shell row: every cell of the run [c-lh, c+lh] inside the box
                            int32_t ta = lo_l, tb = hi_l;
                            if (prune && st.tau < 1.0e300) {
                                // conservative: fl(tau + tau 2^-39) >= tau / LB_SHRINK, and the
                                // reciprocal's rounding is far inside the +1 / -2 slack
                                const double room = __dadd_rn(st.tau, ldexp(st.tau, -39)) - lb;
                                const double G = sqrt(room > 0.0 ? room : 0.0);
                                // compared as integers (ids are within +-2^29, the bounds are
                                // clamped to +-2^30 first)
                                const double ub = floor((Q.v[L] + G) * aLinv) + 1.0;
                                const double lb_t = ceil((Q.v[L] - G) * aLinv) - 2.0;
                                tb = min(tb, (int32_t)fmin(fmax(ub, -0x1p30), 0x1p30));
                                ta = max(ta, (int32_t)fmin(fmax(lb_t, -0x1p30), 0x1p30));
                            }
                            if (ta <= tb) {
                                if constexpr (HASH) {
                                    hash_run(ix, lin, ta, tb, ix.cmin[L], b0, n0, probes_l);
                                } else {
                                    const uint32_t s0 = ix.cell_start[lin + (uint32_t)(ta - ix.cmin[L])];
                                    const uint32_t s1 = ix.cell_start[lin + (uint32_t)(tb - ix.cmin[L]) + 1];
                                    b0 = s0;
                                    n0 = s1 - s0;
                                    probes_l += 2;
                                }
                                if (prune) {
                                    const double g = gap_to_cells(Q.v[L], ta, tb, aL);
                                    key0 = lb_key(__dadd_rn(lb, __dmul_rn(g, g)) * LB_SHRINK);
                                }
                            }
                        } else {
                            // interior row: only the end runs [c-lh, c-l] and [c+l, c+lh] belong to
                            // the layers l .. lh (single cells when lh = l)
                            for (int e = 0; e < 2; ++e) {
                                int32_t t = e == 0 ? cL - l : cL + l;
                                // an empty asm keeps the end cell's bound inside the row loop: the
                                // compiler would otherwise hoist both bounds, and at 64 VGPRs they
                                // spill to scratch on every layer
                                asm volatile("" : "+v"(t));
                                int32_t ta = t, tb = t;
                                if (STOP != GHN_STOP_PAPER && lh > l) {
                                    ta = e == 0 ? max(cL - lh, lo_l) : t;
                                    tb = e == 0 ? t : min(cL + lh, hi_l);
                                }
                                if (tb < lo_l || ta > hi_l) continue;
                                ta = max(ta, lo_l);
                                tb = min(tb, hi_l);
                                double lbe = 0.0;
                                if (prune) {
                                    const double g = gap_to_cells(Q.v[L], ta, tb, aL);
                                    lbe = __dadd_rn(lb, __dmul_rn(g, g)) * LB_SHRINK;
                                    if (lbe > st.tau) continue;
                                }
                                uint32_t s0, sn;
                                if constexpr (HASH) {
                                    hash_run(ix, lin, ta, tb, ix.cmin[L], s0, sn, probes_l);
                                } else {
                                    s0 = ix.cell_start[lin + (uint32_t)(ta - ix.cmin[L])];
                                    sn = ix.cell_start[lin + (uint32_t)(tb - ix.cmin[L]) + 1] - s0;
                                    probes_l += 2;
                                }
                                if (e == 0) { b0 = s0; n0 = sn; key0 = lb_key(lbe); }
                                else { b1 = s0; n1 = sn; key1 = lb_key(lbe); }
                            }
                        }
                    }
                }
                if constexpr (HASH) st.probes += wave_sum_u32(probes_l);
                else st.probes += 2 * (__popcll(ballot(probes_l >= 2)) + __popcll(ballot(probes_l >= 4)));
                score_runs<FT>(ix, Q.q, f, k, b0, n0, key0, b1, n1, key1, prune, s_begin, s_pre, s_key, st);
            }
        }
        if (stop_after_layer<FT, STOP>(ix, Q, f, k, lh, st)) break;
    }
    // only a shifted frame (far query) reaches layer CLAMP or more before its walk ends
    finish_query(ix, io, qi, lh >= (int32_t)CLAMP ? true_layer(lh, far_shift(ix, io.queries, qi, f)) : lh, st);
}

// `preset`: the query's set-up already done (by another lane of the block), or null.
template <int FT, int STOP, bool HASH>
__device__ __forceinline__ void walk_dense(const IndexView& ix, const QueryIO& io, int64_t qi,
                                           uint32_t* s_begin, uint32_t* s_pre, uint32_t* s_key,
                                           const Query<FT>* preset = nullptr) {
    Query<FT> Q;
    if (preset) {
        Q = *preset;
    } else {
        setup_query<FT>(ix, io.queries, qi, FT > 0 ? FT : ix.f, Q);
        if constexpr (FT > 0) uniform_query<FT>(Q);
    }
    if (!Q.finite) {
        write_invalid(ix, io, qi);
        return;
    }
    if (Q.l0 == (int32_t)CLAMP) setup_far<FT>(ix, io.queries, qi, FT > 0 ? FT : ix.f, Q);
    walk_dense_layers<FT, STOP, HASH>(ix, io, qi, s_begin, s_pre, s_key, Q);
}

}  // namespace ghn
