// Per-query layer walk over the cell tree (Section III-B), shared by the
// single-index and the batched kernels.
//
// Layer l is found among the occupied cells: a tree node whose box of cell ids
// spans Chebyshev distances [dmin, dmax] from the central cell can only hold
// cells of layer l if dmin <= l <= dmax, and can only hold a closer point than
// the current k-th if the query's distance to the node's region is below it.
// The wave walks the tree depth first with a stack in LDS (entries: level,
// first node, node count <= 64); the kept cells of layer l are scored with the
// same gather/screen/buffer machinery as the dense walk.
#pragma once

#include "ghn_walk.h"

namespace ghn {

constexpr int TREE_STACK_CAP = TREE_LEVELS_MAX * WAVE;

__device__ __forceinline__ uint64_t pack_entry(int level, uint32_t first, int count) {
    return ((uint64_t)level << 40) | ((uint64_t)count << 32) | first;
}

template <int FT, int STOP>
__device__ __forceinline__ void walk_tree(const IndexView& ix, const QueryIO& io, int64_t qi,
                                          uint32_t* s_begin, uint32_t* s_pre, uint64_t* stack) {
    const int lane = lane_id();
    const int f = FT > 0 ? FT : ix.f;
    const int k = io.k;
    const bool prune = !(io.flags & GHN_FLAG_NO_PRUNE);

    Query<FT> Q;
    setup_query<FT>(ix, io.queries, qi, f, Q);
    if (!Q.finite) {
        write_invalid(ix, io, qi);
        return;
    }
    WaveState st;
    init_state(st);
    const int top = ix.tree_levels;  // level of the root entries (0 = the cells themselves)

    int32_t l = Q.l0;
    for (;; ++l) {
        st.updated = false;
        int sp = 0;
        if (lane == 0) stack[0] = pack_entry(top, 0u, (int)ix.tree_count[top]);
        sp = 1;
        wave_lds_sync();
        while (sp > 0) {
            --sp;
            const uint64_t e = stack[sp];
            wave_lds_sync();
            const int level = (int)(e >> 40);
            const int count = (int)((e >> 32) & 0xff);
            const uint32_t first = (uint32_t)e;
            const bool active = lane < count;
            const int64_t node = (int64_t)first + lane;
            // Chebyshev range of the node's cells from the central cell, and the
            // squared distance from the query to the node's region of space.
            int32_t dmin = 0, dmax = 0;
            double lb = 0.0;
            if (active) {
                const int32_t* lo = level == 0 ? ix.cell_coord + node * f : ix.node_lo + (ix.tree_off[level] + node) * f;
                const int32_t* hi = level == 0 ? lo : ix.node_hi + (ix.tree_off[level] + node) * f;
#pragma unroll
                for (int j = 0; j < (FT > 0 ? FT : F_MAX); ++j) {
                    if (FT == 0 && j >= f) break;
                    const int32_t a = lo[j], b = hi[j], cj = Q.c[j];
                    const int32_t near = cj < a ? a - cj : (cj > b ? cj - b : 0);
                    const int32_t far = max(cj - a, b - cj);
                    dmin = max(dmin, near);
                    dmax = max(dmax, far);
                    const double g = gap_to_cells(Q.v[j], a, b, (double)ix.a[j]);
                    lb = __dadd_rn(lb, __dmul_rn(g, g));
                }
            }
            const bool close = !prune || !(lb * LB_SHRINK > st.tau);
            st.probes += __popcll(ballot(active));
            if (level == 0) {
                uint32_t b0 = 0, n0 = 0;
                if (active && dmin == l && close) {
                    b0 = ix.cell_first[node];
                    n0 = ix.cell_first[node + 1] - b0;
                }
                score_runs<FT>(ix, Q.q, f, k, b0, n0, 0u, 0u, 0u, 0u, false, s_begin, s_pre, nullptr, st);
            } else {
                const bool keep = active && dmin <= l && l <= dmax && close;
                const uint64_t km = ballot(keep);
                if (keep) {
                    const int64_t c0 = node * WAVE;
                    const int cnt = (int)min((int64_t)WAVE, ix.tree_count[level - 1] - c0);
                    stack[sp + __popcll(km & __lanemask_lt())] = pack_entry(level - 1, (uint32_t)c0, cnt);
                }
                sp += __popcll(km);
                wave_lds_sync();
            }
        }
        if (stop_after_layer<FT, STOP>(ix, Q, f, k, l, st)) break;
    }
    finish_query(ix, io, qi, l, st);
}

}  // namespace ghn
