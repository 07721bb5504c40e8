// Per-query layer walk over the cell tree (Section III-B), shared by the
// single-index and the batched kernels.
//
// Layer l is found among the occupied cells: a tree node whose box of cell ids
// spans Chebyshev distances [dmin, dmax] from the central cell holds cells of
// layer l only if dmin <= l <= dmax, and can only hold a closer point than the
// current k-th if the query's distance to the node's region is below it.  The
// wave evaluates a block of up to 64 sibling nodes at a time (one per lane) and
// walks the tree depth first with a stack of blocks in LDS; the cells of layer
// l it reaches are scored with the same gather/screen/buffer machinery as the
// dense walk.
//
// Every node is evaluated at the layer equal to its dmin and no earlier: a
// block whose nodes lie partly in later layers is put on a pending list with
// the smallest dmin among them, and evaluated again when the walk reaches that
// layer (its nodes of earlier layers were handled then and are skipped).  By
// induction every node is first reached at its own dmin, so the walk visits
// each node once instead of once per layer it spans.  The pending list lives in
// LDS; if it fills up, the later layers each walk the tree from the root with
// the dmin <= l <= dmax test instead, which finds the same cells.  With
// FRONTIER = false every layer walks from the root (no pending list: fewer
// registers and less LDS, for kernels that also hold the dense walk).
#pragma once

#include "ghn_walk.h"

namespace ghn {

constexpr int TREE_STACK_CAP = TREE_LEVELS_MAX * WAVE;
constexpr int TREE_PEND_CAP = 512;  // pending blocks per wave
constexpr int32_t PEND_KEY_MAX = (1 << 23) - 1;
static_assert(TREE_LEVELS_MAX <= 8, "pending entries hold the level in 3 bits");

// DFS stack entry: a block of `count` (1..64) nodes of `level`, starting at `first`.
__device__ __forceinline__ uint64_t pack_entry(int level, uint32_t first, int count) {
    return ((uint64_t)level << 40) | ((uint64_t)count << 32) | first;
}

// Pending entry: the same block plus the layer at which to evaluate it again.  A
// key above 2^23 - 1 is stored as that bound; an early evaluation re-defers the
// block and costs only the visit (the walk leaves frontier mode before the
// layer reaches the bound, so the early key cannot repeat within one layer).
__device__ __forceinline__ uint64_t pack_pending(int32_t key, int level, uint32_t first, int count) {
    const uint32_t kk = (uint32_t)(key < PEND_KEY_MAX ? key : PEND_KEY_MAX);
    return ((uint64_t)kk << 41) | ((uint64_t)level << 38) | ((uint64_t)(count - 1) << 32) | first;
}
__device__ __forceinline__ int32_t pending_key(uint64_t p) { return (int32_t)(p >> 41); }
__device__ __forceinline__ uint64_t pending_block(uint64_t p) {
    return pack_entry((int)((p >> 38) & 7), (uint32_t)p, (int)((p >> 32) & 63) + 1);
}

template <int FT, int STOP, bool FRONTIER>
__device__ __forceinline__ void walk_tree_layers(const IndexView& ix, const QueryIO& io, int64_t qi,
                                                 uint32_t* s_begin, uint32_t* s_pre, uint64_t* stack, uint64_t* pend,
                                                 const Query<FT>& Q) {
    const int lane = lane_id();
    const int f = FT > 0 ? FT : ix.f;
    const int k = io.k;
    const bool prune = !(io.flags & GHN_FLAG_NO_PRUNE);
    WaveState st;
    init_state(st);
    const int top = ix.tree_levels;  // level of the root entries (0 = the cells themselves)

    int npend = 0;          // pending blocks (wave-uniform)
    bool frontier = FRONTIER;  // false once the pending list overflowed or keys could saturate
    // ring schedule (EXACT rule only): each step walks the layers l .. lh at once
    RingStep ring(io);
    int32_t l = Q.l0, lh = Q.l0;
    for (;; l = lh + 1) {
        lh = STOP == GHN_STOP_PAPER ? l : ring.last_layer(l, st.count == k, Q.lcover);
        st.updated = false;
        if (lh >= PEND_KEY_MAX - 1) frontier = false;
        bool overflow = false;
        bool root = !frontier || l == Q.l0;  // the root block starts the walk of this step
        int scan = 0;                        // pending entries below `scan` are not due in this step
        for (;;) {
            uint64_t e;
            if (root) {
                e = pack_entry(top, 0u, (int)ix.tree_count[top]);
                root = false;
            } else if (frontier) {
                // next pending block due at this layer
                int found = -1;
                while (scan < npend) {
                    const int idx = scan + lane;
                    const bool due = idx < npend && pending_key(pend[idx]) <= lh;
                    const uint64_t dm = ballot(due);
                    if (dm) {
                        found = scan + __ffsll((unsigned long long)dm) - 1;
                        break;
                    }
                    scan += WAVE;
                }
                if (found < 0) break;
                e = pending_block(pend[found]);
                wave_lds_sync();
                // remove it: the last entry moves into its slot and is checked next
                if (lane == 0) pend[found] = pend[npend - 1];
                --npend;
                scan = found;
                wave_lds_sync();
            } else {
                break;
            }
            int sp = 0;
            if (lane == 0) stack[0] = e;
            sp = 1;
            wave_lds_sync();
            while (sp > 0) {
                --sp;
                const uint64_t se = stack[sp];
                wave_lds_sync();
                const int level = (int)(se >> 40);
                const int count = (int)((se >> 32) & 0xff);
                const uint32_t first = (uint32_t)se;
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
                const bool close = active && (!prune || !(lb * LB_SHRINK > st.tau));
                st.probes += __popcll(ballot(active));
                if (frontier) {
                    // nodes of later steps: the block comes back at the nearest of them
                    const bool later = close && dmin > lh;
                    if (ballot(later)) {
                        const int32_t key = wave_min_nonneg_i32(later ? dmin : INT32_MAX);
                        if (npend < TREE_PEND_CAP) {
                            if (lane == 0) pend[npend] = pack_pending(key, level, first, count);
                            ++npend;
                        } else {
                            overflow = true;
                        }
                    }
                }
                if (level == 0) {
                    uint32_t b0 = 0, n0 = 0;
                    if (close && dmin >= l && dmin <= lh) {
                        b0 = ix.cell_first[node];
                        n0 = ix.cell_first[node + 1] - b0;
                    }
                    score_runs<FT>(ix, Q.q, f, k, b0, n0, 0u, 0u, 0u, 0u, false, s_begin, s_pre, nullptr, st);
                } else {
                    // frontier mode reaches a node first at the step holding its dmin; from the
                    // root, every node whose range meets the step's layers
                    const bool keep = close && (frontier ? (dmin >= l && dmin <= lh) : (dmin <= lh && l <= dmax));
                    const uint64_t km = ballot(keep);
                    if (keep) {
                        const int64_t c0 = node * WAVE;
                        const int cnt = (int)min((int64_t)WAVE, ix.tree_count[level - 1] - c0);
                        stack[sp + __popcll(km & __lanemask_lt())] = pack_entry(level - 1, (uint32_t)c0, cnt);
                    }
                    sp += __popcll(km);
                }
                wave_lds_sync();
            }
        }
        if (overflow) frontier = false;  // blocks were lost: later steps start from the root
        if (stop_after_layer<FT, STOP>(ix, Q, f, k, lh, st)) break;
    }
    // only a shifted frame (far query) reaches layer CLAMP or more before its walk ends
    finish_query(ix, io, qi, lh >= (int32_t)CLAMP ? true_layer(lh, far_shift(ix, io.queries, qi, f)) : lh, st);
}

template <int FT, int STOP, bool FRONTIER>
__device__ __forceinline__ void walk_tree(const IndexView& ix, const QueryIO& io, int64_t qi,
                                          uint32_t* s_begin, uint32_t* s_pre, uint64_t* stack, uint64_t* pend) {
    Query<FT> Q;
    setup_query<FT>(ix, io.queries, qi, FT > 0 ? FT : ix.f, Q);
    if constexpr (FT > 0) uniform_query<FT>(Q);
    if (!Q.finite) {
        write_invalid(ix, io, qi);
        return;
    }
    if (Q.l0 == (int32_t)CLAMP) setup_far<FT>(ix, io.queries, qi, FT > 0 ? FT : ix.f, Q);
    walk_tree_layers<FT, STOP, FRONTIER>(ix, io, qi, s_begin, s_pre, stack, pend, Q);
}

}  // namespace ghn
