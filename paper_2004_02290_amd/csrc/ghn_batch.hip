// Many independent indexes answered in one persistent launch.
//
// The queries of all batch items form one index space: item i owns global query
// positions [first_i, first_i + m_i).  The space is cut into 8 equal ranges, one per
// XCD (blocks are dealt round-robin over the XCDs, so block b runs on XCD b % 8):
// the waves of an XCD take chunks of its range from that range's atomic counter, and
// steal from the next ranges once it is empty, so items of very different cost
// balance while each XCD's L2 mostly serves its own range.  The counters sit 128
// bytes apart: in one cache line their atomics serialised (measured on the 256 3-D
// problems: one counter 4.76 ms, 8 counters in one line 5.80 ms, 8 counters 128 bytes
// apart 3.97 ms).  With a spatial order
// (queries sorted by (item, Morton code of the central cell)) the ranges are regions
// of space.  Each position is walked with its item's own index (dense or tree
// lookup) exactly as the single-index kernels do.  The launch reads only device
// memory, so it can be captured in a graph and replayed.
#include "ghn_walk_dense.h"
#include "ghn_walk_tree.h"

namespace ghn {
namespace {

constexpr int BPT = 256;
constexpr int BWPB = BPT / WAVE;
constexpr int CHUNK = 4;  // queries taken per atomic

constexpr int COUNTER_STRIDE = 16;  // the 8 work counters sit 128 bytes apart

__global__ void k_reset_counter(uint64_t* counter) {
    if (threadIdx.x < NUM_XCD) counter[threadIdx.x * COUNTER_STRIDE] = 0;
}

// A batch whose indexes all use the dense table runs an instance without the tree
// walk, which needs fewer registers: up to 4 dimensions it is held to 96 VGPRs so
// that 5 waves share a SIMD instead of 4 (at f = 4 a few values spill to scratch;
// measured 7 % faster on 256 3-D problems than the instance that can also walk
// trees).  More waves do not pay: at 72 or 64 VGPRs the 3-D instance spills 92 to
// 116 bytes per lane.
// The other instances are held to the occupancy their walk reaches on its own, so that
// the rare set-up of a query far outside the box (setup_far) cannot lower it.
template <int FT, bool TREE>
constexpr int batched_waves_per_eu() {
    return FT < 1 ? 1 : (!TREE ? (FT <= 4 ? 5 : 3) : (FT == 1 ? 7 : (FT == 2 ? 5 : (FT <= 4 ? 4 : 3))));
}

// Lookups of a batch's items: the dense-table walk only, the tree walk only (the tree
// and hash indexes), or both.  A one-kind instance holds only that walk's registers:
// the tree-only one fits the occupancy of the single-index tree kernel (four waves
// per SIMD at f = 8, where the mixed instance runs three and spills).
enum BatchKind { DENSE_ONLY = 0, MIXED = 1, TREE_ONLY = 2 };
template <int FT, int KIND>
constexpr int batch_kind_waves() {
    return KIND == TREE_ONLY ? (FT < 1 ? 1 : 4) : batched_waves_per_eu<FT, KIND == MIXED>();
}

template <int FT, int STOP, int KIND>
__global__ __launch_bounds__(BPT) __attribute__((amdgpu_waves_per_eu(batch_kind_waves<FT, KIND>())))
void k_predict_batched(const BatchItem* __restrict__ items, int n_items, int64_t total,
                       const uint32_t* __restrict__ order, uint64_t* counter) {
    __shared__ uint32_t s_begin[BWPB][RUN_CAP];
    __shared__ uint32_t s_pre[BWPB][RUN_CAP];
    __shared__ uint32_t s_key[BWPB][RUN_CAP];
    constexpr bool TREE = KIND != DENSE_ONLY;
    __shared__ uint64_t s_stack[BWPB][TREE ? TREE_STACK_CAP : 1];
    __shared__ uint64_t s_pend[BWPB][TREE && FT == 8 ? TREE_PEND_CAP : 1];
    const int lane = lane_id();
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x / WAVE);
    const int home = (int)(blockIdx.x % NUM_XCD);
    for (int r = 0; r < NUM_XCD; ++r) {
        const int x = (home + r) % NUM_XCD;
        const int64_t lo = total * x / NUM_XCD, hi = total * (x + 1) / NUM_XCD;
        for (;;) {
            uint64_t c0 = 0;
            if (lane == 0) c0 = atomicAdd((unsigned long long*)&counter[x * COUNTER_STRIDE], (unsigned long long)CHUNK);
            c0 = ((uint64_t)(uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(c0 >> 32)) << 32) |
                 (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)c0);
            const int64_t w0 = lo + (int64_t)c0;
            if (w0 >= hi) break;
            for (int c = 0; c < CHUNK; ++c) {
                const int64_t w = w0 + c;
                if (w >= hi) break;
                const int64_t pos = order ? (int64_t)order[w] : w;
                const BatchItem& it = items[batch_item_of(items, n_items, pos)];
                const IndexView& ix = *it.ix;
                const int64_t qi = pos - it.first;
                // (the host launches a one-kind instance only for batches of that kind)
                if constexpr (KIND == TREE_ONLY) {
                    if (ix.lookup == LOOKUP_DENSE) continue;
                    walk_tree<FT, STOP, FT == 8>(ix, it.io, qi, s_begin[wv], s_pre[wv], s_stack[wv], s_pend[wv]);
                } else if (ix.lookup == LOOKUP_DENSE) {
                    walk_dense<FT, STOP, false>(ix, it.io, qi, s_begin[wv], s_pre[wv], s_key[wv]);
                } else if constexpr (KIND == MIXED) {
                    // the tree walk's pending list only where it costs no occupancy: the f = 8
                    // instance already runs at few waves per SIMD; the others hold the dense
                    // walk at three or four, which the extra state would lower
                    walk_tree<FT, STOP, FT == 8>(ix, it.io, qi, s_begin[wv], s_pre[wv], s_stack[wv], s_pend[wv]);
                }
            }
        }
    }
}

template <int FT, int KIND>
void launch_stop(const BatchItem* items, int n_items, int64_t total, const uint32_t* order, uint64_t* counter,
                 int stop, int blocks, hipStream_t s) {
    if (stop == GHN_STOP_PAPER)
        hipLaunchKernelGGL((k_predict_batched<FT, GHN_STOP_PAPER, KIND>), dim3(blocks), dim3(BPT), 0, s, items, n_items,
                           total, order, counter);
    else
        hipLaunchKernelGGL((k_predict_batched<FT, GHN_STOP_EXACT, KIND>), dim3(blocks), dim3(BPT), 0, s, items, n_items,
                           total, order, counter);
}

template <int FT>
hipError_t launch_ft(const BatchItem* items, int n_items, int64_t total, const uint32_t* order, uint64_t* counter,
                     int stop, bool any_tree, bool any_dense, int blocks, hipStream_t s) {
    if (any_tree && any_dense) launch_stop<FT, MIXED>(items, n_items, total, order, counter, stop, blocks, s);
    else if (any_tree) launch_stop<FT, TREE_ONLY>(items, n_items, total, order, counter, stop, blocks, s);
    else launch_stop<FT, DENSE_ONLY>(items, n_items, total, order, counter, stop, blocks, s);
    return launch_status();
}

}  // namespace

hipError_t launch_predict_batched(const BatchItem* items, int n_items, int64_t total, int f, int stop, bool any_tree,
                                  bool any_dense, const uint32_t* order, int blocks_override, uint64_t* counter,
                                  hipStream_t s) {
    hipLaunchKernelGGL(k_reset_counter, dim3(1), dim3(64), 0, s, counter);
    int64_t blocks = (total + BWPB * CHUNK - 1) / (BWPB * CHUNK);
    if (blocks > 4096) blocks = 4096;
    if (blocks < 1) blocks = 1;
    if (blocks_override > 0) blocks = blocks_override;
    switch (f) {
        case 1: return launch_ft<1>(items, n_items, total, order, counter, stop, any_tree, any_dense, (int)blocks, s);
        case 2: return launch_ft<2>(items, n_items, total, order, counter, stop, any_tree, any_dense, (int)blocks, s);
        case 3: return launch_ft<3>(items, n_items, total, order, counter, stop, any_tree, any_dense, (int)blocks, s);
        case 4: return launch_ft<4>(items, n_items, total, order, counter, stop, any_tree, any_dense, (int)blocks, s);
        case 8: return launch_ft<8>(items, n_items, total, order, counter, stop, any_tree, any_dense, (int)blocks, s);
        default: return launch_ft<0>(items, n_items, total, order, counter, stop, any_tree, any_dense, (int)blocks, s);
    }
}

}  // namespace ghn
