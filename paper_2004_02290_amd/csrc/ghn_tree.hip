// Cell index for many dimensions: occupied cells in Morton order plus a 64-ary
// tree of bounding boxes over them, and the exploration walk that uses it.
//
// Enumerating the cells of a layer by generating their ids stops scaling with
// the dimension: layer 1 alone has 3^f - 1 cells (Eq. 2), 6,560 at f = 8 and
// 43 million at f = 16, almost all of them empty.  Empty cells are not stored
// (Section III-A), so here layer l is found among the occupied cells instead:
// a node of the tree whose box of cell ids spans Chebyshev distances [dmin,
// dmax] from the central cell can only hold cells of layer l if dmin <= l <=
// dmax, and can only hold a closer point than the current k-th if the query's
// distance to the node's region is below it.  Each wave walks the tree depth
// first with a small stack in LDS; the kept cells of layer l are scored with
// the same gather/screen/buffer machinery as the dense walk.
#include "ghn_walk_tree.h"

namespace ghn {
namespace {

constexpr int BT = 256;
constexpr int PT = 256;  // predict: 4 waves = 4 queries per block
constexpr int WPB = PT / WAVE;

__device__ __forceinline__ float load_coord(const void* pts, int64_t idx, int32_t dtype) {
    if (dtype == GHN_BF16) return __uint_as_float((uint32_t)((const uint16_t*)pts)[idx] << 16);
    return ((const float*)pts)[idx];
}

// Morton code of a cell: bit b of dimension j (ids relative to the box minimum)
// for b from the top down, dimensions in order inside each bit; nbits bits in all.
// Codes wider than 64 bits are handled a 64-bit word at a time: word w (0 = the
// most significant) holds code bits [64 (W - 1 - w), 64 (W - w)), W = ceil(nbits / 64).
__global__ __launch_bounds__(BT) void k_morton_keys(const void* pts, int64_t n, int32_t dtype, IndexView iv,
                                                    int nbits, int word, const uint32_t* __restrict__ order,
                                                    uint64_t* keys, uint32_t* vals) {
    const int f = iv.f;
    int bits[F_MAX];
    int maxb = 0;
    for (int j = 0; j < f; ++j) {
        const uint32_t span = (uint32_t)(iv.cmax[j] - iv.cmin[j]);
        bits[j] = span ? 32 - __clz(span) : 0;
        maxb = max(maxb, bits[j]);
    }
    const int nw = (nbits + 63) / 64;
    const int lo = 64 * (nw - 1 - word), hi = min(lo + 64, nbits);
    for (int64_t i = blockIdx.x * (int64_t)BT + threadIdx.x; i < n; i += (int64_t)gridDim.x * BT) {
        const uint32_t p = order ? order[i] : (uint32_t)i;
        uint32_t u[F_MAX];
        for (int j = 0; j < f; ++j) {
            const float x = load_coord(pts, (int64_t)p * f + j, dtype);
            const int64_t c = exact_floor_div(__dadd_rn((double)x, -(double)iv.o[j]), (double)iv.a[j]);
            u[j] = (uint32_t)(c - iv.cmin[j]);
        }
        uint64_t code = 0;
        int pos = nbits;
        for (int b = maxb - 1; b >= 0; --b)
            for (int j = 0; j < f; ++j)
                if (b < bits[j]) {
                    --pos;
                    if (pos >= lo && pos < hi) code = (code << 1) | ((u[j] >> b) & 1u);
                }
        keys[i] = code;
        vals[i] = p;
    }
}

// Cell boundaries of points in cell order, from their cell ids (any code width).
__global__ __launch_bounds__(BT) void k_cell_heads_ids(IndexView iv, int64_t n, uint32_t* heads) {
    const int f = iv.f;
    for (int64_t i = blockIdx.x * (int64_t)BT + threadIdx.x; i < n; i += (int64_t)gridDim.x * BT) {
        bool head = i == 0;
        for (int j = 0; j < f && !head; ++j) {
            const double o = iv.o[j], a = iv.a[j];
            head = exact_floor_div(__dadd_rn((double)iv.spts[i * f + j], -o), a) !=
                   exact_floor_div(__dadd_rn((double)iv.spts[(i - 1) * f + j], -o), a);
        }
        heads[i] = head ? 1u : 0u;
    }
}

__global__ __launch_bounds__(BT) void k_cell_heads(const uint64_t* __restrict__ keys, int64_t n, uint32_t* heads) {
    for (int64_t i = blockIdx.x * (int64_t)BT + threadIdx.x; i < n; i += (int64_t)gridDim.x * BT)
        heads[i] = (i == 0 || keys[i] != keys[i - 1]) ? 1u : 0u;
}

// For every head point: its cell's first point and the cell's ids.
__global__ __launch_bounds__(BT) void k_cell_list(const uint32_t* __restrict__ heads, const uint32_t* __restrict__ rank,
                                                  int64_t n, IndexView iv, uint32_t* cell_start, int32_t* cell_coord) {
    const int f = iv.f;
    for (int64_t i = blockIdx.x * (int64_t)BT + threadIdx.x; i < n; i += (int64_t)gridDim.x * BT) {
        if (!heads[i]) continue;
        const uint32_t c = rank[i];
        cell_start[c] = (uint32_t)i;
        for (int j = 0; j < f; ++j) {
            const int64_t id = exact_floor_div(__dadd_rn((double)iv.spts[i * f + j], -(double)iv.o[j]), (double)iv.a[j]);
            cell_coord[(int64_t)c * f + j] = (int32_t)id;
        }
    }
}

// Boxes of one tree level: node i covers children [64 i, 64 i + 64) of the level below.
__global__ __launch_bounds__(BT) void k_tree_level(const int32_t* __restrict__ child_lo, const int32_t* __restrict__ child_hi,
                                                   int64_t nchild, int32_t f, int32_t* node_lo, int32_t* node_hi,
                                                   int64_t nnode) {
    for (int64_t i = blockIdx.x * (int64_t)BT + threadIdx.x; i < nnode; i += (int64_t)gridDim.x * BT) {
        const int64_t c0 = i * WAVE, c1 = min(c0 + WAVE, nchild);
        for (int j = 0; j < f; ++j) {
            int32_t lo = INT32_MAX, hi = INT32_MIN;
            for (int64_t c = c0; c < c1; ++c) {
                lo = min(lo, child_lo[c * f + j]);
                hi = max(hi, child_hi[c * f + j]);
            }
            node_lo[i * f + j] = lo;
            node_hi[i * f + j] = hi;
        }
    }
}


// At f = 16 the walk is held to 168 VGPRs, three waves per SIMD; left to itself
// the compiler takes 190 and two.
template <int FT> constexpr int tree_waves_per_eu() { return FT == 16 ? 3 : 1; }

template <int FT, int STOP>
__global__ __launch_bounds__(PT) __attribute__((amdgpu_waves_per_eu(tree_waves_per_eu<FT>())))
void k_predict_tree(PredictArgs A) {
    __shared__ uint32_t s_begin[WPB][RUN_CAP];
    __shared__ uint32_t s_pre[WPB][RUN_CAP];
    __shared__ uint64_t s_stack[WPB][TREE_STACK_CAP];
    __shared__ uint64_t s_pend[WPB][FT != 16 ? TREE_PEND_CAP : 1];
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x / WAVE);
    const int64_t slot = wave_slot(A, WPB);
    if (slot >= A.m) return;
    const int64_t qi = A.order ? (int64_t)A.order[slot] : slot;
    // At f = 16 the pending-list state lifts the kernel past 168 VGPRs (3 -> 2 waves per
    // SIMD), which costs more than the revisits it saves there: that instance walks each
    // layer from the root.
    walk_tree<FT, STOP, FT != 16>(A.ix, A.io, qi, s_begin[wv], s_pre[wv], s_stack[wv], s_pend[wv]);
}

template <int FT>
hipError_t launch_ft(const PredictArgs& a, hipStream_t s) {
    const dim3 grid((unsigned)((a.m + WPB - 1) / WPB)), block(PT);
    if (a.stop == GHN_STOP_PAPER)
        hipLaunchKernelGGL((k_predict_tree<FT, GHN_STOP_PAPER>), grid, block, 0, s, a);
    else
        hipLaunchKernelGGL((k_predict_tree<FT, GHN_STOP_EXACT>), grid, block, 0, s, a);
    return launch_status();
}

int grid_for(int64_t work, int threads, int cap = 65536) {
    int64_t g = (work + threads - 1) / threads;
    if (g < 1) g = 1;
    if (g > cap) g = cap;
    return (int)g;
}

}  // namespace

hipError_t launch_morton_keys(const void* pts, int64_t n, int32_t dtype, const IndexView& iv, int nbits, int word,
                              const uint32_t* order, uint64_t* keys, uint32_t* vals, hipStream_t s) {
    hipLaunchKernelGGL(k_morton_keys, dim3(grid_for(n, BT)), dim3(BT), 0, s, pts, n, dtype, iv, nbits, word, order,
                       keys, vals);
    return launch_status();
}

hipError_t launch_cell_heads_ids(const IndexView& iv, int64_t n, uint32_t* heads, hipStream_t s) {
    hipLaunchKernelGGL(k_cell_heads_ids, dim3(grid_for(n, BT)), dim3(BT), 0, s, iv, n, heads);
    return launch_status();
}

hipError_t launch_cell_heads(const uint64_t* sorted_keys, int64_t n, uint32_t* heads, hipStream_t s) {
    hipLaunchKernelGGL(k_cell_heads, dim3(grid_for(n, BT)), dim3(BT), 0, s, sorted_keys, n, heads);
    return launch_status();
}

hipError_t launch_cell_list(const uint32_t* heads, const uint32_t* rank, int64_t n, const IndexView& iv,
                            uint32_t* cell_start, int32_t* cell_coord, hipStream_t s) {
    hipLaunchKernelGGL(k_cell_list, dim3(grid_for(n, BT)), dim3(BT), 0, s, heads, rank, n, iv, cell_start, cell_coord);
    return launch_status();
}

hipError_t launch_tree_level(const int32_t* child_lo, const int32_t* child_hi, int64_t nchild, int32_t f,
                             int32_t* node_lo, int32_t* node_hi, int64_t nnode, hipStream_t s) {
    hipLaunchKernelGGL(k_tree_level, dim3(grid_for(nnode, BT)), dim3(BT), 0, s, child_lo, child_hi, nchild, f, node_lo,
                       node_hi, nnode);
    return launch_status();
}

hipError_t launch_predict_tree(const PredictArgs& a, hipStream_t s) {
    switch (a.ix.f) {
        case 1: return launch_ft<1>(a, s);
        case 2: return launch_ft<2>(a, s);
        case 3: return launch_ft<3>(a, s);
        case 4: return launch_ft<4>(a, s);
        case 8: return launch_ft<8>(a, s);
        case 16: return launch_ft<16>(a, s);
        default: return launch_ft<0>(a, s);
    }
}

}  // namespace ghn
