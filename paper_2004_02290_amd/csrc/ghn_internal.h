// Internal declarations shared by the libghn translation units: the device view
// of an index, launch entry points, and small wave64 helpers for gfx950.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/ghn.h"

namespace ghn {

constexpr int WAVE = 64;
constexpr int F_MAX = GHN_F_MAX;
constexpr int K_MAX = GHN_K_MAX;
// Training-point cell ids must lie in (-COORD_LIMIT, COORD_LIMIT).
constexpr int64_t COORD_LIMIT = int64_t(1) << 27;
// Query cell ids are exact up to CELL_SAT in magnitude and saturated beyond (a
// query coordinate can lie arbitrarily far outside the data).
constexpr double CELL_SAT = 0x1p40;
// A query whose central cell lies more than CLAMP cells outside the occupied box is
// walked in a shifted frame (walk_frame below) whose cell ids stay below 2^29.
constexpr int64_t CLAMP = int64_t(1) << 28;

enum Lookup : int32_t { LOOKUP_DENSE = 0, LOOKUP_TREE = 1, LOOKUP_HASH = 2 };
constexpr uint64_t HASH_EMPTY = ~0ull;  // free slot of the cell hash (keys are < 2^62)
constexpr int TREE_LEVELS_MAX = 6;  // levels of the bounding-box tree, cells included

// Device-side view of an index, passed by value to kernels.
struct IndexView {
    int64_t n;
    int32_t f;
    int32_t dtype;
    int32_t task;
    int32_t lookup;
    const float* spts;          // n x f points in cell order (FP32 copy; exact for bf16 input)
    const int32_t* sid;         // n original row ids, cell order
    const uint32_t* cell_start; // dense: box_cells + 1 offsets into spts; tree: num_cells + 1
    const void* targets;        // n targets, original order
    int64_t box_cells;
    // occupied cells in key order (Morton for the tree lookup, row-major for the
    // dense one) and the bounding boxes above them
    int64_t num_cells;
    const uint32_t* cell_first; // num_cells + 1 offsets into spts
    const int32_t* cell_coord;  // num_cells x f cell ids
    int32_t tree_levels;        // levels above the cells (the root entry's level)
    int64_t tree_count[TREE_LEVELS_MAX];  // nodes per level; level 0 = cells
    int64_t tree_off[TREE_LEVELS_MAX];    // first node of level L (>= 1) in node_lo / node_hi
    const int32_t* node_lo;     // per node, f lowest cell ids of its subtree
    const int32_t* node_hi;     // per node, f highest cell ids
    float a[F_MAX];             // cell width per dimension
    double ainv[F_MAX];         // 1 / a (FP64), for quotient estimates that are then corrected exactly
    float o[F_MAX];             // origin per dimension
    int32_t cmin[F_MAX];
    int32_t cmax[F_MAX];
    uint32_t stride[F_MAX];     // dense-box linear index stride per dimension (last = 1)
    // hash lookup: 64-bit row-major strides over the box, and the open-addressing
    // table of occupied cells (key -> cell index, linear probing from hash_slot)
    uint64_t hstride[F_MAX];
    const uint64_t* hkeys;      // hcap keys, HASH_EMPTY where free
    const uint32_t* hvals;      // hcap cell indexes
    uint64_t hmask;             // hcap - 1 (hcap a power of two >= 2 num_cells)
    // bf16 screen records (grouped matrix-core screen): per point in cell order,
    // x' = fl32(x - c0) split as hi = bf16(x'), lo = bf16(x' - hi), stored as
    // [hi(sp), lo(sp)] with the dimensions past f zero, and xn = |x'|^2 in FP32
    const uint16_t* srec;       // n x 2 sp
    const float* sxn;           // n
    int32_t sp;                 // padded dimension: 8, 16 or 32
    float c0[F_MAX];            // screen centre (centre of the occupied box)
};

// First slot of a cell key in the hash table: the SplitMix64 finalizer (Steele,
// Lea and Flood, 2014) spreads row-major keys, whose low bits are the last
// dimension's id, over the whole table.
__host__ __device__ __forceinline__ uint64_t hash_slot(uint64_t key, uint64_t mask) {
    key ^= key >> 30;
    key *= 0xbf58476d1ce4e5b9ull;
    key ^= key >> 27;
    key *= 0x94d049bb133111ebull;
    key ^= key >> 31;
    return key & mask;
}

// Cell index of a key, or -1 if the cell is empty.  The table is at most half
// full, so a free slot ends every probe sequence; `reads` counts the slots read.
__device__ __forceinline__ int64_t hash_find(const IndexView& ix, uint64_t key, uint32_t& reads) {
    uint64_t h = hash_slot(key, ix.hmask);
    for (uint64_t i = 0; i <= ix.hmask; ++i) {
        const uint64_t k = ix.hkeys[h];
        ++reads;
        if (k == key) return (int64_t)ix.hvals[h];
        if (k == HASH_EMPTY) return -1;
        h = (h + 1) & ix.hmask;
    }
    return -1;
}

// ---------------------------------------------------------------------------------------
// Exact floor of v / a (a > 0 finite, v finite): the largest integer t with t * a <= v.
// The FP64 quotient is rounded, so the candidate is checked against exact products; for
// |t| < 2^29 and an FP32 width, t * a is exact in FP64.
// t * a > v, exactly, for an integer-valued t, an FP32 width a > 0 and a finite v with
// t within two of v / a.  p + e = t * a exactly (e is the FMA residual).  When e = 0
// the sign of the rounded p - v is exact; when e != 0, |t| > 2^29, so p and v lie
// within a factor of two and p - v is exact (Sterbenz).
__device__ __forceinline__ bool prod_gt(double t, double a, double v) {
    const double p = __dmul_rn(t, a);
    const double e = __builtin_fma(t, a, -p);
    const double d = __dadd_rn(p, -v);
    return d > -e;
}

// Cell id of a query coordinate (Eq. 1): the exact floor of v / a, saturated to
// [-CELL_SAT, CELL_SAT], as an integer-valued double.  v * (1 / a) is within 2^-11 of
// v / a while |v / a| <= 2^41, so the floor of the estimate is off by at most one and
// the exact product tests correct it; beyond, only the saturation matters.  A NaN
// gives -CELL_SAT.
__device__ __forceinline__ double cell_floor_sat(double v, double a, double ainv) {
    double t = floor(v * ainv);
    if (fabs(t) <= 0x1p41) {
        if (prod_gt(t, a, v)) t -= 1.0;
        else if (!prod_gt(t + 1.0, a, v)) t += 1.0;
    }
    return fmin(fmax(t, -CELL_SAT), CELL_SAT);
}

// Walk frame of a query far outside the occupied box.  With t the true central cell,
// D_j its distance to [cmin_j, cmax_j] in dimension j and l0 = max_j D_j, the layer of
// a box cell x is L(x) = max_j |x_j - t_j| (Section III-B).  If l0 > CLAMP, let
// s = l0 - CLAMP: a dimension with D_j >= s moves s cells toward the box (its
// distances to every box cell drop by s), and any other dimension is clamped into
// the box.  Box spans are below 2^28 = CLAMP, so the other dimensions' distances stay
// below l0 <= L(x) before and below CLAMP <= L(x) - s after, and the frame layer of
// every box cell is exactly L(x) - s: the layers hold the same cells in the same
// order.  Frame ids lie within CLAMP of the box.
__device__ __forceinline__ double cell_outside(double t, int32_t lo, int32_t hi) {
    return fmax(fmax((double)lo - t, t - (double)hi), 0.0);
}
__device__ __forceinline__ double frame_shift(double l0) { return l0 > (double)CLAMP ? l0 - (double)CLAMP : 0.0; }
__device__ __forceinline__ int32_t frame_id(double t, int32_t lo, int32_t hi, double shift) {
    if (shift == 0.0) return (int32_t)t;
    if (cell_outside(t, lo, hi) >= shift) return (int32_t)(t < (double)lo ? t + shift : t - shift);
    return (int32_t)fmin(fmax(t, (double)lo), (double)hi);
}
// A true layer (frame layer + shift) as reported: saturated to int32.
__device__ __forceinline__ int32_t true_layer(int32_t l, int64_t shift) {
    const int64_t t = (int64_t)l + shift;
    return t < (int64_t)INT32_MAX ? (int32_t)t : INT32_MAX;
}

__device__ __forceinline__ int64_t exact_floor_div(double v, double a) {
    double t = floor(v / a);
    if (!(fabs(t) < 4.0e18)) return t > 0 ? int64_t(4000000000000000000LL) : -int64_t(4000000000000000000LL);
    if (fabs(t) < 536870912.0) {
        if (__dmul_rn(t, a) > v) t -= 1.0;
        else if (__dmul_rn(t + 1.0, a) <= v) t += 1.0;
    }
    return int64_t(t);
}

// ---------------------------------------------------------------------------------------
// wave64 helpers
__device__ __forceinline__ int lane_id() { return __lane_id(); }

__device__ __forceinline__ uint64_t ballot(bool p) { return __ballot(p); }

__device__ __forceinline__ int readlane_i32(int v, int l) { return __builtin_amdgcn_readlane(v, l); }

__device__ __forceinline__ float readlane_f32(float v, int l) {
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), l));
}

__device__ __forceinline__ double readlane_f64(double v, int l) {
    int64_t b = __double_as_longlong(v);
    int lo = __builtin_amdgcn_readlane(int(uint32_t(b)), l);
    int hi = __builtin_amdgcn_readlane(int(uint32_t(uint64_t(b) >> 32)), l);
    return __longlong_as_double(int64_t((uint64_t(uint32_t(hi)) << 32) | uint32_t(lo)));
}

// `v` with the value of lane `l` (wave-uniform) replaced by `x`: one v_writelane.
// The compiler has the intrinsic but no builtin for it, so it is bound by name.
extern "C" __device__ int ghn_amdgcn_writelane(int x, int l, int v) __asm("llvm.amdgcn.writelane.i32");
__device__ __forceinline__ int writelane_i32(int v, int x, int l) { return ghn_amdgcn_writelane(x, l, v); }
__device__ __forceinline__ float writelane_f32(float v, float x, int l) {
    return __int_as_float(ghn_amdgcn_writelane(__float_as_int(x), l, __float_as_int(v)));
}
__device__ __forceinline__ double writelane_f64(double v, double x, int l) {
    const uint64_t bv = (uint64_t)__double_as_longlong(v), bx = (uint64_t)__double_as_longlong(x);
    const uint32_t lo = (uint32_t)ghn_amdgcn_writelane((int)(uint32_t)bx, l, (int)(uint32_t)bv);
    const uint32_t hi = (uint32_t)ghn_amdgcn_writelane((int)(uint32_t)(bx >> 32), l, (int)(uint32_t)(bv >> 32));
    return __longlong_as_double((int64_t)(((uint64_t)hi << 32) | lo));
}

// Value of `v` held by lane (lane - 1); lane 0 gets 0.  DPP wave_shr:1 (a VALU lane
// shift across the whole wave64, no LDS round trip).
constexpr int DPP_WAVE_SHR1 = 0x138;
__device__ __forceinline__ int shfl_up1_i32(int v) {
    return __builtin_amdgcn_mov_dpp(v, DPP_WAVE_SHR1, 0xf, 0xf, true);
}
__device__ __forceinline__ double shfl_up1_f64(double v) {
    int64_t b = __double_as_longlong(v);
    int lo = shfl_up1_i32(int(uint32_t(b)));
    int hi = shfl_up1_i32(int(uint32_t(uint64_t(b) >> 32)));
    return __longlong_as_double(int64_t((uint64_t(uint32_t(hi)) << 32) | uint32_t(lo)));
}

// Minimum over the wave of a non-negative int (uniform result): DPP row_shr
// min-scans inside each 16-lane row, then row broadcasts (the pattern of the
// prefix sum below).
__device__ __forceinline__ int wave_min_nonneg_i32(int m) {
    // lanes with no source lane read INT32_MAX, the identity of min, so each step
    // folds into one DPP min
    m = min(m, __builtin_amdgcn_update_dpp(INT32_MAX, m, 0x111, 0xf, 0xf, false));  // row_shr:1
    m = min(m, __builtin_amdgcn_update_dpp(INT32_MAX, m, 0x112, 0xf, 0xf, false));  // row_shr:2
    m = min(m, __builtin_amdgcn_update_dpp(INT32_MAX, m, 0x114, 0xf, 0xf, false));  // row_shr:4
    m = min(m, __builtin_amdgcn_update_dpp(INT32_MAX, m, 0x118, 0xf, 0xf, false));  // row_shr:8
    // row minima into the later rows: lane 15 into rows 1 and 3, then lane 31 into
    // rows 2 and 3; lane 63 ends with the minimum of the wave
    m = min(m, __builtin_amdgcn_update_dpp(INT32_MAX, m, 0x142, 0xa, 0xf, false));  // row_bcast:15
    m = min(m, __builtin_amdgcn_update_dpp(INT32_MAX, m, 0x143, 0xc, 0xf, false));  // row_bcast:31
    return __builtin_amdgcn_readlane(m, 63);
}

// The same for a non-negative float (its bit pattern orders like the value).
__device__ __forceinline__ float wave_min_nonneg(float v) {
    return __int_as_float(wave_min_nonneg_i32(__float_as_int(v)));
}

// DPP lane patterns (gfx9 encodings).  row_shl:n / row_shr:n read lane i + n / i - n
// of the same 16-lane row, row_ror:n lane (i - n) mod 16, quad_perm a permutation
// inside each group of four, row_bcast:15 / :31 lane 15 of the previous row / lane 31.
constexpr int DPP_QUAD_XOR1 = 0xB1;  // quad_perm [1,0,3,2]
constexpr int DPP_QUAD_XOR2 = 0x4E;  // quad_perm [2,3,0,1]
constexpr int DPP_ROW_SHL4 = 0x104;
constexpr int DPP_ROW_SHR1 = 0x111, DPP_ROW_SHR2 = 0x112, DPP_ROW_SHR4 = 0x114, DPP_ROW_SHR8 = 0x118;
constexpr int DPP_ROW_ROR8 = 0x128;
constexpr int DPP_ROW_BCAST15 = 0x142, DPP_ROW_BCAST31 = 0x143;

// Inclusive prefix sum over the wave: a Hillis-Steele scan inside each row with
// row shifts, then each row adds the totals of the rows before it (row broadcasts
// of lane 15 into rows 1 and 3, then of lane 31 into rows 2 and 3).  Lanes with
// no source lane, and rows outside the row mask, add 0.
__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t v) {
    int x = (int)v;
    x += __builtin_amdgcn_update_dpp(0, x, DPP_ROW_SHR1, 0xf, 0xf, false);
    x += __builtin_amdgcn_update_dpp(0, x, DPP_ROW_SHR2, 0xf, 0xf, false);
    x += __builtin_amdgcn_update_dpp(0, x, DPP_ROW_SHR4, 0xf, 0xf, false);
    x += __builtin_amdgcn_update_dpp(0, x, DPP_ROW_SHR8, 0xf, 0xf, false);
    x += __builtin_amdgcn_update_dpp(0, x, DPP_ROW_BCAST15, 0xa, 0xf, false);
    x += __builtin_amdgcn_update_dpp(0, x, DPP_ROW_BCAST31, 0xc, 0xf, false);
    return (uint32_t)x;
}

// Value of `v` held by lane (lane ^ S), S a power of two below 64: DPP inside a row
// (S <= 8), a swizzle inside each 32-lane half (S = 16), a permute across halves.
template <int S>
__device__ __forceinline__ uint32_t xor_lane(uint32_t v) {
    const int x = (int)v;
    if constexpr (S == 1) {
        return (uint32_t)__builtin_amdgcn_update_dpp(x, x, DPP_QUAD_XOR1, 0xf, 0xf, false);
    } else if constexpr (S == 2) {
        return (uint32_t)__builtin_amdgcn_update_dpp(x, x, DPP_QUAD_XOR2, 0xf, 0xf, false);
    } else if constexpr (S == 4) {
        const int fwd = __builtin_amdgcn_update_dpp(x, x, DPP_ROW_SHL4, 0xf, 0xf, false);
        const int back = __builtin_amdgcn_update_dpp(x, x, DPP_ROW_SHR4, 0xf, 0xf, false);
        return (uint32_t)((lane_id() & 4) ? back : fwd);
    } else if constexpr (S == 8) {
        return (uint32_t)__builtin_amdgcn_update_dpp(x, x, DPP_ROW_ROR8, 0xf, 0xf, false);
    } else if constexpr (S == 16) {
        return (uint32_t)__builtin_amdgcn_ds_swizzle(x, 0x401f);  // bitmask mode: and 0x1f, xor 0x10
    } else {
        static_assert(S == 32, "lane distance must be a power of two below 64");
        // a plain permute (lane ^ 32 is always a lane of the wave): no bounds test, whose
        // lane-limit value would otherwise be kept live across a whole walk
        return (uint32_t)__builtin_amdgcn_ds_bpermute((lane_id() ^ 32) << 2, x);
    }
}

__device__ __forceinline__ uint32_t wave_sum_u32(uint32_t v) {
#pragma unroll
    for (int d = 1; d < WAVE; d <<= 1) v += __shfl_xor(v, d, WAVE);
    return v;
}

// ---------------------------------------------------------------------------------------
// Host-layer environment (ghn_hostenv.hip).  GHN_FAULT=alloc[:N] or launch[:N] makes the
// N-th device allocation or launch check fail; GHN_LOG=1 logs calls and failures.
hipError_t device_alloc(void** p, size_t bytes);  // hipMalloc of max(bytes, 1), or the injected failure
void device_free(void* p);                        // hipFree of a device_alloc block (NULL is ignored)
hipError_t launch_status();                       // hipGetLastError after launches, or the injected failure
bool log_enabled();
void log_line(const char* fmt, ...) __attribute__((format(printf, 1, 2)));

// Static device arrays (ghn_arrays.hip): this device's address of each, looked up once
// per device with hipGetSymbolAddress (hipErrorInvalidDevice above device 255).
hipError_t noalloc_workspace(void** out);        // GHN_NOALLOC_WS_BYTES for ghn_predict_noalloc
hipError_t walk_fault_address(uint32_t** out);   // the walk fault word
hipError_t launch_clear_word(uint32_t* w, hipStream_t s);

// ---------------------------------------------------------------------------------------
// Host-side launchers (defined in the .hip files).
hipError_t launch_cells_minmax(const void* pts, int64_t n, int32_t f, int32_t dtype, const float* a,
                               const float* o, int32_t* d_minmax, int32_t* d_flags, hipStream_t s);
hipError_t launch_hash_build(const uint64_t* sorted_keys, const uint32_t* cell_first, int64_t ncell, uint64_t* hkeys,
                             uint32_t* hvals, uint64_t mask, hipStream_t s);
hipError_t launch_dense_keys(const void* pts, int64_t n, int32_t f, int32_t dtype, const IndexView& iv,
                             uint64_t* keys, uint32_t* vals, hipStream_t s);
size_t radix_sort_temp_bytes(int64_t n);
hipError_t radix_sort_pairs(uint64_t* keys, uint32_t* vals, uint64_t* keys_alt, uint32_t* vals_alt,
                            int64_t n, int nbits, void* temp, bool* result_in_alt, hipStream_t s);
hipError_t launch_gather_points(const void* pts, int64_t n, int32_t f, int32_t dtype, const uint32_t* perm,
                                float* spts, int32_t* sid, hipStream_t s);
hipError_t launch_screen_records(const IndexView& iv, uint16_t* rec, float* xn, hipStream_t s);
hipError_t launch_unsort_points(const float* spts, const int32_t* sid, int64_t n, int32_t f, float* out, hipStream_t s);
hipError_t launch_widen_points(const void* pts, int64_t count, int32_t dtype, float* out, hipStream_t s);
hipError_t launch_merge_points(const uint64_t* okeys, const float* opts, const int32_t* osid, int64_t n,
                               const uint64_t* nkeys, const uint32_t* nperm, const float* npts, int64_t nn, int32_t f,
                               float* mpts, int32_t* msid, hipStream_t s);
hipError_t measure_cells(const void* pts, int64_t n, int32_t f, int32_t dtype, float* width, float* origin,
                         int64_t* splits, bool* nonfinite, hipStream_t s);
hipError_t launch_dense_cell_start(const uint64_t* sorted_keys, int64_t n, int64_t box_cells,
                                   uint32_t* cell_start, hipStream_t s);

hipError_t launch_index_cells(const IndexView& iv, int32_t* out_ids, int64_t* out_counts, int32_t* out_point_cell,
                              hipStream_t s);
// stats[0] += non-empty cells, stats[1] = max points in one cell, over `ncells` offsets.
hipError_t launch_cell_stats(const uint32_t* cell_start, int64_t ncells, int64_t* d_stats, hipStream_t s);
hipError_t exclusive_scan_u32(const uint32_t* in, uint32_t* out, int64_t n, void* temp, hipStream_t s);
size_t exclusive_scan_temp_bytes(int64_t n);
hipError_t launch_morton_keys(const void* pts, int64_t n, int32_t dtype, const IndexView& iv, int nbits, int word,
                              const uint32_t* order, uint64_t* keys, uint32_t* vals, hipStream_t s);
hipError_t launch_cell_heads_ids(const IndexView& iv, int64_t n, uint32_t* heads, hipStream_t s);
hipError_t launch_cell_heads(const uint64_t* sorted_keys, int64_t n, uint32_t* heads, hipStream_t s);
hipError_t launch_cell_list(const uint32_t* heads, const uint32_t* rank, int64_t n, const IndexView& iv,
                            uint32_t* cell_start, int32_t* cell_coord, hipStream_t s);
hipError_t launch_tree_level(const int32_t* child_lo, const int32_t* child_hi, int64_t nchild, int32_t f,
                             int32_t* node_lo, int32_t* node_hi, int64_t nnode, hipStream_t s);

// Per-call query inputs and outputs (device pointers).
struct QueryIO {
    const float* queries;
    int64_t* out_idx;
    double* out_d2;
    void* out_pred;
    int32_t* out_stop_layer;
    int64_t* out_cands;
    int64_t* out_probes;
    int64_t* out_rerank;
    int32_t k;
    uint32_t flags;
    int32_t ring_step;   // EXACT rule: layers per step of the walk (<= 1: one)
    int32_t pad;
    uint32_t* faults;    // the device's walk fault word (GHN_WALK_SHORT), or NULL
};

struct PredictArgs {
    IndexView ix;
    QueryIO io;
    int64_t m;
    int32_t stop;
    const uint32_t* order;  // optional processing order of the queries (NULL = 0..m-1)
};
hipError_t launch_predict_dense(const PredictArgs& a, hipStream_t s);
hipError_t launch_predict_tree(const PredictArgs& a, hipStream_t s);
// One item of a batch over many indexes: global query positions [first, first + m).
struct BatchItem {
    const IndexView* ix;  // device copy of the item's index view
    QueryIO io;
    int64_t first;
    int64_t m;
    // grouped (bf16) batches: the item's query sort key is (item << kb) | its Morton code
    // moved by kshift bits (left if >= 0); groups split where the key >> gshift changes;
    // trunc: the key lost code bits, so the PAPER rule also compares exact cell ids
    int32_t kshift;
    int32_t gshift;
    int32_t trunc;
    int32_t pad;
};

// The item owning global query position w: the last item whose first position is <= w
// (items are in order of first positions; empty items share their successor's).
__device__ __forceinline__ int batch_item_of(const BatchItem* items, int n_items, int64_t w) {
    int lo = 0, hi = n_items;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (items[mid].first <= w) lo = mid;
        else hi = mid;
    }
    return lo;
}

// order: optional walk order of the global positions (a permutation); counter: 8
// work counters (one per XCD range); blocks_override > 0 fixes the grid size.
hipError_t launch_predict_batched(const BatchItem* items, int n_items, int64_t total, int f, int stop, bool any_tree,
                                  bool any_dense, const uint32_t* order, int blocks_override, uint64_t* counter,
                                  hipStream_t s);
// The batch's queries sorted by (item, Morton code of the central cell): *order
// receives the sorted global positions, in `ws` (group_ws_bytes(total) bytes).
hipError_t batch_query_order(const BatchItem* items, int n_items, int64_t total, int kb, int key_bits, void* ws,
                             hipStream_t s, const uint32_t** order);
// Grouped (bf16 screen) walk of a whole batch in one persistent launch, after one sort
// of all its queries by (item, cell) and the grouping; `ws` holds group_ws_bytes(total).
// kb: key bits below the item index; kmax: largest k.
hipError_t run_grouped_batched(const BatchItem* items, int n_items, int64_t total, int f, int kmax, int stop, int kb,
                               int key_bits, int gsize, int tile_w, void* ws, hipStream_t s);

// Per-dimension range of the finite coordinates of n points (synchronises s).
hipError_t coord_range(const void* pts, int64_t n, int32_t f, int32_t dtype, float* lo, float* hi, hipStream_t s);

// Grouped walk with the bf16 matrix-core screen: sort, group and walk the queries.
size_t group_ws_bytes(int64_t m);
hipError_t launch_screen_error(const IndexView& ix, const float* qs, int64_t m, uint32_t nsamp, float* out_abs,
                               float* out_rel, hipStream_t s);
// gsize: most queries per group (1..16); tile_w: candidates per screened tile (32 or 64)
hipError_t run_grouped(const PredictArgs& pa, int group_levels, int gsize, int tile_w, void* ws, hipStream_t s, int* morton_bits,
                       hipEvent_t ev_begin, hipEvent_t ev_end, bool brute);
// Spatial sort key of every query (Morton code of its box-clamped central cell).
hipError_t launch_query_keys(const float* qs, int64_t m, const IndexView& ix, int keep_bits, uint64_t* keys,
                             uint32_t* vals, hipStream_t s);
constexpr int QUERY_KEY_BITS = 16;   // two 8-bit radix passes
constexpr int64_t SORT_MIN_QUERIES = 4096;  // smaller batches run in input order

}  // namespace ghn
