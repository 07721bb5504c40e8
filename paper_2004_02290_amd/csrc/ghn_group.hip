// Grouped exploration with bf16 matrix-core screening (Section III-B with the
// distance step batched over queries).
//
// Queries are sorted by the Morton code of their central cell and cut into
// groups of at most 16 that share a cell (or, under the EXACT rule, a block of
// 2^s cells per dimension).  One wave walks one group: layer l of the group is
// the set of occupied cells at Chebyshev distance l from the group's box of
// central cells, found with the cell tree (or, for dense-table indexes up to 4
// dimensions, as rows of the table).  Every query's own layers 0..l lie
// inside the group's layers 0..l, so each query's stop rule is applied exactly
// as in the per-query walk.  Under the PAPER rule the group is a single cell,
// so group layers are the queries' layers.
//
// The distance step is a matrix-core contraction.  At build time every point
// gets a screen record: x' = fl32(x - c0) (c0 = centre of the occupied box)
// split into bf16 parts h = bf16(x'), l = bf16(x' - h), padded to sp = 8, 16 or
// 32 dimensions, plus xn = |x'|^2.  v_mfma_f32_16x16x32_bf16 then forms, for 16
// queries x 16 candidates at a time, acc = (1 - R) xn - A - 2 q'.x' with
// K = [qh, qh, ql] . [xh, xl, xh] (the lo x lo term is dropped): each lane loads
// its 16-byte slice of a record straight into the B operand, the query parts
// sit in the A operand for the whole walk, and the norms enter as the
// accumulator's initial value.  A pair is admitted when acc <= thr - (1 - R) qn,
// i.e. when s - R (qn + xn) - A <= thr with s = qn + xn - 2 q'.x' and thr the
// query's FP32 admission threshold above its k-th FP64 distance.
//
// Error bound, with N = |q'|^2 + |x'|^2 and u = 2^-8 (bf16 round to nearest):
// each split leaves |x' - h - l| <= u^2 |x'|, so the residues and the dropped
// lo x lo term move q'.x' by at most 3 u^2 sum |q'_j x'_j| <= 1.5 u^2 N, i.e. s
// by 3 u^2 N = 2^-14.4 N; the FP32 accumulation of at most 6 sp / 2 + 1 terms
// whose magnitudes sum to at most 2N adds at most 97 * 2^-23 N < 2^-15.4 N; the
// centring (one FP32 rounding per coordinate) and the FP32 norms add below
// 2^-20 N.  So |s - d| < 2^-13.8 N, and R = 2^-12 (A = 2^-100 for underflow)
// admits every pair whose FP64 distance can still enter the buffer; admitted
// pairs are re-scored in FP64, so the selected set is the exact FP64 one.
//
// In the result tile, lane l holds column l % 16 and rows 4 (l / 16) + i: the
// 16-lane DPP row g holds queries 4g .. 4g+3.  Each query's size-k buffer lives
// in registers of its row (entry e = 16 j + t in register j of lane t), so the
// four rows insert in parallel with row-local DPP shifts.
#include <cstring>
#include <type_traits>

#include "ghn_walk.h"

namespace ghn {
namespace {

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;
typedef __attribute__((__vector_size__(4 * sizeof(float)))) float floatx4;

constexpr int GT = 256;          // threads per block
constexpr int GWPB = GT / WAVE;  // groups (waves) per block
constexpr int GQ = 16;           // queries per group
constexpr int STACK_CAP = TREE_LEVELS_MAX * WAVE;
constexpr int QFLUSH = WAVE;               // queued pairs that trigger the exact check
constexpr int QCAP = GQ * WAVE + QFLUSH;   // one tile can admit every pair
constexpr float SCREEN_REL = 0x1p-12f;   // admission margin, relative to |q'|^2 + |x'|^2
constexpr float SCREEN_ABS = 0x1p-100f;  // absolute margin (FP32 underflow)

// ---- row (16-lane) DPP helpers -------------------------------------------------------------
__device__ __forceinline__ int row_ror1(int v) { return __builtin_amdgcn_update_dpp(v, v, 0x121, 0xf, 0xf, false); }
__device__ __forceinline__ double row_ror1_f64(double v) {
    const int64_t b = __double_as_longlong(v);
    const int lo = row_ror1((int)(uint32_t)b), hi = row_ror1((int)(uint32_t)((uint64_t)b >> 32));
    return __longlong_as_double((int64_t)(((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo));
}
template <int N>
__device__ __forceinline__ int row_bcast_n(int v) { return __builtin_amdgcn_update_dpp(v, v, 0x150 + N, 0xf, 0xf, false); }
// Value of lane n (uniform n in 0..15) of each 16-lane row, to every lane of the row.
__device__ __forceinline__ int row_bcast(int v, int n) {
    switch (n) {
        case 0: return row_bcast_n<0>(v);   case 1: return row_bcast_n<1>(v);
        case 2: return row_bcast_n<2>(v);   case 3: return row_bcast_n<3>(v);
        case 4: return row_bcast_n<4>(v);   case 5: return row_bcast_n<5>(v);
        case 6: return row_bcast_n<6>(v);   case 7: return row_bcast_n<7>(v);
        case 8: return row_bcast_n<8>(v);   case 9: return row_bcast_n<9>(v);
        case 10: return row_bcast_n<10>(v); case 11: return row_bcast_n<11>(v);
        case 12: return row_bcast_n<12>(v); case 13: return row_bcast_n<13>(v);
        case 14: return row_bcast_n<14>(v); default: return row_bcast_n<15>(v);
    }
}
__device__ __forceinline__ double row_bcast_f64(double v, int n) {
    const int64_t b = __double_as_longlong(v);
    const int lo = row_bcast((int)(uint32_t)b, n), hi = row_bcast((int)(uint32_t)((uint64_t)b >> 32), n);
    return __longlong_as_double((int64_t)(((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo));
}

__device__ __forceinline__ float admit_group(double tau) {
    if (!(tau < 1.0e300)) return __int_as_float(0x7f800000);
    return f32_round_up(tau * (1.0 + 0x1p-30)) + 0x1p-125f;
}

// Sort key and flags of a query: the top 64 bits of the Morton code of its central
// cell clamped to the occupied box; flag bit 0 = a coordinate is not finite, bit 1 =
// the central cell lies outside the box (such queries walk alone).
__device__ __forceinline__ uint64_t query_group_code(const IndexView& ix, const float* q, uint32_t& fl) {
    const int f = ix.f;
    int bits[F_MAX];
    int maxb = 0, total = 0;
    for (int j = 0; j < f; ++j) {
        const uint32_t span = (uint32_t)(ix.cmax[j] - ix.cmin[j]);
        bits[j] = span ? 32 - __clz(span) : 0;
        maxb = max(maxb, bits[j]);
        total += bits[j];
    }
    const int drop = total > 64 ? total - 64 : 0;
    uint32_t u[F_MAX];
    fl = 0;
    for (int j = 0; j < f; ++j) {
        const float x = q[j];
        int64_t c = 0;
        if (isfinite(x)) c = exact_floor_div(__dadd_rn((double)x, -(double)ix.o[j]), (double)ix.a[j]);
        else fl |= 1u;
        if (c < ix.cmin[j] || c > ix.cmax[j]) fl |= 2u;
        c = min(max(c, (int64_t)ix.cmin[j]), (int64_t)ix.cmax[j]);
        u[j] = (uint32_t)(c - ix.cmin[j]);
    }
    uint64_t code = 0;
    int pos = total;
    for (int b = maxb - 1; b >= 0; --b)
        for (int j = 0; j < f; ++j)
            if (b < bits[j]) {
                --pos;
                if (pos >= drop) code = (code << 1) | ((u[j] >> b) & 1u);
            }
    return code;
}

__global__ __launch_bounds__(256) void k_group_keys(const float* __restrict__ qs, int64_t m, IndexView ix,
                                                    uint64_t* __restrict__ keys, uint32_t* __restrict__ vals,
                                                    uint32_t* __restrict__ qflags) {
    for (int64_t i = blockIdx.x * 256ll + threadIdx.x; i < m; i += (int64_t)gridDim.x * 256) {
        uint32_t fl;
        keys[i] = query_group_code(ix, qs + i * ix.f, fl);
        vals[i] = (uint32_t)i;
        qflags[i] = fl;
    }
}

// The same over all queries of a batch (global positions): the item's index above
// kb key bits, its code moved by the item's kshift below.
__global__ __launch_bounds__(256) void k_batch_group_keys(const BatchItem* __restrict__ items, int n_items,
                                                          int64_t total, int kb, uint64_t* __restrict__ keys,
                                                          uint32_t* __restrict__ vals, uint32_t* __restrict__ qflags) {
    for (int64_t w = blockIdx.x * 256ll + threadIdx.x; w < total; w += (int64_t)gridDim.x * 256) {
        const int it = batch_item_of(items, n_items, w);
        const BatchItem& B = items[it];
        const IndexView& ix = *B.ix;
        uint32_t fl;
        const uint64_t code = query_group_code(ix, B.io.queries + (w - B.first) * ix.f, fl);
        const uint64_t kc = B.kshift >= 0 ? code << B.kshift : code >> (-B.kshift);
        keys[w] = kb < 64 ? ((uint64_t)it << kb) | kc : kc;
        vals[w] = (uint32_t)w;
        qflags[w] = fl;
    }
}

__global__ void k_zero_u32(uint32_t* p, int n) {
    if ((int)threadIdx.x < n) p[threadIdx.x] = 0u;
}

// Cut the sorted queries into groups: a group starts where the (shifted) key
// changes, at a query that walks alone, or every gsize positions (gsize <= GQ: the
// matrix tile's 16 query rows, of which smaller groups leave some empty).
// Under the PAPER rule a group must share one central cell; when the sort key is a
// truncated code (more than 64 bits), equal keys do not imply equal cells, so the
// cell ids are compared too (`exact`).
__device__ __forceinline__ bool same_cell(const float* qs, const IndexView& ix, uint32_t a, uint32_t b) {
    for (int j = 0; j < ix.f; ++j) {
        const double o = ix.o[j], w = ix.a[j];
        if (exact_floor_div(__dadd_rn((double)qs[(int64_t)a * ix.f + j], -o), w) !=
            exact_floor_div(__dadd_rn((double)qs[(int64_t)b * ix.f + j], -o), w))
            return false;
    }
    return true;
}

__device__ __forceinline__ bool group_start(const uint64_t* keys, const uint32_t* vals, const uint32_t* qflags,
                                            int64_t i, int shift, const float* qs, const IndexView& ix, bool exact,
                                            int gsize) {
    if (i == 0 || (i % gsize) == 0) return true;
    if (qflags[vals[i]] || qflags[vals[i - 1]]) return true;
    if (shift < 64 && (keys[i] >> shift) != (keys[i - 1] >> shift)) return true;
    return exact && !same_cell(qs, ix, vals[i], vals[i - 1]);
}

__global__ __launch_bounds__(256) void k_form_groups(const uint64_t* __restrict__ keys, const uint32_t* __restrict__ vals,
                                                     const uint32_t* __restrict__ qflags, int64_t m, int shift,
                                                     const float* __restrict__ qs, IndexView ix, int exact, int gsize,
                                                     uint2* __restrict__ groups, uint32_t* ngroups) {
    for (int64_t i = blockIdx.x * 256ll + threadIdx.x; i < m; i += (int64_t)gridDim.x * 256) {
        if (!group_start(keys, vals, qflags, i, shift, qs, ix, exact, gsize)) continue;
        int64_t j = i + 1;
        while (j < m && !group_start(keys, vals, qflags, j, shift, qs, ix, exact, gsize)) ++j;
        const uint32_t g = atomicAdd(ngroups, 1u);
        groups[g] = make_uint2((uint32_t)i, (uint32_t)(j - i));
    }
}

// Group starts of a batch: also where the item changes; the key shift and the PAPER
// rule's exact cell check are the item's.
__device__ __forceinline__ bool batch_group_start(const uint64_t* keys, const uint32_t* vals, const uint32_t* qflags,
                                                  int64_t i, const BatchItem* items, int kb, int gsize) {
    if (i == 0 || (i % gsize) == 0) return true;
    if (qflags[vals[i]] || qflags[vals[i - 1]]) return true;
    const int it = kb < 64 ? (int)(keys[i] >> kb) : 0;
    if (kb < 64 && it != (int)(keys[i - 1] >> kb)) return true;
    const BatchItem& B = items[it];
    if (B.gshift < 64 && (keys[i] >> B.gshift) != (keys[i - 1] >> B.gshift)) return true;
    return B.trunc && !same_cell(B.io.queries, *B.ix, (uint32_t)(vals[i] - B.first), (uint32_t)(vals[i - 1] - B.first));
}

__global__ __launch_bounds__(256) void k_batch_form_groups(const uint64_t* __restrict__ keys,
                                                           const uint32_t* __restrict__ vals,
                                                           const uint32_t* __restrict__ qflags, int64_t total,
                                                           const BatchItem* __restrict__ items, int kb, int gsize,
                                                           uint2* __restrict__ groups, uint32_t* ngroups) {
    for (int64_t i = blockIdx.x * 256ll + threadIdx.x; i < total; i += (int64_t)gridDim.x * 256) {
        if (!batch_group_start(keys, vals, qflags, i, items, kb, gsize)) continue;
        int64_t j = i + 1;
        while (j < total && !batch_group_start(keys, vals, qflags, j, items, kb, gsize)) ++j;
        const uint32_t g = atomicAdd(ngroups, 1u);
        groups[g] = make_uint2((uint32_t)i, (uint32_t)(j - i));
    }
}

struct GroupArgs {
    int32_t brute;          // exhaustive KNN: no grid walk, every point screened
    PredictArgs p;          // p.order = queries in sorted order (global positions in a batch)
    const uint2* groups;
    const uint32_t* counters;  // [0] = number of groups
    uint32_t* work;            // next group to take
    const BatchItem* items;    // batch: the items (device), in order of first positions
    int32_t n_items;
    int32_t tile_w;            // candidates per screened tile: 32 or 64 (2 or 4 column blocks)
};

template <int FT>
struct alignas(16) GroupLds {
    static constexpr int FS = FT > 0 ? FT : F_MAX;
    float q[GQ][FS];
    int32_t qc[GQ][FS];
    uint32_t run_begin[WAVE + 1];
    uint32_t run_pre[WAVE + 1];
    uint64_t stack[STACK_CAP];
    int32_t lab[4][K_MAX + 1];  // + 1: the four rows' entries e fall in different banks
    int32_t med[4][2];
    int32_t glo[FS], ghi[FS];
    float qlo[FS], qhi[FS];
    double ad[FS], od[FS];  // cell width and origin (FP64), read inside the walk
    double qd[GQ][FS | 1];  // the queries in FP64 (exact), for the re-rank; an odd row length
                            // puts the rows the re-rank lanes read at once in different banks
    int64_t shift;          // true layer - walk layer (0 unless the query is far outside the box)
    float tq[GQ];           // per query: FP32 threshold >= its k-th distance (+inf while the
                            // buffer is not full), -1 once done or when invalid
    uint32_t qp[QCAP];      // queue of admitted pairs: point position in cell order
    uint8_t qr[QCAP];       //                          and query row of the group
};

// Operand layout of the screen for padded dimension SP (K = [qh, qh, ql] . [xh, xl, xh]
// cut into blocks of 32).  Lane group g = lane / 16 supplies 8 consecutive K values of
// each block: record chunk (8 bf16 = 16 bytes) b_chunk() of its candidate, or zeros
// (-1), and the query part a_part() (0 = hi, 1 = lo, -1 = zeros) of dimensions
// a_dim() .. a_dim() + 7.
template <int SP> struct Screen;
template <> struct Screen<8> {
    static constexpr int NKB = 1, NCH = 1;
    __device__ static int chunk(int c, int g) { return g == 1 ? 1 : 0; }
    __device__ static int b_src(int kb, int g) { return g == 3 ? -1 : 0; }
    __device__ static int a_part(int kb, int g) { return g == 3 ? -1 : (g == 2 ? 1 : 0); }
    __device__ static int a_dim(int kb, int g) { return 0; }
};
template <> struct Screen<16> {
    static constexpr int NKB = 2, NCH = 1;
    __device__ static int chunk(int c, int g) { return g; }
    __device__ static int b_src(int kb, int g) { return kb == 0 ? 0 : (g < 2 ? 0 : -1); }
    __device__ static int a_part(int kb, int g) { return kb == 0 ? 0 : (g < 2 ? 1 : -1); }
    __device__ static int a_dim(int kb, int g) { return kb == 0 ? 8 * (g & 1) : 8 * g; }
};
template <> struct Screen<32> {
    static constexpr int NKB = 3, NCH = 2;
    __device__ static int chunk(int c, int g) { return c == 0 ? g : 4 + g; }
    __device__ static int b_src(int kb, int g) { return kb == 1 ? 1 : 0; }
    __device__ static int a_part(int kb, int g) { return kb == 2 ? 1 : 0; }
    __device__ static int a_dim(int kb, int g) { return 8 * g; }
};

// Integer key ordering float bit patterns as IEEE total order.
__device__ __forceinline__ uint32_t total_key(int32_t bits) {
    const uint32_t u = (uint32_t)bits;
    return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}

// FP32 values at or below / at or above an FP64 value, one extra ulp outward.
__device__ __forceinline__ float f32_below(double x) {
    float r = (float)x;
    if ((double)r > x) r = nextafterf(r, -INFINITY);
    return nextafterf(r, -INFINITY);
}
__device__ __forceinline__ float f32_above(double x) {
    float r = (float)x;
    if ((double)r < x) r = nextafterf(r, INFINITY);
    return nextafterf(r, INFINITY);
}

__device__ __forceinline__ double shfl_f64(double v, int src) {
    const int64_t b = __double_as_longlong(v);
    const int lo = __shfl((int)(uint32_t)b, src, WAVE), hi = __shfl((int)(uint32_t)((uint64_t)b >> 32), src, WAVE);
    return __longlong_as_double((int64_t)(((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo));
}

// Screen of column block cb of a tile: lane (g, t) fetches the record slices of
// candidate 16 cb + t (its run position came from lane 16 cb + t) and the result is
// acc[i] = (1 - R) xn - A - 2 q'.x' for query 4 g + i of the group.
template <int FT, int SP>
__device__ __forceinline__ floatx4 screen_block(const IndexView& ix, const bf16x8* afr, uint32_t pidx, float xinit,
                                                uint32_t base, uint32_t npts, int cb, int g, int t, uint32_t& pc) {
    using SC = Screen<SP>;
    pc = (uint32_t)__shfl((int)pidx, 16 * cb + t, WAVE);
    const float xi = __shfl(xinit, 16 * cb + t, WAVE);
    const bool vc = base + 16 * cb + t < npts;
    bf16x8 ld[SC::NCH];
#pragma unroll
    for (int c = 0; c < SC::NCH; ++c) {
#pragma unroll
        for (int e = 0; e < 8; ++e) ld[c][e] = (__bf16)0.0f;
        if (vc && (SC::NCH > 1 || SC::b_src(0, g) >= 0))
            ld[c] = *(const bf16x8*)(ix.srec + (size_t)pc * (2 * SP) + 8 * SC::chunk(c, g));
    }
    floatx4 acc = {xi, xi, xi, xi};
#pragma unroll
    for (int kb = 0; kb < SC::NKB; ++kb) {
        const int src = SC::b_src(kb, g);
        bf16x8 bb = ld[(SC::NCH > 1 && src > 0) ? SC::NCH - 1 : 0];
        if (src < 0) {
#pragma unroll
            for (int e = 0; e < 8; ++e) bb[e] = (__bf16)0.0f;
        }
        acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(afr[kb], bb, acc, 0, 0, 0);
    }
    return acc;
}

// Screen of the first NB column blocks of a tile, in two halves for a software-pipelined
// walk: the record loads (issued, not waited for), then the matrix instructions, which
// start each column's accumulator at its candidate's initial value.  The loads are not
// guarded: a lane without a candidate has position 0 (a record of the index) and a NaN
// initial value, so its column is never admitted whatever the loaded values are.
template <int SP, int NB>
__device__ __forceinline__ void tile_load(const IndexView& ix, uint32_t pidx, int g, int t,
                                          bf16x8 (&ld)[NB][Screen<SP>::NCH]) {
    using SC = Screen<SP>;
#pragma unroll
    for (int cb = 0; cb < NB; ++cb) {
        const uint32_t pc = (uint32_t)__shfl((int)pidx, 16 * cb + t, WAVE);
#pragma unroll
        for (int c = 0; c < SC::NCH; ++c)
            ld[cb][c] = *(const bf16x8*)(ix.srec + (size_t)pc * (2 * SP) + 8 * SC::chunk(c, g));
    }
}

template <int SP, int NB>
__device__ __forceinline__ void tile_mfma(const bf16x8* afr, const bf16x8 (&ld)[NB][Screen<SP>::NCH], float xinit,
                                          int g, int t, floatx4 (&acc)[NB]) {
    using SC = Screen<SP>;
#pragma unroll
    for (int cb = 0; cb < NB; ++cb) {
        const float xi = __shfl(xinit, 16 * cb + t, WAVE);
        acc[cb] = floatx4{xi, xi, xi, xi};
#pragma unroll
        for (int kb = 0; kb < SC::NKB; ++kb) {
            const int src = SC::b_src(kb, g);
            bf16x8 bb = ld[cb][(SC::NCH > 1 && src > 0) ? SC::NCH - 1 : 0];
            if (src < 0) {
#pragma unroll
                for (int e = 0; e < 8; ++e) bb[e] = (__bf16)0.0f;
            }
            acc[cb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(afr[kb], bb, acc[cb], 0, 0, 0);
        }
    }
}

// BATCH: the groups come from many indexes (a batch); each group belongs to one item,
// found from its first query's global position, and is walked with that item's index,
// queries, k and outputs.  KR covers the largest k of the batch.
template <int FT, int SP, int KR, bool BATCH>
__global__ __launch_bounds__(GT, 2) void k_predict_group(GroupArgs G) {
    __shared__ GroupLds<FT> lds_all[GWPB];
    constexpr int FS = GroupLds<FT>::FS;
    using SC = Screen<SP>;
    constexpr int NKB = SC::NKB;
    constexpr int NCH = SC::NCH;
    const int lane = lane_id();
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x / WAVE);
    GroupLds<FT>& S = lds_all[wv];
    const int g = lane >> 4, t = lane & 15;
    const uint32_t ngroups = G.counters[0];
    const float inf = __int_as_float(0x7f800000);

    for (;;) {
        uint32_t gid = 0;
        if (lane == 0) gid = atomicAdd(G.work, 1u);
        gid = __builtin_amdgcn_readfirstlane(gid);
        if (gid >= ngroups) break;
        const uint2 gd = G.groups[gid];
        const int cnt = (int)gd.y;
        // the group's index, queries and outputs; query positions are global in a batch
        const BatchItem* item = nullptr;
        if constexpr (BATCH) item = &G.items[batch_item_of(G.items, G.n_items, (int64_t)G.p.order[gd.x])];
        const IndexView& ix = BATCH ? *item->ix : G.p.ix;
        const QueryIO& io = BATCH ? item->io : G.p.io;
        const int64_t qbase = BATCH ? item->first : 0;
        const int f = FT > 0 ? FT : ix.f;
        const int k = io.k;
        const bool prune = !(io.flags & GHN_FLAG_NO_PRUNE);

        // ---- group set-up: lane r < cnt loads query r
        bool fin = false;
        {
            const bool act = lane < cnt;
            const int64_t qi = act ? (int64_t)G.p.order[gd.x + lane] - qbase : 0;
            fin = act;
            int32_t cc[FS];
            for (int j = 0; j < f; ++j) {
                const float x = act ? io.queries[qi * f + j] : 0.0f;
                fin = fin && isfinite(x);
                cc[j] = 0;
                if (act) { S.q[lane][j] = x; S.qd[lane][j] = (double)x; }
            }
            for (int j = 0; j < f; ++j) {
                int64_t c = 0;
                if (fin) {
                    const double v = __dadd_rn((double)S.q[lane][j], -(double)ix.o[j]);
                    c = exact_floor_div(v, (double)ix.a[j]);
                    c = max(c, (int64_t)ix.cmin[j] - CLAMP);
                    c = min(c, (int64_t)ix.cmax[j] + CLAMP);
                }
                cc[j] = (int32_t)c;
                if (act) S.qc[lane][j] = cc[j];
            }
            // central cells in the walk frame (walk_frame in ghn_internal.h; the EXACT
            // bound below is then the frame's, see stop_after_layer): the clamped ids
            // are the frame unless a query lies CLAMP or more cells outside the box.
            // Such a query walks alone (k_form_groups), and its ids are redone here one
            // dimension per lane.
            int32_t far0 = 0;
            if (lane == 0 && fin)
                for (int j = 0; j < f; ++j) far0 = max(far0, max(ix.cmin[j] - cc[j], cc[j] - ix.cmax[j]));
            far0 = readlane_i32(far0, 0);
            int64_t gshift = 0;
            if (cnt == 1 && far0 == (int32_t)CLAMP) {
                const int64_t q0 = (int64_t)G.p.order[gd.x] - qbase;
                gshift = far_shift(ix, io.queries, q0, f);
                const int32_t cl = far_frame_id(ix, io.queries, q0, f);
                if (lane < f) S.qc[0][lane] = cl;
                for (int j = 0; j < f; ++j) {
                    const int32_t c0 = readlane_i32(cl, j);
                    if (lane == 0) cc[j] = c0;
                }
            }
            if (lane == 0) S.shift = gshift;
            // group box of central cells and box of query coordinates (finite queries)
            for (int j = 0; j < f; ++j) {
                int32_t lo = fin ? cc[j] : INT32_MAX, hi = fin ? cc[j] : INT32_MIN;
                float ql = fin ? S.q[lane][j] : inf;
                float qh = fin ? S.q[lane][j] : -inf;
                for (int d = 1; d < WAVE; d <<= 1) {
                    lo = min(lo, __shfl_xor(lo, d, WAVE));
                    hi = max(hi, __shfl_xor(hi, d, WAVE));
                    ql = fminf(ql, __shfl_xor(ql, d, WAVE));
                    qh = fmaxf(qh, __shfl_xor(qh, d, WAVE));
                }
                if (lane == 0) {
                    S.glo[j] = lo;
                    S.ghi[j] = hi;
                    S.qlo[j] = ql;
                    S.qhi[j] = qh;
                    S.ad[j] = (double)ix.a[j];
                    S.od[j] = (double)ix.o[j];
                }
            }
        }
        const uint64_t fin_mask = ballot(fin);
        if (lane < GQ) S.tq[lane] = fin ? inf : -1.0f;
        wave_lds_sync();

        // ---- per-slot state (slot i of row g = query 4g + i)
        double bd[4][KR];
        int bi[4][KR];
        double tau[4];
        int taui[4];
        float thr[4], qn[4], bnd[4];
        bool upd[4], done[4];
        int32_t stopl[4];
        int32_t cands[4];
        int32_t rer[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int r = 4 * g + i;
            const bool live = r < cnt && ((fin_mask >> r) & 1);
            done[i] = !live;
            upd[i] = false;
            stopl[i] = -1;
            cands[i] = 0;
            rer[i] = 0;
            tau[i] = __longlong_as_double(0x7ff0000000000000LL);
            taui[i] = INT32_MAX;
            thr[i] = live ? inf : -inf;
#pragma unroll
            for (int j = 0; j < KR; ++j) { bd[i][j] = tau[i]; bi[i][j] = INT32_MAX; }
            float s = 0.0f;
            if (live)
                for (int j = 0; j < f; ++j) {
                    const float d = S.q[r][j] - ix.c0[j];
                    s = __builtin_fmaf(d, d, s);
                }
            qn[i] = s;
            bnd[i] = thr[i];
        }
        // A operand of the 16 queries (row lane % 16): -2 x their bf16 parts
        bf16x8 afr[NKB];
        {
            const int r = lane & 15;
            const bool rlive = r < cnt && ((fin_mask >> r) & 1);
#pragma unroll
            for (int kb = 0; kb < NKB; ++kb) {
                const int part = SC::a_part(kb, g), d0 = SC::a_dim(kb, g);
#pragma unroll
                for (int e = 0; e < 8; ++e) {
                    const int j = d0 + e;
                    float v = 0.0f;
                    if (part >= 0 && rlive && j < f) {
                        const float qp = S.q[r][j] - ix.c0[j];
                        const float hi = (float)(__bf16)qp;
                        v = part == 1 ? (float)(__bf16)(qp - hi) : hi;
                    }
                    afr[kb][e] = (__bf16)(-2.0f * v);
                }
            }
        }
        int32_t l0 = 0, lcover = 0;
        for (int j = 0; j < f; ++j) {
            const int32_t lo = S.glo[j], hi = S.ghi[j];
            l0 = max(l0, max(ix.cmin[j] - hi, lo - ix.cmax[j]));
            lcover = max(lcover, max(hi - ix.cmin[j], ix.cmax[j] - lo));
        }
        int32_t probes = 0;
        int32_t l = l0;
        const bool any_live = (fin_mask & ((cnt >= 64 ? ~0ull : ((1ull << cnt) - 1)))) != 0;

        // Screen, check and insert the points of the run list in LDS (npts points in
        // nrun runs, prefix positions with a sentinel at nrun).
        // Exact FP64 check and insertion of the queued pairs, 64 at a time: each lane
        // scores one pair, then each 16-lane row inserts its query's pairs one by one
        // (the four rows in parallel, one slot at a time).  Deferring the check is
        // exact: thresholds only lag (a superset is admitted), and every queue is
        // flushed before a layer's stop test, so the buffer after layer l and whether
        // layer l changed it do not depend on when pairs are inserted.
        int qcount = 0;
        auto flush = [&]() __attribute__((always_inline)) {
            wave_lds_sync();
            for (int qb = 0; qb < qcount; qb += WAVE) {
                const int e = qb + lane;
                int r = -1;
                double cd = __longlong_as_double(0x7ff0000000000000LL);
                int ci = INT32_MAX;
                if (e < qcount) {
                    r = S.qr[e];
                    const uint32_t pc = S.qp[e];
                    float xv[FS];
                    load_point<FT>(ix.spts + (size_t)pc * f, xv, f);
                    const double* qd = S.qd[r];
                    cd = 0.0;
#pragma unroll
                    for (int j = 0; j < FS; ++j) {
                        if (FT == 0 && j >= f) break;
                        const double d = __dadd_rn(qd[j], -(double)xv[j]);
                        cd = __dadd_rn(cd, __dmul_rn(d, d));
                    }
                    ci = ix.sid[pc];
                }
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const uint64_t m0 = ballot(r == i), m1 = ballot(r == 4 + i), m2 = ballot(r == 8 + i),
                                   m3 = ballot(r == 12 + i);
                    uint64_t mrow = g == 0 ? m0 : (g == 1 ? m1 : (g == 2 ? m2 : m3));
                    while (ballot(mrow != 0)) {
                        bool have = false;
                        int src = lane;
                        if (mrow) {
                            have = true;
                            src = __ffsll((unsigned long long)mrow) - 1;
                            mrow &= mrow - 1;
                        }
                        const double cdb = shfl_f64(cd, src);
                        const int cib = __shfl(ci, src, WAVE);
                        if (have && (cdb < tau[i] || (cdb == tau[i] && cib < taui[i]))) {
                            // entries larger than the candidate move up one place
                            const uint64_t cbits = (uint64_t)__double_as_longlong(cdb);
                            int ngt = 0;
#pragma unroll
                            for (int j = 0; j < KR; ++j) {
                                const int ee = 16 * j + t;
                                const uint64_t bb = (uint64_t)__double_as_longlong(bd[i][j]);
                                const bool gt = ee < k && (bb > cbits || (bb == cbits && bi[i][j] > cib));
                                ngt += __popc((uint32_t)(ballot(gt) >> (16 * g)) & 0xffffu);
                            }
                            const int pos = k - ngt;
                            double rd[KR];
                            int ri[KR];
#pragma unroll
                            for (int j = 0; j < KR; ++j) { rd[j] = row_ror1_f64(bd[i][j]); ri[j] = row_ror1(bi[i][j]); }
#pragma unroll
                            for (int j = KR - 1; j >= 0; --j) {
                                const int ee = 16 * j + t;
                                double nd = rd[j];
                                int ni = ri[j];
                                if (t == 0) {
                                    nd = j > 0 ? rd[j > 0 ? j - 1 : 0] : bd[i][j];
                                    ni = j > 0 ? ri[j > 0 ? j - 1 : 0] : bi[i][j];
                                }
                                if (ee < k && ee >= pos) {
                                    bd[i][j] = ee == pos ? cdb : nd;
                                    bi[i][j] = ee == pos ? cib : ni;
                                }
                            }
                            upd[i] = true;
                            const int jl = (k - 1) >> 4, tl = (k - 1) & 15;
                            double kd = bd[i][0];
                            int ki = bi[i][0];
#pragma unroll
                            for (int j = 1; j < KR; ++j) if (j == jl) { kd = bd[i][j]; ki = bi[i][j]; }
                            tau[i] = row_bcast_f64(kd, tl);
                            taui[i] = row_bcast(ki, tl);
                            thr[i] = taui[i] == INT32_MAX ? inf : admit_group(tau[i]);
                            bnd[i] = thr[i] == inf ? inf : thr[i] - (1.0f - SCREEN_REL) * qn[i];
                            if (t == 0) S.tq[4 * g + i] = thr[i];
                        }
                    }
                }
            }
            qcount = 0;
            wave_lds_sync();
        };

        // Screen the points of the run list in LDS (npts points in nrun runs, prefix
        // positions with a sentinel at nrun) and queue the admitted pairs; `last`
        // flushes the queue at the end (with npts = 0 it only flushes).  A tile holds
        // tw candidates (lanes below tw), screened as tw / 16 column blocks.
        const uint32_t tw = (uint32_t)G.tile_w;
        auto score_tiles = [&](uint32_t npts, uint32_t nrun, bool last) {
            if (npts == 0 && !last) return;
            // With records of 16 or more dimensions the tiles are software-pipelined: the
            // record loads of the next tile are issued before the current tile is screened,
            // so they are in flight while it is (bf16_16d 78.5 -> 70.2 ms).  With 8 the
            // registers this holds cost more than the overlap gains (skew8d 950 -> 983 ms), and
            // a tile's loads are issued once the previous tile is done.
            constexpr bool PIPE = SP >= 16;
            auto run_tiles = [&](auto nbc) __attribute__((always_inline)) {
                constexpr int NB = decltype(nbc)::value;
                constexpr uint32_t TW = 16u * NB;
                uint32_t seg = 0;
                // set-up of the tile at b: candidate b + lane's run (one uniform pass over
                // the runs that start inside the tile), its record position (0 for a lane
                // without a candidate) and its |x'|^2 (a load still in flight)
                auto setup = [&](uint32_t b, uint32_t& pidx, float& xn, bool& valid) __attribute__((always_inline)) {
                    const uint32_t p = b + lane;
                    const uint32_t end = b + TW;
                    uint32_t my = seg;
                    uint32_t s = seg + 1;
                    uint32_t pre_s = (uint32_t)__builtin_amdgcn_readfirstlane((int)S.run_pre[s]);
                    while (pre_s < end && s < nrun) {
                        if (p >= pre_s) my = s;
                        ++s;
                        pre_s = (uint32_t)__builtin_amdgcn_readfirstlane((int)S.run_pre[s]);
                    }
                    seg = (pre_s == end && s < nrun) ? s : s - 1;
                    valid = p < npts && (uint32_t)lane < TW;
                    const uint32_t at = S.run_begin[my] + (p - S.run_pre[my]);
                    pidx = valid ? at : 0u;
                    xn = ix.sxn[pidx];
                    const int nvalid = __popcll(ballot(valid));
#pragma unroll
                    for (int i = 0; i < 4; ++i) if (!done[i]) cands[i] += nvalid;
                };
                bf16x8 ld[NB][Screen<SP>::NCH], ldn[NB][Screen<SP>::NCH];
                uint32_t pidx, pidxn = 0;
                float xn, xnn = 0.0f;
                bool valid, validn = false;
                setup(0u, pidx, xn, valid);
                tile_load<SP, NB>(ix, pidx, g, t, ld);
                for (uint32_t base = 0;; base += TW) {
                    const bool more = base + TW < npts;
                    if (PIPE && more) {
                        setup(base + TW, pidxn, xnn, validn);
                        tile_load<SP, NB>(ix, pidxn, g, t, ldn);
                    }
                    // Fast path: the 16 x TW screen of the tile (lane (g, t) holds candidate
                    // 16 cb + t of column block cb); most tiles admit nothing once the
                    // buffers are full.  A lane without a candidate starts at NaN, which
                    // is never admitted.
                    const float xinit = valid ? __builtin_fmaf(-SCREEN_REL, xn, xn) - SCREEN_ABS
                                              : __int_as_float(0x7fc00000);
                    floatx4 accs[NB];
                    tile_mfma<SP, NB>(afr, ld, xinit, g, t, accs);
                    uint64_t any = 0;
#pragma unroll
                    for (int cb = 0; cb < NB; ++cb)
#pragma unroll
                        for (int i = 0; i < 4; ++i) any |= ballot(accs[cb][i] <= bnd[i]);
                    if (any) {
                        // queue the admitted pairs (query row, point position)
#pragma unroll
                        for (int cb = 0; cb < NB; ++cb) {
                            const uint32_t pc = (uint32_t)__shfl((int)pidx, 16 * cb + t, WAVE);
#pragma unroll
                            for (int i = 0; i < 4; ++i) {
                                const uint64_t M = ballot(accs[cb][i] <= bnd[i]);
                                if ((M >> lane) & 1) {
                                    const int pos = qcount + __popcll(M & __lanemask_lt());
                                    S.qp[pos] = pc;
                                    S.qr[pos] = (uint8_t)(4 * g + i);
                                }
                                qcount += __popcll(M);
                                rer[i] += __popc((uint32_t)(M >> (16 * g)) & 0xffffu);
                            }
                        }
                    }
                    if (qcount >= QFLUSH || (last && qcount > 0 && !more)) {
                        flush();
                        // the next tile's loads are issued again after the flush, so that
                        // they do not hold registers through it (flushes are rare)
                        if (PIPE && more) {
                            xnn = ix.sxn[pidxn];
                            tile_load<SP, NB>(ix, pidxn, g, t, ldn);
                        }
                    }
                    if (!more) break;
                    if constexpr (PIPE) {
#pragma unroll
                        for (int cb = 0; cb < NB; ++cb)
#pragma unroll
                            for (int c = 0; c < Screen<SP>::NCH; ++c) ld[cb][c] = ldn[cb][c];
                        pidx = pidxn;
                        xn = xnn;
                        valid = validn;
                    } else {
                        setup(base + TW, pidx, xn, valid);
                        tile_load<SP, NB>(ix, pidx, g, t, ld);
                    }
                }
            };
            if (tw == 64) run_tiles(std::integral_constant<int, 4>{});
            else run_tiles(std::integral_constant<int, 2>{});
        };

        if (G.brute) {
            // exhaustive KNN: every point is a candidate, in one pass
            if (any_live) {
                if (lane == 0) {
                    S.run_begin[0] = 0u;
                    S.run_pre[0] = 0u;
                    S.run_pre[1] = (uint32_t)ix.n;
                }
                wave_lds_sync();
                score_tiles((uint32_t)ix.n, 1u, true);
                wave_lds_sync();
            }
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                if (!done[i]) stopl[i] = 0;
                done[i] = true;
            }
        }
        for (; any_live && !G.brute; ++l) {
#pragma unroll
            for (int i = 0; i < 4; ++i) upd[i] = false;
            int sp = 0;
            // (instances up to 4 dimensions; wider ones, at their register limit, walk the
            // tree, which every index also holds)
            if (FT >= 1 && FT <= 4 && ix.lookup == LOOKUP_DENSE) {
                // Dense table: layer l of the group is enumerated as in the per-query
                // dense walk, around the box of central cells instead of one cell.  Rows
                // of ids over dimensions 0..f-2 span the box grown by l (clipped to the
                // occupied box); a row at Chebyshev distance l from the group box adds its
                // whole run along the last dimension, a nearer row only the two cells at
                // distance l (pass e = 0 the run or the low cell, e = 1 the high cell).
                const int L = f - 1;
                int32_t blo[FS], bw[FS];
                int64_t rows = 1;
                bool empty = false;
                for (int j = 0; j < f; ++j) {
                    const int32_t a0 = max(S.glo[j] - l, ix.cmin[j]);
                    const int32_t b0 = min(S.ghi[j] + l, ix.cmax[j]);
                    blo[j] = a0;
                    bw[j] = b0 - a0 + 1;
                    if (b0 < a0) empty = true;
                    if (j < L) rows *= (b0 >= a0 ? (int64_t)(b0 - a0 + 1) : 0);
                }
                for (int64_t row0 = 0; !empty && row0 < rows; row0 += WAVE) {
                    for (int e = 0; e < 2; ++e) {
                        double mt = -1.0;
#pragma unroll
                        for (int i = 0; i < 4; ++i) if (!done[i]) mt = fmax(mt, tau[i]);
                        for (int d = 16; d < WAVE; d <<= 1) mt = fmax(mt, __shfl_xor(mt, d, WAVE));
                        const int64_t r = row0 + lane;
                        bool keepc = false;
                        int32_t ids[FS];
                        int32_t ta = 1, tb = 0;
                        uint32_t lin = 0;
                        double lb = 0.0;
                        if (r < rows) {
                            int64_t rem = r;
                            int32_t maxoff = 0;
                            for (int j = L - 1; j >= 0; --j) {
                                const int32_t o = blo[j] + (int32_t)(rem % bw[j]);
                                rem /= bw[j];
                                ids[j] = o;
                                maxoff = max(maxoff, max(S.glo[j] - o, o - S.ghi[j]));
                                lin += (uint32_t)(o - ix.cmin[j]) * ix.stride[j];
                            }
                            if (maxoff == l) {
                                if (e == 0) { ta = blo[L]; tb = blo[L] + bw[L] - 1; }
                            } else {
                                const int32_t tt = e == 0 ? S.glo[L] - l : S.ghi[L] + l;
                                if (tt >= blo[L] && tt <= blo[L] + bw[L] - 1) ta = tb = tt;
                            }
                            if (ta <= tb) {
                                ids[L] = ta;
                                // distance from the box of query coordinates to the run's region
                                for (int j = 0; j < f; ++j) {
                                    const int32_t a = ids[j], b = j == L ? tb : ids[j];
                                    const double aj = S.ad[j], oj = S.od[j];
                                    const double below = __dadd_rn(__dadd_rn(__dmul_rn((double)a, aj), oj), -(double)S.qhi[j]);
                                    const double above = __dadd_rn((double)S.qlo[j], -__dadd_rn(__dmul_rn((double)(b + 1), aj), oj));
                                    double gap = below > above ? below : above;
                                    gap = gap > 0.0 ? gap : 0.0;
                                    lb = __dadd_rn(lb, __dmul_rn(gap, gap));
                                }
                                keepc = !prune || !(lb * LB_SHRINK > mt);
                            }
                        }
                        // the per-query FP32 test of the tree path below, on the run's region
                        if (FT > 0 && FT <= 8 && prune && cnt > 1 && ballot(keepc)) {
                            float clo[FS], chi[FS];
                            if (keepc) {
                                for (int j = 0; j < f; ++j) {
                                    const double aj = S.ad[j], oj = S.od[j];
                                    const int32_t a = ids[j], b = j == L ? tb : ids[j];
                                    clo[j] = f32_below(__dadd_rn(__dmul_rn((double)a, aj), oj));
                                    chi[j] = f32_above(__dadd_rn(__dmul_rn((double)(b + 1), aj), oj));
                                }
                            }
                            bool need = false;
                            for (int qr = 0; qr < cnt; ++qr) {
                                const float tq = S.tq[qr];
                                if (!(tq >= 0.0f)) continue;
                                float lbq = 0.0f;
                                for (int j = 0; j < f; ++j) {
                                    const float q = S.q[qr][j];
                                    const float gp = fmaxf(fmaxf(clo[j] - q, q - chi[j]), 0.0f);
                                    lbq = __builtin_fmaf(gp, gp, lbq);
                                }
                                need = need || lbq * (1.0f - 0x1p-18f) <= tq;
                            }
                            keepc = keepc && need;
                        }
                        uint32_t rb = 0, rn = 0;
                        if (keepc) {
                            rb = ix.cell_start[lin + (uint32_t)(ta - ix.cmin[L])];
                            rn = ix.cell_start[lin + (uint32_t)(tb - ix.cmin[L]) + 1] - rb;
                        }
                        probes += 2 * __popcll(ballot(keepc));
                        const uint32_t incl = wave_incl_scan(rn);
                        const uint32_t npts = readlane_i32((int)incl, WAVE - 1);
                        if (npts == 0) continue;
                        const uint32_t nrun_incl = wave_incl_scan(rn > 0 ? 1u : 0u);
                        const uint32_t nrun = readlane_i32((int)nrun_incl, WAVE - 1);
                        if (rn > 0) {
                            S.run_begin[nrun_incl - 1] = rb;
                            S.run_pre[nrun_incl - 1] = incl - rn;
                        }
                        if (lane == 0) S.run_pre[nrun] = npts;  // sentinel
                        wave_lds_sync();
                        score_tiles(npts, nrun, false);
                        wave_lds_sync();
                    }
                }
            } else {
                if (lane == 0) S.stack[0] = ((uint64_t)ix.tree_levels << 40) | ((uint64_t)ix.tree_count[ix.tree_levels] << 32);
                sp = 1;
                wave_lds_sync();
            }
            while (sp > 0) {
                --sp;
                const uint64_t e = S.stack[sp];
                wave_lds_sync();
                const int level = (int)(e >> 40);
                const int count = (int)((e >> 32) & 0xff);
                const uint32_t node = (uint32_t)e + lane;
                const bool active = lane < count;
                // largest k-th distance over the live queries (+inf while a buffer is not full)
                double mt = -1.0;
#pragma unroll
                for (int i = 0; i < 4; ++i) if (!done[i]) mt = fmax(mt, tau[i]);
                for (int d = 16; d < WAVE; d <<= 1) mt = fmax(mt, __shfl_xor(mt, d, WAVE));
                int32_t dmin = 0, dmax = 0;
                double lb = 0.0;
                if (active) {
                    const int32_t* lo = level == 0 ? ix.cell_coord + (size_t)node * f
                                                   : ix.node_lo + (size_t)(ix.tree_off[level] + node) * f;
                    const int32_t* hi = level == 0 ? lo : ix.node_hi + (size_t)(ix.tree_off[level] + node) * f;
                    for (int j = 0; j < f; ++j) {
                        const int32_t a = lo[j], b = hi[j], ga = S.glo[j], gb = S.ghi[j];
                        dmin = max(dmin, max(a - gb, ga - b));
                        dmax = max(dmax, max(ga - a, b - gb));
                        // distance from the box of query coordinates to the node's region
                        const double aj = S.ad[j], oj = S.od[j];
                        const double below = __dadd_rn(__dadd_rn(__dmul_rn((double)a, aj), oj), -(double)S.qhi[j]);
                        const double above = __dadd_rn((double)S.qlo[j], -__dadd_rn(__dmul_rn((double)(b + 1), aj), oj));
                        double gap = below > above ? below : above;
                        gap = gap > 0.0 ? gap : 0.0;
                        lb = __dadd_rn(lb, __dmul_rn(gap, gap));
                    }
                }
                const bool close = !prune || !(lb * LB_SHRINK > mt);
                probes += __popcll(ballot(active));
                if (level > 0) {
                    const bool keep = active && dmin <= l && l <= dmax && close;
                    const uint64_t km = ballot(keep);
                    if (keep) {
                        const int64_t c0 = (int64_t)node * WAVE;
                        const int nc = (int)min((int64_t)WAVE, ix.tree_count[level - 1] - c0);
                        S.stack[sp + __popcll(km & __lanemask_lt())] =
                            ((uint64_t)(level - 1) << 40) | ((uint64_t)nc << 32) | (uint32_t)c0;
                    }
                    sp += __popcll(km);
                    wave_lds_sync();
                    continue;
                }
                // cells of layer l: one run of points per kept cell.  With several
                // queries a cell is kept only if some live query's own lower bound to
                // it is within that query's threshold (the bound from the box of the
                // group's queries above is weaker).  FP32 bounds: the cell's region is
                // rounded outward and the sum shrunk by (1 - 2^-18), which covers the
                // rounding of f <= 32 differences, squares and sums.  (Up to 8
                // dimensions, where the cell bounds fit in registers.)
                bool keepc = active && dmin == l && close;
                if (FT > 0 && FT <= 8 && prune && cnt > 1 && ballot(keepc)) {
                    float clo[FS], chi[FS];
                    if (keepc) {
                        const int32_t* cid = ix.cell_coord + (size_t)node * f;
                        for (int j = 0; j < f; ++j) {
                            const double aj = S.ad[j], oj = S.od[j];
                            const int32_t c = cid[j];
                            clo[j] = f32_below(__dadd_rn(__dmul_rn((double)c, aj), oj));
                            chi[j] = f32_above(__dadd_rn(__dmul_rn((double)(c + 1), aj), oj));
                        }
                    }
                    bool need = false;
                    for (int r = 0; r < cnt; ++r) {
                        const float tq = S.tq[r];
                        if (!(tq >= 0.0f)) continue;
                        float lbq = 0.0f;
                        for (int j = 0; j < f; ++j) {
                            const float q = S.q[r][j];
                            const float gp = fmaxf(fmaxf(clo[j] - q, q - chi[j]), 0.0f);
                            lbq = __builtin_fmaf(gp, gp, lbq);
                        }
                        need = need || lbq * (1.0f - 0x1p-18f) <= tq;
                    }
                    keepc = keepc && need;
                }
                uint32_t rb = 0, rn = 0;
                if (keepc) {
                    rb = ix.cell_first[node];
                    rn = ix.cell_first[node + 1] - rb;
                }
                const uint32_t incl = wave_incl_scan(rn);
                const uint32_t npts = readlane_i32((int)incl, WAVE - 1);
                if (npts == 0) continue;
                const uint32_t nrun_incl = wave_incl_scan(rn > 0 ? 1u : 0u);
                const uint32_t nrun = readlane_i32((int)nrun_incl, WAVE - 1);
                if (rn > 0) {
                    S.run_begin[nrun_incl - 1] = rb;
                    S.run_pre[nrun_incl - 1] = incl - rn;
                }
                if (lane == 0) S.run_pre[nrun] = npts;  // sentinel
                wave_lds_sync();
                score_tiles(npts, nrun, false);
                wave_lds_sync();
            }
            score_tiles(0u, 0u, true);  // pending exact checks belong to layer l
            // stop rules for every live query of the group, after layer l
            bool any = false;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                if (done[i]) continue;
                const int r = 4 * g + i;
                const bool full = taui[i] != INT32_MAX;
                bool stop = l >= lcover;
                if (!stop && full) {
                    if (G.p.stop == GHN_STOP_PAPER) {
                        stop = !upd[i];
                    } else {
                        double r2 = __longlong_as_double(0x7ff0000000000000LL);
                        for (int j = 0; j < f; ++j) {
                            const double a = S.ad[j];
                            const double v = __dadd_rn((double)S.q[r][j], -S.od[j]);
                            const int32_t c = S.qc[r][j];
                            const double glo = __dadd_rn(v, -__dmul_rn((double)(c - l), a));
                            const double ghi = __dadd_rn(__dmul_rn((double)(c + l + 1), a), -v);
                            double gg = glo < ghi ? glo : ghi;
                            if (gg < 0.0) gg = 0.0;
                            const double g2 = __dmul_rn(gg, gg);
                            if (g2 < r2) r2 = g2;
                        }
                        stop = tau[i] < __dmul_rn(r2, EXACT_SHRINK);
                    }
                }
                if (stop) {
                    done[i] = true;
                    stopl[i] = true_layer(l, S.shift);
                    thr[i] = -inf;
                    bnd[i] = -inf;
                    if (t == 0) S.tq[r] = -1.0f;
                } else {
                    any = true;
                }
            }
            if (!ballot(any)) break;
        }

        // ---- outputs, one slot (four queries, one per row) at a time
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int r = 4 * g + i;
            const bool act = r < cnt;
            const int64_t qi = act ? (int64_t)G.p.order[gd.x + r] - qbase : 0;
            // every walk ends with k rows of the index; one that does not reports it (the
            // buffer fills from the front, so its k-th entry is a row once it is full)
            const bool fin_r = act && ((fin_mask >> r) & 1);
            bool bad = false;
#pragma unroll
            for (int j = 0; j < KR; ++j) bad = bad || (16 * j + t < k && !entry_ok(bi[i][j], ix.n));
            const bool short_r = ((ballot(fin_r && bad) >> (16 * g)) & 0xffffu) != 0;
            const bool live = fin_r && !short_r;
            if (act && !live) {
                write_no_answer_row(io.out_idx, io.out_d2, io.out_pred, io.out_stop_layer, io.out_cands,
                                    io.out_probes, io.out_rerank, ix.task == GHN_CLASSIFY, k, qi, t, 16,
                                    short_r ? STOP_SHORT : STOP_NONFINITE);
                if (short_r && t == 0 && io.faults) atomicOr(io.faults, GHN_WALK_SHORT);
            }
            if (live) {
#pragma unroll
                for (int j = 0; j < KR; ++j) {
                    const int ee = 16 * j + t;
                    if (ee < k) {
                        io.out_idx[qi * k + ee] = bi[i][j];
                        if (io.out_d2) io.out_d2[qi * k + ee] = bd[i][j];
                        S.lab[g][ee] = ((const int32_t*)ix.targets)[bi[i][j]];
                    }
                }
            }
            wave_lds_sync();
            if (live) {
                if (ix.task == GHN_CLASSIFY) {
                    int best = INT32_MAX, best_n = -1;
#pragma unroll
                    for (int j = 0; j < KR; ++j) {
                        const int ee = 16 * j + t;
                        if (ee >= k) continue;
                        const int lab = S.lab[g][ee];
                        int n = 0;
                        for (int e2 = 0; e2 < k; ++e2) n += S.lab[g][e2] == lab;
                        if (n > best_n || (n == best_n && lab < best)) { best = lab; best_n = n; }
                    }
                    for (int d = 1; d < 16; d <<= 1) {
                        const int ob = __shfl_xor(best, d, 16), on = __shfl_xor(best_n, d, 16);
                        if (on > best_n || (on == best_n && ob < best)) { best = ob; best_n = on; }
                    }
                    if (t == 0) ((int32_t*)io.out_pred)[qi] = best;
                } else if (io.flags & GHN_FLAG_MEDIAN) {
                    // the targets at sorted positions (k - 1) / 2 and k / 2 (IEEE total order): each
                    // entry's rank is counted against the row's k targets
                    const int p1 = (k - 1) >> 1, p2 = k >> 1;
#pragma unroll
                    for (int j = 0; j < KR; ++j) {
                        const int ee = 16 * j + t;
                        if (ee >= k) continue;
                        const uint32_t kv = total_key(S.lab[g][ee]);
                        int less = 0, eq = 0;
                        for (int e2 = 0; e2 < k; ++e2) {
                            const uint32_t o = total_key(S.lab[g][e2]);
                            less += o < kv;
                            eq += o == kv;
                        }
                        if (less <= p1 && p1 < less + eq) S.med[g][0] = S.lab[g][ee];
                        if (less <= p2 && p2 < less + eq) S.med[g][1] = S.lab[g][ee];
                    }
                    wave_lds_sync();
                    if (t == 0) {
                        const float a = __int_as_float(S.med[g][0]), b = __int_as_float(S.med[g][1]);
                        ((float*)io.out_pred)[qi] = (k & 1) ? a : (float)(__dadd_rn((double)a, (double)b) / 2.0);
                    }
                } else if (t == 0) {
                    double s = 0.0;
                    for (int e2 = 0; e2 < k; ++e2) s = __dadd_rn(s, (double)__int_as_float(S.lab[g][e2]));
                    ((float*)io.out_pred)[qi] = (float)(s / (double)k);
                }
                if (t == 0) {
                    if (io.out_stop_layer) io.out_stop_layer[qi] = stopl[i];
                    if (io.out_cands) io.out_cands[qi] = cands[i];
                    if (io.out_probes) io.out_probes[qi] = probes;
                    if (io.out_rerank) io.out_rerank[qi] = rer[i];
                }
            }
            wave_lds_sync();
        }
    }
}

// Diagnostic: the grouped screen's error against the exact FP64 distance.  One wave
// takes 16 consecutive queries and `nsamp` points spread evenly over the index (cell
// order), forms s = |q'|^2 + |x'|^2 - 2 q'.x' with the screen's operands and matrix
// instruction (screen_block, accumulator started at |x'|^2), and records per query
// max |s - d| and max |s - d| / (|q'|^2 + |x'|^2).
template <int FT, int SP>
__global__ __launch_bounds__(GT) void k_screen_error(IndexView ix, const float* __restrict__ qs, int64_t m,
                                                     uint32_t nsamp, float* __restrict__ out_abs,
                                                     float* __restrict__ out_rel) {
    constexpr int FS = FT > 0 ? FT : F_MAX;
    using SC = Screen<SP>;
    constexpr int NKB = SC::NKB;
    __shared__ double sqd[GWPB][GQ][FS];
    const int lane = lane_id(), g = lane >> 4, t = lane & 15;
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x / WAVE);
    const int f = FT > 0 ? FT : ix.f;
    const int64_t q0 = ((int64_t)blockIdx.x * GWPB + wv) * GQ;
    if (q0 >= m) return;
    const int cnt = (int)min((int64_t)GQ, m - q0);
    bool fin = lane < cnt;
    for (int j = 0; j < f; ++j) {
        const float x = lane < cnt ? qs[(q0 + lane) * f + j] : 0.0f;
        fin = fin && isfinite(x);
        if (lane < GQ) sqd[wv][lane][j] = (double)x;
    }
    const uint64_t fin_mask = ballot(fin);
    wave_lds_sync();
    bf16x8 afr[NKB];
    {
        const int r = lane & 15;
        const bool rlive = (fin_mask >> r) & 1;
#pragma unroll
        for (int kb = 0; kb < NKB; ++kb) {
            const int part = SC::a_part(kb, g), d0 = SC::a_dim(kb, g);
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                const int j = d0 + e;
                float v = 0.0f;
                if (part >= 0 && rlive && j < f) {
                    const float qp = (float)sqd[wv][r][j] - ix.c0[j];
                    const float hi = (float)(__bf16)qp;
                    v = part == 1 ? (float)(__bf16)(qp - hi) : hi;
                }
                afr[kb][e] = (__bf16)(-2.0f * v);
            }
        }
    }
    float qn[4], mabs[4], mrel[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        float sq = 0.0f;
        if ((fin_mask >> (4 * g + i)) & 1)
            for (int j = 0; j < f; ++j) {
                const float d = (float)sqd[wv][4 * g + i][j] - ix.c0[j];
                sq = __builtin_fmaf(d, d, sq);
            }
        qn[i] = sq;
        mabs[i] = 0.0f;
        mrel[i] = 0.0f;
    }
    for (uint32_t base = 0; base < nsamp; base += WAVE) {
        const uint32_t p = base + lane;
        const bool valid = p < nsamp;
        const uint32_t pidx = valid ? (uint32_t)((uint64_t)p * (uint64_t)ix.n / nsamp) : 0u;
        const float xn = valid ? ix.sxn[pidx] : 0.0f;
#pragma unroll
        for (int cb = 0; cb < 4; ++cb) {
            uint32_t pc;
            const floatx4 acc = screen_block<FT, SP>(ix, afr, pidx, xn, base, nsamp, cb, g, t, pc);
            const float xnc = __shfl(xn, 16 * cb + t, WAVE);
            if (base + 16 * cb + t >= nsamp) continue;
            float xv[FS];
            load_point<FT>(ix.spts + (size_t)pc * f, xv, f);
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                if (!((fin_mask >> (4 * g + i)) & 1)) continue;
                double d = 0.0;
                for (int j = 0; j < f; ++j) {
                    const double dj = __dadd_rn(sqd[wv][4 * g + i][j], -(double)xv[j]);
                    d = __dadd_rn(d, __dmul_rn(dj, dj));
                }
                const double err = fabs(__dadd_rn((double)acc[i] + (double)qn[i], -d));
                mabs[i] = fmaxf(mabs[i], (float)err);
                mrel[i] = fmaxf(mrel[i], (float)(err / ((double)qn[i] + (double)xnc)));
            }
        }
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        for (int d = 1; d < 16; d <<= 1) {
            mabs[i] = fmaxf(mabs[i], __shfl_xor(mabs[i], d, 16));
            mrel[i] = fmaxf(mrel[i], __shfl_xor(mrel[i], d, 16));
        }
        const int r = 4 * g + i;
        if (t == 0 && r < cnt) {
            const bool ok = (fin_mask >> r) & 1;
            out_abs[q0 + r] = ok ? mabs[i] : __int_as_float(0x7fc00000);
            out_rel[q0 + r] = ok ? mrel[i] : __int_as_float(0x7fc00000);
        }
    }
}

template <int FT>
hipError_t launch_err(const IndexView& ix, const float* qs, int64_t m, uint32_t nsamp, float* out_abs,
                      float* out_rel, hipStream_t s) {
    constexpr int SP = FT <= 8 ? 8 : (FT <= 16 ? 16 : 32);
    const int64_t blocks = (m + GQ * GWPB - 1) / (GQ * GWPB);
    if (FT > 0) {
        hipLaunchKernelGGL((k_screen_error<FT, SP>), dim3((unsigned)blocks), dim3(GT), 0, s, ix, qs, m, nsamp, out_abs, out_rel);
    } else if (ix.sp == 8) {
        hipLaunchKernelGGL((k_screen_error<0, 8>), dim3((unsigned)blocks), dim3(GT), 0, s, ix, qs, m, nsamp, out_abs, out_rel);
    } else if (ix.sp == 16) {
        hipLaunchKernelGGL((k_screen_error<0, 16>), dim3((unsigned)blocks), dim3(GT), 0, s, ix, qs, m, nsamp, out_abs, out_rel);
    } else {
        hipLaunchKernelGGL((k_screen_error<0, 32>), dim3((unsigned)blocks), dim3(GT), 0, s, ix, qs, m, nsamp, out_abs, out_rel);
    }
    return launch_status();
}

template <int FT, int SP, bool BATCH>
hipError_t launch_k(const GroupArgs& a, int kmax, int blocks, hipStream_t s) {
    if (kmax <= 16) hipLaunchKernelGGL((k_predict_group<FT, SP, 1, BATCH>), dim3(blocks), dim3(GT), 0, s, a);
    else if (kmax <= 32) hipLaunchKernelGGL((k_predict_group<FT, SP, 2, BATCH>), dim3(blocks), dim3(GT), 0, s, a);
    else hipLaunchKernelGGL((k_predict_group<FT, SP, 4, BATCH>), dim3(blocks), dim3(GT), 0, s, a);
    return launch_status();
}

// sp: the padded screen dimension (every index of a batch has f, so the same sp)
template <int FT, bool BATCH>
hipError_t launch_ft(const GroupArgs& a, int sp, int kmax, int blocks, hipStream_t s) {
    constexpr int SP = FT <= 8 ? 8 : (FT <= 16 ? 16 : 32);
    if (FT > 0) return launch_k<FT, SP, BATCH>(a, kmax, blocks, s);
    if (sp == 8) return launch_k<0, 8, BATCH>(a, kmax, blocks, s);
    if (sp == 16) return launch_k<0, 16, BATCH>(a, kmax, blocks, s);
    return launch_k<0, 32, BATCH>(a, kmax, blocks, s);
}

template <bool BATCH>
hipError_t launch_group_walk(const GroupArgs& ga, int f, int sp, int kmax, int blocks, hipStream_t s) {
    switch (f) {
        case 2: return launch_ft<2, BATCH>(ga, sp, kmax, blocks, s);
        case 3: return launch_ft<3, BATCH>(ga, sp, kmax, blocks, s);
        case 4: return launch_ft<4, BATCH>(ga, sp, kmax, blocks, s);
        case 8: return launch_ft<8, BATCH>(ga, sp, kmax, blocks, s);
        case 16: return launch_ft<16, BATCH>(ga, sp, kmax, blocks, s);
        default: return launch_ft<0, BATCH>(ga, sp, kmax, blocks, s);
    }
}

}  // namespace

size_t group_ws_bytes(int64_t m) {
    auto up = [](size_t b) { return (b + 255) & ~size_t(255); };
    return 2 * up(m * 8) + 3 * up(m * 4) + up(m * 8) + up(64) + up(radix_sort_temp_bytes(m));
}

// Sort + group the queries, then walk the groups.  `ws` holds group_ws_bytes(m).
hipError_t run_grouped(const PredictArgs& pa, int keep_shift_levels, int gsize, int tile_w, void* ws, hipStream_t s,
                       int* morton_bits, hipEvent_t ev_begin, hipEvent_t ev_end, bool brute) {
    const IndexView& ix = pa.ix;
    const int64_t m = pa.m;
    auto up = [](size_t b) { return (b + 255) & ~size_t(255); };
    int bits[F_MAX];
    int total = 0, maxb = 0;
    for (int j = 0; j < ix.f; ++j) {
        const uint32_t span = (uint32_t)(ix.cmax[j] - ix.cmin[j]);
        bits[j] = span ? 32 - __builtin_clz(span) : 0;
        total += bits[j];
        maxb = maxb > bits[j] ? maxb : bits[j];
    }
    *morton_bits = total;
    int shift = 0;  // Morton bits of the lowest `keep_shift_levels` bit levels
    for (int b = 0; b < keep_shift_levels && b < maxb; ++b)
        for (int j = 0; j < ix.f; ++j) shift += bits[j] > b ? 1 : 0;
    // codes wider than 64 bits are kept to their top 64 bits (coarser groups)
    const int kbits = total > 64 ? 64 : total;
    shift = total > 64 ? (shift > total - 64 ? shift - (total - 64) : 0) : shift;
    char* p = (char*)ws;
    uint64_t* k0 = (uint64_t*)p; p += up(m * 8);
    uint64_t* k1 = (uint64_t*)p; p += up(m * 8);
    uint32_t* v0 = (uint32_t*)p; p += up(m * 4);
    uint32_t* v1 = (uint32_t*)p; p += up(m * 4);
    uint32_t* qflags = (uint32_t*)p; p += up(m * 4);
    uint2* groups = (uint2*)p; p += up(m * 8);
    uint32_t* counters = (uint32_t*)p; p += up(64);
    void* rtemp = p;
    int64_t g = (m + 255) / 256;
    if (g > 65536) g = 65536;
    hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(64), 0, s, counters, 2);
    hipLaunchKernelGGL(k_group_keys, dim3((unsigned)g), dim3(256), 0, s, pa.io.queries, m, ix, k0, v0, qflags);
    bool alt = false;
    hipError_t e = radix_sort_pairs(k0, v0, k1, v1, m, kbits, rtemp, &alt, s);
    if (e != hipSuccess) return e;
    const uint64_t* sk = alt ? k1 : k0;
    const uint32_t* sv = alt ? v1 : v0;
    const int exact = pa.stop == GHN_STOP_PAPER && total > 64 ? 1 : 0;
    hipLaunchKernelGGL(k_form_groups, dim3((unsigned)g), dim3(256), 0, s, sk, sv, qflags, m, shift, pa.io.queries,
                       ix, exact, gsize, groups, counters);
    GroupArgs ga;
    ga.brute = brute ? 1 : 0;
    ga.p = pa;
    ga.p.order = sv;
    ga.groups = groups;
    ga.counters = counters;
    ga.work = counters + 1;
    ga.items = nullptr;
    ga.n_items = 0;
    ga.tile_w = tile_w;
    int64_t blocks = (m + GQ * GWPB - 1) / (GQ * GWPB);
    if (blocks > 2048) blocks = 2048;
    if (ev_begin && (e = hipEventRecord(ev_begin, s)) != hipSuccess) return e;
    e = launch_group_walk<false>(ga, ix.f, ix.sp, pa.io.k, (int)blocks, s);
    if (e == hipSuccess && ev_end) e = hipEventRecord(ev_end, s);
    return e;
}

hipError_t batch_query_order(const BatchItem* items, int n_items, int64_t total, int kb, int key_bits, void* ws,
                             hipStream_t s, const uint32_t** order) {
    auto up = [](size_t b) { return (b + 255) & ~size_t(255); };
    const int64_t m = total;
    char* p = (char*)ws;
    uint64_t* k0 = (uint64_t*)p; p += up(m * 8);
    uint64_t* k1 = (uint64_t*)p; p += up(m * 8);
    uint32_t* v0 = (uint32_t*)p; p += up(m * 4);
    uint32_t* v1 = (uint32_t*)p; p += up(m * 4);
    uint32_t* qflags = (uint32_t*)p; p += up(m * 4);
    p += up(m * 8) + up(64);  // (groups and counters of the grouped form)
    void* rtemp = p;
    int64_t g = (m + 255) / 256;
    if (g > 65536) g = 65536;
    hipLaunchKernelGGL(k_batch_group_keys, dim3((unsigned)g), dim3(256), 0, s, items, n_items, m, kb, k0, v0, qflags);
    bool alt = false;
    const hipError_t e = radix_sort_pairs(k0, v0, k1, v1, m, key_bits, rtemp, &alt, s);
    *order = alt ? v1 : v0;
    return e;
}

hipError_t run_grouped_batched(const BatchItem* items, int n_items, int64_t total, int f, int kmax, int stop, int kb,
                               int key_bits, int gsize, int tile_w, void* ws, hipStream_t s) {
    auto up = [](size_t b) { return (b + 255) & ~size_t(255); };
    const int64_t m = total;
    char* p = (char*)ws;
    uint64_t* k0 = (uint64_t*)p; p += up(m * 8);
    uint64_t* k1 = (uint64_t*)p; p += up(m * 8);
    uint32_t* v0 = (uint32_t*)p; p += up(m * 4);
    uint32_t* v1 = (uint32_t*)p; p += up(m * 4);
    uint32_t* qflags = (uint32_t*)p; p += up(m * 4);
    uint2* groups = (uint2*)p; p += up(m * 8);
    uint32_t* counters = (uint32_t*)p; p += up(64);
    void* rtemp = p;
    int64_t g = (m + 255) / 256;
    if (g > 65536) g = 65536;
    hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(64), 0, s, counters, 2);
    hipLaunchKernelGGL(k_batch_group_keys, dim3((unsigned)g), dim3(256), 0, s, items, n_items, m, kb, k0, v0, qflags);
    bool alt = false;
    hipError_t e = radix_sort_pairs(k0, v0, k1, v1, m, key_bits, rtemp, &alt, s);
    if (e != hipSuccess) return e;
    const uint64_t* sk = alt ? k1 : k0;
    const uint32_t* sv = alt ? v1 : v0;
    hipLaunchKernelGGL(k_batch_form_groups, dim3((unsigned)g), dim3(256), 0, s, sk, sv, qflags, m, items, kb, gsize,
                       groups, counters);
    GroupArgs ga;
    std::memset(&ga, 0, sizeof ga);
    ga.brute = 0;
    ga.p.m = m;
    ga.p.stop = stop;
    ga.p.order = sv;
    ga.groups = groups;
    ga.counters = counters;
    ga.work = counters + 1;
    ga.items = items;
    ga.n_items = n_items;
    ga.tile_w = tile_w;
    int64_t blocks = (m + GQ * GWPB - 1) / (GQ * GWPB);
    if (blocks > 2048) blocks = 2048;
    if (blocks < 1) blocks = 1;
    const int sp = f <= 8 ? 8 : (f <= 16 ? 16 : 32);
    return launch_group_walk<true>(ga, f, sp, kmax, (int)blocks, s);
}

hipError_t launch_screen_error(const IndexView& ix, const float* qs, int64_t m, uint32_t nsamp, float* out_abs,
                               float* out_rel, hipStream_t s) {
    switch (ix.f) {
        case 2: return launch_err<2>(ix, qs, m, nsamp, out_abs, out_rel, s);
        case 3: return launch_err<3>(ix, qs, m, nsamp, out_abs, out_rel, s);
        case 4: return launch_err<4>(ix, qs, m, nsamp, out_abs, out_rel, s);
        case 8: return launch_err<8>(ix, qs, m, nsamp, out_abs, out_rel, s);
        case 16: return launch_err<16>(ix, qs, m, nsamp, out_abs, out_rel, s);
        default: return launch_err<0>(ix, qs, m, nsamp, out_abs, out_rel, s);
    }
}

}  // namespace ghn
