// Device pieces shared by the exploration kernels (Section III-B): query set-up,
// the FP32 screen + FP64 size-k buffer, the load-balanced gather of a list of
// point runs, the stop rules, and the prediction from the buffer.
//
// One wave64 walks one query.  The size-k buffer (the paper's heap) lives in
// lanes 0..k-1 sorted by (FP64 distance, row id).  Candidates are screened with
// an FP32 distance; only those that may still enter the buffer get their FP64
// distance and an exact (distance, id) comparison, so the buffer always holds
// exactly the k best of everything scored so far.
#pragma once

#include "ghn_guard.h"
#include "ghn_internal.h"

namespace ghn {

constexpr int NUM_XCD = 8;
constexpr double LB_SHRINK = 1.0 - 0x1p-40;    // cell lower bounds are shrunk by this before pruning
constexpr double EXACT_SHRINK = 1.0 - 0x1p-44; // squared ring distance is shrunk by this (EXACT rule)
constexpr int RUN_CAP = 2 * WAVE + 1;          // point runs listed per batch (+ sentinel)
constexpr int32_t RING_STEP_MAX = 64;          // most layers one step of the ring schedule walks

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
#pragma unroll
    for (int j = 0; j < (FT > 0 ? FT : F_MAX); ++j) {
        if (FT == 0 && j >= f) break;
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

// Distance from v to the id interval [lo*a, (hi+1)*a) in FP64 (0 inside).
__device__ __forceinline__ double gap_to_cells(double v, int64_t lo, int64_t hi, double a) {
    double below = __dadd_rn(__dmul_rn((double)lo, a), -v);
    double above = __dadd_rn(v, -__dmul_rn((double)(hi + 1), a));
    double g = below > above ? below : above;
    return g > 0.0 ? g : 0.0;
}

// Ring schedule of the EXACT rule: a step walks the layers l .. last_layer(l) at once:
// io.ring_step layers (at least 1), and with GHN_FLAG_RING_GROW twice as many as the
// step before while the buffer still holds fewer than k entries (no stop test can fire
// then), never past the layer that covers the box.  The stop test runs after each
// step with the step's last layer, so the result stays the brute-force one.  (Growing
// only after steps that held no point was measured too: on the skew8d queries it
// kept the dense half faster but lost more on the sparse half, 320 against 314 ms.)
struct RingStep {
    int32_t base, cur;
    bool grow;
    __device__ __forceinline__ explicit RingStep(const QueryIO& io)
        : base(io.ring_step > 1 ? io.ring_step : 1), cur(io.ring_step > 1 ? io.ring_step : 1),
          grow((io.flags & GHN_FLAG_RING_GROW) != 0) {}
    __device__ __forceinline__ int32_t last_layer(int32_t l, bool full, int32_t lcover) {
        const int32_t lh = min(l + cur - 1, max(lcover, l));
        cur = grow && !full ? min(cur * 2, RING_STEP_MAX) : base;
        return lh;
    }
};

struct WaveState {
    double bd;      // this lane's buffer slot: distance (lanes < k)
    int bi;         // this lane's buffer slot: row id
    double tau;     // k-th distance (+inf while the buffer is not full)
    int tau_i;      // k-th row id
    float t32;      // FP32 admission threshold derived from tau
    int count;      // entries in the buffer (<= k)
    bool updated;   // an insertion happened in the current layer
    int32_t cands;  // candidates scored
    int32_t probes; // index entries read to find cells
    int32_t rerank; // candidates re-scored in FP64
};

__device__ __forceinline__ void init_state(WaveState& st) {
    st.bd = __longlong_as_double(0x7ff0000000000000LL);
    st.bi = INT32_MAX;
    st.tau = st.bd;
    st.tau_i = INT32_MAX;
    st.t32 = __int_as_float(0x7f800000);
    st.count = 0;
    st.updated = false;
    st.cands = 0;
    st.probes = 0;
    st.rerank = 0;
}

// Query set-up: coordinates, central cell (Eq. 1) in the walk frame (walk_frame in
// ghn_internal.h: the true cell unless it lies more than CLAMP cells outside the
// occupied box), first layer that reaches the box and layer that covers it, both in
// the frame; the true layer is the frame layer + shift.  setup_query alone clamps the
// ids to CLAMP cells outside the box, which is the frame unless l0 comes out as
// CLAMP; the walk then calls setup_far.
template <int FT>
struct Query {
    float q[FT > 0 ? FT : F_MAX];
    double v[FT > 0 ? FT : F_MAX];   // q - origin, FP64
    int32_t c[FT > 0 ? FT : F_MAX];  // central cell id in the walk frame (|c| < 2^29)
    int32_t l0, lcover;              // a shifted frame has l0 = CLAMP and layers >= CLAMP
    bool finite;
};

// Cell id of coordinate v clamped to [lo, hi] (lo and hi within 2^29 of 0): the floor
// of the quotient estimate, corrected with exact products (exact for |t| < 2^29),
// clamped while still an integer-valued double.  A NaN clamps to lo.
__device__ __forceinline__ int32_t clamped_cell_id(double v, double a, double ainv, int32_t lo, int32_t hi) {
    double t = floor(v * ainv);
    if (fabs(t) < 536870912.0) {
        if (__dmul_rn(t, a) > v) t -= 1.0;
        else if (__dmul_rn(t + 1.0, a) <= v) t += 1.0;
    }
    return (int32_t)fmin(fmax(t, (double)lo), (double)hi);
}

// Lane j < f: the exact central cell id of query qi in dimension j (cell_floor_sat)
// and its distance to the occupied box; other lanes 0.  The far-query paths below
// work one dimension per lane from the query in memory, so they add almost nothing
// to the registers a walk holds.
__device__ __forceinline__ void far_dim(const IndexView& ix, const float* queries, int64_t qi, int f, double& t,
                                        double& d) {
    const int j = lane_id();
    t = 0.0;
    d = 0.0;
    if (j < f) {
        const double v = __dadd_rn((double)queries[qi * f + j], -(double)ix.o[j]);
        t = cell_floor_sat(v, (double)ix.a[j], ix.ainv[j]);
        d = cell_outside(t, ix.cmin[j], ix.cmax[j]);
    }
}

__device__ __forceinline__ double wave_max_f64(double x) {
    // the permute addresses are formed here: shared with the walk's own lane terms, they
    // were held across the whole walk for this rare path and spilled to scratch per query
    int lane = lane_id();
    asm volatile("" : "+v"(lane));
#pragma unroll
    for (int m = 1; m < WAVE; m <<= 1) {
        // plain permutes (lane ^ m is always a lane of the wave)
        const int64_t b = __double_as_longlong(x);
        const int lo = __builtin_amdgcn_ds_bpermute((lane ^ m) << 2, (int)(uint32_t)b);
        const int hi = __builtin_amdgcn_ds_bpermute((lane ^ m) << 2, (int)(uint32_t)((uint64_t)b >> 32));
        x = fmax(x, __longlong_as_double((int64_t)(((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo)));
    }
    return x;
}

// True layer - frame layer of a finite query (walk_frame).
__device__ __forceinline__ int64_t far_shift(const IndexView& ix, const float* queries, int64_t qi, int f) {
    double t, d;
    far_dim(ix, queries, qi, f, t, d);
    return (int64_t)frame_shift(wave_max_f64(d));
}

// Lane j < f: the frame id of dimension j of a finite query (walk_frame).
__device__ __forceinline__ int32_t far_frame_id(const IndexView& ix, const float* queries, int64_t qi, int f) {
    double t, d;
    far_dim(ix, queries, qi, f, t, d);
    const double sh = frame_shift(wave_max_f64(d));
    const int j = lane_id();
    return j < f ? frame_id(t, ix.cmin[j], ix.cmax[j], sh) : 0;
}

// The frame of a set-up query whose l0 is CLAMP (it may lie further out): ids
// recomputed exactly and moved by walk_frame's rule.  Wave-uniform call.
template <int FT>
__device__ __forceinline__ void setup_far(const IndexView& ix, const float* queries, int64_t qi, int f, Query<FT>& Q) {
    const int32_t cl = far_frame_id(ix, queries, qi, f);
    Q.l0 = 0;
    Q.lcover = 0;
#pragma unroll
    for (int i = 0; i < (FT > 0 ? FT : F_MAX); ++i) {
        if (FT == 0 && i >= f) break;
        const int32_t c32 = readlane_i32(cl, i);
        Q.c[i] = c32;
        Q.l0 = max(Q.l0, max(ix.cmin[i] - c32, c32 - ix.cmax[i]));
        Q.lcover = max(Q.lcover, max(c32 - ix.cmin[i], ix.cmax[i] - c32));
    }
}

template <int FT>
__device__ __forceinline__ void setup_query(const IndexView& ix, const float* queries, int64_t qi, int f, Query<FT>& Q) {
    Q.finite = true;
    Q.l0 = 0;
    Q.lcover = 0;
#pragma unroll
    for (int j = 0; j < (FT > 0 ? FT : F_MAX); ++j) {
        if (FT == 0 && j >= f) break;
        Q.q[j] = queries[qi * f + j];
        Q.finite = Q.finite && isfinite(Q.q[j]);
        Q.v[j] = __dadd_rn((double)Q.q[j], -(double)ix.o[j]);
        // the frame id unless the query lies CLAMP or more cells outside the box
        const int32_t c32 = clamped_cell_id(Q.v[j], (double)ix.a[j], ix.ainv[j], ix.cmin[j] - (int32_t)CLAMP,
                                            ix.cmax[j] + (int32_t)CLAMP);
        Q.c[j] = c32;
        Q.l0 = max(Q.l0, max(ix.cmin[j] - c32, c32 - ix.cmax[j]));
        Q.lcover = max(Q.lcover, max(c32 - ix.cmin[j], ix.cmax[j] - c32));
    }
}

// The "no answer" row of query qi, written by the wave (entry e by lane e).
__device__ __forceinline__ void write_no_answer(const IndexView& ix, const QueryIO& io, int64_t qi, int32_t stop) {
    write_no_answer_row(io.out_idx, io.out_d2, io.out_pred, io.out_stop_layer, io.out_cands, io.out_probes,
                        io.out_rerank, ix.task == GHN_CLASSIFY, io.k, qi, lane_id(), WAVE, stop);
}

// Outputs of a query with a non-finite coordinate.
__device__ __forceinline__ void write_invalid(const IndexView& ix, const QueryIO& io, int64_t qi) {
    write_no_answer(ix, io, qi, STOP_NONFINITE);
}

// A walk that ended without k rows of the index: the "no answer" row, and the
// device's fault word records it.
__device__ __forceinline__ void report_short_walk(const IndexView& ix, const QueryIO& io, int64_t qi) {
    write_no_answer(ix, io, qi, STOP_SHORT);
    if (lane_id() == 0 && io.faults) atomicOr(io.faults, GHN_WALK_SHORT);
}

// Which query this wave walks.  With a spatial query order each XCD (blocks are
// dealt round-robin over the 8 XCDs) gets one contiguous range of blocks, so
// each XCD's L2 serves one region of space.
__device__ __forceinline__ int64_t wave_slot(const PredictArgs& A, int waves_per_block) {
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x / WAVE);
    int64_t blk = blockIdx.x;
    if (A.order) {
        const int64_t nb = gridDim.x, x = blk % NUM_XCD, t = blk / NUM_XCD;
        blk = x * (nb / NUM_XCD) + min(x, nb % NUM_XCD) + t;
    }
    return blk * waves_per_block + wv;
}

// One 64-wide chunk of candidates.
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

// (d, i) before (t, ti) in the exact (distance, row id) order; bitwise, so it
// compiles to compares without branches.
__device__ __forceinline__ bool before(double d, int i, double t, int ti) {
    return (d < t) | ((d == t) & (i < ti));
}

// The lanes for which before(d, i, t, ti) holds: the three compares are balloted
// one by one and combined as masks, so no per-lane boolean is built for the ballot.
__device__ __forceinline__ uint64_t ballot_before(double d, int i, double t, int ti) {
    return ballot(d < t) | (ballot(d == t) & ballot(i < ti));
}

// Insert (cd, ci) into the sorted buffer: the entries after it move up one lane
// (the k-th leaves the buffer; free slots hold +inf), then its lane is written.
// The caller guarantees that it beats the k-th entry, so it lands below lane k.
__device__ __forceinline__ void insert_entry(WaveState& st, uint64_t kmask, int k, int lane, double cd, int ci) {
    const bool gt = (lane < k) & before(cd, ci, st.bd, st.bi);
    const int pos = k - __popcll(ballot_before(cd, ci, st.bd, st.bi) & kmask);
    const double ud = shfl_up1_f64(st.bd);
    const int ui = shfl_up1_i32(st.bi);
    st.bd = gt ? ud : st.bd;
    st.bi = gt ? ui : st.bi;
    st.bd = writelane_f64(st.bd, cd, pos);
    st.bi = writelane_i32(st.bi, ci, pos);
}

// Screen a chunk in FP32; candidates that may enter the buffer get their FP64
// distance and are inserted one at a time (exact (distance, id) comparison).
template <int FT>
__device__ __forceinline__ void score_chunk(const float* q, int f, int k, const Chunk<FT>& c, WaveState& st) {
    const int lane = lane_id();
    // lanes without a candidate get NaN, which fails the admission compare (a real
    // candidate's FP32 distance is never NaN: the coordinates are finite)
    float d32 = __int_as_float(0x7fc00000);
    if (c.valid) d32 = dist32<FT>(q, c.x, f);
    const bool adm = d32 <= st.t32;
    uint64_t mask = ballot(adm);
    if (mask == 0) return;
    st.rerank += __popcll(mask);
    double d64 = 0.0;
    if (adm) d64 = dist64<FT>(q, c.x, f);
    // Only candidates that beat the current k-th entry in the exact (distance, id)
    // order can enter; the mask is narrowed to them now and after every insertion
    // into a full buffer, so each candidate left in it is inserted.
    if (st.count == k) mask &= ballot_before(d64, c.id, st.tau, st.tau_i);
    if (mask == 0) return;
    st.updated = true;
    const uint64_t kmask = ballot(lane < k);
    if (st.count < k) {
        // Free slots first.  With more candidates than free slots the nearest go
        // first, so the buffer fills with near points and the rest drop out of the
        // mask without an insertion.  (count + candidates left stays constant here.)
        const bool nearest = st.count + __popcll(mask) > k;
        float mine = ((mask >> lane) & 1) ? d32 : __int_as_float(0x7f800000);
        while (mask && st.count < k) {
            int src;
            if (nearest) {
                const float mn = wave_min_nonneg(mine);
                src = __ffsll((unsigned long long)(ballot(mine == mn) & mask)) - 1;
                mine = writelane_f32(mine, __int_as_float(0x7f800000), src);
            } else {
                src = __ffsll((unsigned long long)mask) - 1;
            }
            mask &= ~(1ull << src);
            insert_entry(st, kmask, k, lane, readlane_f64(d64, src), readlane_i32(c.id, src));
            ++st.count;
        }
        if (mask) mask &= ballot_before(d64, c.id, readlane_f64(st.bd, k - 1), readlane_i32(st.bi, k - 1));
    }
    while (mask) {
        const int src = __ffsll((unsigned long long)mask) - 1;
        mask &= ~(1ull << src);
        insert_entry(st, kmask, k, lane, readlane_f64(d64, src), readlane_i32(c.id, src));
        // the candidates that no longer beat the new k-th entry drop out
        if (mask) mask &= ballot_before(d64, c.id, readlane_f64(st.bd, k - 1), readlane_i32(st.bi, k - 1));
    }
    if (st.count == k) {
        st.tau = readlane_f64(st.bd, k - 1);
        st.tau_i = readlane_i32(st.bi, k - 1);
        st.t32 = admit_threshold(st.tau);
    }
}

__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Key of a run for the nearest-first order: its distance lower bound (>= 0,
// already shrunk), rounded down to FP32 with the low 7 bits cleared; the bit
// pattern orders like the value and the low bits carry the run's slot.
__device__ __forceinline__ uint32_t lb_key(double lb) {
    float f = (float)lb;
    if ((double)f > lb) f = __uint_as_float(__float_as_uint(f) - 1u);
    return __float_as_uint(f) & ~127u;
}

// One compare-exchange step of a bitonic sort: merge blocks of SIZE lanes at lane
// distance S; a lane keeps the smaller key when its position in the pair (lane & S)
// and the block's direction (lane & SIZE) agree.
template <int SIZE, int S>
__device__ __forceinline__ uint32_t bitonic_step(uint32_t key, int lane) {
    const uint32_t other = xor_lane<S>(key);
    const bool up = (lane & SIZE) == 0;
    const bool low = (lane & S) == 0;
    return low == up ? min(key, other) : max(key, other);
}

// Ascending bitonic sort of one 32-bit key per lane over blocks of `width`
// lanes (a power of two, 2 <= width <= 64; lanes past the data hold 0xffffffff).
__device__ __forceinline__ uint32_t wave_sort_asc(uint32_t key, int lane, int width) {
    key = bitonic_step<2, 1>(key, lane);
    if (width >= 4) {
        key = bitonic_step<4, 2>(key, lane);
        key = bitonic_step<4, 1>(key, lane);
    }
    if (width >= 8) {
        key = bitonic_step<8, 4>(key, lane);
        key = bitonic_step<8, 2>(key, lane);
        key = bitonic_step<8, 1>(key, lane);
    }
    if (width >= 16) {
        key = bitonic_step<16, 8>(key, lane);
        key = bitonic_step<16, 4>(key, lane);
        key = bitonic_step<16, 2>(key, lane);
        key = bitonic_step<16, 1>(key, lane);
    }
    if (width >= 32) {
        key = bitonic_step<32, 16>(key, lane);
        key = bitonic_step<32, 8>(key, lane);
        key = bitonic_step<32, 4>(key, lane);
        key = bitonic_step<32, 2>(key, lane);
        key = bitonic_step<32, 1>(key, lane);
    }
    if (width >= 64) {
        key = bitonic_step<64, 32>(key, lane);
        key = bitonic_step<64, 16>(key, lane);
        key = bitonic_step<64, 8>(key, lane);
        key = bitonic_step<64, 4>(key, lane);
        key = bitonic_step<64, 2>(key, lane);
        key = bitonic_step<64, 1>(key, lane);
    }
    return key;
}

// Lane-held runs of points (begin b0/b1, length n0/n1; 0 = none) are listed in
// the wave's LDS arrays and scored in 64-wide chunks, each lane finding its
// point by a binary search over the run prefixes.
//
// With `order` set the runs carry lower-bound keys (lb_key of a lower bound of
// every point's distance in the run): they are scored nearest run first, and
// before each chunk the runs whose bound exceeds the current k-th distance are
// cut off the end of the list (none of their points could enter the buffer).
template <int FT>
__device__ __forceinline__ void score_runs(const IndexView& ix, const float* q, int f, int k, uint32_t b0, uint32_t n0,
                                           uint32_t key0, uint32_t b1, uint32_t n1, uint32_t key1, bool order,
                                           uint32_t* s_begin, uint32_t* s_pre, uint32_t* s_key, WaveState& st) {
    const int lane = lane_id();
    const uint32_t nseg_l = (n0 > 0) + (n1 > 0);
    const uint32_t npts_l = n0 + n1;
    const uint32_t seg_incl = wave_incl_scan(nseg_l);
    const uint32_t pts_incl = wave_incl_scan(npts_l);
    const uint32_t nseg = readlane_i32((int)seg_incl, WAVE - 1);
    const uint32_t npts = readlane_i32((int)pts_incl, WAVE - 1);
    if (npts == 0) return;
    uint32_t sidx = seg_incl - nseg_l, pofs = pts_incl - npts_l;
    const bool sorted = order && nseg > 1 && nseg <= WAVE;
    float lbk = __int_as_float(0x7f800000);  // sorted: this lane's run bound (lanes < nseg)
    uint32_t spre = 0xffffffffu;              // sorted: this lane's run offset (lanes < nseg)
    if (sorted) {
        if (n0 > 0) { s_begin[sidx] = b0; s_pre[sidx] = n0; s_key[sidx] = key0 | sidx; ++sidx; }
        if (n1 > 0) { s_begin[sidx] = b1; s_pre[sidx] = n1; s_key[sidx] = key1 | sidx; }
        wave_lds_sync();
        uint32_t key = (uint32_t)lane < nseg ? s_key[lane] : 0xffffffffu;
        int width = 2;
        while ((uint32_t)width < nseg) width <<= 1;
        key = wave_sort_asc(key, lane, width);
        uint32_t rb = 0, rn = 0;
        if ((uint32_t)lane < nseg) {
            rb = s_begin[key & 127u];
            rn = s_pre[key & 127u];
            lbk = __uint_as_float(key & ~127u);
        }
        const uint32_t incl = wave_incl_scan(rn);
        wave_lds_sync();
        if ((uint32_t)lane < nseg) {
            spre = incl - rn;
            s_begin[lane] = rb;
            s_pre[lane] = spre;
        }
    } else {
        if (n0 > 0) { s_begin[sidx] = b0; s_pre[sidx] = pofs; ++sidx; pofs += n0; }
        if (n1 > 0) { s_begin[sidx] = b1; s_pre[sidx] = pofs; }
    }
    if (lane == 0) s_pre[nseg] = npts;  // sentinel
    wave_lds_sync();
    // Chunk [base, base + 64): `seg` is the run holding `base`; the runs that start
    // inside the chunk are few, so each lane finds its run with one uniform pass
    // over them.  Sorted lists hold the run offsets in lanes (strictly increasing,
    // runs are non-empty), unsorted ones only in LDS.
    uint32_t seg = 0;
    uint32_t limit = npts;
    for (uint32_t base = 0; base < limit; base += WAVE) {
        const uint32_t p = base + lane;
        const uint32_t end = base + WAVE;
        uint32_t my = seg;
        if (sorted) {
            const uint64_t far = ballot((double)lbk > st.tau);
            if (far) {
                // lanes past the list hold an infinite bound, so the first far lane is
                // at most nseg: the end of the list
                const int cut = __ffsll((unsigned long long)far) - 1;
                limit = cut < (int)nseg ? (uint32_t)readlane_i32((int)spre, cut) : npts;
                if (base >= limit) break;
            }
            for (uint64_t in = ballot(spre > base) & ballot(spre < end); in; in &= in - 1) {
                const int r = __ffsll((unsigned long long)in) - 1;
                if (p >= (uint32_t)readlane_i32((int)spre, r)) my = (uint32_t)r;
            }
            seg = (uint32_t)__popcll(ballot(spre <= end)) - 1;  // the run holding `end`
        } else {
            uint32_t s = seg + 1;
            uint32_t pre_s = (uint32_t)__builtin_amdgcn_readfirstlane((int)s_pre[s]);
            while (pre_s < end && s < nseg) {
                if (p >= pre_s) my = s;
                ++s;
                pre_s = (uint32_t)__builtin_amdgcn_readfirstlane((int)s_pre[s]);
            }
            seg = (pre_s == end && s < nseg) ? s : s - 1;
        }
        const bool valid = p < limit;
        const uint32_t pidx = valid ? s_begin[my] + (p - s_pre[my]) : 0u;
        Chunk<FT> cur;
        fetch_chunk<FT>(ix, f, valid, pidx, cur);
        st.cands += (int32_t)min((uint32_t)WAVE, limit - base);  // the lanes with p < limit
        score_chunk<FT>(q, f, k, cur, st);
    }
    wave_lds_sync();
}

// A query's set-up is the same on every lane of its wave.  Made wave-uniform after it
// is computed, its values live in scalar registers for the walk instead of taking
// vector registers (the walks that set up their own query; the single-index dense
// kernel reads a block-shared set-up).
template <int FT>
__device__ __forceinline__ void uniform_query(Query<FT>& Q) {
    static_assert(FT > 0, "per-dimension instances only");
#pragma unroll
    for (int j = 0; j < FT; ++j) {
        Q.q[j] = __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(Q.q[j])));
        const uint64_t b = (uint64_t)__double_as_longlong(Q.v[j]);
        const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)b);
        const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(b >> 32));
        Q.v[j] = __longlong_as_double((int64_t)(((uint64_t)hi << 32) | lo));
        Q.c[j] = __builtin_amdgcn_readfirstlane(Q.c[j]);
    }
    Q.l0 = __builtin_amdgcn_readfirstlane(Q.l0);
    Q.lcover = __builtin_amdgcn_readfirstlane(Q.lcover);
    Q.finite = __builtin_amdgcn_readfirstlane((int)Q.finite) != 0;
}

// Stop rules, checked after every complete layer l of the walk frame.  In a shifted
// frame the EXACT bound is that of the frame's layer box, which lies inside the true
// layer box in every dimension: the bound is smaller (often 0) and the walk stops no
// earlier than with the true box, so the neighbours stay exact.
template <int FT, int STOP>
__device__ __forceinline__ bool stop_after_layer(const IndexView& ix, const Query<FT>& Q, int f, int k, int32_t l,
                                                 const WaveState& st) {
    if (l >= Q.lcover) return true;  // every occupied cell has been visited
    if (st.count != k) return false;
    if (STOP == GHN_STOP_PAPER) return !st.updated;
    // r_l: the query's distance to the nearest face of the layer box.  Rounding a
    // square is monotonic on [0, inf), so squaring the smallest face distance gives
    // the smallest of the squared ones.
    double g = __longlong_as_double(0x7ff0000000000000LL);
#pragma unroll
    for (int j = 0; j < (FT > 0 ? FT : F_MAX); ++j) {
        if (FT == 0 && j >= f) break;
        const double a = ix.a[j];
        const double glo = __dadd_rn(Q.v[j], -__dmul_rn((double)(Q.c[j] - l), a));
        const double ghi = __dadd_rn(__dmul_rn((double)(Q.c[j] + l + 1), a), -Q.v[j]);
        g = fmin(g, fmin(glo, ghi));
    }
    g = fmax(g, 0.0);
    return st.tau < __dmul_rn(__dmul_rn(g, g), EXACT_SHRINK);
}

// Neighbours in (distance, id) order, then the majority vote (ties -> smallest
// label) or the mean (FP64 sum in neighbour order, / k, rounded to FP32).
__device__ __forceinline__ void finish_query(const IndexView& ix, const QueryIO& io, int64_t qi, int32_t l,
                                             const WaveState& st) {
    const int lane = lane_id();
    const int k = io.k;
    if (ballot(lane < k && !entry_ok(st.bi, ix.n))) {
        report_short_walk(ix, io, qi);
        return;
    }
    const bool have = lane < k;
    if (lane < k) {
        io.out_idx[qi * k + lane] = st.bi;
        if (io.out_d2) io.out_d2[qi * k + lane] = st.bd;
    }
    if (ix.task == GHN_CLASSIFY) {
        const int32_t* lab = (const int32_t*)ix.targets;
        const int my = have ? lab[st.bi] : INT32_MAX;
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
        if (lane == 0) ((int32_t*)io.out_pred)[qi] = best;
    } else if (io.flags & GHN_FLAG_MEDIAN) {
        // sort the k targets across the wave in IEEE total order (padding last)
        const float* y = (const float*)ix.targets;
        const uint32_t u = have ? __float_as_uint(y[st.bi]) : 0u;
        uint32_t key = lane < k ? ((u & 0x80000000u) ? ~u : (u | 0x80000000u)) : 0xffffffffu;
        key = wave_sort_asc(key, lane, WAVE);
        const float v = __uint_as_float((key & 0x80000000u) ? (key & 0x7fffffffu) : ~key);
        float mid;
        if (k & 1) {
            mid = readlane_f32(v, k >> 1);
        } else {
            const double a = readlane_f32(v, (k >> 1) - 1), b = readlane_f32(v, k >> 1);
            mid = (float)(__dadd_rn(a, b) / 2.0);
        }
        if (lane == 0) ((float*)io.out_pred)[qi] = mid;
    } else {
        const float* y = (const float*)ix.targets;
        const float my = have ? y[st.bi] : 0.0f;
        double s = 0.0;
        for (int t = 0; t < k; ++t) s = __dadd_rn(s, (double)readlane_f32(my, t));
        if (lane == 0) ((float*)io.out_pred)[qi] = (float)(s / (double)k);
    }
    if (lane == 0) {
        if (io.out_stop_layer) io.out_stop_layer[qi] = (int32_t)l;
        if (io.out_cands) io.out_cands[qi] = st.cands;
        if (io.out_probes) io.out_probes[qi] = st.probes;
        if (io.out_rerank) io.out_rerank[qi] = st.rerank;
    }
}

}  // namespace ghn
