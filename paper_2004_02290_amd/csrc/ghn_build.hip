// Cell sampling on the GPU (Eq. 1, Algorithm 1): every training point gets its
// cell id; points are then grouped by cell with a stable LSD radix sort on the
// cell key, copied in cell order, and an offset table maps each cell of the
// occupied box to its run of points.  Empty cells own empty runs and store no
// points (Section III-A keeps no information about empty cells).
#include "ghn_internal.h"

namespace ghn {
namespace {

constexpr int BT = 256;  // threads per block for the simple build kernels

__device__ __forceinline__ float load_coord(const void* pts, int64_t idx, int32_t dtype) {
    if (dtype == GHN_BF16) {
        uint32_t b = ((const uint16_t*)pts)[idx];
        return __uint_as_float(b << 16);
    }
    return ((const float*)pts)[idx];
}

// Per-dimension range of cell ids plus data checks.
// minmax[j] = min cell id of dimension j, minmax[F_MAX + j] = max.
// flags[0] = a coordinate is NaN/Inf, flags[1] = a cell id is outside (-COORD_LIMIT, COORD_LIMIT).
__global__ __launch_bounds__(BT) void k_cells_minmax(const void* pts, int64_t n, int32_t f, int32_t dtype,
                                                     const float* __restrict__ a, const float* __restrict__ o,
                                                     int32_t* minmax, int32_t* flags) {
    __shared__ int32_t smin[F_MAX], smax[F_MAX];
    __shared__ int32_t sflag[2];
    if (threadIdx.x < F_MAX) { smin[threadIdx.x] = INT32_MAX; smax[threadIdx.x] = INT32_MIN; }
    if (threadIdx.x < 2) sflag[threadIdx.x] = 0;
    __syncthreads();
    for (int j = 0; j < f; ++j) {
        const double aj = a[j], oj = o[j];
        int32_t lmin = INT32_MAX, lmax = INT32_MIN;
        int32_t nonfinite = 0, overflow = 0;
        for (int64_t i = blockIdx.x * (int64_t)BT + threadIdx.x; i < n; i += (int64_t)gridDim.x * BT) {
            float x = load_coord(pts, i * f + j, dtype);
            if (!isfinite(x)) { nonfinite = 1; continue; }
            int64_t c = exact_floor_div(__dadd_rn((double)x, -oj), aj);
            if (c <= -COORD_LIMIT || c >= COORD_LIMIT) { overflow = 1; continue; }
            lmin = min(lmin, (int32_t)c);
            lmax = max(lmax, (int32_t)c);
        }
        if (lmin != INT32_MAX) atomicMin(&smin[j], lmin);
        if (lmax != INT32_MIN) atomicMax(&smax[j], lmax);
        if (nonfinite) sflag[0] = 1;
        if (overflow) sflag[1] = 1;
    }
    __syncthreads();
    if (threadIdx.x < (unsigned)f) {
        atomicMin(&minmax[threadIdx.x], smin[threadIdx.x]);
        atomicMax(&minmax[F_MAX + threadIdx.x], smax[threadIdx.x]);
    }
    if (threadIdx.x < 2 && sflag[threadIdx.x]) atomicOr(&flags[threadIdx.x], 1);
}

// Dense-box key of every point: linear index of its cell inside the occupied box.
__global__ __launch_bounds__(BT) void k_dense_keys(const void* pts, int64_t n, int32_t dtype, IndexView iv,
                                                   uint64_t* keys, uint32_t* vals) {
    const int32_t f = iv.f;
    for (int64_t i = blockIdx.x * (int64_t)BT + threadIdx.x; i < n; i += (int64_t)gridDim.x * BT) {
        uint64_t key = 0;
        for (int j = 0; j < f; ++j) {
            float x = load_coord(pts, i * f + j, dtype);
            int64_t c = exact_floor_div(__dadd_rn((double)x, -(double)iv.o[j]), (double)iv.a[j]);
            key += (uint64_t)(c - iv.cmin[j]) * (iv.lookup == LOOKUP_HASH ? iv.hstride[j] : (uint64_t)iv.stride[j]);
        }
        keys[i] = key;
        vals[i] = (uint32_t)i;
    }
}

// ------------------------------------------------------------------------------------------
// Stable LSD radix sort of (u64 key, u32 value) pairs, 8-bit digits, reduce-then-scan
// (per pass: block digit histograms, one exclusive scan over digit-major counts, then a
// stable scatter in which each block ranks its keys with wave ballots).
constexpr int RS_T = 256;
constexpr int RS_ITEMS = 16;
constexpr int RS_TILE = RS_T * RS_ITEMS;

__global__ __launch_bounds__(RS_T) void k_radix_hist(const uint64_t* __restrict__ keys, int64_t n, int shift,
                                                     uint32_t* __restrict__ counts, int nblocks) {
    __shared__ uint32_t h[256];
    h[threadIdx.x] = 0;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * RS_TILE;
    for (int it = 0; it < RS_ITEMS; ++it) {
        int64_t i = base + it * RS_T + threadIdx.x;
        if (i < n) atomicAdd(&h[(keys[i] >> shift) & 255u], 1u);
    }
    __syncthreads();
    counts[(int64_t)threadIdx.x * nblocks + blockIdx.x] = h[threadIdx.x];
}

constexpr int SCAN_T = 1024;

// Exclusive scan of `total` counts in place, one block.
__global__ __launch_bounds__(SCAN_T) void k_exclusive_scan_u32(uint32_t* data, int64_t total) {
    __shared__ uint32_t part[SCAN_T];
    const int64_t chunk = (total + SCAN_T - 1) / SCAN_T;
    const int64_t b = threadIdx.x * chunk;
    const int64_t e = min(b + chunk, total);
    uint32_t s = 0;
    for (int64_t i = b; i < e; ++i) s += data[i];
    part[threadIdx.x] = s;
    __syncthreads();
    for (int d = 1; d < SCAN_T; d <<= 1) {
        uint32_t t = threadIdx.x >= (unsigned)d ? part[threadIdx.x - d] : 0u;
        __syncthreads();
        part[threadIdx.x] += t;
        __syncthreads();
    }
    uint32_t run = part[threadIdx.x] - s;
    for (int64_t i = b; i < e; ++i) {
        uint32_t v = data[i];
        data[i] = run;
        run += v;
    }
}

__global__ __launch_bounds__(RS_T) void k_radix_scatter(const uint64_t* __restrict__ kin,
                                                        const uint32_t* __restrict__ vin,
                                                        uint64_t* __restrict__ kout, uint32_t* __restrict__ vout,
                                                        int64_t n, int shift, const uint32_t* __restrict__ offs,
                                                        int nblocks) {
    __shared__ uint32_t run[256];
    __shared__ uint32_t wc[RS_T / WAVE][256];
    const int t = threadIdx.x, w = t / WAVE;
    run[t] = offs[(int64_t)t * nblocks + blockIdx.x];
    for (int i = 0; i < RS_T / WAVE; ++i) wc[i][t] = 0;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * RS_TILE;
    const uint64_t lt = __lanemask_lt();
    for (int r = 0; r < RS_ITEMS; ++r) {
        const int64_t i = base + r * RS_T + t;
        const bool valid = i < n;
        uint64_t key = 0;
        uint32_t val = 0;
        uint32_t d = 0;
        if (valid) {
            key = kin[i];
            val = vin[i];
            d = (uint32_t)(key >> shift) & 255u;
        }
        uint64_t peers = ballot(valid);
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            const bool bit = (d >> b) & 1u;
            const uint64_t m = ballot(valid && bit);
            peers &= bit ? m : ~m;
        }
        const uint32_t rank = __popcll(peers & lt);
        if (valid && rank == 0) wc[w][d] = __popcll(peers);
        __syncthreads();
        if (valid) {
            uint32_t pre = 0;
            for (int ww = 0; ww < w; ++ww) pre += wc[ww][d];
            const uint32_t pos = run[d] + pre + rank;
            kout[pos] = key;
            vout[pos] = val;
        }
        __syncthreads();
        uint32_t tot = 0;
        for (int ww = 0; ww < RS_T / WAVE; ++ww) { tot += wc[ww][t]; wc[ww][t] = 0; }
        run[t] += tot;
        __syncthreads();
    }
}

// Multi-block exclusive scan: per-tile sums, one scan of the sums, per-tile scan.
constexpr int SC_ITEMS = 16;
constexpr int SC_TILE = BT * SC_ITEMS;

__global__ __launch_bounds__(BT) void k_tile_sums(const uint32_t* __restrict__ in, int64_t n, uint32_t* sums) {
    __shared__ uint32_t red[BT / WAVE];
    const int64_t base = (int64_t)blockIdx.x * SC_TILE;
    uint32_t s = 0;
    for (int it = 0; it < SC_ITEMS; ++it) {
        const int64_t i = base + it * BT + threadIdx.x;
        if (i < n) s += in[i];
    }
    s = wave_sum_u32(s);
    if (lane_id() == 0) red[threadIdx.x / WAVE] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t t = 0;
        for (int w = 0; w < BT / WAVE; ++w) t += red[w];
        sums[blockIdx.x] = t;
    }
}

__global__ __launch_bounds__(BT) void k_tile_scan(const uint32_t* __restrict__ in, uint32_t* __restrict__ out,
                                                  int64_t n, const uint32_t* __restrict__ offs) {
    __shared__ uint32_t part[BT];
    const int64_t base = (int64_t)blockIdx.x * SC_TILE + (int64_t)threadIdx.x * SC_ITEMS;
    uint32_t v[SC_ITEMS];
    uint32_t s = 0;
    for (int it = 0; it < SC_ITEMS; ++it) {
        const int64_t i = base + it;
        v[it] = i < n ? in[i] : 0u;
        s += v[it];
    }
    part[threadIdx.x] = s;
    __syncthreads();
    for (int d = 1; d < BT; d <<= 1) {
        const uint32_t t = threadIdx.x >= (unsigned)d ? part[threadIdx.x - d] : 0u;
        __syncthreads();
        part[threadIdx.x] += t;
        __syncthreads();
    }
    uint32_t run = offs[blockIdx.x] + part[threadIdx.x] - s;
    for (int it = 0; it < SC_ITEMS; ++it) {
        const int64_t i = base + it;
        if (i < n) out[i] = run;
        run += v[it];
    }
}

__global__ __launch_bounds__(BT) void k_gather_points(const void* pts, int64_t n, int32_t f, int32_t dtype,
                                                      const uint32_t* __restrict__ perm, float* __restrict__ spts,
                                                      int32_t* __restrict__ sid) {
    for (int64_t r = blockIdx.x * (int64_t)BT + threadIdx.x; r < n; r += (int64_t)gridDim.x * BT) {
        const uint32_t src = perm[r];
        for (int j = 0; j < f; ++j) spts[r * f + j] = load_coord(pts, (int64_t)src * f + j, dtype);
        sid[r] = (int32_t)src;
    }
}

// Points back in their original row order: out[sid[r]] = spts[r].
__global__ __launch_bounds__(BT) void k_unsort_points(const float* __restrict__ spts, const int32_t* __restrict__ sid,
                                                      int64_t n, int32_t f, float* __restrict__ out) {
    for (int64_t r = blockIdx.x * (int64_t)BT + threadIdx.x; r < n; r += (int64_t)gridDim.x * BT)
        for (int j = 0; j < f; ++j) out[(int64_t)sid[r] * f + j] = spts[r * f + j];
}

// Points as float32 (bf16 widened exactly).
__global__ __launch_bounds__(BT) void k_widen_points(const void* pts, int64_t count, int32_t dtype, float* __restrict__ out) {
    for (int64_t i = blockIdx.x * (int64_t)BT + threadIdx.x; i < count; i += (int64_t)gridDim.x * BT)
        out[i] = load_coord(pts, i, dtype);
}

// bf16 round to nearest, ties to even, of a finite float.
__device__ __forceinline__ uint16_t bf16_rne(float x) {
    const uint32_t u = __float_as_uint(x);
    return (uint16_t)((u + 0x7fffu + ((u >> 16) & 1u)) >> 16);
}

// Screen record of every point (cell order): x' = fl32(x - c0), hi = bf16(x'),
// lo = bf16(x' - hi), dimensions f..sp-1 zero; xn = |x'|^2 (FP64 sum, rounded).
__global__ __launch_bounds__(BT) void k_screen_records(IndexView iv, uint16_t* __restrict__ rec,
                                                       float* __restrict__ xn) {
    const int f = iv.f, sp = iv.sp;
    for (int64_t r = blockIdx.x * (int64_t)BT + threadIdx.x; r < iv.n; r += (int64_t)gridDim.x * BT) {
        double nn = 0.0;
        uint16_t* out = rec + r * 2 * sp;
        for (int j = 0; j < sp; ++j) {
            uint16_t h = 0, l = 0;
            if (j < f) {
                const float xp = iv.spts[r * f + j] - iv.c0[j];
                h = bf16_rne(xp);
                l = bf16_rne(xp - __uint_as_float((uint32_t)h << 16));
                nn += (double)xp * (double)xp;
            }
            out[j] = h;
            out[sp + j] = l;
        }
        xn[r] = (float)nn;
    }
}

// cell_start[L] = first position whose key is >= L, for L in [0, box_cells].
__global__ __launch_bounds__(BT) void k_dense_cell_start(const uint64_t* __restrict__ keys, int64_t n,
                                                         int64_t box_cells, uint32_t* __restrict__ cs) {
    for (int64_t L = blockIdx.x * (int64_t)BT + threadIdx.x; L <= box_cells; L += (int64_t)gridDim.x * BT) {
        int64_t lo = 0, hi = n;
        while (lo < hi) {
            int64_t mid = (lo + hi) >> 1;
            if (keys[mid] < (uint64_t)L) lo = mid + 1;
            else hi = mid;
        }
        cs[L] = (uint32_t)lo;
    }
}

// Hash table of the occupied cells: every slot free, then each cell claims the
// first free slot of its probe sequence (keys are distinct, and the table has
// more slots than cells, so every insertion ends).
__global__ __launch_bounds__(BT) void k_hash_clear(uint64_t* __restrict__ hkeys, int64_t cap) {
    for (int64_t i = blockIdx.x * (int64_t)BT + threadIdx.x; i < cap; i += (int64_t)gridDim.x * BT)
        hkeys[i] = HASH_EMPTY;
}

__global__ __launch_bounds__(BT) void k_hash_insert(const uint64_t* __restrict__ skeys,
                                                    const uint32_t* __restrict__ cell_first, int64_t ncell,
                                                    uint64_t* hkeys, uint32_t* __restrict__ hvals, uint64_t mask) {
    for (int64_t c = blockIdx.x * (int64_t)BT + threadIdx.x; c < ncell; c += (int64_t)gridDim.x * BT) {
        const uint64_t key = skeys[cell_first[c]];
        uint64_t h = hash_slot(key, mask);
        for (uint64_t i = 0; i <= mask; ++i) {
            const unsigned long long prev = atomicCAS((unsigned long long*)&hkeys[h], (unsigned long long)HASH_EMPTY,
                                                      (unsigned long long)key);
            if (prev == HASH_EMPTY) {
                hvals[h] = (uint32_t)c;
                break;
            }
            h = (h + 1) & mask;
        }
    }
}

// stats[0] += non-empty cells, stats[1] = max(points in one cell).
__global__ __launch_bounds__(BT) void k_dense_cell_stats(const uint32_t* __restrict__ cs, int64_t box_cells,
                                                         int64_t* stats) {
    int64_t cnt = 0, mx = 0;
    for (int64_t L = blockIdx.x * (int64_t)BT + threadIdx.x; L < box_cells; L += (int64_t)gridDim.x * BT) {
        const int64_t occ = (int64_t)cs[L + 1] - (int64_t)cs[L];
        if (occ > 0) { cnt += 1; mx = max(mx, occ); }
    }
    for (int d = 1; d < WAVE; d <<= 1) {
        cnt += __shfl_xor(cnt, d, WAVE);
        mx = max(mx, (int64_t)__shfl_xor(mx, d, WAVE));
    }
    if (lane_id() == 0) {
        atomicAdd((unsigned long long*)&stats[0], (unsigned long long)cnt);
        atomicMax((unsigned long long*)&stats[1], (unsigned long long)mx);
    }
}

int grid_for(int64_t work, int threads, int cap = 65536) {
    int64_t g = (work + threads - 1) / threads;
    if (g < 1) g = 1;
    if (g > cap) g = cap;
    return (int)g;
}

}  // namespace

hipError_t launch_cells_minmax(const void* pts, int64_t n, int32_t f, int32_t dtype, const float* a,
                               const float* o, int32_t* d_minmax, int32_t* d_flags, hipStream_t s) {
    hipLaunchKernelGGL(k_cells_minmax, dim3(grid_for(n, BT, 4096)), dim3(BT), 0, s, pts, n, f, dtype, a, o,
                       d_minmax, d_flags);
    return launch_status();
}

hipError_t launch_dense_keys(const void* pts, int64_t n, int32_t f, int32_t dtype, const IndexView& iv,
                             uint64_t* keys, uint32_t* vals, hipStream_t s) {
    (void)f;
    hipLaunchKernelGGL(k_dense_keys, dim3(grid_for(n, BT)), dim3(BT), 0, s, pts, n, dtype, iv, keys, vals);
    return launch_status();
}

size_t radix_sort_temp_bytes(int64_t n) {
    const int64_t nblocks = (n + RS_TILE - 1) / RS_TILE;
    return (size_t)(256 * nblocks) * sizeof(uint32_t);
}

hipError_t radix_sort_pairs(uint64_t* keys, uint32_t* vals, uint64_t* keys_alt, uint32_t* vals_alt, int64_t n,
                            int nbits, void* temp, bool* result_in_alt, hipStream_t s) {
    const int nblocks = (int)((n + RS_TILE - 1) / RS_TILE);
    uint32_t* counts = (uint32_t*)temp;
    uint64_t *ki = keys, *ko = keys_alt;
    uint32_t *vi = vals, *vo = vals_alt;
    bool alt = false;
    for (int shift = 0; shift < nbits; shift += 8) {
        hipLaunchKernelGGL(k_radix_hist, dim3(nblocks), dim3(RS_T), 0, s, ki, n, shift, counts, nblocks);
        hipLaunchKernelGGL(k_exclusive_scan_u32, dim3(1), dim3(SCAN_T), 0, s, counts, (int64_t)256 * nblocks);
        hipLaunchKernelGGL(k_radix_scatter, dim3(nblocks), dim3(RS_T), 0, s, ki, vi, ko, vo, n, shift, counts,
                           nblocks);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        uint64_t* tk = ki; ki = ko; ko = tk;
        uint32_t* tv = vi; vi = vo; vo = tv;
        alt = !alt;
    }
    *result_in_alt = alt;
    return hipSuccess;
}

size_t exclusive_scan_temp_bytes(int64_t n) {
    return (size_t)((n + SC_TILE - 1) / SC_TILE + 1) * sizeof(uint32_t);
}

hipError_t exclusive_scan_u32(const uint32_t* in, uint32_t* out, int64_t n, void* temp, hipStream_t s) {
    const int nb = (int)((n + SC_TILE - 1) / SC_TILE);
    uint32_t* sums = (uint32_t*)temp;
    hipLaunchKernelGGL(k_tile_sums, dim3(nb), dim3(BT), 0, s, in, n, sums);
    hipLaunchKernelGGL(k_exclusive_scan_u32, dim3(1), dim3(SCAN_T), 0, s, sums, (int64_t)nb);
    hipLaunchKernelGGL(k_tile_scan, dim3(nb), dim3(BT), 0, s, in, out, n, sums);
    return launch_status();
}

hipError_t launch_gather_points(const void* pts, int64_t n, int32_t f, int32_t dtype, const uint32_t* perm,
                                float* spts, int32_t* sid, hipStream_t s) {
    hipLaunchKernelGGL(k_gather_points, dim3(grid_for(n, BT)), dim3(BT), 0, s, pts, n, f, dtype, perm, spts, sid);
    return launch_status();
}

hipError_t launch_unsort_points(const float* spts, const int32_t* sid, int64_t n, int32_t f, float* out, hipStream_t s) {
    hipLaunchKernelGGL(k_unsort_points, dim3(grid_for(n, BT)), dim3(BT), 0, s, spts, sid, n, f, out);
    return launch_status();
}

hipError_t launch_widen_points(const void* pts, int64_t count, int32_t dtype, float* out, hipStream_t s) {
    hipLaunchKernelGGL(k_widen_points, dim3(grid_for(count, BT)), dim3(BT), 0, s, pts, count, dtype, out);
    return launch_status();
}

hipError_t launch_screen_records(const IndexView& iv, uint16_t* rec, float* xn, hipStream_t s) {
    hipLaunchKernelGGL(k_screen_records, dim3(grid_for(iv.n, BT)), dim3(BT), 0, s, iv, rec, xn);
    return launch_status();
}

hipError_t launch_hash_build(const uint64_t* sorted_keys, const uint32_t* cell_first, int64_t ncell, uint64_t* hkeys,
                             uint32_t* hvals, uint64_t mask, hipStream_t s) {
    const int64_t cap = (int64_t)mask + 1;
    hipLaunchKernelGGL(k_hash_clear, dim3(grid_for(cap, BT)), dim3(BT), 0, s, hkeys, cap);
    hipLaunchKernelGGL(k_hash_insert, dim3(grid_for(ncell, BT)), dim3(BT), 0, s, sorted_keys, cell_first, ncell, hkeys,
                       hvals, mask);
    return launch_status();
}

hipError_t launch_dense_cell_start(const uint64_t* sorted_keys, int64_t n, int64_t box_cells, uint32_t* cell_start,
                                   hipStream_t s) {
    hipLaunchKernelGGL(k_dense_cell_start, dim3(grid_for(box_cells + 1, BT)), dim3(BT), 0, s, sorted_keys, n,
                       box_cells, cell_start);
    return launch_status();
}

// An insert's merge (Algorithm 1 appends every new point to its cell): the index's
// points, in cell order with ascending keys `okeys`, and the new points, sorted by key
// (`nkeys`, ties in row order, `nperm` their rows), into one cell order.  A new point
// follows the points already in its cell (their row ids are smaller), which is the
// order a build of all the points gives.  Each element finds its place with a binary
// search in the other list.
__global__ __launch_bounds__(BT) void k_merge_points(const uint64_t* __restrict__ okeys, const float* __restrict__ opts,
                                                     const int32_t* __restrict__ osid, int64_t n,
                                                     const uint64_t* __restrict__ nkeys,
                                                     const uint32_t* __restrict__ nperm, const float* __restrict__ npts,
                                                     int64_t nn, int32_t f, float* __restrict__ mpts,
                                                     int32_t* __restrict__ msid) {
    for (int64_t i = blockIdx.x * (int64_t)BT + threadIdx.x; i < n + nn; i += (int64_t)gridDim.x * BT) {
        int64_t pos;
        const float* src;
        int32_t id;
        if (i < n) {
            // new points strictly below this key come first
            const uint64_t key = okeys[i];
            int64_t lo = 0, hi = nn;
            while (lo < hi) {
                const int64_t mid = (lo + hi) >> 1;
                if (nkeys[mid] < key) lo = mid + 1;
                else hi = mid;
            }
            pos = i + lo;
            src = opts + i * f;
            id = osid[i];
        } else {
            // the index's points at or below this key come first
            const int64_t j = i - n;
            const uint64_t key = nkeys[j];
            int64_t lo = 0, hi = n;
            while (lo < hi) {
                const int64_t mid = (lo + hi) >> 1;
                if (okeys[mid] <= key) lo = mid + 1;
                else hi = mid;
            }
            pos = j + lo;
            src = npts + (int64_t)nperm[j] * f;
            id = (int32_t)(n + nperm[j]);
        }
        for (int c = 0; c < f; ++c) mpts[pos * f + c] = src[c];
        msid[pos] = id;
    }
}

hipError_t launch_merge_points(const uint64_t* okeys, const float* opts, const int32_t* osid, int64_t n,
                               const uint64_t* nkeys, const uint32_t* nperm, const float* npts, int64_t nn, int32_t f,
                               float* mpts, int32_t* msid, hipStream_t s) {
    hipLaunchKernelGGL(k_merge_points, dim3(grid_for(n + nn, BT)), dim3(BT), 0, s, okeys, opts, osid, n, nkeys, nperm,
                       npts, nn, f, mpts, msid);
    return launch_status();
}

// The index's occupied cells in its cell order: ids and point counts per cell, and for
// every training point (original row id) the position of its cell.
__global__ void k_index_cells(const uint32_t* __restrict__ cell_first, const int32_t* __restrict__ coord,
                              const int32_t* __restrict__ sid, int64_t ncells, int32_t f, int32_t* __restrict__ out_ids,
                              int64_t* __restrict__ out_counts, int32_t* __restrict__ out_point_cell) {
    for (int64_t c = blockIdx.x * (int64_t)BT + threadIdx.x; c < ncells; c += (int64_t)gridDim.x * BT) {
        const uint32_t b = cell_first[c], e = cell_first[c + 1];
        if (out_ids)
            for (int j = 0; j < f; ++j) out_ids[c * f + j] = coord[c * f + j];
        if (out_counts) out_counts[c] = (int64_t)(e - b);
        if (out_point_cell)
            for (uint32_t p = b; p < e; ++p) out_point_cell[sid[p]] = (int32_t)c;
    }
}

hipError_t launch_index_cells(const IndexView& iv, int32_t* out_ids, int64_t* out_counts, int32_t* out_point_cell,
                              hipStream_t s) {
    if (iv.num_cells == 0) return hipSuccess;
    hipLaunchKernelGGL(k_index_cells, dim3(grid_for(iv.num_cells, BT, 4096)), dim3(BT), 0, s, iv.cell_first,
                       iv.cell_coord, iv.sid, iv.num_cells, iv.f, out_ids, out_counts, out_point_cell);
    return launch_status();
}

hipError_t launch_cell_stats(const uint32_t* cell_start, int64_t ncells, int64_t* d_stats, hipStream_t s) {
    hipLaunchKernelGGL(k_dense_cell_stats, dim3(grid_for(ncells, BT, 4096)), dim3(BT), 0, s, cell_start, ncells, d_stats);
    return launch_status();
}

}  // namespace ghn
