// Host side of the libghn C ABI: argument checks, device memory of an index,
// the build sequence, and dispatch of predict kernels.
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "ghn_internal.h"

struct ghn_index {
    ghn::IndexView view;
    ghn_index_info info;
    std::vector<void*> allocs;
};

namespace {

thread_local std::string g_err;

ghn_status fail(ghn_status st, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
ghn_status fail(ghn_status st, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return st;
}

ghn_status hip_fail(hipError_t e, const char* what) {
    return fail(GHN_E_HIP, "%s: %s", what, hipGetErrorString(e));
}

// Device allocations released together unless kept.
struct DevPool {
    std::vector<void*> ptrs;
    ~DevPool() {
        for (void* p : ptrs) (void)hipFree(p);
    }
    hipError_t alloc(void** p, size_t bytes) {
        *p = nullptr;
        hipError_t e = hipMalloc(p, bytes ? bytes : 1);
        if (e == hipSuccess) ptrs.push_back(*p);
        return e;
    }
    void release(std::vector<void*>& to) {
        to.insert(to.end(), ptrs.begin(), ptrs.end());
        ptrs.clear();
    }
};

// Dense tables larger than this many cells are not built.
int64_t dense_limit(int64_t n) {
    int64_t lim = 16 * n;
    return lim < (int64_t(1) << 24) ? (int64_t(1) << 24) : lim;
}

}  // namespace

extern "C" {

const char* ghn_last_error(void) { return g_err.c_str(); }

ghn_status ghn_build(const void* points, int64_t n, int32_t f, int32_t dtype, const void* targets, int32_t task,
                     const float* cell_width, int32_t n_width, const float* origin, void* stream,
                     ghn_index** out) {
    using namespace ghn;
    if (!out) return fail(GHN_E_INVALID_ARG, "ghn_build: out is NULL");
    *out = nullptr;
    if (!points || !targets) return fail(GHN_E_INVALID_ARG, "ghn_build: points and targets must not be NULL");
    if (n < 1 || n >= (int64_t(1) << 31)) return fail(GHN_E_INVALID_ARG, "ghn_build: n=%lld outside [1, 2^31)", (long long)n);
    if (f < 1 || f > F_MAX) return fail(GHN_E_INVALID_ARG, "ghn_build: f=%d outside [1, %d]", f, F_MAX);
    if (dtype != GHN_F32 && dtype != GHN_BF16) return fail(GHN_E_INVALID_ARG, "ghn_build: bad dtype %d", dtype);
    if (task != GHN_CLASSIFY && task != GHN_REGRESS) return fail(GHN_E_INVALID_ARG, "ghn_build: bad task %d", task);
    if (!cell_width || (n_width != 1 && n_width != f))
        return fail(GHN_E_INVALID_ARG, "ghn_build: cell_width must hold 1 or f values (n_width=%d)", n_width);
    if (((uintptr_t)points % (dtype == GHN_BF16 ? 2 : 4)) || ((uintptr_t)targets % 4))
        return fail(GHN_E_INVALID_ARG, "ghn_build: misaligned points or targets");
    float a[F_MAX], o[F_MAX];
    for (int j = 0; j < f; ++j) {
        a[j] = cell_width[n_width == 1 ? 0 : j];
        if (!(std::isfinite(a[j]) && a[j] > 0.0f))
            return fail(GHN_E_INVALID_ARG, "ghn_build: cell width of dimension %d is %g (must be finite and > 0)", j, (double)a[j]);
        o[j] = origin ? origin[j] : 0.0f;
        if (!std::isfinite(o[j])) return fail(GHN_E_INVALID_ARG, "ghn_build: origin of dimension %d is not finite", j);
    }
    hipStream_t s = (hipStream_t)stream;
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "ghn_build: pending HIP error");

    DevPool tmp, keep;
    // 1. cell id range and data checks
    struct Small { float a[F_MAX]; float o[F_MAX]; int32_t minmax[2 * F_MAX]; int32_t flags[2]; int64_t stats[2]; };
    Small h;
    std::memset(&h, 0, sizeof h);
    std::memcpy(h.a, a, sizeof a);
    std::memcpy(h.o, o, sizeof o);
    for (int j = 0; j < F_MAX; ++j) { h.minmax[j] = INT32_MAX; h.minmax[F_MAX + j] = INT32_MIN; }
    Small* d_small = nullptr;
    if ((e = tmp.alloc((void**)&d_small, sizeof(Small))) != hipSuccess) return fail(GHN_E_NOMEM, "ghn_build: hipMalloc failed");
    if ((e = hipMemcpyAsync(d_small, &h, sizeof h, hipMemcpyHostToDevice, s)) != hipSuccess) return hip_fail(e, "ghn_build: upload");
    if ((e = launch_cells_minmax(points, n, f, dtype, d_small->a, d_small->o, d_small->minmax, d_small->flags, s)) != hipSuccess)
        return hip_fail(e, "ghn_build: cell range kernel");
    if ((e = hipMemcpyAsync(&h, d_small, sizeof h, hipMemcpyDeviceToHost, s)) != hipSuccess) return hip_fail(e, "ghn_build: readback");
    if ((e = hipStreamSynchronize(s)) != hipSuccess) return hip_fail(e, "ghn_build: sync");
    if (h.flags[0]) return fail(GHN_E_NONFINITE, "ghn_build: a training point has a NaN or infinite coordinate");
    if (h.flags[1]) return fail(GHN_E_KEY_OVERFLOW, "ghn_build: a cell id is outside (-2^27, 2^27); use a larger cell width");

    // 2. occupied box and dense-table strides
    IndexView iv;
    std::memset(&iv, 0, sizeof iv);
    iv.n = n; iv.f = f; iv.dtype = dtype; iv.task = task; iv.lookup = LOOKUP_DENSE;
    int64_t box = 1;
    bool too_big = false;
    for (int j = f - 1; j >= 0; --j) {
        iv.a[j] = a[j];
        iv.o[j] = o[j];
        iv.cmin[j] = h.minmax[j];
        iv.cmax[j] = h.minmax[F_MAX + j];
        iv.stride[j] = box;
        const int64_t wj = (int64_t)iv.cmax[j] - iv.cmin[j] + 1;
        if (box > (int64_t(1) << 40) / wj) too_big = true;
        else box *= wj;
    }
    if (too_big || box > dense_limit(n))
        return fail(GHN_E_UNSUPPORTED, "ghn_build: the occupied box holds more than %lld cells; this build only has the "
                    "dense cell table (use a larger cell width or fewer dimensions)", (long long)dense_limit(n));
    iv.box_cells = box;
    int nbits = 0;
    while (nbits < 64 && (uint64_t(1) << nbits) < (uint64_t)box) ++nbits;

    // 3. keys, sort, gather, table
    uint64_t *keys, *keys2;
    uint32_t *vals, *vals2;
    void* rtemp;
    if (tmp.alloc((void**)&keys, n * 8) || tmp.alloc((void**)&keys2, n * 8) || tmp.alloc((void**)&vals, n * 4) ||
        tmp.alloc((void**)&vals2, n * 4) || tmp.alloc(&rtemp, radix_sort_temp_bytes(n)))
        return fail(GHN_E_NOMEM, "ghn_build: out of device memory for the sort");
    float* spts;
    int32_t* sid;
    uint32_t* cs;
    void* tg;
    if (keep.alloc((void**)&spts, (size_t)n * f * 4) || keep.alloc((void**)&sid, (size_t)n * 4) ||
        keep.alloc((void**)&cs, (size_t)(box + 1) * 4) || keep.alloc(&tg, (size_t)n * 4))
        return fail(GHN_E_NOMEM, "ghn_build: out of device memory for the index");
    if ((e = launch_dense_keys(points, n, f, dtype, iv, keys, vals, s)) != hipSuccess) return hip_fail(e, "ghn_build: keys");
    bool in_alt = false;
    if ((e = radix_sort_pairs(keys, vals, keys2, vals2, n, nbits, rtemp, &in_alt, s)) != hipSuccess)
        return hip_fail(e, "ghn_build: radix sort");
    const uint64_t* skeys = in_alt ? keys2 : keys;
    const uint32_t* perm = in_alt ? vals2 : vals;
    if ((e = launch_gather_points(points, n, f, dtype, perm, spts, sid, s)) != hipSuccess) return hip_fail(e, "ghn_build: gather");
    if ((e = launch_dense_cell_start(skeys, n, box, cs, d_small->stats, s)) != hipSuccess) return hip_fail(e, "ghn_build: table");
    if ((e = hipMemcpyAsync(tg, targets, (size_t)n * 4, hipMemcpyDeviceToDevice, s)) != hipSuccess) return hip_fail(e, "ghn_build: targets");
    if ((e = hipMemcpyAsync(&h, d_small, sizeof h, hipMemcpyDeviceToHost, s)) != hipSuccess) return hip_fail(e, "ghn_build: readback");
    if ((e = hipStreamSynchronize(s)) != hipSuccess) return hip_fail(e, "ghn_build: sync");

    iv.spts = spts; iv.sid = sid; iv.cell_start = cs; iv.targets = tg;
    ghn_index* ix = new ghn_index();
    ix->view = iv;
    std::memset(&ix->info, 0, sizeof ix->info);
    ix->info.n = n; ix->info.f = f; ix->info.dtype = dtype; ix->info.task = task; ix->info.lookup = LOOKUP_DENSE;
    ix->info.num_cells = h.stats[0];
    ix->info.box_cells = box;
    ix->info.max_occupancy = h.stats[1];
    for (int j = 0; j < f; ++j) {
        ix->info.cell_min[j] = iv.cmin[j];
        ix->info.cell_max[j] = iv.cmax[j];
        ix->info.cell_width[j] = a[j];
        ix->info.origin[j] = o[j];
    }
    ix->info.device_bytes = (size_t)n * f * 4 + (size_t)n * 4 + (size_t)(box + 1) * 4 + (size_t)n * 4;
    keep.release(ix->allocs);
    *out = ix;
    return GHN_OK;
}

ghn_status ghn_index_get_info(const ghn_index* index, ghn_index_info* out) {
    if (!index || !out) return fail(GHN_E_INVALID_ARG, "ghn_index_get_info: NULL argument");
    *out = index->info;
    return GHN_OK;
}

void ghn_destroy(ghn_index* index) {
    if (!index) return;
    for (void* p : index->allocs) (void)hipFree(p);
    delete index;
}

namespace {
// Workspace of the query sort: keys, values, their alternates, radix counts.
size_t sort_ws_bytes(int64_t m) {
    auto up = [](size_t b) { return (b + 255) & ~size_t(255); };
    return 2 * up(m * 8) + 2 * up(m * 4) + up(ghn::radix_sort_temp_bytes(m));
}
bool wants_sort(int64_t m, uint32_t flags) { return m >= ghn::SORT_MIN_QUERIES && !(flags & GHN_FLAG_NO_SORT); }

// Keys + radix sort in `ws` (sort_ws_bytes(m) bytes); *order points into ws.
hipError_t sort_queries(const ghn_index* index, const float* queries, int64_t m, void* ws, uint32_t** order,
                        hipStream_t s) {
    using namespace ghn;
    auto up = [](size_t b) { return (b + 255) & ~size_t(255); };
    char* p = (char*)ws;
    uint64_t* k0 = (uint64_t*)p; p += up(m * 8);
    uint64_t* k1 = (uint64_t*)p; p += up(m * 8);
    uint32_t* v0 = (uint32_t*)p; p += up(m * 4);
    uint32_t* v1 = (uint32_t*)p; p += up(m * 4);
    hipError_t e = launch_query_keys(queries, m, index->view, QUERY_KEY_BITS, k0, v0, s);
    if (e != hipSuccess) return e;
    bool alt = false;
    e = radix_sort_pairs(k0, v0, k1, v1, m, QUERY_KEY_BITS, p, &alt, s);
    *order = alt ? v1 : v0;
    return e;
}
}  // namespace

size_t ghn_predict_workspace_bytes(const ghn_index* index, int64_t m, int32_t k, const ghn_predict_opts* opts) {
    (void)index; (void)k;
    const uint32_t flags = opts ? opts->flags : 0u;
    if (opts && opts->order) return 0;
    return wants_sort(m, flags) ? sort_ws_bytes(m) : 0;
}

size_t ghn_query_order_workspace_bytes(int64_t m) { return m > 0 ? sort_ws_bytes(m) : 0; }

ghn_status ghn_query_order(const ghn_index* index, const float* queries, int64_t m, uint32_t* out_order, void* ws,
                           size_t ws_bytes, void* stream) {
    if (!index) return fail(GHN_E_INVALID_ARG, "ghn_query_order: index is NULL");
    if (m < 0 || m >= (int64_t(1) << 32)) return fail(GHN_E_INVALID_ARG, "ghn_query_order: m=%lld outside [0, 2^32)", (long long)m);
    if (m == 0) return GHN_OK;
    if (!queries || !out_order) return fail(GHN_E_INVALID_ARG, "ghn_query_order: queries and out_order must not be NULL");
    const size_t need = sort_ws_bytes(m);
    if (!ws || ws_bytes < need)
        return fail(GHN_E_WORKSPACE, "ghn_query_order: workspace of %zu bytes needed, %zu given", need, ws ? ws_bytes : (size_t)0);
    if ((uintptr_t)ws % 256 || (uintptr_t)queries % 4 || (uintptr_t)out_order % 4)
        return fail(GHN_E_INVALID_ARG, "ghn_query_order: misaligned pointer");
    hipStream_t s = (hipStream_t)stream;
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "ghn_query_order: pending HIP error");
    uint32_t* order = nullptr;
    if ((e = sort_queries(index, queries, m, ws, &order, s)) != hipSuccess) return hip_fail(e, "ghn_query_order: sort");
    if ((e = hipMemcpyAsync(out_order, order, (size_t)m * 4, hipMemcpyDeviceToDevice, s)) != hipSuccess)
        return hip_fail(e, "ghn_query_order: copy");
    return GHN_OK;
}

ghn_status ghn_predict(const ghn_index* index, const float* queries, int64_t m, int32_t k,
                       const ghn_predict_opts* opts, int64_t* out_idx, double* out_d2, void* out_pred, void* ws,
                       size_t ws_bytes, void* stream) {
    using namespace ghn;
    (void)ws; (void)ws_bytes;
    if (!index) return fail(GHN_E_INVALID_ARG, "ghn_predict: index is NULL");
    if (m < 0) return fail(GHN_E_INVALID_ARG, "ghn_predict: m=%lld < 0", (long long)m);
    if (k < 1 || k > K_MAX) return fail(GHN_E_INVALID_ARG, "ghn_predict: k=%d outside [1, %d]", k, K_MAX);
    if (k > index->info.n) return fail(GHN_E_K_GT_N, "ghn_predict: k=%d exceeds n=%lld", k, (long long)index->info.n);
    ghn_predict_opts o = {GHN_STOP_EXACT, GHN_PREC_FP32, 0u, nullptr, nullptr, nullptr, nullptr};
    if (opts) o = *opts;
    if (o.stop != GHN_STOP_EXACT && o.stop != GHN_STOP_PAPER) return fail(GHN_E_INVALID_ARG, "ghn_predict: bad stop rule %d", o.stop);
    if (o.prec != GHN_PREC_FP32 && o.prec != GHN_PREC_BF16_MFMA) return fail(GHN_E_INVALID_ARG, "ghn_predict: bad precision %d", o.prec);
    if (o.flags & ~(GHN_FLAG_NO_PRUNE | GHN_FLAG_NO_SORT)) return fail(GHN_E_INVALID_ARG, "ghn_predict: unknown flags 0x%x", o.flags);
    if (m == 0) return GHN_OK;
    if (!queries || !out_idx || !out_pred) return fail(GHN_E_INVALID_ARG, "ghn_predict: queries, out_idx and out_pred must not be NULL");
    if (((uintptr_t)queries % 4) || ((uintptr_t)out_idx % 8) || ((uintptr_t)out_pred % 4) || ((uintptr_t)out_d2 % 8))
        return fail(GHN_E_INVALID_ARG, "ghn_predict: misaligned array");
    if (o.prec == GHN_PREC_BF16_MFMA) return fail(GHN_E_UNSUPPORTED, "ghn_predict: the bf16 matrix-core screen is not built yet");
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "ghn_predict: pending HIP error");
    PredictArgs pa;
    pa.ix = index->view;
    pa.queries = queries;
    pa.m = m;
    pa.k = k;
    pa.stop = o.stop;
    pa.flags = o.flags;
    pa.out_idx = out_idx;
    pa.out_d2 = out_d2;
    pa.out_pred = out_pred;
    pa.out_stop_layer = o.out_stop_layer;
    pa.out_cands = o.out_cands;
    pa.out_probes = o.out_probes;
    pa.order = o.order;
    hipStream_t s = (hipStream_t)stream;
    if (!o.order && wants_sort(m, o.flags)) {
        const size_t need = sort_ws_bytes(m);
        if (!ws || ws_bytes < need)
            return fail(GHN_E_WORKSPACE, "ghn_predict: workspace of %zu bytes needed, %zu given", need, ws ? ws_bytes : (size_t)0);
        if ((uintptr_t)ws % 256) return fail(GHN_E_INVALID_ARG, "ghn_predict: workspace must be 256-byte aligned");
        uint32_t* order = nullptr;
        if ((e = sort_queries(index, queries, m, ws, &order, s)) != hipSuccess) return hip_fail(e, "ghn_predict: query sort");
        pa.order = order;
    }
    if ((e = launch_predict_dense(pa, s)) != hipSuccess) return hip_fail(e, "ghn_predict: launch");
    return GHN_OK;
}

}  // extern "C"
