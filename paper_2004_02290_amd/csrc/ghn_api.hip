// Host side of the libghn C ABI: argument checks, device memory of an index,
// the build sequence, and dispatch of predict kernels.
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <memory>
#include <string>
#include <utility>
#include <vector>

#include "ghn_internal.h"

struct ghn_index {
    ghn::IndexView view;
    ghn::IndexView* view_dev;  // device copy of `view` (for batched launches)
    ghn_index_info info;
    std::vector<void*> allocs;
    int32_t want_lookup;       // the lookup asked for at build (GHN_LOOKUP_AUTO may re-choose on insert)
};

struct ghn_batch {
    ghn::BatchItem* items_dev;
    uint64_t* counter_dev;
    int32_t n_items;
    int64_t total;
    int32_t f;
    int32_t stop;
    bool any_tree;  // some item's index uses the cell tree
    bool any_dense; // some item's index uses the dense table
    // bf16 screen: one grouped launch over all items' query groups
    int32_t prec;
    int32_t kmax;
    int32_t kb;         // key bits below the item index
    int32_t key_bits;   // bits of the sort key
    void* group_ws;     // group_ws_bytes(total) bytes of the caller's workspace
    int32_t group_size; // bf16 screen: most queries per group
    int32_t tile_width; // bf16 screen: candidates per screened tile
    bool sorted;        // FP32 screen: walk the queries in spatial order (sorted by the key)
    int32_t blocks;     // grid size of the FP32 launch (0 = by the query count)
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
    ghn::log_line("error %d: %s", (int)st, buf);
    return st;
}

ghn_status hip_fail(hipError_t e, const char* what) {
    return fail(GHN_E_HIP, "%s: %s", what, hipGetErrorString(e));
}

// The device's walk fault word (GHN_WALK_SHORT).
ghn_status fault_word(uint32_t** out) {
    const hipError_t e = ghn::walk_fault_address(out);
    if (e == hipErrorInvalidDevice) return fail(GHN_E_UNSUPPORTED, "walk fault word: device index above 255");
    if (e != hipSuccess) return hip_fail(e, "walk fault word address");
    return GHN_OK;
}

// Device memory of a build: hipMalloc'd blocks released together unless kept, or
// (carve) 256-byte aligned pieces of a caller's buffer, which is never freed here.
struct DevPool {
    std::vector<void*> ptrs;
    char* base = nullptr;  // carve mode: the caller's buffer
    size_t cap = 0, used = 0;
    const char* what = nullptr;  // carve mode: name of the buffer, for errors
    DevPool() = default;
    DevPool(void* buffer, size_t bytes, const char* name) : base((char*)buffer), cap(bytes), what(name) {}
    DevPool(const DevPool&) = delete;
    DevPool& operator=(const DevPool&) = delete;
    ~DevPool() {
        for (void* p : ptrs) ghn::device_free(p);
    }
    bool carving() const { return base != nullptr; }
    hipError_t alloc(void** p, size_t bytes) {
        *p = nullptr;
        if (carving()) {
            const size_t at = (used + 255) & ~(size_t)255;
            if (at > cap || cap - at < bytes) return hipErrorOutOfMemory;
            *p = base + at;
            used = at + bytes;
            return hipSuccess;
        }
        hipError_t e = ghn::device_alloc(p, bytes);
        if (e == hipSuccess) ptrs.push_back(*p);
        return e;
    }
    void release(std::vector<void*>& to) {
        to.insert(to.end(), ptrs.begin(), ptrs.end());
        ptrs.clear();
    }
};

// Status of a failed DevPool::alloc: out of device memory, or a caller's buffer too small.
ghn_status no_memory(const DevPool& pool, const char* fn, const char* purpose) {
    if (pool.carving())
        return fail(GHN_E_WORKSPACE, "%s: the %s (%zu bytes) is too small for the %s", fn, pool.what, pool.cap, purpose);
    return fail(GHN_E_NOMEM, "%s: out of device memory for the %s", fn, purpose);
}

constexpr size_t ALIGN_SLACK = 256;  // per piece carved from a caller's buffer
inline size_t up256(size_t b) { return (b + 255) & ~(size_t)255; }

// Padded dimension of the bf16 screen records.
inline int screen_pad(int f) { return f <= 8 ? 8 : (f <= 16 ? 16 : 32); }

// Device bytes of an index of n points in f dimensions with the given lookup: exact
// for the points, targets and screen records, an upper bound (num_cells <= n) for the
// cell list, the tree and the hash table; `box` = cells of the dense table's box.
size_t index_bytes_bound(int64_t n, int f, int lookup, int64_t box) {
    const size_t un = (size_t)n;
    size_t b = 0;
    b += up256(un * f * 4) + up256(un * 4) + up256(un * 4);           // points, row ids, targets
    b += up256(un * 2 * screen_pad(f) * 2) + up256(un * 4);           // screen records and norms
    b += up256((un + 1) * 4) + up256(un * f * 4);                     // cell list: first points, ids
    const size_t nodes = un / (ghn::WAVE - 1) + ghn::TREE_LEVELS_MAX + 1;
    b += 2 * up256(nodes * f * 4);                                     // tree node boxes
    if (lookup == GHN_LOOKUP_HASH) {
        size_t cap = 64;
        while (cap < 2 * un) cap <<= 1;
        b += up256(cap * 8) + up256(cap * 4);
    }
    if (lookup == GHN_LOOKUP_DENSE) b += up256(((size_t)box + 1) * 4);
    b += up256(sizeof(ghn::IndexView));
    return b + 16 * ALIGN_SLACK;
}

// Build temporaries (bytes of the caller workspace of ghn_build_into).
struct BuildSmall { float a[ghn::F_MAX]; float o[ghn::F_MAX]; int32_t minmax[2 * ghn::F_MAX]; int32_t flags[2]; int64_t stats[2]; };
size_t build_ws_bytes(int64_t n) {
    const size_t un = (size_t)n;
    return up256(sizeof(BuildSmall)) + 2 * up256(un * 8) + 2 * up256(un * 4) + up256(ghn::radix_sort_temp_bytes(n)) +
           2 * up256(un * 4) + up256(ghn::exclusive_scan_temp_bytes(n)) + 16 * ALIGN_SLACK;
}

size_t sort_ws_bytes(int64_t m);  // workspace of the spatial query sort (defined below)

constexpr size_t BATCH_COUNTER_BYTES = 1024;  // the FP32 batch's 8 work counters, 128 bytes apart

// The ring schedule (ghn_predict_opts.ring_step, GHN_FLAG_RING_GROW) is for the EXACT rule.
bool tile_width_ok(int32_t tw) { return tw == 0 || tw == 32 || tw == 64; }

bool ring_ok(const ghn_predict_opts& o) {
    if (o.ring_step < 0 || o.ring_step > 64) return false;
    return o.stop != GHN_STOP_PAPER || (o.ring_step <= 1 && !(o.flags & GHN_FLAG_RING_GROW));
}

// Dense tables larger than this many cells are not built (linear cell indices stay 32-bit).
int64_t dense_limit(int64_t n) {
    int64_t lim = 16 * n;
    if (lim < (int64_t(1) << 24)) lim = int64_t(1) << 24;
    if (lim > (int64_t(1) << 32) - 2) lim = (int64_t(1) << 32) - 2;
    return lim;
}

}  // namespace

extern "C" {

const char* ghn_last_error(void) { return g_err.c_str(); }

size_t ghn_batch_workspace_bytes(int32_t n_items) {
    if (n_items <= 0) return 0;
    return (((size_t)n_items * sizeof(ghn::BatchItem) + 255) & ~(size_t)255) + BATCH_COUNTER_BYTES;
}

namespace {
// FP32 batches walk their queries in spatial order unless GHN_FLAG_NO_SORT is set or
// they hold fewer than SORT_MIN_QUERIES queries.
bool batch_sorts(int64_t total, uint32_t flags) { return total >= ghn::SORT_MIN_QUERIES && !(flags & GHN_FLAG_NO_SORT); }
}  // namespace

size_t ghn_batch_workspace_bytes_for(const ghn_batch_item* items, int32_t n_items, const ghn_predict_opts* opts) {
    if (n_items <= 0 || !items) return 0;
    const size_t base = ghn_batch_workspace_bytes(n_items);
    int64_t total = 0;
    for (int32_t i = 0; i < n_items; ++i) total += items[i].m > 0 ? items[i].m : 0;
    const bool bf16 = opts && opts->prec == GHN_PREC_BF16_MFMA;
    if (!bf16 && !batch_sorts(total, opts ? opts->flags : 0u)) return base;
    return base + (total > 0 ? ghn::group_ws_bytes(total) : 0);
}

ghn_status ghn_batch_prepare(const ghn_batch_item* items, int32_t n_items, const ghn_predict_opts* opts, void* ws,
                             size_t ws_bytes, void* stream, ghn_batch** out) {
    using namespace ghn;
    if (!out) return fail(GHN_E_INVALID_ARG, "ghn_batch_prepare: out is NULL");
    *out = nullptr;
    if (!items || n_items < 1) return fail(GHN_E_INVALID_ARG, "ghn_batch_prepare: no items");
    ghn_predict_opts o = {GHN_STOP_EXACT, GHN_PREC_FP32, 0u, nullptr, nullptr, nullptr, nullptr, -1, nullptr, nullptr};
    if (opts) o = *opts;
    if (o.stop != GHN_STOP_EXACT && o.stop != GHN_STOP_PAPER) return fail(GHN_E_INVALID_ARG, "ghn_batch_prepare: bad stop rule %d", o.stop);
    if (o.prec != GHN_PREC_FP32 && o.prec != GHN_PREC_BF16_MFMA) return fail(GHN_E_INVALID_ARG, "ghn_batch_prepare: bad precision %d", o.prec);
    if (o.group_levels < -1 || o.group_levels > 16) return fail(GHN_E_INVALID_ARG, "ghn_batch_prepare: group_levels=%d outside [-1, 16]", o.group_levels);
    if (o.flags & ~(GHN_FLAG_NO_PRUNE | GHN_FLAG_NO_SORT | GHN_FLAG_MEDIAN | GHN_FLAG_RING_GROW)) return fail(GHN_E_INVALID_ARG, "ghn_batch_prepare: unknown flags 0x%x", o.flags);
    if (!ring_ok(o)) return fail(GHN_E_INVALID_ARG, "ghn_batch_prepare: ring_step=%d (0..64, and 0 or 1 without GHN_FLAG_RING_GROW under the PAPER rule)", o.ring_step);
    if (o.group_size < 0 || o.group_size > 16) return fail(GHN_E_INVALID_ARG, "ghn_batch_prepare: group_size=%d outside [0, 16]", o.group_size);
    if (!tile_width_ok(o.tile_width)) return fail(GHN_E_INVALID_ARG, "ghn_batch_prepare: tile_width=%d (0, 32 or 64)", o.tile_width);
    const size_t base = ghn_batch_workspace_bytes(n_items);
    ghn_predict_opts oo = o;
    const size_t need = ghn_batch_workspace_bytes_for(items, n_items, &oo);
    if (!ws || ws_bytes < need)
        return fail(GHN_E_WORKSPACE, "ghn_batch_prepare: workspace of %zu bytes needed, %zu given", need, ws ? ws_bytes : (size_t)0);
    if ((uintptr_t)ws % 256) return fail(GHN_E_INVALID_ARG, "ghn_batch_prepare: workspace must be 256-byte aligned");
    uint32_t* faults = nullptr;
    if (const ghn_status fs = fault_word(&faults); fs != GHN_OK) return fs;
    std::vector<BatchItem> h((size_t)n_items);
    int64_t total = 0;
    int32_t f = -1;
    bool any_tree = false, any_dense = false;
    for (int32_t i = 0; i < n_items; ++i) {
        const ghn_batch_item& it = items[i];
        if (!it.index) return fail(GHN_E_INVALID_ARG, "ghn_batch_prepare: item %d has no index", i);
        if (f < 0) f = it.index->info.f;
        if (it.index->info.f != f) return fail(GHN_E_INVALID_ARG, "ghn_batch_prepare: item %d has f=%d, item 0 f=%d", i, it.index->info.f, f);
        if (it.m < 0) return fail(GHN_E_INVALID_ARG, "ghn_batch_prepare: item %d has m < 0", i);
        if (it.k < 1 || it.k > K_MAX) return fail(GHN_E_INVALID_ARG, "ghn_batch_prepare: item %d has k=%d outside [1, %d]", i, it.k, K_MAX);
        if (it.k > it.index->info.n) return fail(GHN_E_K_GT_N, "ghn_batch_prepare: item %d has k=%d > n=%lld", i, it.k, (long long)it.index->info.n);
        if ((o.flags & GHN_FLAG_MEDIAN) && it.index->info.task != GHN_REGRESS)
            return fail(GHN_E_INVALID_ARG, "ghn_batch_prepare: GHN_FLAG_MEDIAN needs regression indexes (item %d)", i);
        if (it.m > 0 && (!it.queries || !it.out_idx || !it.out_pred))
            return fail(GHN_E_INVALID_ARG, "ghn_batch_prepare: item %d has a NULL array", i);
        if (((uintptr_t)it.queries % 4) || ((uintptr_t)it.out_idx % 8) || ((uintptr_t)it.out_pred % 4) || ((uintptr_t)it.out_d2 % 8))
            return fail(GHN_E_INVALID_ARG, "ghn_batch_prepare: item %d has a misaligned array", i);
        BatchItem& b = h[(size_t)i];
        b.ix = it.index->view_dev;
        b.io.queries = it.queries;
        b.io.out_idx = it.out_idx;
        b.io.out_d2 = it.out_d2;
        b.io.out_pred = it.out_pred;
        b.io.out_stop_layer = nullptr;
        b.io.out_cands = nullptr;
        b.io.out_probes = nullptr;
        b.io.out_rerank = nullptr;
        b.io.k = it.k;
        b.io.flags = o.flags;
        b.io.ring_step = o.ring_step;
        b.io.faults = faults;
        b.first = total;
        b.m = it.m;
        total += it.m;
        if (it.m > 0 && it.index->view.lookup != LOOKUP_DENSE) any_tree = true;
        if (it.m > 0 && it.index->view.lookup == LOOKUP_DENSE) any_dense = true;
    }
    // the sort key of every item's queries (item index above kb bits, then the item's
    // Morton code of the central cell, aligned) and its group shift (bf16 groups)
    int32_t kmax = 1, kb = 0, key_bits = 1;
    const bool sorted = o.prec == GHN_PREC_FP32 && batch_sorts(total, o.flags);
    if (o.prec == GHN_PREC_BF16_MFMA || sorted) {
        int item_bits = 0;
        while ((int64_t(1) << item_bits) < (int64_t)n_items) ++item_bits;
        std::vector<int> cbits((size_t)n_items), scode((size_t)n_items), tot((size_t)n_items);
        const int levels = o.stop == GHN_STOP_PAPER ? 0 : (o.group_levels >= 0 ? o.group_levels : (f >= 12 ? 3 : 1));
        int maxc = 0;
        for (int32_t i = 0; i < n_items; ++i) {
            const IndexView& v = items[i].index->view;
            int bits[F_MAX], total = 0, maxb = 0;
            for (int j = 0; j < f; ++j) {
                const uint32_t span = (uint32_t)(v.cmax[j] - v.cmin[j]);
                bits[j] = span ? 32 - __builtin_clz(span) : 0;
                total += bits[j];
                maxb = maxb > bits[j] ? maxb : bits[j];
            }
            int sh = 0;
            for (int b = 0; b < levels && b < maxb; ++b)
                for (int j = 0; j < f; ++j) sh += bits[j] > b ? 1 : 0;
            cbits[(size_t)i] = total > 64 ? 64 : total;
            scode[(size_t)i] = total > 64 ? (sh > total - 64 ? sh - (total - 64) : 0) : sh;
            tot[(size_t)i] = total;
            if (items[i].m > 0 && cbits[(size_t)i] > maxc) maxc = cbits[(size_t)i];
            if (items[i].k > kmax) kmax = items[i].k;
        }
        kb = 64 - item_bits < maxc ? 64 - item_bits : maxc;
        key_bits = item_bits + kb > 0 ? item_bits + kb : 1;
        for (int32_t i = 0; i < n_items; ++i) {
            BatchItem& b = h[(size_t)i];
            b.kshift = kb - cbits[(size_t)i];
            b.gshift = b.kshift >= 0 ? scode[(size_t)i] + b.kshift
                                     : (scode[(size_t)i] + b.kshift > 0 ? scode[(size_t)i] + b.kshift : 0);
            b.trunc = o.stop == GHN_STOP_PAPER && (tot[(size_t)i] > cbits[(size_t)i] || b.kshift < 0) ? 1 : 0;
            b.pad = 0;
        }
    }
    hipStream_t s = (hipStream_t)stream;
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "ghn_batch_prepare: pending HIP error");
    if ((e = hipMemcpyAsync(ws, h.data(), h.size() * sizeof(BatchItem), hipMemcpyHostToDevice, s)) != hipSuccess ||
        (e = hipStreamSynchronize(s)) != hipSuccess)
        return hip_fail(e, "ghn_batch_prepare: upload");
    ghn_batch* b = new ghn_batch();
    b->items_dev = (BatchItem*)ws;
    b->counter_dev = (uint64_t*)((char*)ws + base - BATCH_COUNTER_BYTES);
    b->n_items = n_items;
    b->total = total;
    b->f = f;
    b->stop = o.stop;
    b->any_tree = any_tree;
    b->any_dense = any_dense;
    b->prec = o.prec;
    b->kmax = kmax;
    b->kb = kb;
    b->key_bits = key_bits;
    b->group_ws = (char*)ws + base;
    b->sorted = sorted;
    b->group_size = o.group_size > 0 ? o.group_size : 16;
    b->tile_width = o.tile_width > 0 ? o.tile_width : 64;
    b->blocks = 0;
    if (const char* env = std::getenv("GHN_BATCH_BLOCKS")) b->blocks = std::atoi(env) > 0 ? std::atoi(env) : 0;
    ghn::log_line("batch_prepare items=%d queries=%lld f=%d kmax=%d stop=%d prec=%d flags=0x%x sorted=%d", n_items,
                  (long long)total, f, kmax, o.stop, o.prec, o.flags, (int)sorted);
    *out = b;
    return GHN_OK;
}

ghn_status ghn_predict_batched(const ghn_batch* batch, void* stream) {
    if (!batch) return fail(GHN_E_INVALID_ARG, "ghn_predict_batched: batch is NULL");
    ghn::log_line("predict_batched items=%d queries=%lld prec=%d", batch->n_items, (long long)batch->total, batch->prec);
    if (batch->total == 0) return GHN_OK;
    if (batch->prec == GHN_PREC_BF16_MFMA) {
        const hipError_t e = ghn::run_grouped_batched(batch->items_dev, batch->n_items, batch->total, batch->f,
                                                      batch->kmax, batch->stop, batch->kb, batch->key_bits,
                                                      batch->group_size, batch->tile_width, batch->group_ws,
                                                      (hipStream_t)stream);
        if (e != hipSuccess) return hip_fail(e, "ghn_predict_batched: grouped launch");
        return GHN_OK;
    }
    const uint32_t* order = nullptr;
    hipError_t e = hipSuccess;
    if (batch->sorted && (e = ghn::batch_query_order(batch->items_dev, batch->n_items, batch->total, batch->kb,
                                                    batch->key_bits, batch->group_ws, (hipStream_t)stream,
                                                    &order)) != hipSuccess)
        return hip_fail(e, "ghn_predict_batched: query order");
    e = ghn::launch_predict_batched(batch->items_dev, batch->n_items, batch->total, batch->f, batch->stop,
                                    batch->any_tree, batch->any_dense, order, batch->blocks, batch->counter_dev,
                                    (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "ghn_predict_batched: launch");
    return GHN_OK;
}

void ghn_batch_destroy(ghn_batch* batch) { delete batch; }

ghn_status ghn_autotune(const void* points, int64_t n, int32_t f, int32_t dtype, const void* targets, int32_t task,
                        const float* queries, int64_t m, int32_t k, int32_t stop, const float* widths,
                        int32_t n_widths, ghn_tune_trial* best, ghn_tune_trial* trials, int32_t max_trials,
                        int32_t* n_trials, void* stream) {
    using namespace ghn;
    if (n_trials) *n_trials = 0;
    if (!best) return fail(GHN_E_INVALID_ARG, "ghn_autotune: best is NULL");
    if (!points || !targets || !queries) return fail(GHN_E_INVALID_ARG, "ghn_autotune: NULL array");
    if (n < 1 || f < 1 || f > F_MAX || m < 1) return fail(GHN_E_INVALID_ARG, "ghn_autotune: bad sizes");
    if (k < 1 || k > K_MAX) return fail(GHN_E_INVALID_ARG, "ghn_autotune: k=%d outside [1, %d]", k, K_MAX);
    if (k > n) return fail(GHN_E_K_GT_N, "ghn_autotune: k=%d exceeds n=%lld", k, (long long)n);
    if (stop != GHN_STOP_EXACT && stop != GHN_STOP_PAPER) return fail(GHN_E_INVALID_ARG, "ghn_autotune: bad stop rule");
    if (stop == GHN_STOP_PAPER && (!widths || n_widths != 1))
        return fail(GHN_E_INVALID_ARG, "ghn_autotune: the PAPER rule needs exactly one cell width");
    hipStream_t s = (hipStream_t)stream;
    std::vector<float> cand;
    if (widths && n_widths > 0) {
        cand.assign(widths, widths + n_widths);
    } else {
        float lo[F_MAX], hi[F_MAX];
        hipError_t e = coord_range(points, n, f, dtype, lo, hi, s);
        if (e != hipSuccess) return hip_fail(e, "ghn_autotune: coordinate range");
        double logvol = 0.0;
        for (int j = 0; j < f; ++j) {
            double r = (double)hi[j] - (double)lo[j];
            logvol += std::log(r > 1e-30 ? r : 1e-30);
        }
        const double w0 = std::exp((logvol + std::log(8.0 / (double)n)) / f);
        for (int i = -3; i <= 2; ++i) cand.push_back((float)(w0 * std::ldexp(1.0, i)));
    }
    struct Setting { int32_t prec, levels; uint32_t flags; int32_t ring, gsize, tw; };
    std::vector<Setting> settings = {{GHN_PREC_FP32, -1, GHN_FLAG_NO_SORT, 0, 0, 0}, {GHN_PREC_FP32, -1, 0u, 0, 0, 0}};
    // bf16 group and tile shapes: 16 queries x 64 candidates, 8 x 64, 16 x 32
    const int shapes[3][2] = {{16, 64}, {8, 64}, {16, 32}};
    if (stop == GHN_STOP_PAPER) {
        for (const auto& sh : shapes) settings.push_back({GHN_PREC_BF16_MFMA, 0, 0u, 0, sh[0], sh[1]});
    } else {
        // the EXACT walk's ring schedule: 2 layers a step, doubling steps until the buffer is
        // full, or both (input and spatial order)
        for (uint32_t order : {(uint32_t)GHN_FLAG_NO_SORT, 0u}) {
            settings.push_back({GHN_PREC_FP32, -1, order, 2, 0, 0});
            settings.push_back({GHN_PREC_FP32, -1, order | GHN_FLAG_RING_GROW, 1, 0, 0});
            settings.push_back({GHN_PREC_FP32, -1, order | GHN_FLAG_RING_GROW, 2, 0, 0});
        }
        // bf16: groups of 2^lv cells per dimension, in each group and tile shape
        for (const auto& sh : shapes)
            for (int lv = 0; lv <= 3; ++lv) settings.push_back({GHN_PREC_BF16_MFMA, lv, 0u, 0, sh[0], sh[1]});
    }

    // outputs and a workspace large enough for every setting
    int64_t* oi = nullptr;
    void* op = nullptr;
    void* ws = nullptr;
    size_t ws_bytes = sort_ws_bytes(m) > group_ws_bytes(m) ? sort_ws_bytes(m) : group_ws_bytes(m);
    hipEvent_t e0 = nullptr, e1 = nullptr;
    ghn_status result = GHN_OK;
    bool have_best = false;
    int32_t nt = 0;
    if (device_alloc((void**)&oi, (size_t)m * k * 8) != hipSuccess || device_alloc(&op, (size_t)m * 4) != hipSuccess ||
        device_alloc(&ws, ws_bytes) != hipSuccess || hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
        result = fail(GHN_E_NOMEM, "ghn_autotune: out of device memory");
    } else {
        for (float w : cand) {
            ghn_index* ix = nullptr;
            if (ghn_build(points, n, f, dtype, targets, task, &w, 1, nullptr, stream, &ix) != GHN_OK) {
                if (trials && nt < max_trials) trials[nt] = {w, -1, -1, -1, 0u, 0, 0, 0, -1.0};
                ++nt;
                continue;
            }
            for (const Setting& st : settings) {
                ghn_predict_opts o = {stop, st.prec, st.flags, nullptr, nullptr, nullptr, nullptr, st.levels, nullptr, nullptr,
                                      nullptr, st.ring, st.gsize, st.tw};
                double ms = -1.0;
                if (ghn_predict(ix, queries, m, k, &o, oi, nullptr, op, ws, ws_bytes, stream) == GHN_OK &&
                    hipStreamSynchronize(s) == hipSuccess) {
                    float best_ms = 1e30f;
                    for (int rep = 0; rep < 3; ++rep) {
                        float t = 0.0f;
                        (void)hipEventRecord(e0, s);
                        (void)ghn_predict(ix, queries, m, k, &o, oi, nullptr, op, ws, ws_bytes, stream);
                        (void)hipEventRecord(e1, s);
                        if (hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&t, e0, e1) != hipSuccess) break;
                        best_ms = t < best_ms ? t : best_ms;
                    }
                    if (best_ms < 1e29f) ms = best_ms;
                }
                const ghn_tune_trial tr = {w, ix->info.lookup, st.prec, st.levels, st.flags, st.ring, st.gsize, st.tw, ms};
                if (trials && nt < max_trials) trials[nt] = tr;
                ++nt;
                if (ms >= 0.0 && (!have_best || ms < best->ms)) { *best = tr; have_best = true; }
            }
            const bool tree = ix->info.lookup == GHN_LOOKUP_TREE;
            ghn_destroy(ix);
            // a grid too fine for the dense table in few dimensions: also the hash lookup
            // (FP32 walk; the grouped screen walks the tree either way)
            const ghn_build_opts ho = {GHN_LOOKUP_HASH};
            if (tree && f <= 6 && ghn_build_ex(points, n, f, dtype, targets, task, &w, 1, nullptr, &ho, stream, &ix) == GHN_OK) {
                for (const Setting& st : settings) {
                    if (st.prec != GHN_PREC_FP32) continue;
                    ghn_predict_opts o = {stop, st.prec, st.flags, nullptr, nullptr, nullptr, nullptr, st.levels, nullptr, nullptr,
                                      nullptr, st.ring, st.gsize, st.tw};
                    double ms = -1.0;
                    if (ghn_predict(ix, queries, m, k, &o, oi, nullptr, op, ws, ws_bytes, stream) == GHN_OK &&
                        hipStreamSynchronize(s) == hipSuccess) {
                        float best_ms = 1e30f;
                        for (int rep = 0; rep < 3; ++rep) {
                            float t = 0.0f;
                            (void)hipEventRecord(e0, s);
                            (void)ghn_predict(ix, queries, m, k, &o, oi, nullptr, op, ws, ws_bytes, stream);
                            (void)hipEventRecord(e1, s);
                            if (hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&t, e0, e1) != hipSuccess) break;
                            best_ms = t < best_ms ? t : best_ms;
                        }
                        if (best_ms < 1e29f) ms = best_ms;
                    }
                    const ghn_tune_trial tr = {w, GHN_LOOKUP_HASH, st.prec, st.levels, st.flags, st.ring, st.gsize, st.tw, ms};
                    if (trials && nt < max_trials) trials[nt] = tr;
                    ++nt;
                    if (ms >= 0.0 && (!have_best || ms < best->ms)) { *best = tr; have_best = true; }
                }
                ghn_destroy(ix);
            }
        }
        if (!have_best) result = fail(GHN_E_UNSUPPORTED, "ghn_autotune: no candidate setting could be built and run");
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (oi) ghn::device_free(oi);
    if (op) ghn::device_free(op);
    if (ws) ghn::device_free(ws);
    if (n_trials) *n_trials = nt;
    if (result == GHN_OK)
        log_line("autotune trials=%d best: width=%g lookup=%d prec=%d group_levels=%d flags=0x%x ring_step=%d "
                 "group_size=%d tile_width=%d ms=%.4f", nt, best->cell_width, best->lookup, best->prec, best->group_levels,
                 best->flags, best->ring_step, best->group_size, best->tile_width, best->ms);
    return result;
}

ghn_status ghn_cell_measure(const void* points, int64_t n, int32_t f, int32_t dtype, float* out_width,
                            float* out_origin, int64_t* out_splits, void* stream) {
    using namespace ghn;
    if (!points || !out_width || !out_origin || !out_splits)
        return fail(GHN_E_INVALID_ARG, "ghn_cell_measure: NULL pointer argument");
    if (n < 1 || n >= (int64_t(1) << 32)) return fail(GHN_E_INVALID_ARG, "ghn_cell_measure: n=%lld outside [1, 2^32)", (long long)n);
    if (f < 1 || f > F_MAX) return fail(GHN_E_INVALID_ARG, "ghn_cell_measure: f=%d outside [1, %d]", f, F_MAX);
    if (dtype != GHN_F32 && dtype != GHN_BF16) return fail(GHN_E_INVALID_ARG, "ghn_cell_measure: bad dtype %d", dtype);
    if ((uintptr_t)points % (dtype == GHN_F32 ? 4 : 2)) return fail(GHN_E_INVALID_ARG, "ghn_cell_measure: misaligned points");
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "ghn_cell_measure: pending HIP error");
    bool nonfinite = false;
    e = measure_cells(points, n, f, dtype, out_width, out_origin, out_splits, &nonfinite, (hipStream_t)stream);
    if (e == hipErrorOutOfMemory) return fail(GHN_E_NOMEM, "ghn_cell_measure: out of device memory");
    if (e != hipSuccess) return hip_fail(e, "ghn_cell_measure");
    if (nonfinite) return fail(GHN_E_NONFINITE, "ghn_cell_measure: a coordinate is NaN or infinite");
    return GHN_OK;
}

ghn_status ghn_build(const void* points, int64_t n, int32_t f, int32_t dtype, const void* targets, int32_t task,
                     const float* cell_width, int32_t n_width, const float* origin, void* stream,
                     ghn_index** out) {
    return ghn_build_ex(points, n, f, dtype, targets, task, cell_width, n_width, origin, nullptr, stream, out);
}

}  // extern "C"

namespace {

// Points already in cell order (an insert's merge): FP32 coordinates and row ids.
// The build then computes their keys, which come out ascending, and skips the sort.
struct Presorted {
    const float* spts;
    const int32_t* sid;
};

// The build (Eq. 1, Algorithm 1).  Temporaries come from `tmp`, the index's memory
// from `keep` (hipMalloc'd, or carved from caller buffers).  With `size_only` set,
// only the cell range is computed and *size_only receives the index's device bytes
// (index_bytes_bound for the lookup the build would use); nothing is kept.  With
// `pre` the points come in cell order; only the dense-table and hash lookups take
// them (the tree's Morton order differs): GHN_E_UNSUPPORTED otherwise.
ghn_status build_impl(const void* points, int64_t n, int32_t f, int32_t dtype, const void* targets, int32_t task,
                      const float* cell_width, int32_t n_width, const float* origin, const ghn_build_opts* bopts,
                      void* stream, DevPool& tmp, DevPool& keep, size_t* size_only, ghn_index** out,
                      const Presorted* pre = nullptr) {
    using namespace ghn;
    if (!out && !size_only) return fail(GHN_E_INVALID_ARG, "ghn_build: out is NULL");
    if (out) *out = nullptr;
    if (!points || (!targets && !size_only)) return fail(GHN_E_INVALID_ARG, "ghn_build: points and targets must not be NULL");
    if (n < 1 || n >= (int64_t(1) << 31)) return fail(GHN_E_INVALID_ARG, "ghn_build: n=%lld outside [1, 2^31)", (long long)n);
    if (f < 1 || f > F_MAX) return fail(GHN_E_INVALID_ARG, "ghn_build: f=%d outside [1, %d]", f, F_MAX);
    if (dtype != GHN_F32 && dtype != GHN_BF16) return fail(GHN_E_INVALID_ARG, "ghn_build: bad dtype %d", dtype);
    if (task != GHN_CLASSIFY && task != GHN_REGRESS) return fail(GHN_E_INVALID_ARG, "ghn_build: bad task %d", task);
    if (!cell_width || (n_width != 1 && n_width != f))
        return fail(GHN_E_INVALID_ARG, "ghn_build: cell_width must hold 1 or f values (n_width=%d)", n_width);
    if (((uintptr_t)points % (dtype == GHN_BF16 ? 2 : 4)) || ((uintptr_t)targets % 4))
        return fail(GHN_E_INVALID_ARG, "ghn_build: misaligned points or targets");
    const int32_t want_lookup = bopts ? bopts->lookup : GHN_LOOKUP_AUTO;
    if (want_lookup != GHN_LOOKUP_AUTO && want_lookup != GHN_LOOKUP_DENSE && want_lookup != GHN_LOOKUP_TREE &&
        want_lookup != GHN_LOOKUP_HASH)
        return fail(GHN_E_INVALID_ARG, "ghn_build: bad lookup %d", want_lookup);
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

    // 1. cell id range and data checks
    typedef BuildSmall Small;
    Small h;
    std::memset(&h, 0, sizeof h);
    std::memcpy(h.a, a, sizeof a);
    std::memcpy(h.o, o, sizeof o);
    for (int j = 0; j < F_MAX; ++j) { h.minmax[j] = INT32_MAX; h.minmax[F_MAX + j] = INT32_MIN; }
    Small* d_small = nullptr;
    if ((e = tmp.alloc((void**)&d_small, sizeof(Small))) != hipSuccess) return no_memory(tmp, "ghn_build", "cell range");
    if ((e = hipMemcpyAsync(d_small, &h, sizeof h, hipMemcpyHostToDevice, s)) != hipSuccess) return hip_fail(e, "ghn_build: upload");
    if ((e = launch_cells_minmax(pre ? (const void*)pre->spts : points, n, f, pre ? (int32_t)GHN_F32 : dtype, d_small->a,
                                 d_small->o, d_small->minmax, d_small->flags, s)) != hipSuccess)
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
    uint64_t hbox = 1;  // the same product for the hash keys, up to 2^62
    bool hash_too_big = false;
    for (int j = f - 1; j >= 0; --j) {
        iv.a[j] = a[j];
        iv.ainv[j] = 1.0 / (double)a[j];
        iv.o[j] = o[j];
        iv.cmin[j] = h.minmax[j];
        iv.cmax[j] = h.minmax[F_MAX + j];
        iv.stride[j] = (uint32_t)box;
        const int64_t wj = (int64_t)iv.cmax[j] - iv.cmin[j] + 1;
        if (box > (int64_t(1) << 40) / wj) too_big = true;
        else box *= wj;
        iv.hstride[j] = hbox;
        if (hbox > (uint64_t(1) << 62) / (uint64_t)wj) hash_too_big = true;
        else hbox *= (uint64_t)wj;
    }
    const bool dense_ok = !too_big && box <= dense_limit(n);
    const int32_t lookup = want_lookup == GHN_LOOKUP_AUTO ? (dense_ok ? GHN_LOOKUP_DENSE : GHN_LOOKUP_TREE) : want_lookup;
    if (lookup == GHN_LOOKUP_DENSE && !dense_ok)
        return fail(GHN_E_UNSUPPORTED, "ghn_build: the occupied box holds more than %lld cells, too many for the dense "
                    "table (use the tree lookup or a larger cell width)", (long long)dense_limit(n));
    if (lookup == GHN_LOOKUP_HASH && hash_too_big)
        return fail(GHN_E_KEY_OVERFLOW, "ghn_build: the occupied box holds more than 2^62 cells, too many for the "
                    "hash keys (use the tree lookup or a larger cell width)");
    iv.lookup = lookup;
    if (pre && lookup == GHN_LOOKUP_TREE)
        return fail(GHN_E_UNSUPPORTED, "ghn_build: points in cell order need the dense table or the hash lookup");
    const size_t need = index_bytes_bound(n, f, lookup, box);
    if (size_only) {
        *size_only = need;
        return GHN_OK;
    }
    if (keep.carving() && keep.cap < need)
        return fail(GHN_E_WORKSPACE, "ghn_build: index storage of %zu bytes needed (ghn_index_bytes_for), %zu given",
                    need, keep.cap);
    // memory the library allocates for the index is one block of that size, carved like
    // caller storage: one allocation, and one release when the index goes
    std::unique_ptr<DevPool> block_pool;
    DevPool* kp = &keep;
    if (!keep.carving()) {
        void* block = nullptr;
        if (keep.alloc(&block, need)) return no_memory(keep, "ghn_build", "index");
        block_pool.reset(new DevPool(block, need, "index block"));
        kp = block_pool.get();
    }
    int nbits = 0;
    if (lookup == GHN_LOOKUP_DENSE) {
        iv.box_cells = box;
        while (nbits < 64 && (uint64_t(1) << nbits) < (uint64_t)box) ++nbits;
    } else if (lookup == GHN_LOOKUP_HASH) {
        iv.box_cells = (int64_t)hbox;
        while (nbits < 64 && (uint64_t(1) << nbits) < hbox) ++nbits;
    } else {
        iv.box_cells = too_big ? -1 : box;
        for (int j = 0; j < f; ++j) {
            const uint32_t span = (uint32_t)(iv.cmax[j] - iv.cmin[j]);
            nbits += span ? 32 - __builtin_clz(span) : 0;
        }
    }

    // 3. keys, sort, gather
    uint64_t *keys, *keys2;
    uint32_t *vals, *vals2;
    void* rtemp;
    if (tmp.alloc((void**)&keys, n * 8) || tmp.alloc((void**)&keys2, n * 8) || tmp.alloc((void**)&vals, n * 4) ||
        tmp.alloc((void**)&vals2, n * 4) || tmp.alloc(&rtemp, radix_sort_temp_bytes(n)))
        return no_memory(tmp, "ghn_build", "sort");
    float* spts;
    int32_t* sid;
    void* tg;
    if (kp->alloc((void**)&spts, (size_t)n * f * 4) || kp->alloc((void**)&sid, (size_t)n * 4) ||
        kp->alloc(&tg, (size_t)n * 4))
        return no_memory(*kp, "ghn_build", "index");
    const uint64_t* skeys = nullptr;
    const uint32_t* perm = nullptr;
    if (pre) {
        // row-major keys (last dimension fastest) of points in cell order are ascending
        if ((e = launch_dense_keys(pre->spts, n, f, GHN_F32, iv, keys, vals, s)) != hipSuccess)
            return hip_fail(e, "ghn_build: keys");
        skeys = keys;
    } else if (lookup == GHN_LOOKUP_DENSE || lookup == GHN_LOOKUP_HASH || nbits <= 64) {
        e = lookup != GHN_LOOKUP_TREE ? launch_dense_keys(points, n, f, dtype, iv, keys, vals, s)
                                       : launch_morton_keys(points, n, dtype, iv, nbits, 0, nullptr, keys, vals, s);
        if (e != hipSuccess) return hip_fail(e, "ghn_build: keys");
        bool in_alt = false;
        if ((e = radix_sort_pairs(keys, vals, keys2, vals2, n, nbits, rtemp, &in_alt, s)) != hipSuccess)
            return hip_fail(e, "ghn_build: radix sort");
        skeys = in_alt ? keys2 : keys;
        perm = in_alt ? vals2 : vals;
    } else {
        // wide Morton codes: stable LSD sort one 64-bit word at a time, least significant
        // word first, each pass recomputing its word in the order of the previous pass
        uint64_t *ka = keys, *kb = keys2;
        uint32_t *va = vals, *vb = vals2;
        const int nw = (nbits + 63) / 64;
        for (int w = nw - 1; w >= 0; --w) {
            const int wbits = w == 0 ? nbits - 64 * (nw - 1) : 64;
            if ((e = launch_morton_keys(points, n, dtype, iv, nbits, w, perm, ka, va, s)) != hipSuccess)
                return hip_fail(e, "ghn_build: keys");
            bool in_alt = false;
            if ((e = radix_sort_pairs(ka, va, kb, vb, n, wbits, rtemp, &in_alt, s)) != hipSuccess)
                return hip_fail(e, "ghn_build: radix sort");
            if (in_alt) { std::swap(ka, kb); std::swap(va, vb); }
            perm = va;  // the sorted order; the next word is written to the other buffers
            std::swap(ka, kb);
            std::swap(va, vb);
        }
    }
    if (pre) {
        if ((e = hipMemcpyAsync(spts, pre->spts, (size_t)n * f * 4, hipMemcpyDeviceToDevice, s)) != hipSuccess ||
            (e = hipMemcpyAsync(sid, pre->sid, (size_t)n * 4, hipMemcpyDeviceToDevice, s)) != hipSuccess)
            return hip_fail(e, "ghn_build: points in cell order");
    } else if ((e = launch_gather_points(points, n, f, dtype, perm, spts, sid, s)) != hipSuccess) {
        return hip_fail(e, "ghn_build: gather");
    }
    if ((e = hipMemcpyAsync(tg, targets, (size_t)n * 4, hipMemcpyDeviceToDevice, s)) != hipSuccess) return hip_fail(e, "ghn_build: targets");
    iv.spts = spts; iv.sid = sid; iv.targets = tg;

    // bf16 screen records, centred on the occupied box
    iv.sp = screen_pad(f);
    for (int j = 0; j < F_MAX; ++j) iv.c0[j] = 0.0f;
    for (int j = 0; j < f; ++j)
        iv.c0[j] = (float)((double)o[j] + ((double)iv.cmin[j] + (double)iv.cmax[j] + 1.0) * 0.5 * (double)a[j]);
    uint16_t* srec;
    float* sxn;
    if (kp->alloc((void**)&srec, (size_t)n * 2 * iv.sp * 2) || kp->alloc((void**)&sxn, (size_t)n * 4))
        return no_memory(*kp, "ghn_build", "screen records");
    if ((e = launch_screen_records(iv, srec, sxn, s)) != hipSuccess) return hip_fail(e, "ghn_build: screen records");
    iv.srec = srec;
    iv.sxn = sxn;

    // 4. occupied cells (every lookup): heads of equal-key runs, their ranks, first
    //    points and ids, then the bounding-box levels above them
    uint32_t *heads, *rank;
    void* stemp;
    if (tmp.alloc((void**)&heads, n * 4) || tmp.alloc((void**)&rank, n * 4) ||
        tmp.alloc(&stemp, exclusive_scan_temp_bytes(n)))
        return no_memory(tmp, "ghn_build", "cell list");
    e = skeys ? launch_cell_heads(skeys, n, heads, s) : launch_cell_heads_ids(iv, n, heads, s);
    if (e != hipSuccess) return hip_fail(e, "ghn_build: heads");
    if ((e = exclusive_scan_u32(heads, rank, n, stemp, s)) != hipSuccess) return hip_fail(e, "ghn_build: scan");
    uint32_t last[2] = {0, 0};
    if ((e = hipMemcpyAsync(&last[0], rank + n - 1, 4, hipMemcpyDeviceToHost, s)) != hipSuccess ||
        (e = hipMemcpyAsync(&last[1], heads + n - 1, 4, hipMemcpyDeviceToHost, s)) != hipSuccess ||
        (e = hipStreamSynchronize(s)) != hipSuccess)
        return hip_fail(e, "ghn_build: cell count");
    const int64_t ncell = (int64_t)last[0] + last[1];
    uint32_t* cf;
    int32_t* coord;
    if (kp->alloc((void**)&cf, (size_t)(ncell + 1) * 4) || kp->alloc((void**)&coord, (size_t)ncell * f * 4))
        return no_memory(*kp, "ghn_build", "cell list");
    if ((e = launch_cell_list(heads, rank, n, iv, cf, coord, s)) != hipSuccess) return hip_fail(e, "ghn_build: cell list");
    const uint32_t n32 = (uint32_t)n;
    if ((e = hipMemcpyAsync(cf + ncell, &n32, 4, hipMemcpyHostToDevice, s)) != hipSuccess) return hip_fail(e, "ghn_build: cell end");
    int64_t count[TREE_LEVELS_MAX] = {0};
    int64_t off[TREE_LEVELS_MAX] = {0};
    count[0] = ncell;
    int top = 0;
    int64_t total = 0;
    while (count[top] > WAVE) {
        if (top + 1 >= TREE_LEVELS_MAX) return fail(GHN_E_UNSUPPORTED, "ghn_build: too many cells for the tree");
        count[top + 1] = (count[top] + WAVE - 1) / WAVE;
        off[top + 1] = total;
        total += count[top + 1];
        ++top;
    }
    int32_t *nlo = nullptr, *nhi = nullptr;
    if (total > 0 && (kp->alloc((void**)&nlo, (size_t)total * f * 4) || kp->alloc((void**)&nhi, (size_t)total * f * 4)))
        return no_memory(*kp, "ghn_build", "tree");
    for (int L = 1; L <= top; ++L) {
        const int32_t* clo = L == 1 ? coord : nlo + off[L - 1] * f;
        const int32_t* chi = L == 1 ? coord : nhi + off[L - 1] * f;
        if ((e = launch_tree_level(clo, chi, count[L - 1], f, nlo + off[L] * f, nhi + off[L] * f, count[L], s)) != hipSuccess)
            return hip_fail(e, "ghn_build: tree level");
    }
    if ((e = launch_cell_stats(cf, ncell, d_small->stats, s)) != hipSuccess) return hip_fail(e, "ghn_build: stats");
    iv.cell_first = cf;
    iv.num_cells = ncell;
    iv.cell_coord = coord;
    iv.tree_levels = top;
    for (int L = 0; L < TREE_LEVELS_MAX; ++L) { iv.tree_count[L] = count[L]; iv.tree_off[L] = off[L]; }
    iv.node_lo = nlo;
    iv.node_hi = nhi;
    size_t table_bytes = (size_t)(ncell + 1) * 4 + (size_t)ncell * f * 4 + (size_t)total * f * 8;
    // 5. dense table over the whole box, or the hash table of the occupied cells
    iv.cell_start = cf;
    if (lookup == GHN_LOOKUP_HASH) {
        uint64_t cap = 64;
        while (cap < 2 * (uint64_t)ncell) cap <<= 1;
        uint64_t* hk;
        uint32_t* hv;
        if (kp->alloc((void**)&hk, (size_t)cap * 8) || kp->alloc((void**)&hv, (size_t)cap * 4))
            return no_memory(*kp, "ghn_build", "hash table");
        if ((e = launch_hash_build(skeys, cf, ncell, hk, hv, cap - 1, s)) != hipSuccess) return hip_fail(e, "ghn_build: hash table");
        iv.hkeys = hk;
        iv.hvals = hv;
        iv.hmask = cap - 1;
        table_bytes += (size_t)cap * 12;
    }
    if (lookup == GHN_LOOKUP_DENSE) {
        uint32_t* cs;
        if (kp->alloc((void**)&cs, (size_t)(box + 1) * 4)) return no_memory(*kp, "ghn_build", "table");
        if ((e = launch_dense_cell_start(skeys, n, box, cs, s)) != hipSuccess) return hip_fail(e, "ghn_build: table");
        iv.cell_start = cs;
        table_bytes += (size_t)(box + 1) * 4;
    }
    if ((e = hipMemcpyAsync(&h, d_small, sizeof h, hipMemcpyDeviceToHost, s)) != hipSuccess) return hip_fail(e, "ghn_build: readback");
    if ((e = hipStreamSynchronize(s)) != hipSuccess) return hip_fail(e, "ghn_build: sync");

    ghn::IndexView* ivd;
    if (kp->alloc((void**)&ivd, sizeof(IndexView))) return no_memory(*kp, "ghn_build", "index view");
    if ((e = hipMemcpyAsync(ivd, &iv, sizeof iv, hipMemcpyHostToDevice, s)) != hipSuccess ||
        (e = hipStreamSynchronize(s)) != hipSuccess)
        return hip_fail(e, "ghn_build: index view upload");
    ghn_index* ix = new ghn_index();
    ix->view = iv;
    ix->view_dev = ivd;
    std::memset(&ix->info, 0, sizeof ix->info);
    ix->info.n = n; ix->info.f = f; ix->info.dtype = dtype; ix->info.task = task; ix->info.lookup = lookup;
    ix->info.num_cells = iv.num_cells;
    ix->info.box_cells = iv.box_cells;
    ix->info.max_occupancy = h.stats[1];
    for (int j = 0; j < f; ++j) {
        ix->info.cell_min[j] = iv.cmin[j];
        ix->info.cell_max[j] = iv.cmax[j];
        ix->info.cell_width[j] = a[j];
        ix->info.origin[j] = o[j];
    }
    ix->info.device_bytes = (size_t)n * f * 4 + (size_t)n * 4 + (size_t)n * 4 + table_bytes +
                           (size_t)n * 2 * iv.sp * 2 + (size_t)n * 4;
    keep.release(ix->allocs);
    ix->want_lookup = want_lookup;
    ix->info.device_bytes = keep.carving() ? keep.used : need;
    ghn::log_line("build n=%lld f=%d dtype=%d task=%d lookup=%d cells=%lld max_occupancy=%lld device_bytes=%zu%s",
                  (long long)n, f, dtype, task, lookup, (long long)iv.num_cells, (long long)h.stats[1],
                  ix->info.device_bytes, keep.carving() ? " (caller storage)" : "");
    *out = ix;
    return GHN_OK;
}

// Checks of ghn_build_into's caller buffers.
ghn_status check_buffer(const char* fn, const char* name, const void* p, size_t bytes, size_t need) {
    if (!p || bytes < need)
        return fail(GHN_E_WORKSPACE, "%s: %s of %zu bytes needed, %zu given", fn, name, need, p ? bytes : (size_t)0);
    if ((uintptr_t)p % 256) return fail(GHN_E_INVALID_ARG, "%s: %s must be 256-byte aligned", fn, name);
    return GHN_OK;
}

}  // namespace

extern "C" {

ghn_status ghn_build_ex(const void* points, int64_t n, int32_t f, int32_t dtype, const void* targets, int32_t task,
                        const float* cell_width, int32_t n_width, const float* origin, const ghn_build_opts* bopts,
                        void* stream, ghn_index** out) {
    DevPool tmp, keep;
    return build_impl(points, n, f, dtype, targets, task, cell_width, n_width, origin, bopts, stream, tmp, keep,
                      nullptr, out);
}

size_t ghn_build_workspace_bytes(int64_t n, int32_t f) {
    (void)f;
    return n < 1 ? 0 : build_ws_bytes(n);
}

size_t ghn_index_bytes(int64_t n, int32_t f, int32_t dtype, int32_t task) {
    (void)dtype; (void)task;
    if (n < 1 || f < 1 || f > ghn::F_MAX) return 0;
    const size_t dense = index_bytes_bound(n, f, GHN_LOOKUP_DENSE, dense_limit(n));
    const size_t hash = index_bytes_bound(n, f, GHN_LOOKUP_HASH, 0);
    return dense > hash ? dense : hash;
}

ghn_status ghn_index_bytes_for(const void* points, int64_t n, int32_t f, int32_t dtype, int32_t task,
                               const float* cell_width, int32_t n_width, const float* origin,
                               const ghn_build_opts* opts, void* ws, size_t ws_bytes, void* stream,
                               size_t* out_bytes) {
    if (!out_bytes) return fail(GHN_E_INVALID_ARG, "ghn_index_bytes_for: out_bytes is NULL");
    *out_bytes = 0;
    if (n < 1) return fail(GHN_E_INVALID_ARG, "ghn_index_bytes_for: n=%lld < 1", (long long)n);
    ghn_status st = check_buffer("ghn_index_bytes_for", "workspace", ws, ws_bytes, up256(sizeof(BuildSmall)));
    if (st != GHN_OK) return st;
    DevPool tmp(ws, ws_bytes, "workspace"), keep(nullptr, 0, "index storage");
    return build_impl(points, n, f, dtype, nullptr, task, cell_width, n_width, origin, opts, stream, tmp, keep,
                      out_bytes, nullptr);
}

ghn_status ghn_build_into(const void* points, int64_t n, int32_t f, int32_t dtype, const void* targets, int32_t task,
                          const float* cell_width, int32_t n_width, const float* origin, const ghn_build_opts* opts,
                          void* index_storage, size_t index_bytes, void* ws, size_t ws_bytes, void* stream,
                          ghn_index** out) {
    if (!out) return fail(GHN_E_INVALID_ARG, "ghn_build_into: out is NULL");
    *out = nullptr;
    if (n < 1 || n >= (int64_t(1) << 31)) return fail(GHN_E_INVALID_ARG, "ghn_build_into: n=%lld outside [1, 2^31)", (long long)n);
    ghn_status st = check_buffer("ghn_build_into", "workspace", ws, ws_bytes, build_ws_bytes(n));
    if (st != GHN_OK) return st;
    if ((st = check_buffer("ghn_build_into", "index storage", index_storage, index_bytes, 1)) != GHN_OK) return st;
    DevPool tmp(ws, ws_bytes, "workspace"), keep(index_storage, index_bytes, "index storage");
    return build_impl(points, n, f, dtype, targets, task, cell_width, n_width, origin, opts, stream, tmp, keep,
                      nullptr, out);
}


ghn_status ghn_index_cells(const ghn_index* index, int32_t* out_ids, int64_t* out_counts, int32_t* out_point_cell,
                           void* stream) {
    if (!index) return fail(GHN_E_INVALID_ARG, "ghn_index_cells: index is NULL");
    if (((uintptr_t)out_ids % 4) || ((uintptr_t)out_counts % 8) || ((uintptr_t)out_point_cell % 4))
        return fail(GHN_E_INVALID_ARG, "ghn_index_cells: misaligned array");
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "ghn_index_cells: pending HIP error");
    if ((e = ghn::launch_index_cells(index->view, out_ids, out_counts, out_point_cell, (hipStream_t)stream)) != hipSuccess)
        return hip_fail(e, "ghn_index_cells");
    return GHN_OK;
}

ghn_status ghn_index_get_info(const ghn_index* index, ghn_index_info* out) {
    if (!index || !out) return fail(GHN_E_INVALID_ARG, "ghn_index_get_info: NULL argument");
    *out = index->info;
    return GHN_OK;
}

void ghn_destroy(ghn_index* index) {
    if (!index) return;
    for (void* p : index->allocs) ghn::device_free(p);
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
    if (m <= 0) return 0;
    if (opts && opts->prec == GHN_PREC_BF16_MFMA) return ghn::group_ws_bytes(m);
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

// ghn_predict and ghn_bruteforce (brute: every point is screened, no grid walk).
static ghn_status predict_common(const ghn_index* index, const float* queries, int64_t m, int32_t k,
                                 const ghn_predict_opts* opts, int64_t* out_idx, double* out_d2, void* out_pred,
                                 void* ws, size_t ws_bytes, void* stream, bool brute) {
    using namespace ghn;
    (void)ws; (void)ws_bytes;
    if (!index) return fail(GHN_E_INVALID_ARG, "ghn_predict: index is NULL");
    if (m < 0) return fail(GHN_E_INVALID_ARG, "ghn_predict: m=%lld < 0", (long long)m);
    if (k < 1 || k > K_MAX) return fail(GHN_E_INVALID_ARG, "ghn_predict: k=%d outside [1, %d]", k, K_MAX);
    if (k > index->info.n) return fail(GHN_E_K_GT_N, "ghn_predict: k=%d exceeds n=%lld", k, (long long)index->info.n);
    ghn_predict_opts o = {GHN_STOP_EXACT, GHN_PREC_FP32, 0u, nullptr, nullptr, nullptr, nullptr, -1, nullptr, nullptr};
    if (opts) o = *opts;
    if (o.stop != GHN_STOP_EXACT && o.stop != GHN_STOP_PAPER) return fail(GHN_E_INVALID_ARG, "ghn_predict: bad stop rule %d", o.stop);
    if (o.prec != GHN_PREC_FP32 && o.prec != GHN_PREC_BF16_MFMA) return fail(GHN_E_INVALID_ARG, "ghn_predict: bad precision %d", o.prec);
    if (o.flags & ~(GHN_FLAG_NO_PRUNE | GHN_FLAG_NO_SORT | GHN_FLAG_MEDIAN | GHN_FLAG_RING_GROW)) return fail(GHN_E_INVALID_ARG, "ghn_predict: unknown flags 0x%x", o.flags);
    if (!ring_ok(o)) return fail(GHN_E_INVALID_ARG, "ghn_predict: ring_step=%d (0..64, and 0 or 1 without GHN_FLAG_RING_GROW under the PAPER rule)", o.ring_step);
    if (o.group_size < 0 || o.group_size > 16) return fail(GHN_E_INVALID_ARG, "ghn_predict: group_size=%d outside [0, 16]", o.group_size);
    if (!tile_width_ok(o.tile_width)) return fail(GHN_E_INVALID_ARG, "ghn_predict: tile_width=%d (0, 32 or 64)", o.tile_width);
    if ((o.flags & GHN_FLAG_MEDIAN) && index->info.task != GHN_REGRESS)
        return fail(GHN_E_INVALID_ARG, "ghn_predict: GHN_FLAG_MEDIAN needs a regression index");
    if (m == 0) return GHN_OK;
    if (m >= (int64_t(1) << 32)) return fail(GHN_E_INVALID_ARG, "ghn_predict: m=%lld too large for one call (< 2^32)", (long long)m);
    if (!queries || !out_idx || !out_pred) return fail(GHN_E_INVALID_ARG, "ghn_predict: queries, out_idx and out_pred must not be NULL");
    if (((uintptr_t)queries % 4) || ((uintptr_t)out_idx % 8) || ((uintptr_t)out_pred % 4) || ((uintptr_t)out_d2 % 8))
        return fail(GHN_E_INVALID_ARG, "ghn_predict: misaligned array");
    if (o.group_levels < -1 || o.group_levels > 16) return fail(GHN_E_INVALID_ARG, "ghn_predict: group_levels=%d outside [-1, 16]", o.group_levels);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "ghn_predict: pending HIP error");
    PredictArgs pa;
    pa.ix = index->view;
    pa.io.queries = queries;
    pa.m = m;
    pa.io.k = k;
    pa.stop = o.stop;
    pa.io.flags = o.flags;
    pa.io.ring_step = o.ring_step;
    pa.io.out_idx = out_idx;
    pa.io.out_d2 = out_d2;
    pa.io.out_pred = out_pred;
    pa.io.out_stop_layer = o.out_stop_layer;
    pa.io.out_cands = o.out_cands;
    pa.io.out_probes = o.out_probes;
    pa.io.out_rerank = o.out_rerank;
    pa.io.pad = 0;
    if (const ghn_status fs = fault_word(&pa.io.faults); fs != GHN_OK) return fs;
    pa.order = o.order;
    hipStream_t s = (hipStream_t)stream;
    if (brute) {
        o.prec = GHN_PREC_BF16_MFMA;
        pa.order = nullptr;
    }
    if (log_enabled())
        log_line("%s m=%lld k=%d stop=%d prec=%d flags=0x%x ring_step=%d group_levels=%d group_size=%d tile_width=%d "
                 "lookup=%d order=%s",
                 brute ? "bruteforce" : "predict", (long long)m, k, o.stop, o.prec, o.flags, o.ring_step,
                 o.group_levels, o.group_size, o.tile_width, index->view.lookup,
                 o.order ? "given" : (o.prec == GHN_PREC_FP32 && wants_sort(m, o.flags)) ? "sorted" : "input");
    if (o.prec == GHN_PREC_BF16_MFMA) {
        const size_t need = group_ws_bytes(m);
        if (!ws || ws_bytes < need)
            return fail(GHN_E_WORKSPACE, "ghn_predict: workspace of %zu bytes needed, %zu given", need, ws ? ws_bytes : (size_t)0);
        if ((uintptr_t)ws % 256) return fail(GHN_E_INVALID_ARG, "ghn_predict: workspace must be 256-byte aligned");
        const int levels = brute ? 32 : o.stop == GHN_STOP_PAPER ? 0 : (o.group_levels >= 0 ? o.group_levels : (index->info.f >= 12 ? 3 : 1));
        int bits = 0;
        const int gsize = o.group_size > 0 ? o.group_size : 16;
        const int tw = o.tile_width > 0 ? o.tile_width : 64;
        e = run_grouped(pa, levels, gsize, tw, ws, s, &bits, (hipEvent_t)o.walk_event_begin, (hipEvent_t)o.walk_event_end,
                        brute);
        if (e != hipSuccess) return hip_fail(e, "ghn_predict: grouped walk");
        return GHN_OK;
    }
    if (!o.order && wants_sort(m, o.flags)) {
        const size_t need = sort_ws_bytes(m);
        if (!ws || ws_bytes < need)
            return fail(GHN_E_WORKSPACE, "ghn_predict: workspace of %zu bytes needed, %zu given", need, ws ? ws_bytes : (size_t)0);
        if ((uintptr_t)ws % 256) return fail(GHN_E_INVALID_ARG, "ghn_predict: workspace must be 256-byte aligned");
        uint32_t* order = nullptr;
        if ((e = sort_queries(index, queries, m, ws, &order, s)) != hipSuccess) return hip_fail(e, "ghn_predict: query sort");
        pa.order = order;
    }
    if (o.walk_event_begin && (e = hipEventRecord((hipEvent_t)o.walk_event_begin, s)) != hipSuccess)
        return hip_fail(e, "ghn_predict: walk_event_begin");
    e = index->view.lookup == LOOKUP_TREE ? launch_predict_tree(pa, s) : launch_predict_dense(pa, s);
    if (e != hipSuccess) return hip_fail(e, "ghn_predict: launch");
    if (o.walk_event_end && (e = hipEventRecord((hipEvent_t)o.walk_event_end, s)) != hipSuccess)
        return hip_fail(e, "ghn_predict: walk_event_end");
    return GHN_OK;
}

ghn_status ghn_predict(const ghn_index* index, const float* queries, int64_t m, int32_t k,
                       const ghn_predict_opts* opts, int64_t* out_idx, double* out_d2, void* out_pred, void* ws,
                       size_t ws_bytes, void* stream) {
    return predict_common(index, queries, m, k, opts, out_idx, out_d2, out_pred, ws, ws_bytes, stream, false);
}

ghn_status ghn_bruteforce(const ghn_index* index, const float* queries, int64_t m, int32_t k,
                          const ghn_predict_opts* opts, int64_t* out_idx, double* out_d2, void* out_pred, void* ws,
                          size_t ws_bytes, void* stream) {
    return predict_common(index, queries, m, k, opts, out_idx, out_d2, out_pred, ws, ws_bytes, stream, true);
}

}  // extern "C"

namespace {

// Workspace of ghn_predict_noalloc: the device's static array (ghn_arrays.hip).
ghn_status scratch_address(void** out) {
    const hipError_t e = ghn::noalloc_workspace(out);
    if (e == hipErrorInvalidDevice) return fail(GHN_E_UNSUPPORTED, "ghn_predict_noalloc: device index above 255");
    if (e != hipSuccess) return hip_fail(e, "ghn_predict_noalloc: address of the workspace array");
    return GHN_OK;
}

}  // namespace

extern "C" {

ghn_status ghn_walk_faults(uint32_t* out_flags, int clear, void* stream) {
    if (!out_flags) return fail(GHN_E_INVALID_ARG, "ghn_walk_faults: out_flags is NULL");
    uint32_t* w = nullptr;
    if (const ghn_status fs = fault_word(&w); fs != GHN_OK) return fs;
    hipStream_t s = (hipStream_t)stream;
    uint32_t v = 0;
    hipError_t e = hipMemcpyAsync(&v, w, sizeof v, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess && clear) e = ghn::launch_clear_word(w, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(e, "ghn_walk_faults");
    *out_flags = v;
    return GHN_OK;
}

ghn_status ghn_predict_noalloc(const ghn_index* index, const float* queries, int64_t m, int32_t k,
                               const ghn_predict_opts* opts, int64_t* out_idx, double* out_d2, void* out_pred,
                               void* stream) {
    if (!index) return fail(GHN_E_INVALID_ARG, "ghn_predict_noalloc: index is NULL");
    if (m < 0 || m >= (int64_t(1) << 32))
        return fail(GHN_E_INVALID_ARG, "ghn_predict_noalloc: m=%lld outside [0, 2^32)", (long long)m);
    const size_t need = ghn_predict_workspace_bytes(index, m, k, opts);
    if (need > GHN_NOALLOC_WS_BYTES)
        return fail(GHN_E_WORKSPACE, "ghn_predict_noalloc: m=%lld needs %zu bytes of workspace, more than the %zu "
                    "bytes the library holds (use ghn_predict with a caller workspace)", (long long)m, need,
                    (size_t)GHN_NOALLOC_WS_BYTES);
    void* ws = nullptr;
    if (need > 0) {
        const ghn_status st = scratch_address(&ws);
        if (st != GHN_OK) return st;
    }
    return predict_common(index, queries, m, k, opts, out_idx, out_d2, out_pred, ws, ws ? GHN_NOALLOC_WS_BYTES : 0,
                          stream, false);
}

ghn_status ghn_screen_error(const ghn_index* index, const float* queries, int64_t m, int64_t sample,
                            float* out_abs, float* out_rel, void* stream) {
    using namespace ghn;
    if (!index || !queries || !out_abs || !out_rel) return fail(GHN_E_INVALID_ARG, "ghn_screen_error: NULL argument");
    if (m < 0) return fail(GHN_E_INVALID_ARG, "ghn_screen_error: m < 0");
    if (sample < 1 || sample >= (int64_t(1) << 31))
        return fail(GHN_E_INVALID_ARG, "ghn_screen_error: sample=%lld outside [1, 2^31)", (long long)sample);
    if (((uintptr_t)queries % 4) || ((uintptr_t)out_abs % 4) || ((uintptr_t)out_rel % 4))
        return fail(GHN_E_INVALID_ARG, "ghn_screen_error: misaligned array");
    if (m == 0) return GHN_OK;
    const int64_t nsamp = sample < index->info.n ? sample : index->info.n;
    hipError_t e = launch_screen_error(index->view, queries, m, (uint32_t)nsamp, out_abs, out_rel, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "ghn_screen_error");
    return GHN_OK;
}

// ---- persistence and insertion: the model is the training data plus the grid
// parameters (Section III-A); the grid is rebuilt from them, deterministically.

namespace {

struct SavedHeader {
    char magic[8];           // "GHNIDX01"
    uint32_t version;        // 1
    int32_t f;
    int64_t n;
    int32_t dtype;           // ghn_dtype of the points as built
    int32_t task;
    int32_t want_lookup;
    int32_t reserved;
    float width[GHN_F_MAX];
    float origin[GHN_F_MAX];
};
static_assert(sizeof(SavedHeader) == 296, "saved index header layout");

// Points of an index in their original row order (float32, n x f) into `out`.
hipError_t original_points(const ghn_index* index, float* out, hipStream_t s) {
    return ghn::launch_unsort_points(index->view.spts, index->view.sid, index->info.n, index->info.f, out, s);
}

// Insert by merge (Algorithm 1 appends each new point to its cell): only the new points
// are sorted; they are merged into the index's cell order, and the cell structures are
// rebuilt from the merged order.  The result equals a build of all the points.  Needs
// an index in row-major cell order (dense table or hash) and an enlarged index that
// takes one of those lookups with keys in 64 bits: GHN_E_UNSUPPORTED otherwise, with
// nothing changed (the caller then rebuilds from all the points).
ghn_status insert_merge(const ghn_index* index, const void* points, int64_t nn, int32_t dtype, const void* targets,
                        hipStream_t s, ghn_index** fresh) {
    using namespace ghn;
    *fresh = nullptr;
    const IndexView& iv = index->view;
    if (iv.lookup == LOOKUP_TREE) return fail(GHN_E_UNSUPPORTED, "ghn_insert: the tree index is in Morton order");
    const int64_t n = index->info.n, total = n + nn;
    const int32_t f = index->info.f;
    hipError_t e;
    // one device block for the merge's temporaries and the build's (one allocation and
    // one release instead of one per array)
    const size_t un = (size_t)n, unn = (size_t)nn, ut = (size_t)total;
    const size_t merge_bytes = up256(sizeof(BuildSmall)) + up256(un * 8) + up256(un * 4) + 2 * up256(unn * 8) +
                               2 * up256(unn * 4) + up256(radix_sort_temp_bytes(nn)) + up256(unn * f * 4) +
                               up256(ut * f * 4) + 2 * up256(ut * 4) + 16 * ALIGN_SLACK;
    const size_t build_bytes = build_ws_bytes(total);
    DevPool block;
    void* base = nullptr;
    if (block.alloc(&base, merge_bytes + build_bytes)) return no_memory(block, "ghn_insert", "merge workspace");
    DevPool tmp(base, merge_bytes, "merge workspace");
    // 1. cell range of the new points
    BuildSmall h;
    std::memset(&h, 0, sizeof h);
    for (int j = 0; j < f; ++j) { h.a[j] = index->info.cell_width[j]; h.o[j] = index->info.origin[j]; }
    for (int j = 0; j < F_MAX; ++j) { h.minmax[j] = INT32_MAX; h.minmax[F_MAX + j] = INT32_MIN; }
    BuildSmall* d_small = nullptr;
    if (tmp.alloc((void**)&d_small, sizeof h)) return no_memory(tmp, "ghn_insert", "cell range");
    if ((e = hipMemcpyAsync(d_small, &h, sizeof h, hipMemcpyHostToDevice, s)) != hipSuccess ||
        (e = launch_cells_minmax(points, nn, f, dtype, d_small->a, d_small->o, d_small->minmax, d_small->flags, s)) !=
            hipSuccess ||
        (e = hipMemcpyAsync(&h, d_small, sizeof h, hipMemcpyDeviceToHost, s)) != hipSuccess ||
        (e = hipStreamSynchronize(s)) != hipSuccess)
        return hip_fail(e, "ghn_insert: cell range");
    if (h.flags[0]) return fail(GHN_E_NONFINITE, "ghn_insert: a new point has a NaN or infinite coordinate");
    if (h.flags[1]) return fail(GHN_E_KEY_OVERFLOW, "ghn_insert: a cell id is outside (-2^27, 2^27)");
    // 2. row-major keys over the box of all the points (last dimension fastest)
    IndexView mv = iv;
    mv.lookup = LOOKUP_HASH;  // the keys kernel takes the 64-bit strides
    uint64_t box = 1;
    for (int j = f - 1; j >= 0; --j) {
        mv.cmin[j] = std::min(iv.cmin[j], h.minmax[j]);
        mv.cmax[j] = std::max(iv.cmax[j], h.minmax[F_MAX + j]);
        mv.hstride[j] = box;
        const uint64_t w = (uint64_t)((int64_t)mv.cmax[j] - mv.cmin[j] + 1);
        if (box > (uint64_t(1) << 62) / w) return fail(GHN_E_UNSUPPORTED, "ghn_insert: keys wider than 64 bits");
        box *= w;
    }
    int nbits = 0;
    while (nbits < 64 && (uint64_t(1) << nbits) < box) ++nbits;
    // 3. keys of the index's points (ascending) and of the new points (sorted), merge
    uint64_t *okeys, *nk, *nk2;
    uint32_t *ovals, *nv, *nv2;
    void* rtemp;
    float *npts, *mpts;
    int32_t* msid;
    void* mtg;
    if (tmp.alloc((void**)&okeys, (size_t)n * 8) || tmp.alloc((void**)&ovals, (size_t)n * 4) ||
        tmp.alloc((void**)&nk, (size_t)nn * 8) || tmp.alloc((void**)&nk2, (size_t)nn * 8) ||
        tmp.alloc((void**)&nv, (size_t)nn * 4) || tmp.alloc((void**)&nv2, (size_t)nn * 4) ||
        tmp.alloc(&rtemp, radix_sort_temp_bytes(nn)) || tmp.alloc((void**)&npts, (size_t)nn * f * 4) ||
        tmp.alloc((void**)&mpts, (size_t)total * f * 4) || tmp.alloc((void**)&msid, (size_t)total * 4) ||
        tmp.alloc(&mtg, (size_t)total * 4))
        return no_memory(tmp, "ghn_insert", "merge");
    bool alt = false;
    if ((e = launch_dense_keys(iv.spts, n, f, GHN_F32, mv, okeys, ovals, s)) != hipSuccess ||
        (e = launch_dense_keys(points, nn, f, dtype, mv, nk, nv, s)) != hipSuccess ||
        (e = radix_sort_pairs(nk, nv, nk2, nv2, nn, nbits, rtemp, &alt, s)) != hipSuccess ||
        (e = launch_widen_points(points, nn * f, dtype, npts, s)) != hipSuccess ||
        (e = launch_merge_points(okeys, iv.spts, iv.sid, n, alt ? nk2 : nk, alt ? nv2 : nv, npts, nn, f, mpts, msid,
                                 s)) != hipSuccess ||
        (e = hipMemcpyAsync(mtg, iv.targets, (size_t)n * 4, hipMemcpyDeviceToDevice, s)) != hipSuccess ||
        (e = hipMemcpyAsync((char*)mtg + (size_t)n * 4, targets, (size_t)nn * 4, hipMemcpyDeviceToDevice, s)) !=
            hipSuccess)
        return hip_fail(e, "ghn_insert: merge");
    // 4. the cell structures of the merged order
    const Presorted pre = {mpts, msid};
    const ghn_build_opts bo = {index->want_lookup};
    DevPool btmp((char*)base + merge_bytes, build_bytes, "build workspace"), keep;
    return build_impl(mpts, total, f, GHN_F32, mtg, index->info.task, index->info.cell_width, f, index->info.origin,
                      &bo, s, btmp, keep, nullptr, fresh, &pre);
}

// Replace the contents of `dst` by those of `src` (which is consumed).
void adopt(ghn_index* dst, ghn_index* src) {
    for (void* p : dst->allocs) ghn::device_free(p);
    *dst = *src;
    src->allocs.clear();
    delete src;
}

}  // namespace

size_t ghn_index_save_bytes(const ghn_index* index) {
    if (!index) return 0;
    return sizeof(SavedHeader) + (size_t)index->info.n * index->info.f * 4 + (size_t)index->info.n * 4;
}

ghn_status ghn_index_save(const ghn_index* index, void* buffer, size_t bytes, void* stream) {
    using namespace ghn;
    if (!index || !buffer) return fail(GHN_E_INVALID_ARG, "ghn_index_save: NULL argument");
    const size_t need = ghn_index_save_bytes(index);
    if (bytes < need) return fail(GHN_E_WORKSPACE, "ghn_index_save: %zu bytes needed, %zu given", need, bytes);
    const int64_t n = index->info.n;
    const int32_t f = index->info.f;
    SavedHeader h;
    std::memset(&h, 0, sizeof h);
    std::memcpy(h.magic, "GHNIDX01", 8);
    h.version = 1;
    h.f = f;
    h.n = n;
    h.dtype = index->info.dtype;
    h.task = index->info.task;
    h.want_lookup = index->want_lookup;
    for (int j = 0; j < f; ++j) { h.width[j] = index->info.cell_width[j]; h.origin[j] = index->info.origin[j]; }
    hipStream_t s = (hipStream_t)stream;
    DevPool tmp;
    float* pts = nullptr;
    if (tmp.alloc((void**)&pts, (size_t)n * f * 4)) return fail(GHN_E_NOMEM, "ghn_index_save: out of device memory");
    char* out = (char*)buffer;
    std::memcpy(out, &h, sizeof h);
    hipError_t e;
    if ((e = original_points(index, pts, s)) != hipSuccess ||
        (e = hipMemcpyAsync(out + sizeof h, pts, (size_t)n * f * 4, hipMemcpyDeviceToHost, s)) != hipSuccess ||
        (e = hipMemcpyAsync(out + sizeof h + (size_t)n * f * 4, index->view.targets, (size_t)n * 4,
                            hipMemcpyDeviceToHost, s)) != hipSuccess ||
        (e = hipStreamSynchronize(s)) != hipSuccess)
        return hip_fail(e, "ghn_index_save");
    return GHN_OK;
}

ghn_status ghn_index_load(const void* buffer, size_t bytes, void* stream, ghn_index** out) {
    using namespace ghn;
    if (!out) return fail(GHN_E_INVALID_ARG, "ghn_index_load: out is NULL");
    *out = nullptr;
    if (!buffer || bytes < sizeof(SavedHeader)) return fail(GHN_E_INVALID_ARG, "ghn_index_load: buffer too small");
    SavedHeader h;
    std::memcpy(&h, buffer, sizeof h);
    if (std::memcmp(h.magic, "GHNIDX01", 8) != 0 || h.version != 1)
        return fail(GHN_E_INVALID_ARG, "ghn_index_load: not a saved index (bad magic or version)");
    if (h.f < 1 || h.f > GHN_F_MAX || h.n < 1 || h.n >= (int64_t(1) << 31))
        return fail(GHN_E_INVALID_ARG, "ghn_index_load: corrupt header (n=%lld, f=%d)", (long long)h.n, h.f);
    const size_t need = sizeof h + (size_t)h.n * h.f * 4 + (size_t)h.n * 4;
    if (bytes < need) return fail(GHN_E_INVALID_ARG, "ghn_index_load: %zu bytes needed, %zu given", need, bytes);
    hipStream_t s = (hipStream_t)stream;
    DevPool tmp;
    void *pts = nullptr, *tg = nullptr;
    if (tmp.alloc(&pts, (size_t)h.n * h.f * 4) || tmp.alloc(&tg, (size_t)h.n * 4))
        return fail(GHN_E_NOMEM, "ghn_index_load: out of device memory");
    const char* in = (const char*)buffer;
    hipError_t e;
    if ((e = hipMemcpyAsync(pts, in + sizeof h, (size_t)h.n * h.f * 4, hipMemcpyHostToDevice, s)) != hipSuccess ||
        (e = hipMemcpyAsync(tg, in + sizeof h + (size_t)h.n * h.f * 4, (size_t)h.n * 4, hipMemcpyHostToDevice, s)) !=
            hipSuccess)
        return hip_fail(e, "ghn_index_load: upload");
    ghn_build_opts bo = {h.want_lookup};
    ghn_status st = ghn_build_ex(pts, h.n, h.f, GHN_F32, tg, h.task, h.width, h.f, h.origin, &bo, stream, out);
    if (st != GHN_OK) return st;
    (*out)->info.dtype = h.dtype;
    return GHN_OK;
}

ghn_status ghn_insert(ghn_index* index, const void* points, int64_t n_new, int32_t dtype, const void* targets,
                      void* stream) {
    using namespace ghn;
    if (!index) return fail(GHN_E_INVALID_ARG, "ghn_insert: index is NULL");
    if (n_new < 0) return fail(GHN_E_INVALID_ARG, "ghn_insert: n_new < 0");
    if (n_new == 0) return GHN_OK;
    if (index->allocs.empty())
        return fail(GHN_E_UNSUPPORTED, "ghn_insert: the index lives in caller storage; build the enlarged index with "
                    "ghn_build_into");
    if (!points || !targets) return fail(GHN_E_INVALID_ARG, "ghn_insert: points and targets must not be NULL");
    if (dtype != GHN_F32 && dtype != GHN_BF16) return fail(GHN_E_INVALID_ARG, "ghn_insert: bad dtype %d", dtype);
    if (((uintptr_t)points % (dtype == GHN_BF16 ? 2 : 4)) || ((uintptr_t)targets % 4))
        return fail(GHN_E_INVALID_ARG, "ghn_insert: misaligned points or targets");
    const int64_t n = index->info.n, total = n + n_new;
    const int32_t f = index->info.f;
    if (total >= (int64_t(1) << 31)) return fail(GHN_E_INVALID_ARG, "ghn_insert: %lld points in all (>= 2^31)", (long long)total);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "ghn_insert: pending HIP error");
    hipStream_t s = (hipStream_t)stream;
    const int32_t dt = index->info.dtype == GHN_BF16 && dtype == GHN_BF16 ? GHN_BF16 : GHN_F32;
    {
        ghn_index* merged = nullptr;
        const ghn_status st = insert_merge(index, points, n_new, dtype, targets, s, &merged);
        if (st == GHN_OK) {
            adopt(index, merged);
            index->info.dtype = dt;
            log_line("insert n=%lld n_new=%lld: merged into the cell order", (long long)n, (long long)n_new);
            return GHN_OK;
        }
        if (st != GHN_E_UNSUPPORTED) return st;  // the index is left as it was
    }
    // a tree index (Morton order), or an enlarged box beyond the merge: rebuild from all points
    DevPool tmp;
    float* pts = nullptr;
    void* tg = nullptr;
    if (tmp.alloc((void**)&pts, (size_t)total * f * 4) || tmp.alloc(&tg, (size_t)total * 4))
        return fail(GHN_E_NOMEM, "ghn_insert: out of device memory");
    if ((e = original_points(index, pts, s)) != hipSuccess ||
        (e = launch_widen_points(points, n_new * f, dtype, pts + (size_t)n * f, s)) != hipSuccess ||
        (e = hipMemcpyAsync(tg, index->view.targets, (size_t)n * 4, hipMemcpyDeviceToDevice, s)) != hipSuccess ||
        (e = hipMemcpyAsync((char*)tg + (size_t)n * 4, targets, (size_t)n_new * 4, hipMemcpyDeviceToDevice, s)) !=
            hipSuccess)
        return hip_fail(e, "ghn_insert: staging");
    ghn_build_opts bo = {index->want_lookup};
    ghn_index* fresh = nullptr;
    const ghn_status st = ghn_build_ex(pts, total, f, GHN_F32, tg, index->info.task, index->info.cell_width, f,
                                       index->info.origin, &bo, stream, &fresh);
    if (st != GHN_OK) return st;  // the index is left as it was
    adopt(index, fresh);
    index->info.dtype = dt;
    log_line("insert n=%lld n_new=%lld: rebuilt from all points", (long long)n, (long long)n_new);
    return GHN_OK;
}

}  // extern "C"
