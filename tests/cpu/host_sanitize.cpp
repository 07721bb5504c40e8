// The library's host code under AddressSanitizer, LeakSanitizer and UBSan.
//
// Linked against a libghn whose host-side entry points (ghn_api.hip, ghn_hostenv.hip)
// are compiled with -fsanitize=address,undefined; the kernels are the ordinary ones
// (no device sanitizer).  Phase 1 needs no GPU: argument checks, size queries and
// NULL handles of every entry point.  Phase 2 runs when a GPU is present: every entry
// point on a small problem, results checked against ghn_bruteforce, and the failure
// paths forced with GHN_FAULT.  Any memory error, leak or undefined behaviour in the
// host code aborts the program with a report.  Prints "host sanitize ok (...)" at the end.
#include <hip/hip_runtime_api.h>

#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <random>
#include <vector>

#include "ghn.h"

static int failures = 0;
#define CHECK(c)                                                                  \
    do {                                                                          \
        if (!(c)) {                                                               \
            std::printf("FAIL %s:%d: %s (%s)\n", __FILE__, __LINE__, #c, ghn_last_error()); \
            ++failures;                                                           \
        }                                                                         \
    } while (0)

static void phase_no_gpu() {
    const float w = 0.5f;
    ghn_index* ix = (ghn_index*)0x1;
    CHECK(ghn_build(nullptr, 10, 2, GHN_F32, nullptr, GHN_CLASSIFY, &w, 1, nullptr, nullptr, &ix) == GHN_E_INVALID_ARG);
    CHECK(ix == nullptr && std::strlen(ghn_last_error()) > 0);
    CHECK(ghn_build_ex(nullptr, 10, 0, GHN_F32, nullptr, GHN_CLASSIFY, &w, 1, nullptr, nullptr, nullptr, &ix) ==
          GHN_E_INVALID_ARG);
    CHECK(ghn_build_into(nullptr, 10, 2, GHN_F32, nullptr, GHN_CLASSIFY, &w, 1, nullptr, nullptr, nullptr, 0, nullptr,
                         0, nullptr, &ix) == GHN_E_WORKSPACE);
    CHECK(ghn_build_into(nullptr, 0, 2, GHN_F32, nullptr, GHN_CLASSIFY, &w, 1, nullptr, nullptr, nullptr, 0, nullptr,
                         0, nullptr, &ix) == GHN_E_INVALID_ARG);
    CHECK(ghn_index_get_info(nullptr, nullptr) == GHN_E_INVALID_ARG);
    CHECK(ghn_index_cells(nullptr, nullptr, nullptr, nullptr, nullptr) == GHN_E_INVALID_ARG);
    CHECK(ghn_predict(nullptr, nullptr, 1, 1, nullptr, nullptr, nullptr, nullptr, nullptr, 0, nullptr) ==
          GHN_E_INVALID_ARG);
    CHECK(ghn_predict_noalloc(nullptr, nullptr, 1, 1, nullptr, nullptr, nullptr, nullptr, nullptr) ==
          GHN_E_INVALID_ARG);
    CHECK(ghn_bruteforce(nullptr, nullptr, 1, 1, nullptr, nullptr, nullptr, nullptr, nullptr, 0, nullptr) ==
          GHN_E_INVALID_ARG);
    CHECK(ghn_query_order(nullptr, nullptr, 1, nullptr, nullptr, 0, nullptr) == GHN_E_INVALID_ARG);
    ghn_batch* b = (ghn_batch*)0x1;
    CHECK(ghn_batch_prepare(nullptr, 1, nullptr, nullptr, 0, nullptr, &b) == GHN_E_INVALID_ARG);
    CHECK(ghn_predict_batched(nullptr, nullptr) == GHN_E_INVALID_ARG);
    ghn_tune_trial best;
    CHECK(ghn_autotune(nullptr, 10, 2, GHN_F32, nullptr, GHN_CLASSIFY, nullptr, 1, 1, GHN_STOP_EXACT, nullptr, 0,
                       nullptr, nullptr, 0, nullptr, nullptr) == GHN_E_INVALID_ARG);
    (void)best;
    CHECK(ghn_cell_measure(nullptr, 10, 2, GHN_F32, nullptr, nullptr, nullptr, nullptr) == GHN_E_INVALID_ARG);
    CHECK(ghn_screen_error(nullptr, nullptr, 1, 1, nullptr, nullptr, nullptr) == GHN_E_INVALID_ARG);
    CHECK(ghn_index_save(nullptr, nullptr, 0, nullptr) == GHN_E_INVALID_ARG);
    CHECK(ghn_index_load(nullptr, 0, nullptr, &ix) == GHN_E_INVALID_ARG);
    std::vector<unsigned char> junk(200, 0xab);
    ix = (ghn_index*)0x1;
    CHECK(ghn_index_load(junk.data(), junk.size(), nullptr, &ix) != GHN_OK && ix == nullptr);
    CHECK(ghn_insert(nullptr, nullptr, 1, GHN_F32, nullptr, nullptr) == GHN_E_INVALID_ARG);
    CHECK(ghn_walk_faults(nullptr, 0, nullptr) == GHN_E_INVALID_ARG);
    CHECK(ghn_index_save_bytes(nullptr) == 0);
    CHECK(ghn_batch_workspace_bytes(0) == 0 && ghn_batch_workspace_bytes(3) > 0);
    CHECK(ghn_build_workspace_bytes(1000, 3) > 0);
    CHECK(ghn_index_bytes(1000, 3, GHN_F32, GHN_CLASSIFY) > ghn_index_bytes(10, 3, GHN_F32, GHN_CLASSIFY));
    CHECK(ghn_query_order_workspace_bytes(100000) > 0);
    ghn_destroy(nullptr);
    ghn_batch_destroy(nullptr);
}

struct Dev {
    void* p = nullptr;
    explicit Dev(size_t bytes) { (void)hipMalloc(&p, bytes ? bytes : 1); }
    ~Dev() { (void)hipFree(p); }
    template <class T> T* as() { return (T*)p; }
};

template <class T> static std::vector<T> down(const Dev& d, size_t count) {
    std::vector<T> h(count);
    (void)hipMemcpy(h.data(), d.p, count * sizeof(T), hipMemcpyDeviceToHost);
    return h;
}

static void phase_gpu() {
    const int64_t n = 6000, m = 700;
    const int32_t f = 3, k = 7;
    std::mt19937 rng(5);
    std::normal_distribution<float> g(0.f, 1.f);
    std::vector<float> pts((size_t)n * f), qs((size_t)m * f);
    std::vector<int32_t> lab((size_t)n);
    for (auto& x : pts) x = g(rng);
    for (auto& x : qs) x = 1.2f * g(rng);
    for (int64_t i = 0; i < n; ++i) lab[(size_t)i] = (int32_t)(rng() % 5);
    Dev dp(pts.size() * 4), dq(qs.size() * 4), dl(lab.size() * 4);
    (void)hipMemcpy(dp.p, pts.data(), pts.size() * 4, hipMemcpyHostToDevice);
    (void)hipMemcpy(dq.p, qs.data(), qs.size() * 4, hipMemcpyHostToDevice);
    (void)hipMemcpy(dl.p, lab.data(), lab.size() * 4, hipMemcpyHostToDevice);
    const float w = 0.25f;
    Dev oi((size_t)m * k * 8), od((size_t)m * k * 8), op((size_t)m * 4), bi((size_t)m * k * 8),
        bd((size_t)m * k * 8), bp((size_t)m * 4);

    // brute force (the reference for every EXACT form below)
    ghn_index* ix = nullptr;
    CHECK(ghn_build(dp.p, n, f, GHN_F32, dl.p, GHN_CLASSIFY, &w, 1, nullptr, nullptr, &ix) == GHN_OK);
    if (!ix) return;
    ghn_predict_opts o;
    std::memset(&o, 0, sizeof o);
    o.group_levels = -1;
    size_t wsb = ghn_predict_workspace_bytes(ix, m, k, &o);
    {
        ghn_predict_opts ob = o;
        ob.prec = GHN_PREC_BF16_MFMA;
        const size_t w2 = ghn_predict_workspace_bytes(ix, m, k, &ob);
        if (w2 > wsb) wsb = w2;
    }
    Dev ws(wsb);
    CHECK(ghn_bruteforce(ix, dq.as<float>(), m, k, nullptr, bi.as<int64_t>(), bd.as<double>(), bp.p, ws.p, wsb,
                         nullptr) == GHN_OK);
    const std::vector<int64_t> want = down<int64_t>(bi, (size_t)m * k);

    // every lookup, both screens, both rules
    for (int lookup = GHN_LOOKUP_DENSE; lookup <= GHN_LOOKUP_HASH; ++lookup) {
        ghn_build_opts bo = {lookup};
        ghn_index* jx = nullptr;
        CHECK(ghn_build_ex(dp.p, n, f, GHN_F32, dl.p, GHN_CLASSIFY, &w, 1, nullptr, &bo, nullptr, &jx) == GHN_OK);
        if (!jx) continue;
        for (int stop = 0; stop < 2; ++stop)
            for (int prec = 0; prec < 2; ++prec) {
                ghn_predict_opts q = o;
                q.stop = stop;
                q.prec = prec;
                q.tile_width = lookup == GHN_LOOKUP_TREE ? 32 : 0;  // both screen tile widths
                CHECK(ghn_predict(jx, dq.as<float>(), m, k, &q, oi.as<int64_t>(), od.as<double>(), op.p, ws.p, wsb,
                                  nullptr) == GHN_OK);
                if (stop == GHN_STOP_EXACT) CHECK(down<int64_t>(oi, (size_t)m * k) == want);
            }
        CHECK(ghn_predict_noalloc(jx, dq.as<float>(), m, k, &o, oi.as<int64_t>(), od.as<double>(), op.p, nullptr) ==
              GHN_OK);
        CHECK(down<int64_t>(oi, (size_t)m * k) == want);
        ghn_index_info info;
        CHECK(ghn_index_get_info(jx, &info) == GHN_OK && info.n == n && info.lookup == lookup);
        Dev ids((size_t)info.num_cells * f * 4), cnt((size_t)info.num_cells * 8), pc((size_t)n * 4);
        CHECK(ghn_index_cells(jx, ids.as<int32_t>(), cnt.as<int64_t>(), pc.as<int32_t>(), nullptr) == GHN_OK);
        int64_t total = 0;
        for (int64_t c : down<int64_t>(cnt, (size_t)info.num_cells)) total += c;
        CHECK(total == n);
        ghn_destroy(jx);
    }
    // argument checks with a live index
    CHECK(ghn_predict(ix, dq.as<float>(), m, 0, &o, oi.as<int64_t>(), nullptr, op.p, ws.p, wsb, nullptr) ==
          GHN_E_INVALID_ARG);
    CHECK(ghn_predict(ix, dq.as<float>(), m, GHN_K_MAX + 1, &o, oi.as<int64_t>(), nullptr, op.p, ws.p, wsb, nullptr) ==
          GHN_E_INVALID_ARG);
    {
        ghn_predict_opts q = o;
        q.flags = 0x100;
        CHECK(ghn_predict(ix, dq.as<float>(), m, k, &q, oi.as<int64_t>(), nullptr, op.p, ws.p, wsb, nullptr) ==
              GHN_E_INVALID_ARG);
        q = o;
        q.prec = GHN_PREC_BF16_MFMA;
        CHECK(ghn_predict(ix, dq.as<float>(), m, k, &q, oi.as<int64_t>(), nullptr, op.p, nullptr, 0, nullptr) ==
              GHN_E_WORKSPACE);
        q.tile_width = 48;
        CHECK(ghn_predict(ix, dq.as<float>(), m, k, &q, oi.as<int64_t>(), nullptr, op.p, ws.p, wsb, nullptr) ==
              GHN_E_INVALID_ARG);
    }

    // a batch of two items
    {
        ghn_batch_item items[2] = {{ix, dq.as<float>(), m / 2, k, oi.as<int64_t>(), nullptr, op.p},
                                   {ix, dq.as<float>() + (m / 2) * f, m - m / 2, k, oi.as<int64_t>() + (m / 2) * k,
                                    nullptr, (int32_t*)op.p + m / 2}};
        for (int prec = 0; prec < 2; ++prec) {
            ghn_predict_opts q = o;
            q.prec = prec;
            const size_t bb = ghn_batch_workspace_bytes_for(items, 2, &q);
            Dev bws(bb);
            ghn_batch* batch = nullptr;
            CHECK(ghn_batch_prepare(items, 2, &q, bws.p, bb, nullptr, &batch) == GHN_OK);
            if (batch) {
                CHECK(ghn_predict_batched(batch, nullptr) == GHN_OK);
                (void)hipDeviceSynchronize();
                CHECK(down<int64_t>(oi, (size_t)m * k) == want);
                ghn_batch_destroy(batch);
            }
        }
    }

    // save, load, insert
    {
        const size_t sb = ghn_index_save_bytes(ix);
        std::vector<unsigned char> buf(sb);
        CHECK(ghn_index_save(ix, buf.data(), sb, nullptr) == GHN_OK);
        ghn_index* lx = nullptr;
        CHECK(ghn_index_load(buf.data(), sb, nullptr, &lx) == GHN_OK);
        if (lx) {
            CHECK(ghn_predict(lx, dq.as<float>(), m, k, &o, oi.as<int64_t>(), nullptr, op.p, ws.p, wsb, nullptr) ==
                  GHN_OK);
            CHECK(down<int64_t>(oi, (size_t)m * k) == want);
            ghn_destroy(lx);
        }
        buf.resize(sb / 2);
        lx = (ghn_index*)0x1;
        CHECK(ghn_index_load(buf.data(), buf.size(), nullptr, &lx) != GHN_OK && lx == nullptr);
        ghn_index* hx = nullptr;
        CHECK(ghn_build(dp.p, n / 2, f, GHN_F32, dl.p, GHN_CLASSIFY, &w, 1, nullptr, nullptr, &hx) == GHN_OK);
        if (hx) {
            CHECK(ghn_insert(hx, dp.as<float>() + (n / 2) * f, n - n / 2, GHN_F32, dl.as<int32_t>() + n / 2,
                             nullptr) == GHN_OK);
            CHECK(ghn_predict(hx, dq.as<float>(), m, k, &o, oi.as<int64_t>(), nullptr, op.p, ws.p, wsb, nullptr) ==
                  GHN_OK);
            CHECK(down<int64_t>(oi, (size_t)m * k) == want);
            ghn_destroy(hx);
        }
    }

    // caller storage
    {
        size_t need = 0;
        const size_t bw = ghn_build_workspace_bytes(n, f);
        Dev bws(bw);
        CHECK(ghn_index_bytes_for(dp.p, n, f, GHN_F32, GHN_CLASSIFY, &w, 1, nullptr, nullptr, bws.p, bw, nullptr,
                                  &need) == GHN_OK);
        Dev store(need);
        ghn_index* cx = nullptr;
        CHECK(ghn_build_into(dp.p, n, f, GHN_F32, dl.p, GHN_CLASSIFY, &w, 1, nullptr, nullptr, store.p, need, bws.p, bw,
                             nullptr, &cx) == GHN_OK);
        if (cx) {
            CHECK(ghn_predict(cx, dq.as<float>(), m, k, &o, oi.as<int64_t>(), nullptr, op.p, ws.p, wsb, nullptr) ==
                  GHN_OK);
            CHECK(down<int64_t>(oi, (size_t)m * k) == want);
            CHECK(ghn_insert(cx, dp.p, 10, GHN_F32, dl.p, nullptr) == GHN_E_UNSUPPORTED);
            ghn_destroy(cx);
        }
        cx = (ghn_index*)0x1;
        CHECK(ghn_build_into(dp.p, n, f, GHN_F32, dl.p, GHN_CLASSIFY, &w, 1, nullptr, nullptr, store.p, need / 4,
                             bws.p, bw, nullptr, &cx) == GHN_E_WORKSPACE && cx == nullptr);
    }

    // measurement, autotune, screen error, order, walk faults
    {
        float mw[GHN_F_MAX], mo[GHN_F_MAX];
        int64_t ms[GHN_F_MAX];
        CHECK(ghn_cell_measure(dp.p, n, f, GHN_F32, mw, mo, ms, nullptr) == GHN_OK);
        ghn_tune_trial best;
        std::vector<ghn_tune_trial> trials(300);
        int32_t nt = 0;
        const float widths[2] = {0.2f, 0.4f};
        CHECK(ghn_autotune(dp.p, n, f, GHN_F32, dl.p, GHN_CLASSIFY, dq.as<float>(), m, k, GHN_STOP_EXACT, widths, 2,
                           &best, trials.data(), (int32_t)trials.size(), &nt, nullptr) == GHN_OK);
        CHECK(nt > 0 && best.ms >= 0.0);
        Dev ea((size_t)m * 4), er((size_t)m * 4);
        CHECK(ghn_screen_error(ix, dq.as<float>(), m, 512, ea.as<float>(), er.as<float>(), nullptr) == GHN_OK);
        const size_t qb = ghn_query_order_workspace_bytes(m);
        Dev qws(qb), ord((size_t)m * 4);
        CHECK(ghn_query_order(ix, dq.as<float>(), m, ord.as<uint32_t>(), qws.p, qb, nullptr) == GHN_OK);
        uint32_t fl = 7;
        CHECK(ghn_walk_faults(&fl, 1, nullptr) == GHN_OK && fl == 0);
    }

    // failure paths forced from the host: every allocation and launch check of a build
    for (int kind = 0; kind < 2; ++kind)
        for (int at = 1; at < 100; ++at) {
            char v[32];
            std::snprintf(v, sizeof v, "%s:%d", kind ? "launch" : "alloc", at);
            setenv("GHN_FAULT", v, 1);
            ghn_build_opts bo = {GHN_LOOKUP_TREE};
            ghn_index* fx = (ghn_index*)0x1;
            const ghn_status st =
                ghn_build_ex(dp.p, n, f, GHN_F32, dl.p, GHN_CLASSIFY, &w, 1, nullptr, &bo, nullptr, &fx);
            unsetenv("GHN_FAULT");
            if (st == GHN_OK) {
                ghn_destroy(fx);
                break;
            }
            CHECK(st == (kind ? GHN_E_HIP : GHN_E_NOMEM) && fx == nullptr);
        }
    for (int at = 1; at <= 4; ++at) {
        char v[32];
        std::snprintf(v, sizeof v, "alloc:%d", at);
        setenv("GHN_FAULT", v, 1);
        ghn_tune_trial best;
        const float widths[1] = {0.3f};
        const ghn_status st = ghn_autotune(dp.p, n, f, GHN_F32, dl.p, GHN_CLASSIFY, dq.as<float>(), m, k,
                                           GHN_STOP_EXACT, widths, 1, &best, nullptr, 0, nullptr, nullptr);
        unsetenv("GHN_FAULT");
        // the sample's outputs fail (NOMEM), or the one width's build does (no candidate left)
        CHECK(st == GHN_E_NOMEM || st == GHN_E_UNSUPPORTED || st == GHN_OK);
    }
    ghn_destroy(ix);
}

int main() {
    phase_no_gpu();
    int devices = 0;
    const bool gpu = hipGetDeviceCount(&devices) == hipSuccess && devices > 0;
    if (gpu) {
        phase_gpu();
        (void)hipDeviceSynchronize();
    }
    if (failures) {
        std::printf("%d checks failed\n", failures);
        return 1;
    }
    std::printf("host sanitize ok (%s)\n", gpu ? "argument checks and GPU phase" : "argument checks; no GPU");
    return 0;
}
