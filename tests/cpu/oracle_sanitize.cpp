// The oracle under AddressSanitizer, LeakSanitizer and UBSan: every exported function
// on seeded inputs (1 to 5 dimensions, clustered and lattice points with ties, k from
// 1 to n, all three prediction tasks, both stop rules, far queries), with the checks
// that hold whatever the inputs: the EXACT grid walk equals brute force, the cells
// partition the points, the layer trace ends at the walk's stop layer.  Compiled with
// g++ together with oracle/ghn_oracle.cpp by tests/test_sanitize_cpu.py.
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <random>
#include <vector>

extern "C" {
int ghn_oracle_cells(const float* pts, int64_t n, int32_t f, const float* widths, int32_t n_width,
                     const float* origin, int64_t* out);
int64_t ghn_oracle_count_cells(const float* pts, int64_t n, int32_t f, const float* widths, int32_t n_width,
                               const float* origin);
int ghn_oracle_bruteforce(const float* pts, int64_t n, int32_t f, const void* targets, int32_t task, const float* qs,
                          int64_t m, int32_t k, int64_t* out_idx, double* out_d2, void* out_pred, int32_t nthreads);
void* ghn_oracle_grid_build(const float* pts, int64_t n, int32_t f, const void* targets, int32_t task,
                            const float* widths, int32_t n_width, const float* origin);
int64_t ghn_oracle_grid_num_cells(const void* h);
int ghn_oracle_grid_cells(const void* h, int64_t* ids, int64_t* counts);
int ghn_oracle_grid_predict(const void* h, const float* qs, int64_t m, int32_t k, int32_t stop, int64_t* out_idx,
                            double* out_d2, void* out_pred, int32_t* out_stop_layer, int64_t* out_cells,
                            int64_t* out_cands, int32_t nthreads);
int32_t ghn_oracle_grid_trace(const void* h, const float* q, int32_t k, int32_t stop, int64_t* layer_cells,
                              int32_t* layer_updated, int32_t max_layers);
void ghn_oracle_grid_free(void* h);
int ghn_oracle_cell_measure(const float* pts, int64_t n, int32_t f, float* width, float* origin, int64_t* splits);
}

static int failures = 0;
#define CHECK(c)                                                    \
    do {                                                            \
        if (!(c)) {                                                 \
            std::printf("FAIL %s:%d: %s\n", __FILE__, __LINE__, #c); \
            ++failures;                                             \
        }                                                           \
    } while (0)

static void run_case(int f, int64_t n, int64_t m, bool lattice, unsigned seed) {
    std::mt19937 rng(seed);
    std::normal_distribution<float> g(0.f, 1.f);
    std::vector<float> pts((size_t)(n * f)), qs((size_t)(m * f));
    for (auto& x : pts) x = lattice ? (float)(int)(4.f * g(rng)) * 0.25f : g(rng);
    for (auto& x : qs) x = 1.3f * g(rng);
    if (m > 1) for (int j = 0; j < f; ++j) qs[(size_t)j] = 1e9f;  // a far query
    std::vector<int32_t> lab((size_t)n);
    std::vector<float> y((size_t)n);
    for (int64_t i = 0; i < n; ++i) {
        lab[(size_t)i] = (int32_t)(rng() % 4);
        y[(size_t)i] = g(rng);
    }
    const float w = lattice ? 0.5f : 0.35f;
    // cells partition the points
    std::vector<int64_t> cid((size_t)(n * f));
    CHECK(ghn_oracle_cells(pts.data(), n, f, &w, 1, nullptr, cid.data()) == 0);
    const int64_t nc = ghn_oracle_count_cells(pts.data(), n, f, &w, 1, nullptr);
    for (int task = 0; task < 3; ++task) {
        const void* tg = task == 0 ? (const void*)lab.data() : (const void*)y.data();
        void* h = ghn_oracle_grid_build(pts.data(), n, f, tg, task, &w, 1, nullptr);
        CHECK(h != nullptr);
        CHECK(ghn_oracle_grid_num_cells(h) == nc);
        std::vector<int64_t> ids((size_t)(nc * f)), counts((size_t)nc);
        CHECK(ghn_oracle_grid_cells(h, ids.data(), counts.data()) == 0);
        int64_t total = 0;
        for (int64_t c : counts) total += c;
        CHECK(total == n);
        for (int32_t k : {1, 3, 17, 64}) {
            if (k > n) k = (int32_t)n;
            std::vector<int64_t> bi((size_t)(m * k)), gi((size_t)(m * k)), cells((size_t)m), cands((size_t)m);
            std::vector<double> bd((size_t)(m * k)), gd((size_t)(m * k));
            std::vector<int32_t> bp((size_t)m), gp((size_t)m), sl((size_t)m);
            CHECK(ghn_oracle_bruteforce(pts.data(), n, f, tg, task, qs.data(), m, k, bi.data(), bd.data(), bp.data(),
                                        2) == 0);
            for (int stop = 0; stop < 2; ++stop) {
                CHECK(ghn_oracle_grid_predict(h, qs.data(), m, k, stop, gi.data(), gd.data(), gp.data(), sl.data(),
                                              cells.data(), cands.data(), 2) == 0);
                if (stop == 0) {
                    CHECK(gi == bi);
                    CHECK(std::memcmp(gd.data(), bd.data(), gd.size() * 8) == 0);
                    CHECK(std::memcmp(gp.data(), bp.data(), gp.size() * 4) == 0);
                }
                for (int64_t q = 0; q < (m < 4 ? m : 4); ++q) {
                    std::vector<int64_t> lc(4096);
                    std::vector<int32_t> lu(4096);
                    const int32_t last = ghn_oracle_grid_trace(h, qs.data() + q * f, k, stop, lc.data(), lu.data(),
                                                               4096);
                    CHECK(last == sl[(size_t)q]);
                }
            }
        }
        CHECK(ghn_oracle_grid_predict(h, qs.data(), m, (int32_t)n + 1, 0, nullptr, nullptr, nullptr, nullptr, nullptr,
                                      nullptr, 1) != 0);
        ghn_oracle_grid_free(h);
    }
    std::vector<float> mw((size_t)f), mo((size_t)f);
    std::vector<int64_t> ms((size_t)f);
    CHECK(ghn_oracle_cell_measure(pts.data(), n, f, mw.data(), mo.data(), ms.data()) == 0);
    for (int j = 0; j < f; ++j) CHECK(ms[(size_t)j] >= 1);
}

int main() {
    run_case(1, 300, 50, false, 1);
    run_case(2, 500, 40, true, 2);
    run_case(3, 800, 30, false, 3);
    run_case(5, 400, 20, false, 4);
    run_case(2, 5, 3, true, 5);
    run_case(3, 1, 1, false, 6);
    if (failures) {
        std::printf("%d checks failed\n", failures);
        return 1;
    }
    std::printf("oracle sanitize ok\n");
    return 0;
}
