// GHN oracle: a plain, slow, obviously correct FP64 CPU reference for the Grid
// Hashing Neighborhood KNN method (Tchaye-Kondi, Zhai, Zhu, "A new hashing based
// nearest neighbors selection technique for big datasets", arXiv 2004.02290).
//
// TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the CPU
// baseline leg of the benchmark may load this library.  It shares no code with
// the GPU library: no headers, kernels, helpers or tables.
//
// What it computes, and where the paper says so:
//   * cell coordinate of a point (Eq. 1, Section III-A): per dimension the
//     integer division of the point by the cell measurement; read as the exact
//     floor of the real quotient (x - o) / a, with x - o evaluated in FP64,
//     saturated to +-2^40 (only far query coordinates reach that).
//   * cell sampling (Algorithm 1): a hash table from cell id to the list of its
//     points; empty cells are never stored (Section III-A).
//   * exploration (Section III-B, Algorithm 2): start at the query's central
//     cell, visit the stored cells layer by layer (layer l = the cells whose
//     Chebyshev index distance to the central cell is l), keep the k nearest
//     candidates seen so far in a size-k buffer, and stop by one of two rules:
//       PAPER: after a layer that left the buffer unchanged while it holds k
//              (Section III-B, and the k = 3 walk-through of Fig. 2c);
//       EXACT: after a layer l once the buffer holds k and its k-th distance is
//              below the squared distance from the query to the outside of the
//              box of layers 0..l (a sound bound; the result then equals brute
//              force).
//     Both rules also stop once every stored cell has been visited.
//   * prediction (Section I, Section III-D): majority class of the k neighbours
//     (ties -> smallest label), their mean (FP64 sum in result order, / k,
//     rounded to FP32) or their median (the paper names both statistics for
//     regression): the middle target in IEEE total order, or for even k the
//     FP64 mean of the two middle targets rounded to FP32.
//   * cell measurements (Section III-A, Fig. 3): per dimension the largest
//     number of equal splits of the range covered by the points that leaves no
//     split empty; the split width is the cell measurement.
//   * brute force: the plain KNN definition (Section I) over all n points.
//
// Distances are squared Euclidean, d(q,x) = sum_j (q_j - x_j)^2 computed in FP64
// in order j = 0..f-1 with no fused multiply-add (built with -ffp-contract=off).
// Neighbours are ordered by (distance, original row index).

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <map>
#include <utility>
#include <vector>

#include <omp.h>

namespace {

enum { TASK_CLASSIFY = 0, TASK_REGRESS = 1, TASK_REGRESS_MEDIAN = 2 };
enum { STOP_EXACT = 0, STOP_PAPER = 1 };

// Cell ids are saturated to [-CELL_LIMIT, CELL_LIMIT]: a query coordinate can lie
// arbitrarily far outside the data, and no finite id range holds every quotient of
// two floats.  Below the limit the id is the exact floor.
const int64_t CELL_LIMIT = int64_t(1) << 40;

// Exact floor of v / a for a > 0 finite and v finite, via fmod in x87 extended
// precision (64-bit significand): r = fmodl(v, a) is exact and v = t*a + r with
// |r| < a and r carrying the sign of v.  While |t| <= 2^40 the product t*a needs
// at most 40 + 24 bits (a is a float32 width), so v - r = t*a is exact, and so is
// the division by a; the floor is t - 1 when r < 0.  Beyond 2^40 the (then
// rounded) quotient only decides the saturation.
int64_t floor_div(double v, double a) {
    const long double lv = v, la = a;
    const long double r = fmodl(lv, la);
    long double t = (lv - r) / la;
    if (r < 0) t -= 1;
    if (t > (long double)CELL_LIMIT) return CELL_LIMIT;
    if (t < -(long double)CELL_LIMIT) return -CELL_LIMIT;
    return (int64_t)t;
}

struct Params {
    int f;
    std::vector<double> a;  // cell measurement per dimension
    std::vector<double> o;  // grid origin per dimension (0 = Eq. 1 as printed)
};

Params make_params(int f, const float* widths, int n_width, const float* origin) {
    Params p;
    p.f = f;
    p.a.resize(f);
    p.o.resize(f);
    for (int j = 0; j < f; ++j) {
        p.a[j] = (double)(n_width == 1 ? widths[0] : widths[j]);
        p.o[j] = origin ? (double)origin[j] : 0.0;
    }
    return p;
}

// Eq. 1: the cell id of a point.
std::vector<int64_t> cell_of(const Params& p, const float* x) {
    std::vector<int64_t> c(p.f);
    for (int j = 0; j < p.f; ++j) c[j] = floor_div((double)x[j] - p.o[j], p.a[j]);
    return c;
}

double sqdist(const float* q, const float* x, int f) {
    double s = 0.0;
    for (int j = 0; j < f; ++j) {
        double d = (double)q[j] - (double)x[j];
        s = s + d * d;
    }
    return s;
}

typedef std::pair<double, int64_t> Cand;  // (distance, original row index)

// The size-k buffer of Section III-B, kept sorted ascending by (distance, index).
// Returns true when the candidate entered the buffer.
bool buffer_offer(std::vector<Cand>& buf, int k, const Cand& c) {
    if ((int)buf.size() == k && !(c < buf.back())) return false;
    buf.insert(std::upper_bound(buf.begin(), buf.end(), c), c);
    if ((int)buf.size() > k) buf.pop_back();
    return true;
}

// Integer key ordering floats as IEEE total order.
int64_t total_key(float x) {
    uint32_t u;
    std::memcpy(&u, &x, 4);
    return (u & 0x80000000u) ? -(int64_t)(u & 0x7fffffffu) - 1 : (int64_t)u;
}

void predict_from(const std::vector<Cand>& buf, int k, int task, const void* targets,
                  void* out_pred, int64_t qi) {
    if (task == TASK_CLASSIFY) {
        const int32_t* lab = (const int32_t*)targets;
        std::map<int32_t, int> count;
        for (int t = 0; t < k; ++t) count[lab[buf[t].second]] += 1;
        int32_t best = 0;
        int best_n = -1;
        for (const auto& kv : count)  // ascending label order: first maximum = smallest label
            if (kv.second > best_n) { best = kv.first; best_n = kv.second; }
        ((int32_t*)out_pred)[qi] = best;
    } else if (task == TASK_REGRESS) {
        const float* y = (const float*)targets;
        double s = 0.0;
        for (int t = 0; t < k; ++t) s = s + (double)y[buf[t].second];
        ((float*)out_pred)[qi] = (float)(s / (double)k);
    } else {
        // median in IEEE total order (negative NaN < -inf < ... < +inf < NaN)
        const float* y = (const float*)targets;
        std::vector<float> v;
        for (int t = 0; t < k; ++t) v.push_back(y[buf[t].second]);
        std::sort(v.begin(), v.end(), [](float a, float b) { return total_key(a) < total_key(b); });
        const float mid = (k % 2) ? v[(size_t)k / 2]
                                  : (float)(((double)v[(size_t)k / 2 - 1] + (double)v[(size_t)k / 2]) / 2.0);
        ((float*)out_pred)[qi] = mid;
    }
}

void write_result(const std::vector<Cand>& buf, int k, int64_t qi, int64_t* out_idx, double* out_d2) {
    for (int t = 0; t < k; ++t) {
        if (out_idx) out_idx[qi * k + t] = buf[t].second;
        if (out_d2) out_d2[qi * k + t] = buf[t].first;
    }
}

struct Grid {
    Params p;
    int64_t n;
    std::vector<float> pts;                                   // n x f, original order
    std::vector<unsigned char> targets;                       // n targets (4 bytes each)
    int task;
    std::map<std::vector<int64_t>, std::vector<int64_t>> table;  // Algorithm 1's `grid`
    // The stored cells as a flat list (same content as `table`), for scanning.
    std::vector<std::vector<int64_t>> keys;
    std::vector<const std::vector<int64_t>*> members;
};

struct WalkStats {
    int32_t stop_layer = -1;
    int64_t cells = 0;       // stored cells visited
    int64_t cands = 0;       // points whose distance was computed
};

// Exploration for one query (Section III-B).  `layer_cells` / `layer_updated`,
// when not null, receive per-layer traces for layers 0..max_layers-1.
std::vector<Cand> walk(const Grid& g, const float* q, int k, int stop, WalkStats* st,
                       int64_t* layer_cells, int32_t* layer_updated, int32_t max_layers) {
    const int f = g.p.f;
    std::vector<int64_t> c = cell_of(g.p, q);  // the central cell

    // Layer of every stored cell = Chebyshev distance of its id to the central id.
    const size_t nc = g.keys.size();
    std::vector<std::pair<int64_t, size_t>> by_layer(nc);
    for (size_t i = 0; i < nc; ++i) {
        int64_t l = 0;
        for (int j = 0; j < f; ++j) {
            int64_t d = g.keys[i][j] - c[j];
            if (d < 0) d = -d;
            if (d > l) l = d;
        }
        by_layer[i] = std::make_pair(l, i);
    }
    std::sort(by_layer.begin(), by_layer.end());
    const int64_t l_first = by_layer.front().first;
    const int64_t l_last = by_layer.back().first;

    std::vector<Cand> buf;
    size_t pos = 0;
    WalkStats s;
    for (int64_t l = 0;; ++l) {
        if (l < l_first) {  // layers before the first stored cell are empty and the buffer stays
            l = l_first - 1;  // empty, so no stop rule can fire there: go straight to l_first
            continue;
        }
        bool updated = false;
        int64_t visited = 0;
        while (pos < nc && by_layer[pos].first == l) {
            const std::vector<int64_t>& pts = *g.members[by_layer[pos].second];
            for (int64_t i : pts) {
                Cand cd(sqdist(q, &g.pts[(size_t)i * f], f), i);
                if (buffer_offer(buf, k, cd)) updated = true;
                s.cands += 1;
            }
            visited += 1;
            ++pos;
        }
        s.cells += visited;
        if (layer_cells && l < max_layers) { layer_cells[l] = visited; layer_updated[l] = updated ? 1 : 0; }

        const bool full = (int)buf.size() == k;
        bool done = (l >= l_last);  // every stored cell has been visited
        if (!done && full && stop == STOP_PAPER) done = !updated;
        if (!done && full && stop == STOP_EXACT) {
            // Squared distance from q to the outside of the box of cells c +- l.
            double r2 = INFINITY;
            for (int j = 0; j < f; ++j) {
                double v = (double)q[j] - g.p.o[j];
                double lo = v - (double)(c[j] - l) * g.p.a[j];
                double hi = (double)(c[j] + l + 1) * g.p.a[j] - v;
                double gj = lo < hi ? lo : hi;
                double g2 = gj * gj;
                if (g2 < r2) r2 = g2;
            }
            done = buf.back().first < r2 * (1.0 - 0x1p-44);
        }
        if (done) {  // the stop layer is reported as int32, saturated
            s.stop_layer = l < (int64_t)INT32_MAX ? (int32_t)l : INT32_MAX;
            break;
        }
    }
    if (st) *st = s;
    return buf;
}

}  // namespace

extern "C" {

// Cell coordinates (Eq. 1) of n points: out[i*f + j].
int ghn_oracle_cells(const float* pts, int64_t n, int32_t f, const float* widths, int32_t n_width,
                     const float* origin, int64_t* out) {
    Params p = make_params(f, widths, n_width, origin);
    for (int64_t i = 0; i < n; ++i) {
        std::vector<int64_t> c = cell_of(p, pts + i * f);
        for (int j = 0; j < f; ++j) out[i * f + j] = c[j];
    }
    return 0;
}

// Number of distinct (non-empty) cells.
int64_t ghn_oracle_count_cells(const float* pts, int64_t n, int32_t f, const float* widths,
                               int32_t n_width, const float* origin) {
    Params p = make_params(f, widths, n_width, origin);
    std::map<std::vector<int64_t>, int64_t> t;
    for (int64_t i = 0; i < n; ++i) t[cell_of(p, pts + i * f)] += 1;
    return (int64_t)t.size();
}

// Plain KNN (Section I): all n distances, the k smallest by (distance, index).
int ghn_oracle_bruteforce(const float* pts, int64_t n, int32_t f, const void* targets, int32_t task,
                          const float* qs, int64_t m, int32_t k, int64_t* out_idx, double* out_d2,
                          void* out_pred, int32_t nthreads) {
    if (k < 1 || k > n) return -1;
    if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t qi = 0; qi < m; ++qi) {
        const float* q = qs + qi * f;
        std::vector<Cand> all((size_t)n);
        for (int64_t i = 0; i < n; ++i) all[(size_t)i] = Cand(sqdist(q, pts + i * f, f), i);
        std::partial_sort(all.begin(), all.begin() + k, all.end());
        all.resize((size_t)k);
        write_result(all, k, qi, out_idx, out_d2);
        if (out_pred) predict_from(all, k, task, targets, out_pred, qi);
    }
    return 0;
}

// Algorithm 1: hash every training point into the cell table.
void* ghn_oracle_grid_build(const float* pts, int64_t n, int32_t f, const void* targets, int32_t task,
                            const float* widths, int32_t n_width, const float* origin) {
    Grid* g = new Grid();
    g->p = make_params(f, widths, n_width, origin);
    g->n = n;
    g->task = task;
    g->pts.assign(pts, pts + n * f);
    g->targets.assign((const unsigned char*)targets, (const unsigned char*)targets + n * 4);
    for (int64_t i = 0; i < n; ++i) {
        std::vector<int64_t> id = cell_of(g->p, pts + i * f);
        auto it = g->table.find(id);
        if (it == g->table.end()) it = g->table.emplace(id, std::vector<int64_t>()).first;
        it->second.push_back(i);
    }
    for (const auto& kv : g->table) {
        g->keys.push_back(kv.first);
        g->members.push_back(&kv.second);
    }
    return g;
}

int64_t ghn_oracle_grid_num_cells(const void* h) { return (int64_t)((const Grid*)h)->keys.size(); }

// Stored cells: ids (num_cells x f, ascending) and point counts.
int ghn_oracle_grid_cells(const void* h, int64_t* ids, int64_t* counts) {
    const Grid* g = (const Grid*)h;
    for (size_t i = 0; i < g->keys.size(); ++i) {
        for (int j = 0; j < g->p.f; ++j) ids[i * g->p.f + j] = g->keys[i][j];
        counts[i] = (int64_t)g->members[i]->size();
    }
    return 0;
}

// Exploration (Section III-B) for m queries.  Optional per-query outputs: the
// layer at which the walk stopped, stored cells visited and points evaluated.
int ghn_oracle_grid_predict(const void* h, const float* qs, int64_t m, int32_t k, int32_t stop,
                            int64_t* out_idx, double* out_d2, void* out_pred, int32_t* out_stop_layer,
                            int64_t* out_cells, int64_t* out_cands, int32_t nthreads) {
    const Grid* g = (const Grid*)h;
    if (k < 1 || k > g->n) return -1;
    if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t qi = 0; qi < m; ++qi) {
        WalkStats st;
        std::vector<Cand> buf = walk(*g, qs + qi * g->p.f, k, stop, &st, nullptr, nullptr, 0);
        write_result(buf, k, qi, out_idx, out_d2);
        if (out_pred) predict_from(buf, k, g->task, g->targets.data(), out_pred, qi);
        if (out_stop_layer) out_stop_layer[qi] = st.stop_layer;
        if (out_cells) out_cells[qi] = st.cells;
        if (out_cands) out_cands[qi] = st.cands;
    }
    return 0;
}

// Per-layer trace of one query's walk: stored cells visited in layer l and whether
// the buffer changed in it, for l < max_layers.  Returns the stop layer.
int32_t ghn_oracle_grid_trace(const void* h, const float* q, int32_t k, int32_t stop,
                              int64_t* layer_cells, int32_t* layer_updated, int32_t max_layers) {
    const Grid* g = (const Grid*)h;
    for (int32_t l = 0; l < max_layers; ++l) { layer_cells[l] = 0; layer_updated[l] = 0; }
    WalkStats st;
    walk(*g, q, k, stop, &st, layer_cells, layer_updated, max_layers);
    return st.stop_layer;
}

void ghn_oracle_grid_free(void* h) { delete (Grid*)h; }

// The paper's cell measurement rule (Section III-A, Fig. 3), per dimension j:
// the range [mn, mx] covered by the points is cut into s equal splits of width
// w = fl32((mx - mn) / s); a point x belongs to split min(floor((x - mn) / w), s - 1)
// (exact floor; the last split is closed at mx).  The answer is the largest s
// that leaves no split empty, found here by trying every s from the number of
// distinct values down to 1.  The grid origin is mn, so cells are the splits.
// A dimension whose points all coincide gets s = 1 and width 1.
int ghn_oracle_cell_measure(const float* pts, int64_t n, int32_t f, float* width, float* origin, int64_t* splits) {
    if (n < 1 || f < 1) return -1;
    for (int j = 0; j < f; ++j) {
        std::vector<double> v((size_t)n);
        for (int64_t i = 0; i < n; ++i) v[(size_t)i] = (double)pts[i * f + j];
        std::sort(v.begin(), v.end());
        const double mn = v.front(), mx = v.back();
        const int64_t distinct = (int64_t)(std::unique(v.begin(), v.end()) - v.begin());
        origin[j] = (float)mn;
        splits[j] = 1;
        width[j] = 1.0f;
        if (!(mx > mn)) continue;
        for (int64_t s = distinct; s >= 1; --s) {
            const float w = (float)((mx - mn) / (double)s);
            if (!(w > 0.0f)) continue;
            std::vector<char> hit((size_t)s, 0);
            for (int64_t i = 0; i < n; ++i) {
                int64_t c = floor_div((double)pts[i * f + j] - mn, (double)w);
                if (c > s - 1) c = s - 1;
                hit[(size_t)c] = 1;
            }
            if (std::find(hit.begin(), hit.end(), 0) == hit.end()) {
                splits[j] = s;
                width[j] = w;
                break;
            }
        }
    }
    return 0;
}

}  // extern "C"
