// Host check of the code plan behind gfbp_code_build (built with g++ and the
// address and undefined-behaviour sanitizers by tests/test_sanitizers.py):
// seeded random codes of every field with random visiting orders and source
// chains, and malformed descriptions.  For a valid description the plan's
// column index must list every edge once, the SUS levels must put a column
// after every earlier-visited column it shares a check with (and, in the
// second levelisation, after its earlier-visited chain neighbours), and the
// records must describe each column's edges; a malformed one must be refused.
// Also the LDS layout of the whole decode in LDS over random code shapes.
// Prints "ok <codes checked>" and exits 0, or names the failure and exits 1.
#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <set>
#include <string>
#include <vector>

#include "../paper_cs_0605069_amd/csrc/gfbp_plan.h"

using namespace gfbp;

static uint64_t rng_state = 0x9E3779B97F4A7C15ull;
static uint32_t rnd() {  // xorshift64*
    rng_state ^= rng_state >> 12;
    rng_state ^= rng_state << 25;
    rng_state ^= rng_state >> 27;
    return uint32_t((rng_state * 0x2545F4914F6CDD1Dull) >> 32);
}

#define CHECK(c, msg)                                               \
    do {                                                            \
        if (!(c)) {                                                 \
            std::printf("FAIL %s (code %d)\n", msg, code_id);       \
            return false;                                           \
        }                                                           \
    } while (0)

static bool check_valid(int code_id) {
    const int p = 1 + int(rnd() % 6), q = 1 << p;
    const int n = 4 + int(rnd() % 60), m = 2 + int(rnd() % (n - 1));
    std::vector<int32_t> row_ptr(m + 1, 0), col;
    std::vector<uint8_t> coef;
    for (int i = 0; i < m; ++i) {
        std::set<int> cols;
        const int dc = 1 + int(rnd() % 6);
        while (int(cols.size()) < std::min(dc, n)) cols.insert(int(rnd() % n));
        for (int j : cols) {
            col.push_back(j);
            coef.push_back(uint8_t(1 + rnd() % (q - 1)));
        }
        row_ptr[i + 1] = int32_t(col.size());
    }
    // column degrees within the kernels' limit
    std::vector<int> deg(n, 0);
    for (int j : col) deg[j]++;
    for (int j = 0; j < n; ++j)
        if (deg[j] > GFBP_MAX_COL_DEGREE) return true;  // not a case for this check
    const int K = int(rnd() % (n + 1));
    std::vector<int32_t> visit(n), src;
    for (int j = 0; j < n; ++j) visit[j] = j;
    for (int j = n - 1; j > 0; --j) std::swap(visit[j], visit[rnd() % (j + 1)]);
    std::vector<int32_t> perm(n);
    for (int j = 0; j < n; ++j) perm[j] = j;
    for (int j = n - 1; j > 0; --j) std::swap(perm[j], perm[rnd() % (j + 1)]);
    src.assign(perm.begin(), perm.begin() + K);
    gfbp_code_desc d{};
    d.q = q;
    d.n = n;
    d.m = m;
    d.n_info = K;
    d.row_ptr = row_ptr.data();
    d.col = col.data();
    d.coef = coef.data();
    d.visit_order = (rnd() & 1) ? visit.data() : nullptr;
    d.source_cols = (rnd() & 1) ? src.data() : nullptr;
    CodePlan pl;
    std::string err;
    const gfbp_status st = build_plan(&d, pl, err);
    CHECK(st == GFBP_OK, ("valid code refused: " + err).c_str());
    const int E = row_ptr[m];
    CHECK(pl.E == E && pl.col_ptr[n] == E, "edge count");
    std::vector<int> seen(E, 0);
    for (int j = 0; j < n; ++j)
        for (int t = pl.col_ptr[j]; t < pl.col_ptr[j + 1]; ++t) {
            const int e = pl.col_edge[t];
            CHECK(e >= 0 && e < E && col[e] == j, "column index");
            seen[e]++;
        }
    for (int e = 0; e < E; ++e) CHECK(seen[e] == 1 && row_ptr[pl.edge_row[e]] <= e && e < row_ptr[pl.edge_row[e] + 1], "edge rows");
    std::vector<int> vpos(n);
    for (int t = 0; t < n; ++t) vpos[pl.visit[t]] = t;
    for (int chain = 0; chain < 2; ++chain) {
        const LevelPlan &L = pl.lv[chain];
        const int RS = std::max(1, pl.max_dv);
        CHECK(int(pl.recs[chain].size()) == n * RS && L.ptr.back() == n, "record count");
        std::vector<int> level(n, -1);
        for (size_t l = 0; l + 1 < L.ptr.size(); ++l)
            for (int pos = L.ptr[l]; pos < L.ptr[l + 1]; ++pos) {
                const SusRec &r0 = pl.recs[chain][size_t(pos) * RS];
                CHECK(r0.j >= 0 && r0.j < n && level[r0.j] < 0, "each column once");
                level[r0.j] = int(l);
                CHECK(r0.dv == pl.col_ptr[r0.j + 1] - pl.col_ptr[r0.j], "record degree");
                for (int t = 0; t < r0.dv; ++t) {
                    const SusRec &r = pl.recs[chain][size_t(pos) * RS + t];
                    CHECK(r.e == pl.col_edge[pl.col_ptr[r0.j] + t] && r.rs + r.self == r.e &&
                              r.dc == row_ptr[r.i + 1] - row_ptr[r.i], "record edge");
                }
            }
        for (int i = 0; i < m; ++i)  // columns sharing check i: levels increase with the visiting order
            for (int a = row_ptr[i]; a < row_ptr[i + 1]; ++a)
                for (int b = row_ptr[i]; b < row_ptr[i + 1]; ++b)
                    if (vpos[col[a]] < vpos[col[b]]) CHECK(level[col[a]] < level[col[b]], "level order in a check");
        if (chain)
            for (int k = 0; k + 1 < K; ++k) {
                const int x = pl.chain_col[k], y = pl.chain_col[k + 1];
                const int first = vpos[x] < vpos[y] ? x : y, second = first == x ? y : x;
                CHECK(level[first] < level[second], "chain neighbours");
            }
    }
    return true;
}

static bool check_refusals(int code_id) {
    const int32_t row_ptr[4] = {0, 3, 6, 9};
    const int32_t col_ok[9] = {0, 1, 2, 2, 3, 4, 4, 5, 0};
    const uint8_t coef_ok[9] = {1, 2, 3, 1, 2, 3, 1, 2, 3};
    struct Case {
        const char *what;
        int q, n_info;
        const int32_t *col;
        const uint8_t *coef;
        std::vector<int32_t> visit, src;
    };
    const int32_t col_rep[9] = {0, 0, 2, 2, 3, 4, 4, 5, 0}, col_oob[9] = {0, 1, 9, 2, 3, 4, 4, 5, 0};
    const uint8_t coef_zero[9] = {1, 0, 3, 1, 2, 3, 1, 2, 3}, coef_big[9] = {1, 4, 3, 1, 2, 3, 1, 2, 3};
    const std::vector<Case> cases = {
        {"q not a power of two", 6, 0, col_ok, coef_ok, {}, {}},
        {"repeated column", 4, 0, col_rep, coef_ok, {}, {}},
        {"column out of range", 4, 0, col_oob, coef_ok, {}, {}},
        {"zero coefficient", 4, 0, col_ok, coef_zero, {}, {}},
        {"coefficient beyond q", 4, 0, col_ok, coef_big, {}, {}},
        {"visit order not a permutation", 4, 0, col_ok, coef_ok, {0, 1, 2, 3, 4, 4}, {}},
        {"visit order out of range", 4, 0, col_ok, coef_ok, {0, 1, 2, 3, 4, 6}, {}},
        {"source chain repeated", 4, 2, col_ok, coef_ok, {}, {1, 1}},
        {"source chain out of range", 4, 2, col_ok, coef_ok, {}, {0, 7}},
    };
    for (const Case &c : cases) {
        gfbp_code_desc d{};
        d.q = c.q;
        d.n = 6;
        d.m = 3;
        d.n_info = c.n_info;
        d.row_ptr = row_ptr;
        d.col = c.col;
        d.coef = c.coef;
        d.visit_order = c.visit.empty() ? nullptr : c.visit.data();
        d.source_cols = c.src.empty() ? nullptr : c.src.data();
        CodePlan pl;
        std::string err;
        CHECK(build_plan(&d, pl, err) != GFBP_OK && !err.empty(), c.what);
    }
    return true;
}

// The LDS layout of the whole decode in LDS: every array the decode uses
// lies inside the workgroup's bytes, 16-byte aligned, apart from every other;
// the total fits the limit; the frames per workgroup are the most that fit
// in half the limit (at most four, at most the batch), else one if one fits
// at all, else none.
static bool check_onchip_layout(int code_id) {
    const int q = 2 << (rnd() % 3);
    const int n = 8 + int(rnd() % 3000), m = 4 + int(rnd() % (n / 2 + 1)), K = int(rnd() % (n + 1));
    const int max_dv = 1 + int(rnd() % 8), E = n * (1 + int(rnd() % max_dv)), nlev = 1 + int(rnd() % n);
    const bool pus = rnd() % 2, prior_on = rnd() % 2, markov = prior_on && (rnd() % 2);
    const int frames = 1 + int(rnd() % 3000), limit = (rnd() % 2) ? 163840 : 65536;
    const OnchipLayout ly = onchip_layout_for(q, E, n, m, K, max_dv, nlev, pus, prior_on, markov, frames, limit);
    // the arrays and their sizes, restated from the decode's use of them
    struct Arr {
        int off;
        size_t bytes;
        bool used;
        bool per_frame;
    };
    const size_t Q = size_t(q);
    const Arr arrs[] = {
        {ly.qm, E * Q * 4, true, true},   {ly.r, E * Q * 4, pus, true},        {ly.l, n * Q * 4, true, true},
        {ly.pr, K * Q * 4, prior_on, true}, {ly.qp, K * Q * 4, markov, true}, {ly.xh, size_t(n), true, true},
        {ly.z, size_t(m), true, true},     {ly.mul, Q * Q, true, false},      {ly.flags, 5 * 4 * 4, true, false},
        {ly.rsh, 256 * Q * 4, !pus, false}, {ly.eg, size_t(E) * 4, true, false}, {ly.erow, size_t(E) * 2, true, false},
        {ly.ecol, size_t(E) * 2, true, false}, {ly.cedge, size_t(E) * 2, true, false},
        {ly.cg, size_t(n) * 4, true, false}, {ly.ck, size_t(n) * 2, true, false}, {ly.rrow, size_t(m) * 4, true, false},
        {ly.kcol, size_t(K) * 2, true, false}, {ly.lcol, size_t(n) * 2, !pus, false},
        {ly.lptr, size_t(nlev + 1) * 2, !pus, false}, {ly.pe, size_t(n) * max_dv * 4, !pus, false},
        {ly.mk, (4 + Q + Q * Q) * 4, markov, false}};
    size_t frame = 0, shared = 0;
    for (const Arr &a : arrs) (a.per_frame ? frame : shared) += a.used ? (a.bytes + 15) / 16 * 16 : 0;
    const size_t one = frame + shared;
    if (ly.fw == 0) {
        CHECK(one > size_t(limit), "no frames per workgroup although one frame fits");
        return true;
    }
    CHECK(ly.fw >= 1 && ly.fw <= 4 && ly.fw <= frames, "frames per workgroup out of range");
    CHECK(size_t(ly.frame) == frame, "frame block size");
    CHECK(size_t(ly.total) == ly.fw * frame + shared && ly.total <= limit, "total bytes");
    const int best_half = [&] {
        for (int k = 4; k >= 1; --k)
            if (k * frame + shared <= size_t(limit) / 2) return k;
        return 0;
    }();
    CHECK(ly.fw == std::min(best_half > 0 ? best_half : 1, frames), "frames per workgroup not the most that fit");
    // every used array inside the workgroup's bytes, aligned, and apart
    std::vector<std::pair<size_t, size_t>> spans;
    for (const Arr &a : arrs) {
        if (!a.used) {
            CHECK(a.off == -1, "an unused array has an offset");
            continue;
        }
        CHECK(a.off >= 0 && a.off % 16 == 0, "array offset negative or unaligned");
        for (int w = 0; w < (a.per_frame ? ly.fw : 1); ++w) {
            const size_t b0 = size_t(a.off) + (a.per_frame ? size_t(w) * frame : 0);
            CHECK(b0 + a.bytes <= size_t(ly.total), "array beyond the workgroup's LDS");
            if (a.bytes) spans.push_back({b0, b0 + a.bytes});
        }
    }
    std::sort(spans.begin(), spans.end());
    for (size_t k = 1; k < spans.size(); ++k) CHECK(spans[k].first >= spans[k - 1].second, "arrays overlap");
    return true;
}

int main(int argc, char **argv) {
    const int count = argc > 1 ? std::atoi(argv[1]) : 400;
    if (!check_refusals(-1)) return 1;
    for (int k = 0; k < count; ++k)
        if (!check_valid(k)) return 1;
    for (int k = 0; k < 4 * count; ++k)
        if (!check_onchip_layout(k)) return 1;
    std::printf("ok %d\n", count);
    return 0;
}
