// Host-side plan of a code for gfbp_code_build: the checks of the
// description, the field's tables, the column index, each edge's coefficient
// maps, the visiting order and source chain, and the SUS dependency levels
// with their per-edge records.  Plain C++ (no device code), so that it also
// builds and runs on the host alone.
#pragma once
#include <stdint.h>

#include <algorithm>
#include <string>
#include <vector>

#include "../../include/gfbp.h"

namespace gfbp {

// One edge slot of a column in the sequential schedule, precomputed so that
// a column step starts from a single wave-uniform load: the column j and its
// degree dv, and for slots below dv the edge e, its row i, the row's first
// edge rs, the row degree dc, e's place in its row (self) and the packed
// images of the basis under h_e^-1 and h_e.
struct SusRec {
    int32_t j, dv, e, i, rs, dc, self, pad;
    uint64_t hinv, h;
};

// SUS levels with at most this many columns are walked in runs (k_sus_run):
// one launch then costs more than walking a couple of columns in a row
constexpr int kThinLevel = 2;

// One levelisation of the SUS sweep.
struct LevelPlan {
    std::vector<int32_t> ptr;   // level l: the columns at positions ptr[l]..ptr[l+1]-1 of the records
    std::vector<double> sibs;   // per level: sibling vectors read (sum over its edges of d_c - 1)
    std::vector<double> edges;  // per level: edges
    std::vector<double> src;    // per level: source columns
    // launches of one sweep: a wide level alone (one workgroup per column
    // and tile), or a run of consecutive thin levels (one per tile)
    struct Seg {
        int c0, nc, run;
        double sibs, edges, src;
    };
    std::vector<Seg> segs;
};

struct CodePlan {
    int q = 0, p = 0, n = 0, m = 0, E = 0, K = 0, max_dc = 0, max_dv = 0;
    unsigned poly = 0;
    double sum_dc2 = 0;                      // sum over checks of d_c (d_c - 1)
    std::vector<uint8_t> mul, inv;           // [q][q] products, [q] inverses
    std::vector<int32_t> col_ptr, col_edge, edge_row, visit, chain_col, col_chain;
    std::vector<uint64_t> emap;              // [E][2] basis images under h^-1 and h
    LevelPlan lv[2];                         // [0] shared checks; [1] also the source chain
    std::vector<SusRec> recs[2];             // [n][max(1, max_dv)] records in level order
};

inline gfbp_status plan_fail(std::string &err, gfbp_status s, const char *msg) {
    err = msg;
    return s;
}

// GF(2^p) tables of a primitive polynomial (false if it is not primitive of degree p).
inline bool field_tables(int p, unsigned poly, std::vector<uint8_t> &mul, std::vector<uint8_t> &inv) {
    const int q = 1 << p;
    if (poly >> p != 1u) return false;
    std::vector<int> ex(2 * q), lg(q, -1);
    int v = 1;
    for (int i = 0; i < q - 1; ++i) {
        if (lg[v] != -1) return false;  // x is not primitive
        ex[i] = ex[i + q - 1] = v;
        lg[v] = i;
        v <<= 1;
        if (v & q) v ^= int(poly);
    }
    if (v != 1) return false;
    mul.assign(size_t(q) * q, 0);
    inv.assign(q, 0);
    for (int a = 1; a < q; ++a) {
        for (int b = 1; b < q; ++b) mul[a * q + b] = uint8_t(ex[lg[a] + lg[b]]);
        inv[a] = uint8_t(ex[(q - 1 - lg[a]) % (q - 1)]);
    }
    return true;
}

inline constexpr unsigned kDefaultPoly[7] = {0, 0x3, 0x7, 0xB, 0x13, 0x25, 0x43};

// Validate the description and build the plan; on failure returns the status
// and sets err.
inline gfbp_status build_plan(const gfbp_code_desc *d, CodePlan &pl, std::string &err) {
    const int q = d->q;
    int p = 0;
    while ((1 << p) < q) ++p;
    if (q < 2 || q > GFBP_MAX_Q || (1 << p) != q) return plan_fail(err, GFBP_EUNSUPPORTED, "q must be 2^p with 1 <= p <= 6");
    if (d->n <= 0 || d->m <= 0 || d->n_info < 0 || d->n_info > d->n)
        return plan_fail(err, GFBP_EINVAL, "bad n, m or n_info");
    if (!d->row_ptr || !d->col || !d->coef) return plan_fail(err, GFBP_EINVAL, "null row_ptr/col/coef");
    const unsigned poly = d->poly ? unsigned(d->poly) : kDefaultPoly[p];
    std::vector<uint8_t> mul, inv;
    if (!field_tables(p, poly, mul, inv)) return plan_fail(err, GFBP_EINVAL, "polynomial is not primitive of degree p");
    const int n = d->n, m = d->m;
    if (d->row_ptr[0] != 0) return plan_fail(err, GFBP_EINVAL, "row_ptr[0] must be 0");
    for (int i = 0; i < m; ++i)
        if (d->row_ptr[i + 1] < d->row_ptr[i]) return plan_fail(err, GFBP_EINVAL, "row_ptr not nondecreasing");
    const int E = d->row_ptr[m];
    int max_dc = 0;
    double sum_dc2 = 0;
    std::vector<int> col_deg(n, 0), seen(n, -1);
    for (int i = 0; i < m; ++i) {
        const int dc = d->row_ptr[i + 1] - d->row_ptr[i];
        max_dc = dc > max_dc ? dc : max_dc;
        sum_dc2 += double(dc) * (dc - 1);
        for (int e = d->row_ptr[i]; e < d->row_ptr[i + 1]; ++e) {
            const int j = d->col[e];
            if (j < 0 || j >= n) return plan_fail(err, GFBP_EINVAL, "column index out of range");
            if (d->coef[e] == 0 || d->coef[e] >= q) return plan_fail(err, GFBP_EINVAL, "coefficient not in GF(q)\\{0}");
            if (seen[j] == i) return plan_fail(err, GFBP_EINVAL, "column repeated in a row");
            seen[j] = i;
            col_deg[j]++;
        }
    }
    int max_dv = 0;
    for (int j = 0; j < n; ++j) max_dv = col_deg[j] > max_dv ? col_deg[j] : max_dv;
    if (max_dc > GFBP_MAX_ROW_DEGREE) return plan_fail(err, GFBP_EUNSUPPORTED, "row degree above GFBP_MAX_ROW_DEGREE");
    if (max_dv > GFBP_MAX_COL_DEGREE) return plan_fail(err, GFBP_EUNSUPPORTED, "column degree above GFBP_MAX_COL_DEGREE");

    std::vector<int32_t> col_ptr(n + 1, 0), col_edge(E), edge_row(E), fill(n, 0);
    for (int j = 0; j < n; ++j) col_ptr[j + 1] = col_ptr[j] + col_deg[j];
    for (int i = 0; i < m; ++i)
        for (int e = d->row_ptr[i]; e < d->row_ptr[i + 1]; ++e) {
            edge_row[e] = i;
            const int j = d->col[e];
            col_edge[col_ptr[j] + fill[j]++] = e;
        }
    // per-edge images of the basis x^b under multiplication by h^-1 and h
    std::vector<uint64_t> emap(2 * size_t(E));
    for (int e = 0; e < E; ++e) {
        const int h = d->coef[e], hi = inv[h];
        uint64_t wi = 0, wm = 0;
        for (int b = 0; b < p; ++b) {
            wi |= uint64_t(mul[hi * q + (1 << b)]) << (6 * b);
            wm |= uint64_t(mul[h * q + (1 << b)]) << (6 * b);
        }
        emap[2 * size_t(e)] = wi;
        emap[2 * size_t(e) + 1] = wm;
    }

    // visiting order and source chain (defaults: 0..n-1 and 0..n_info-1)
    const int K = d->n_info;
    std::vector<int32_t> visit(n), chain_col(std::max(K, 1), 0), col_chain(n, -1), vpos(n, -1);
    for (int t = 0; t < n; ++t) {
        const int j = d->visit_order ? d->visit_order[t] : t;
        if (j < 0 || j >= n || vpos[j] >= 0) return plan_fail(err, GFBP_EINVAL, "visit_order is not a permutation of 0..n-1");
        visit[t] = j;
        vpos[j] = t;
    }
    for (int k = 0; k < K; ++k) {
        const int j = d->source_cols ? d->source_cols[k] : k;
        if (j < 0 || j >= n || col_chain[j] >= 0) return plan_fail(err, GFBP_EINVAL, "source_cols out of range or repeated");
        chain_col[k] = j;
        col_chain[j] = k;
    }

    // SUS dependency levels, taking the columns in visiting order:
    // level(j) = 1 + the highest level among columns visited earlier that
    // share a check with j (0 if none); with chain = 1 a source column also
    // comes after its chain neighbours visited earlier (their pseudo-
    // posteriors of the same sweep give its prior).  Then the sequential-
    // schedule records, columns in level order, RS slots each.
    const int RS = std::max(1, max_dv);
    LevelPlan *lvs = pl.lv;
    std::vector<SusRec> *recs = pl.recs;
    for (int chain = 0; chain < 2; ++chain) {
        std::vector<int32_t> level(n, 0), row_top(m, -1);
        int nlev = 0;
        for (int t = 0; t < n; ++t) {
            const int j = visit[t];
            int lv = 0;
            for (int u = col_ptr[j]; u < col_ptr[j + 1]; ++u) lv = std::max(lv, row_top[edge_row[col_edge[u]]] + 1);
            const int k = col_chain[j];
            if (chain && k >= 0)
                for (int kk = k - 1; kk <= k + 1; kk += 2)
                    if (kk >= 0 && kk < K && vpos[chain_col[kk]] < t) lv = std::max(lv, level[chain_col[kk]] + 1);
            for (int u = col_ptr[j]; u < col_ptr[j + 1]; ++u) row_top[edge_row[col_edge[u]]] = lv;
            level[j] = lv;
            nlev = std::max(nlev, lv + 1);
        }
        LevelPlan &L = lvs[chain];
        L.ptr.assign(nlev + 1, 0);
        L.sibs.assign(nlev, 0.0);
        L.edges.assign(nlev, 0.0);
        L.src.assign(nlev, 0.0);
        std::vector<int32_t> cols(n);
        for (int j = 0; j < n; ++j) L.ptr[level[j] + 1]++;
        for (int l = 0; l < nlev; ++l) L.ptr[l + 1] += L.ptr[l];
        std::vector<int32_t> fillp(L.ptr.begin(), L.ptr.end() - 1);
        for (int t = 0; t < n; ++t) {
            const int j = visit[t];
            const int l = level[j];
            cols[fillp[l]++] = j;
            L.src[l] += col_chain[j] >= 0 ? 1.0 : 0.0;
            for (int u = col_ptr[j]; u < col_ptr[j + 1]; ++u) {
                const int i = edge_row[col_edge[u]];
                L.sibs[l] += d->row_ptr[i + 1] - d->row_ptr[i] - 1;
                L.edges[l] += 1;
            }
        }
        // levels of at most kThinLevel columns are walked in runs
        for (int l = 0; l < nlev; ++l) {
            const int c0 = L.ptr[l], nc = L.ptr[l + 1] - c0;
            const bool thin = nc <= kThinLevel;
            if (thin && !L.segs.empty() && L.segs.back().run) {
                LevelPlan::Seg &g = L.segs.back();
                g.nc += nc;
                g.sibs += L.sibs[l];
                g.edges += L.edges[l];
                g.src += L.src[l];
            } else {
                L.segs.push_back({c0, nc, thin ? 1 : 0, L.sibs[l], L.edges[l], L.src[l]});
            }
        }
        recs[chain].resize(size_t(n) * RS);
        for (int p = 0; p < n; ++p) {
            const int j = cols[p], dv = col_ptr[j + 1] - col_ptr[j];
            for (int t = 0; t < RS; ++t) {
                SusRec r{};
                r.j = j;
                r.dv = dv;
                if (t < dv) {
                    const int e = col_edge[col_ptr[j] + t], i = edge_row[e];
                    r.e = e;
                    r.i = i;
                    r.rs = d->row_ptr[i];
                    r.dc = d->row_ptr[i + 1] - d->row_ptr[i];
                    r.self = e - r.rs;
                    r.hinv = emap[2 * size_t(e)];
                    r.h = emap[2 * size_t(e) + 1];
                }
                recs[chain][size_t(p) * RS + t] = r;
            }
        }
    }

    pl.q = q;
    pl.p = p;
    pl.n = n;
    pl.m = m;
    pl.E = E;
    pl.K = K;
    pl.max_dc = max_dc;
    pl.max_dv = max_dv;
    pl.poly = poly;
    pl.sum_dc2 = sum_dc2;
    pl.mul = std::move(mul);
    pl.inv = std::move(inv);
    pl.col_ptr = std::move(col_ptr);
    pl.col_edge = std::move(col_edge);
    pl.edge_row = std::move(edge_row);
    pl.visit = std::move(visit);
    pl.chain_col = std::move(chain_col);
    pl.col_chain = std::move(col_chain);
    pl.emap = std::move(emap);
    return GFBP_OK;
}

// LDS layout of a whole decode in LDS (gfbp_onchip.h): byte offsets of every
// array, in a frame block (qm .. z) or from the start of LDS (mul .. mk);
// -1 for an array the decode does not use.  fw = 0: one frame does not fit.
struct OnchipLayout {
    int fw;                          // frames per workgroup
    int frame;                       // bytes per frame block (16-byte multiple)
    int qm, r, l, pr, qp, xh, z;     // frame block: Qm [E][q], R [E][q] (PUS), L [n][q], Pr [K][q] (prior),
                                     // Qp [K][q] (Markov) floats; xh [n], z [m] bytes
    int mul, flags, rsh;             // the field table [q][q]; frame flags; SUS r scratch [threads][q]
    int eg, erow, ecol, cedge, cg, ck, rrow, kcol, lcol, lptr;  // the packed graph (lcol, lptr: SUS)
    int pe;                          // SUS: [n][rs] u32, the edge of each (position, slot) | degree << 16
    int mk;                          // Markov source: shape [4], pi [q], M [q][q] floats
    int total;                       // bytes of LDS per workgroup
};

constexpr int kOnchipThreads = 256;
constexpr int kOnchipMaxFW = 4;
constexpr int kOnchipFlags = 5;  // int32 [kOnchipMaxFW] each: active, unsat, guards, iterations, converged

// The layout for a code (q, E edges, n columns, m rows, K source symbols,
// column degree up to max_dv, nlev SUS levels), a schedule and prior, a batch
// of `frames` frames and `limit` bytes of LDS per workgroup.  Frames per
// workgroup: as many (up to kOnchipMaxFW) as fit in half the limit (two
// workgroups per compute unit), else one if one fits in all of it.
inline OnchipLayout onchip_layout_for(int q_, int E_, int n_, int m_, int K_, int max_dv, int nlev, bool pus,
                                      bool prior_on, bool markov, int frames, int limit) {
    OnchipLayout ly{};
    const size_t q = size_t(q_), E = size_t(E_), n = size_t(n_), m = size_t(m_), K = size_t(K_);
    size_t off = 0;
    auto take = [&](size_t bytes, bool on) -> int {
        if (!on) return -1;
        const size_t o = off;
        off += (bytes + 15) & ~size_t(15);
        return int(std::min<size_t>(o, size_t(1) << 30));
    };
    ly.qm = take(E * q * 4, true);
    ly.r = take(E * q * 4, pus);
    ly.l = take(n * q * 4, true);
    ly.pr = take(K * q * 4, prior_on);
    ly.qp = take(K * q * 4, markov);
    ly.xh = take(n, true);
    ly.z = take(m, true);
    const size_t frame = off;
    off = 0;  // the shared part, offsets from its start
    const int o_mul = take(q * q, true);
    const int o_flags = take(size_t(kOnchipFlags) * kOnchipMaxFW * 4, true);
    const int o_rsh = take(size_t(kOnchipThreads) * q * 4, !pus);
    const int o_eg = take(E * 4, true);
    const int o_erow = take(E * 2, true);
    const int o_ecol = take(E * 2, true);
    const int o_cedge = take(E * 2, true);
    const int o_cg = take(n * 4, true);
    const int o_ck = take(n * 2, true);
    const int o_rrow = take(m * 4, true);
    const int o_kcol = take(K * 2, true);
    const int o_lcol = take(n * 2, !pus);
    const int o_lptr = take((size_t(std::max(0, nlev)) + 1) * 2, !pus);
    const int o_pe = take(n * size_t(std::max(1, max_dv)) * 4, !pus);
    const int o_mk = take((4 + q + q * q) * 4, markov);
    const size_t shared = off;
    const size_t lim = size_t(std::max(0, limit));
    int fw = 0;
    for (int k = kOnchipMaxFW; k >= 1 && fw == 0; --k)
        if (size_t(k) * frame + shared <= lim / 2) fw = k;
    if (fw == 0 && frame + shared <= lim) fw = 1;
    fw = std::min(fw, std::max(1, frames));
    if (fw == 0) return OnchipLayout{};
    ly.fw = fw;
    ly.frame = int(frame);
    const int base = int(size_t(fw) * frame);
    auto at = [&](int o) { return o < 0 ? -1 : base + o; };
    ly.mul = at(o_mul);
    ly.flags = at(o_flags);
    ly.rsh = at(o_rsh);
    ly.eg = at(o_eg);
    ly.erow = at(o_erow);
    ly.ecol = at(o_ecol);
    ly.cedge = at(o_cedge);
    ly.cg = at(o_cg);
    ly.ck = at(o_ck);
    ly.rrow = at(o_rrow);
    ly.kcol = at(o_kcol);
    ly.lcol = at(o_lcol);
    ly.lptr = at(o_lptr);
    ly.pe = at(o_pe);
    ly.mk = at(o_mk);
    ly.total = int(size_t(fw) * frame + shared);
    return ly;
}

}  // namespace gfbp
