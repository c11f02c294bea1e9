// Decoding with the frames' whole message state in LDS.
//
// When one frame's messages, evidence, priors and decisions fit in a part of
// a compute unit's 160 KB of LDS (small codes over GF(2), GF(4), GF(8)), a
// workgroup decodes FW frames from their initial messages to their final
// decisions in one launch: every iteration's schedule (A3-A4 for PUS, the
// dependency levels of A6 for SUS), the H x = z test and retirement (A5) and
// the Markov refresh (A7) run between workgroup barriers, and HBM is touched
// only to load the initial state (written by the initialisation kernel) and
// to store the results.  The iterations cost no launches and no host round
// trips, which is what bounds such codes on the tiled kernels (a few
// microseconds of work per launch, dozens of launches per SUS iteration).
//
// A q-vector (q <= 8) is held in registers by the lanes of an item (PUS: one
// lane; SUS: q/2 lanes of two entries), laid out as the tiled kernels lay out
// a frame's lanes, and the arithmetic is theirs at that shape: the same
// transforms and lane exchanges, products in the same order, the same
// normalisation and clipping, float32 storage of every message; so the
// results are bitwise those of the tiled decode at the same entries per lane.
//
// LDS of a workgroup: FW frame blocks, then the shared part.  A frame block
// holds (floats, [node][a]) Qm [E][q] (weighted domain, as in global memory),
// R [E][q] (PUS), L [n][q], Pr [K][q] (with a prior), Qp [K][q] (Markov: the
// pseudo-posterior of each source symbol's column), then bytes xh [n] and
// z [m].  The shared part holds the field's multiplication table, the
// frames' flags and counters, for SUS the r-messages of the columns of one
// pass over a level ([threads][q] floats), and the graph, packed, so that no
// iteration reads global memory: per edge its row's first edge, the row's
// degree, the edge's place in the row, its coefficient h and h^-1 (one word),
// its row, its column and the edges of each column in column order (16 bits
// each); per column its first edge and degree, and its source symbol + 1;
// per row its first edge and degree; per source symbol its column; for SUS
// the columns in level order, the first position of each level and, per
// (position, edge slot), the slot's edge and the column's degree.
#pragma once
#include "gfbp_tiled.h"

namespace gfbp {
namespace onchip {

constexpr int kThreads = kOnchipThreads;
constexpr int kMaxFW = kOnchipMaxFW;  // frames per workgroup, at most
constexpr int kMaxP = 3;              // q <= 8: a thread's vectors stay in registers

// Byte offsets of the LDS arrays, computed on the host (onchip_layout_for).
using Layout = OnchipLayout;

// log2 of the lanes holding one vector.  PUS: one lane per vector (every
// phase has work for all the workgroup's lanes; spreading a vector over more
// lanes only adds exchanges: GF(4) N = 504, 2048 frames running, 41 against
// 69 us per iteration).  SUS: two entries per lane (a dependency level has
// few columns, and the lanes of a vector shorten each one's dependent chain:
// 10.3 against 11.0 ms for 2000 frames).
template <int P>
constexpr int lanes_log(int schedule) {
    return schedule == GFBP_SUS ? P - 1 : 0;
}

// One edge's word of the packed graph.
__device__ __forceinline__ uint32_t pack_edge(int rs, int dc, int self, int h, int hinv) {
    return uint32_t(rs) | (uint32_t(dc) << 16) | (uint32_t(self) << 21) | (uint32_t(h) << 26) |
           (uint32_t(hinv) << 29);
}
__device__ __forceinline__ int eg_rs(uint32_t w) { return int(w & 0xffffu); }
__device__ __forceinline__ int eg_dc(uint32_t w) { return int((w >> 16) & 31u); }
__device__ __forceinline__ int eg_self(uint32_t w) { return int((w >> 21) & 31u); }
__device__ __forceinline__ int eg_h(uint32_t w) { return int((w >> 26) & 7u); }
__device__ __forceinline__ int eg_hinv(uint32_t w) { return int(w >> 29); }

// Per-frame flags in the shared part: int32 [kMaxFW] each.
enum { F_ACTIVE = 0, F_UNSAT = 1, F_GUARDS = 2, F_ITERS = 3, F_CONV = 4, F_NFLAGS = 5 };
static_assert(F_NFLAGS == kOnchipFlags, "the layout's flag words");

struct Args {
    DevCode c;
    const float *Qm, *L, *Pr;  // initial state in global memory, [node][Fp][q]
    const int32_t *guards0;    // [F] guard events of the initialisation
    int F, Fp;
    const uint8_t *z;          // [F][m] syndromes, or null for z = 0
    int schedule, max_iter, early_stop, prior_on, markov, wantQ;
    const float *M, *pi, *mshape;  // Markov source (markov != 0)
    const SusRec *recs;        // SUS: columns in level order, rs records each
    const int32_t *lvl;        // [nlev + 1] first record position of each level
    int nlev, rs;
    uint8_t *xhat;             // [F][n]
    int32_t *iters;            // [F]
    uint8_t *conv;             // [F]
    int32_t *guards;           // [F] or null
    Layout lay;
};

// Lane geometry (that of the tiled kernels): an item (an edge, a column, a
// source symbol of one frame) is held by G = 2^LG lanes with EL = q/G entries
// each; a wavefront holds TF = 64/G items, lane = g*TF + item, and lane g
// holds entries g*EL .. g*EL + EL - 1 of the item's vectors.

// Normalise the item's distributed vector to sum 1 (the tiled kernels'
// order: each lane's entries, then across the lanes); uniform and false when
// the sum is zero or not finite.
template <int P, int LG>
__device__ __forceinline__ bool normalise_l(double *v) {
    using Gm = tiled::Geo<P, LG>;
    double s = 0.0;
#pragma unroll
    for (int r = 0; r < Gm::EL; ++r) s += v[r];
    s = tiled::lanes_sum<P, LG>(s);
    if (!(s > 0.0) || !isfinite(s)) {
#pragma unroll
        for (int r = 0; r < Gm::EL; ++r) v[r] = 1.0 / double(Gm::Q);
        return false;
    }
    const double inv = 1.0 / s;
#pragma unroll
    for (int r = 0; r < Gm::EL; ++r) v[r] *= inv;
    return true;
}

// This lane's EL entries of a q-vector in LDS, in one access.
template <int EL>
__device__ __forceinline__ void lds_vec(const float *p, float *v) {
    if constexpr (EL == 1) {
        v[0] = p[0];
    } else if constexpr (EL == 2) {
        const tiled::f32x2 t = *reinterpret_cast<const tiled::f32x2 *>(p);
        v[0] = t.x;
        v[1] = t.y;
    } else {
#pragma unroll
        for (int k = 0; k < EL / 4; ++k) {
            const tiled::f32x4 t = reinterpret_cast<const tiled::f32x4 *>(p)[k];
            v[4 * k] = t.x;
            v[4 * k + 1] = t.y;
            v[4 * k + 2] = t.z;
            v[4 * k + 3] = t.w;
        }
    }
}

// a x (g*EL + r) for this lane's entries r, from row a of the multiplication
// table, read as one word.
template <int P, int LG>
__device__ __forceinline__ void mul_pos(const uint8_t *mul, int a, int g, int *out) {
    using Gm = tiled::Geo<P, LG>;
    const uint8_t *row = mul + a * Gm::Q + g * Gm::EL;
    uint64_t w;
    if constexpr (Gm::EL == 1) w = row[0];
    else if constexpr (Gm::EL == 2) w = *reinterpret_cast<const uint16_t *>(row);
    else if constexpr (Gm::EL == 4) w = *reinterpret_cast<const uint32_t *>(row);
    else w = *reinterpret_cast<const uint64_t *>(row);
    static_assert(Gm::EL <= 8, "entries per lane");
#pragma unroll
    for (int r = 0; r < Gm::EL; ++r) out[r] = int((w >> (8 * r)) & 0xffu);
}

// A3 for one edge: r from the siblings (row positions 0..dc-1 except `self`)
// in row order, T = WHT(signs(z) x prod WHT(q~)), r(h^-1 y) = T(y) / q.
// Where registers allow, every sibling is requested before the first is used.
template <int P, int LG, int DCM>
__device__ __forceinline__ void edge_r(const float *qm, int rs, int dc, int self, int zi, const uint8_t *mul,
                                       int hinv, int g, float *rout) {
    using Gm = tiled::Geo<P, LG>;
    constexpr int Q = Gm::Q, EL = Gm::EL;
    constexpr bool kPre = (DCM - 1) * EL <= 40;
    int pos[EL];
    mul_pos<P, LG>(mul, hinv, g, pos);
    double T[EL];
    tiled::syndrome_signs<P, LG>(zi, g, T);
    const float *base = qm + g * EL;
    if constexpr (kPre) {
        float raw[DCM - 1][EL];
#pragma unroll
        for (int u = 0; u < DCM - 1; ++u)
            if (u < dc - 1) lds_vec<EL>(base + size_t(rs + (u < self ? u : u + 1)) * Q, raw[u]);
#pragma unroll
        for (int u = 0; u < DCM - 1; ++u)
            if (u < dc - 1) {
                double W[EL];
#pragma unroll
                for (int r = 0; r < EL; ++r) W[r] = double(raw[u][r]);
                tiled::wht<P, LG>(W, g);
#pragma unroll
                for (int r = 0; r < EL; ++r) T[r] *= W[r];
            }
    } else {
        for (int u = 0; u < dc; ++u) {
            if (u == self) continue;
            float raw[EL];
            lds_vec<EL>(base + size_t(rs + u) * Q, raw);
            double W[EL];
#pragma unroll
            for (int r = 0; r < EL; ++r) W[r] = double(raw[r]);
            tiled::wht<P, LG>(W, g);
#pragma unroll
            for (int r = 0; r < EL; ++r) T[r] *= W[r];
        }
    }
    tiled::wht<P, LG>(T, g);
#pragma unroll
    for (int r = 0; r < EL; ++r) rout[pos[r]] = float(fmax(T[r] * (1.0 / double(Q)), 0.0));
}

// Two edges at once (independent chains interleaved); the second one's result
// is stored only when st1.  Rows of at most DCM entries; a missing sibling
// multiplies by 1 (exact).
template <int P, int LG, int DCM>
__device__ __forceinline__ void edge_r_pair(const float *qm0, const float *qm1, uint32_t ge0, uint32_t ge1, int z0,
                                            int z1, const uint8_t *mul, int g, float *rout0, float *rout1, bool st1) {
    using Gm = tiled::Geo<P, LG>;
    constexpr int Q = Gm::Q, EL = Gm::EL;
    const float *qm[2] = {qm0 + g * EL, qm1 + g * EL};
    const uint32_t ge[2] = {ge0, ge1};
    const int zi[2] = {z0, z1};
    int pos[2][EL];
    double T[2][EL];
    float raw[2][DCM - 1][EL];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        mul_pos<P, LG>(mul, eg_hinv(ge[h]), g, pos[h]);
        tiled::syndrome_signs<P, LG>(zi[h], g, T[h]);
        const int rs = eg_rs(ge[h]), dc = eg_dc(ge[h]), self = eg_self(ge[h]);
#pragma unroll
        for (int u = 0; u < DCM - 1; ++u) {
            const int t = u < dc - 1 ? (u < self ? u : u + 1) : self;
            lds_vec<EL>(qm[h] + size_t(rs + t) * Q, raw[h][u]);
        }
    }
#pragma unroll
    for (int u = 0; u < DCM - 1; ++u)
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            double W[EL];
#pragma unroll
            for (int r = 0; r < EL; ++r) W[r] = double(raw[h][u][r]);
            tiled::wht<P, LG>(W, g);
            const bool use = u < eg_dc(ge[h]) - 1;
#pragma unroll
            for (int r = 0; r < EL; ++r) T[h][r] *= use ? W[r] : 1.0;
        }
#pragma unroll
    for (int h = 0; h < 2; ++h) tiled::wht<P, LG>(T[h], g);
#pragma unroll
    for (int r = 0; r < EL; ++r) rout0[pos[0][r]] = float(fmax(T[0][r] * (1.0 / double(Q)), 0.0));
    if (st1)
#pragma unroll
        for (int r = 0; r < EL; ++r) rout1[pos[1][r]] = float(fmax(T[1][r] * (1.0 / double(Q)), 0.0));
}

// A4/A5 for a column from its r-vectors rv[0..dv) (this lane's entries,
// column edge order) and its prior row pv: the pseudo-posterior (Eq. (5)),
// into Qp_k (this lane's entries) when not null, and the decision (lane 0).
template <int P, int LG, int DVM>
__device__ __forceinline__ void posterior_step(const float (&rv)[DVM][tiled::Geo<P, LG>::EL], int dv,
                                               const double *pv, float *Qp_k, uint8_t *xh_j, int g, int *gd) {
    using Gm = tiled::Geo<P, LG>;
    double acc[Gm::EL];
#pragma unroll
    for (int q = 0; q < Gm::EL; ++q) acc[q] = pv[q];
#pragma unroll
    for (int d2 = 0; d2 < DVM; ++d2)
        if (d2 < dv)
#pragma unroll
            for (int q = 0; q < Gm::EL; ++q) acc[q] *= double(rv[d2][q]);
    if (!normalise_l<P, LG>(acc)) ++*gd;
    if (Qp_k)
#pragma unroll
        for (int q = 0; q < Gm::EL; ++q) Qp_k[q] = float(acc[q]);
    const int best = tiled::clip<P, LG>(acc, g);
    if (g == 0) *xh_j = uint8_t(best);
}

// Eq. (4) for edge slot d of the column: q from the prior and the other
// edges' r, normalised, this lane's entries stored at positions h (g*EL + r)
// of the edge's vector dst.
template <int P, int LG, int DVM>
__device__ __forceinline__ void edge_q_step(const float (&rv)[DVM][tiled::Geo<P, LG>::EL], int dv, const double *pv,
                                            int d, float *dst, const int *hpos, int *gd) {
    using Gm = tiled::Geo<P, LG>;
    double qv[Gm::EL];
#pragma unroll
    for (int q = 0; q < Gm::EL; ++q) qv[q] = pv[q];
#pragma unroll
    for (int d2 = 0; d2 < DVM; ++d2)
        if (d2 < dv && d2 != d)
#pragma unroll
            for (int q = 0; q < Gm::EL; ++q) qv[q] *= double(rv[d2][q]);
    if (!normalise_l<P, LG>(qv)) ++*gd;
#pragma unroll
    for (int q = 0; q < Gm::EL; ++q) dst[hpos[q]] = float(qv[q]);
}

// A7 for source symbol k (Eq. (7)): the neighbours' pseudo-posteriors
// Qp[k -+ 1] through M (O(q) when M is self-transition plus uniform), times
// the evidence of its column Lj, into pr (this lane's entries of each);
// guard events counted in *gd.
template <int P, int LG>
__device__ __forceinline__ void markov_row(const float *Qp, const float *Lj, int k, int K, const float *M,
                                           const float *pi, const float *mshape, float *pr, int g, int *gd) {
    using Gm = tiled::Geo<P, LG>;
    constexpr int Q = Gm::Q, EL = Gm::EL;
    double u[EL], v[EL];
#pragma unroll
    for (int q = 0; q < EL; ++q) {
        u[q] = k == 0 ? double(pi[g * EL + q]) : 0.0;
        v[q] = k == K - 1 ? 1.0 : 0.0;
    }
    if (mshape[0] != 0.0f) {
        const double sd = mshape[1], od = mshape[2];
        float nb[2][EL];
        double S[2] = {0.0, 0.0};
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int kk = h == 0 ? k - 1 : k + 1;
            if (kk >= 0 && kk < K)
                lds_vec<EL>(Qp + size_t(kk) * Q + g * EL, nb[h]);
            else
#pragma unroll
                for (int q = 0; q < EL; ++q) nb[h][q] = 0.0f;
#pragma unroll
            for (int q = 0; q < EL; ++q) S[h] += double(nb[h][q]);
            S[h] = tiled::lanes_sum<P, LG>(S[h]);
        }
        if (k > 0)
#pragma unroll
            for (int q = 0; q < EL; ++q) u[q] = sd * double(nb[0][q]) + od * (S[0] - double(nb[0][q]));
        if (k < K - 1)
#pragma unroll
            for (int q = 0; q < EL; ++q) v[q] = sd * double(nb[1][q]) + od * (S[1] - double(nb[1][q]));
    } else {
        if (k > 0) {
            const float *qp = Qp + size_t(k - 1) * Q;
#pragma unroll 2
            for (int a = 0; a < Q; ++a) {
                const double qa = qp[a];
#pragma unroll
                for (int q = 0; q < EL; ++q) u[q] += qa * double(M[a * Q + g * EL + q]);
            }
        }
        if (k < K - 1) {
            const float *qp = Qp + size_t(k + 1) * Q;
#pragma unroll 2
            for (int cc = 0; cc < Q; ++cc) {
                const double qc = qp[cc];
#pragma unroll
                for (int q = 0; q < EL; ++q) v[q] += double(M[(g * EL + q) * Q + cc]) * qc;
            }
        }
    }
#pragma unroll
    for (int q = 0; q < EL; ++q) u[q] *= v[q];
    if (!normalise_l<P, LG>(u)) ++*gd;
    float lf[EL];
    lds_vec<EL>(Lj + g * EL, lf);
#pragma unroll
    for (int q = 0; q < EL; ++q) u[q] *= double(lf[q]);
    if (!normalise_l<P, LG>(u)) ++*gd;
#pragma unroll
    for (int q = 0; q < EL; ++q) pr[g * EL + q] = float(u[q]);
}

template <int P, int LG, int DCM, int DVM>
__global__ __launch_bounds__(kThreads) void k_onchip(const Args a) {
    using Gm = tiled::Geo<P, LG>;
    constexpr int Q = Gm::Q, EL = Gm::EL;
    constexpr int NI = (kThreads / kWave) * Gm::TF;  // items a pass of the workgroup covers
    extern __shared__ __align__(16) unsigned char lds[];
    const DevCode &c = a.c;
    const Layout &ly = a.lay;
    const int tid = int(threadIdx.x);
    const int lane = tid % kWave;
    const int g = lane >> Gm::LTF;                                  // this lane's part of its item
    const int xi = (tid / kWave) * Gm::TF + (lane & (Gm::TF - 1));  // this lane's item
    const int f0 = int(blockIdx.x) * ly.fw;
    const int fw = min(ly.fw, a.F - f0);  // >= 1: the grid covers F exactly
    const int E = c.E, n = c.n, m = c.m, K = c.n_info;
    uint8_t *mul = lds + ly.mul;
    int32_t *flags = reinterpret_cast<int32_t *>(lds + ly.flags);
    int32_t *active = flags + F_ACTIVE * kMaxFW, *unsat = flags + F_UNSAT * kMaxFW,
            *gcount = flags + F_GUARDS * kMaxFW, *fiters = flags + F_ITERS * kMaxFW,
            *fconv = flags + F_CONV * kMaxFW;
    uint32_t *eg = reinterpret_cast<uint32_t *>(lds + ly.eg);
    uint16_t *erow = reinterpret_cast<uint16_t *>(lds + ly.erow);
    uint16_t *ecol = reinterpret_cast<uint16_t *>(lds + ly.ecol);
    uint16_t *cedge = reinterpret_cast<uint16_t *>(lds + ly.cedge);
    uint32_t *cg = reinterpret_cast<uint32_t *>(lds + ly.cg);
    uint16_t *ck = reinterpret_cast<uint16_t *>(lds + ly.ck);
    uint32_t *rrow = reinterpret_cast<uint32_t *>(lds + ly.rrow);
    uint16_t *kcol = reinterpret_cast<uint16_t *>(lds + ly.kcol);
    float *mk = reinterpret_cast<float *>(lds + ly.mk);  // Markov: shape [4], pi [q], M [q][q]
    auto blk = [&](int w) { return lds + size_t(w) * ly.frame; };
    auto Qm = [&](int w) { return reinterpret_cast<float *>(blk(w) + ly.qm); };
    auto Rr = [&](int w) { return reinterpret_cast<float *>(blk(w) + ly.r); };
    auto Lv = [&](int w) { return reinterpret_cast<float *>(blk(w) + ly.l); };
    auto Pr = [&](int w) { return reinterpret_cast<float *>(blk(w) + ly.pr); };
    auto Qp = [&](int w) { return reinterpret_cast<float *>(blk(w) + ly.qp); };
    auto Xh = [&](int w) { return blk(w) + ly.xh; };
    auto Zs = [&](int w) { return blk(w) + ly.z; };
    // prior-weighted evidence of column j (Pr for a source symbol with a prior)
    auto prow = [&](int w, int j) -> const float * {
        const int k1 = ck[j];
        return a.prior_on && k1 > 0 ? Pr(w) + size_t(k1 - 1) * Q : Lv(w) + size_t(j) * Q;
    };

    // ---- load: tables, graph, flags, the initial state
    for (int t = tid; t < Q * Q; t += kThreads) mul[t] = c.mul[t];
    for (int e = tid; e < E; e += kThreads) {
        const int i = c.edge_row[e], rs = c.row_ptr[i];
        const int h = int(c.coef[e]), hinv = int(c.emap[2 * size_t(e)] & 63u);  // images of 1
        eg[e] = pack_edge(rs, c.row_ptr[i + 1] - rs, e - rs, h, hinv);
        erow[e] = uint16_t(i);
        ecol[e] = uint16_t(c.col[e]);
        cedge[e] = uint16_t(c.col_edge[e]);
    }
    for (int j = tid; j < n; j += kThreads) {
        const int cs = c.col_ptr[j];
        cg[j] = uint32_t(cs) | (uint32_t(c.col_ptr[j + 1] - cs) << 16);
        ck[j] = uint16_t(c.col_chain[j] + 1);
    }
    for (int i = tid; i < m; i += kThreads) {
        const int rs = c.row_ptr[i];
        rrow[i] = uint32_t(rs) | (uint32_t(c.row_ptr[i + 1] - rs) << 16);
    }
    for (int k = tid; k < K; k += kThreads) kcol[k] = uint16_t(c.chain_col[k]);
    if (a.schedule == GFBP_SUS) {
        uint16_t *lcol = reinterpret_cast<uint16_t *>(lds + ly.lcol);
        uint16_t *lptr = reinterpret_cast<uint16_t *>(lds + ly.lptr);
        uint32_t *pe = reinterpret_cast<uint32_t *>(lds + ly.pe);
        for (int p = tid; p < n; p += kThreads) lcol[p] = uint16_t(a.recs[size_t(p) * a.rs].j);
        for (int l = tid; l <= a.nlev; l += kThreads) lptr[l] = uint16_t(a.lvl[l]);
        for (int t = tid; t < n * a.rs; t += kThreads) {  // edge of each (position, slot), and the degree
            const SusRec &r = a.recs[t];
            pe[t] = uint32_t(t % a.rs < r.dv ? r.e : 0) | (uint32_t(r.dv) << 16);
        }
    }
    if (a.markov) {
        for (int t = tid; t < 4; t += kThreads) mk[t] = a.mshape[t];
        for (int t = tid; t < Q; t += kThreads) mk[4 + t] = a.pi[t];
        for (int t = tid; t < Q * Q; t += kThreads) mk[4 + Q + t] = a.M[t];
    }
    if (tid < kMaxFW) {
        const bool on = tid < fw;
        active[tid] = on ? 1 : 0;
        unsat[tid] = 0;
        gcount[tid] = on ? a.guards0[f0 + tid] : 0;
        fiters[tid] = 0;
        fconv[tid] = 0;
    }
    // consecutive threads read the frames' adjacent vectors of one node
    for (int t = tid; t < E * fw * Q; t += kThreads) {
        const int q = t % Q, w = (t / Q) % fw, e = t / (Q * fw);
        Qm(w)[size_t(e) * Q + q] = a.Qm[(size_t(e) * a.Fp + size_t(f0 + w)) * Q + q];
    }
    for (int t = tid; t < n * fw * Q; t += kThreads) {
        const int q = t % Q, w = (t / Q) % fw, j = t / (Q * fw);
        Lv(w)[size_t(j) * Q + q] = a.L[(size_t(j) * a.Fp + size_t(f0 + w)) * Q + q];
    }
    if (a.prior_on)
        for (int t = tid; t < K * fw * Q; t += kThreads) {
            const int q = t % Q, w = (t / Q) % fw, k = t / (Q * fw);
            Pr(w)[size_t(k) * Q + q] = a.Pr[(size_t(k) * a.Fp + size_t(f0 + w)) * Q + q];
        }
    for (int t = tid; t < m * fw; t += kThreads) {
        const int w = t / m, i = t % m;
        Zs(w)[i] = a.z ? a.z[size_t(f0 + w) * m + i] : 0;
    }
    __syncthreads();

    for (int t = 1; t <= a.max_iter; ++t) {
        if (a.schedule == GFBP_PUS) {
            // A3: every edge's r from the previous iteration's q
            if constexpr (DCM <= 6) {
                for (int x = xi; x < E * fw; x += 2 * NI) {
                    const int x1 = min(x + NI, E * fw - 1);
                    const int w0 = x % fw, e0 = x / fw, w1 = x1 % fw, e1 = x1 / fw;
                    const bool a0 = active[w0] != 0, a1 = x + NI < E * fw && active[w1] != 0;
                    if (!a0 && !a1) continue;
                    // two edges' chains interleaved; an edge of a stopped
                    // frame (or past the end) is computed but not stored
                    const uint32_t g0 = eg[e0], g1 = eg[e1];
                    float scratch[Q];
                    edge_r_pair<P, LG, DCM>(Qm(w0), Qm(w1), g0, g1, Zs(w0)[erow[e0]], Zs(w1)[erow[e1]], mul, g,
                                            a0 ? Rr(w0) + size_t(e0) * Q : scratch, Rr(w1) + size_t(e1) * Q, a1);
                }
            } else {
                for (int x = xi; x < E * fw; x += NI) {
                    const int w = x % fw, e = x / fw;
                    if (!active[w]) continue;
                    const uint32_t ge = eg[e];
                    edge_r<P, LG, DCM>(Qm(w), eg_rs(ge), eg_dc(ge), eg_self(ge), Zs(w)[erow[e]], mul, eg_hinv(ge),
                                       g, Rr(w) + size_t(e) * Q);
                }
            }
            __syncthreads();
            // A4: every column's pseudo-posterior, decision and q
            for (int x = xi; x < n * fw; x += NI) {
                const int w = x % fw, j = x / fw;
                if (!active[w]) continue;
                const uint32_t gc = cg[j];
                const int cs = int(gc & 0xffffu), dv = int(gc >> 16);
                const float *R = Rr(w) + g * EL;
                float rv[DVM][EL];
                int es[DVM];
#pragma unroll
                for (int d = 0; d < DVM; ++d)
                    if (d < dv) {
                        es[d] = cedge[cs + d];
                        lds_vec<EL>(R + size_t(es[d]) * Q, rv[d]);
                    }
                float pf[EL];
                lds_vec<EL>(prow(w, j) + g * EL, pf);
                double pv[EL];
#pragma unroll
                for (int q = 0; q < EL; ++q) pv[q] = pf[q];
                int gd = 0;
                const int k1 = ck[j];
                posterior_step<P, LG, DVM>(rv, dv, pv,
                                           a.wantQ && k1 > 0 ? Qp(w) + size_t(k1 - 1) * Q + g * EL : nullptr,
                                           Xh(w) + j, g, &gd);
#pragma unroll
                for (int d = 0; d < DVM; ++d)
                    if (d < dv) {
                        int hp[EL];
                        mul_pos<P, LG>(mul, eg_h(eg[es[d]]), g, hp);
                        edge_q_step<P, LG, DVM>(rv, dv, pv, d, Qm(w) + size_t(es[d]) * Q, hp, &gd);
                    }
                if (gd && g == 0) atomicAdd(&gcount[w], gd);
            }
            __syncthreads();
        } else {
            // A6: the dependency levels in order; a level's columns share no
            // check, so each column's step is the one of the strict sweep.
            // Items (column of the pass, frame, edge slot); a pass holds as
            // many columns as the threads cover.
            const uint16_t *lcol = reinterpret_cast<const uint16_t *>(lds + ly.lcol);
            const uint16_t *lptr = reinterpret_cast<const uint16_t *>(lds + ly.lptr);
            const uint32_t *pe = reinterpret_cast<const uint32_t *>(lds + ly.pe);
            float *rsh = reinterpret_cast<float *>(lds + ly.rsh);
            const int per = fw * a.rs;
            const int cw = NI / per;
            const int col = xi / per, w = (xi % per) / a.rs, d = xi % a.rs;  // this lane's item
            for (int l = 0; l < a.nlev; ++l) {
                const int p0 = lptr[l], p1 = lptr[l + 1];
                for (int c0 = p0; c0 < p1; c0 += cw) {
                    const int nc = min(cw, p1 - c0);
                    const bool in = xi < nc * per;
                    const int p = c0 + (in ? col : 0);
                    const uint32_t pw = pe[size_t(p) * a.rs + d];
                    const int e = int(pw & 0xffffu), dv = int(pw >> 16);
                    const bool live = in && active[w] != 0;
                    if (live && d < dv) {
                        const uint32_t ge = eg[e];
                        edge_r<P, LG, DCM>(Qm(w), eg_rs(ge), eg_dc(ge), eg_self(ge), Zs(w)[erow[e]], mul,
                                           eg_hinv(ge), g, rsh + size_t(xi) * Q);
                    }
                    __syncthreads();
                    if (live && (d < dv || d == 0)) {
                        const int j = lcol[p];
                        float rv[DVM][EL];
#pragma unroll
                        for (int d2 = 0; d2 < DVM; ++d2)
                            if (d2 < dv) lds_vec<EL>(rsh + size_t(xi - d + d2) * Q + g * EL, rv[d2]);
                        float pf[EL];
                        lds_vec<EL>(prow(w, j) + g * EL, pf);
                        double pv[EL];
#pragma unroll
                        for (int q = 0; q < EL; ++q) pv[q] = pf[q];
                        int gd = 0;
                        if (d == 0) {
                            const int k1 = ck[j];
                            posterior_step<P, LG, DVM>(
                                rv, dv, pv, a.wantQ && k1 > 0 ? Qp(w) + size_t(k1 - 1) * Q + g * EL : nullptr,
                                Xh(w) + j, g, &gd);
                        }
                        if (d < dv) {
                            int hp[EL];
                            mul_pos<P, LG>(mul, eg_h(eg[e]), g, hp);
                            edge_q_step<P, LG, DVM>(rv, dv, pv, d, Qm(w) + size_t(e) * Q, hp, &gd);
                        }
                        if (gd && g == 0) atomicAdd(&gcount[w], gd);
                    }
                    __syncthreads();
                }
            }
        }
        // A5: H x = z on the decisions of this iteration
        for (int x = tid; x < m * fw; x += kThreads) {
            const int w = x % fw, i = x / fw;
            if (!active[w]) continue;
            const uint8_t *xh = Xh(w);
            const uint32_t gr = rrow[i];
            const int rs = int(gr & 0xffffu), re = rs + int(gr >> 16);
            int acc = 0;
            for (int e = rs; e < re; ++e) acc ^= mul[eg_h(eg[e]) * Q + xh[ecol[e]]];
            if (acc != Zs(w)[i]) unsat[w] = 1;
        }
        __syncthreads();
        if (tid < fw && active[tid]) {
            const bool ok = unsat[tid] == 0;
            if (ok && !fconv[tid]) {
                fconv[tid] = 1;
                fiters[tid] = t;
            }
            if ((ok && a.early_stop) || t >= a.max_iter) {
                active[tid] = 0;
                if (!fconv[tid]) fiters[tid] = a.max_iter;
                a.iters[f0 + tid] = fiters[tid];
                a.conv[f0 + tid] = uint8_t(fconv[tid]);
                if (a.guards) a.guards[f0 + tid] = gcount[tid];
            }
        }
        if (tid < kMaxFW) unsat[tid] = 0;
        __syncthreads();
        bool any = false;
        for (int w = 0; w < fw; ++w) any = any || active[w] != 0;
        if (!any || t == a.max_iter) break;  // uniform: every thread read the same flags
        if (a.markov) {
            // A7: every source symbol's prior for the next iteration
            for (int x = xi; x < K * fw; x += NI) {
                const int w = x % fw, k = x / fw;
                if (!active[w]) continue;
                int gd = 0;
                markov_row<P, LG>(Qp(w), Lv(w) + size_t(kcol[k]) * Q, k, K, mk + 4 + Q, mk + 4, mk,
                                  Pr(w) + size_t(k) * Q, g, &gd);
                if (gd && g == 0) atomicAdd(&gcount[w], gd);
            }
            __syncthreads();
        }
    }
    // ---- the decisions
    for (int x = tid; x < n * fw; x += kThreads) {
        const int w = x / n, j = x % n;
        a.xhat[size_t(f0 + w) * n + j] = Xh(w)[j];
    }
}

}  // namespace onchip
}  // namespace gfbp
