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
// One thread holds a whole q-vector (q <= 8) in registers.  The arithmetic is
// that of the tiled kernels at one lane per frame (entries per lane = q): the
// same transforms, products in the same order, the same normalisation and
// clipping, float32 storage of every message; so the results are bitwise
// those of the tiled decode at that shape.
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

template <int Q>
__device__ __forceinline__ bool normalise_q(double *v) {
    double s = 0.0;
#pragma unroll
    for (int r = 0; r < Q; ++r) s += v[r];
    if (!(s > 0.0) || !isfinite(s)) {
#pragma unroll
        for (int r = 0; r < Q; ++r) v[r] = 1.0 / double(Q);
        return false;
    }
    const double inv = 1.0 / s;
#pragma unroll
    for (int r = 0; r < Q; ++r) v[r] *= inv;
    return true;
}

template <int Q>
__device__ __forceinline__ int clip_q(const double *acc) {
    int best = 0;
    double bv = acc[0];
#pragma unroll
    for (int r = 1; r < Q; ++r)
        if (acc[r] > bv) {
            bv = acc[r];
            best = r;
        }
    return best;
}

// One q-vector from LDS (its q floats are 4q-byte aligned) in one access.
template <int Q>
__device__ __forceinline__ void lds_vec(const float *p, float *v) {
    if constexpr (Q == 2) {
        const tiled::f32x2 t = *reinterpret_cast<const tiled::f32x2 *>(p);
        v[0] = t.x;
        v[1] = t.y;
    } else {
#pragma unroll
        for (int k = 0; k < Q / 4; ++k) {
            const tiled::f32x4 t = reinterpret_cast<const tiled::f32x4 *>(p)[k];
            v[4 * k] = t.x;
            v[4 * k + 1] = t.y;
            v[4 * k + 2] = t.z;
            v[4 * k + 3] = t.w;
        }
    }
}

// Row a of the multiplication table (a x y for every y), read as one word.
template <int Q>
__device__ __forceinline__ void mul_row(const uint8_t *mul, int a, int *out) {
    const uint8_t *row = mul + a * Q;
    uint64_t w;
    if constexpr (Q == 2) w = *reinterpret_cast<const uint16_t *>(row);
    else if constexpr (Q == 4) w = *reinterpret_cast<const uint32_t *>(row);
    else w = *reinterpret_cast<const uint64_t *>(row);
#pragma unroll
    for (int y = 0; y < Q; ++y) out[y] = int((w >> (8 * y)) & 0xffu);
}

// A3 for one edge: r from the siblings (row positions 0..dc-1 except `self`)
// in row order, T = WHT(signs(z) x prod WHT(q~)), r(h^-1 y) = T(y) / q.
// Where registers allow (rows of at most DCM entries, few entries), every
// sibling is requested before the first is used.
template <int P, int DCM>
__device__ __forceinline__ void edge_r(const float *qm, int rs, int dc, int self, int zi, const uint8_t *mul,
                                       int hinv, float *rout) {
    constexpr int Q = 1 << P;
    constexpr bool kPre = (DCM - 1) * Q <= 40;
    int pos[Q];
    mul_row<Q>(mul, hinv, pos);
    double T[Q];
#pragma unroll
    for (int r = 0; r < Q; ++r) T[r] = (__popc(unsigned(zi & r)) & 1) ? -1.0 : 1.0;
    if constexpr (kPre) {
        float raw[DCM - 1][Q];
#pragma unroll
        for (int u = 0; u < DCM - 1; ++u)
            if (u < dc - 1) lds_vec<Q>(qm + size_t(rs + (u < self ? u : u + 1)) * Q, raw[u]);
#pragma unroll
        for (int u = 0; u < DCM - 1; ++u)
            if (u < dc - 1) {
                double W[Q];
#pragma unroll
                for (int r = 0; r < Q; ++r) W[r] = double(raw[u][r]);
                tiled::wht_regs<Q>(W);
#pragma unroll
                for (int r = 0; r < Q; ++r) T[r] *= W[r];
            }
    } else {
        for (int u = 0; u < dc; ++u) {
            if (u == self) continue;
            float raw[Q];
            lds_vec<Q>(qm + size_t(rs + u) * Q, raw);
            double W[Q];
#pragma unroll
            for (int r = 0; r < Q; ++r) W[r] = double(raw[r]);
            tiled::wht_regs<Q>(W);
#pragma unroll
            for (int r = 0; r < Q; ++r) T[r] *= W[r];
        }
    }
    tiled::wht_regs<Q>(T);
#pragma unroll
    for (int y = 0; y < Q; ++y) rout[pos[y]] = float(fmax(T[y] * (1.0 / double(Q)), 0.0));
}

// A4/A5 for a column from its r-vectors rv[0..dv) (natural order, column
// edge order) and its prior row pv: the pseudo-posterior (Eq. (5)), into
// Qp_k when not null, and the decision.
template <int P, int DVM>
__device__ __forceinline__ void posterior_step(const float (&rv)[DVM][1 << P], int dv, const double *pv,
                                               float *Qp_k, uint8_t *xh_j, int *g) {
    constexpr int Q = 1 << P;
    double acc[Q];
#pragma unroll
    for (int q = 0; q < Q; ++q) acc[q] = pv[q];
#pragma unroll
    for (int d2 = 0; d2 < DVM; ++d2)
        if (d2 < dv)
#pragma unroll
            for (int q = 0; q < Q; ++q) acc[q] *= double(rv[d2][q]);
    if (!normalise_q<Q>(acc)) ++*g;
    if (Qp_k)
#pragma unroll
        for (int q = 0; q < Q; ++q) Qp_k[q] = float(acc[q]);
    *xh_j = uint8_t(clip_q<Q>(acc));
}

// Eq. (4) for edge slot d of the column: q from the prior and the other
// edges' r, normalised, stored at position h a (hpos[a]) of its vector.
template <int P, int DVM>
__device__ __forceinline__ void edge_q_step(const float (&rv)[DVM][1 << P], int dv, const double *pv, int d,
                                            float *dst, const int *hpos, int *g) {
    constexpr int Q = 1 << P;
    double qv[Q];
#pragma unroll
    for (int q = 0; q < Q; ++q) qv[q] = pv[q];
#pragma unroll
    for (int d2 = 0; d2 < DVM; ++d2)
        if (d2 < dv && d2 != d)
#pragma unroll
            for (int q = 0; q < Q; ++q) qv[q] *= double(rv[d2][q]);
    if (!normalise_q<Q>(qv)) ++*g;
#pragma unroll
    for (int q = 0; q < Q; ++q) dst[hpos[q]] = float(qv[q]);
}

// A7 for source symbol k (Eq. (7)): the neighbours' pseudo-posteriors
// Qp[k -+ 1] through M (O(q) when M is self-transition plus uniform), times
// the evidence of its column, into pr; guard events counted in *g.
template <int P>
__device__ __forceinline__ void markov_row(const float *Qp, const float *Lj, int k, int K, const float *M,
                                           const float *pi, const float *mshape, float *pr, int *g) {
    constexpr int Q = 1 << P;
    double u[Q], v[Q];
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        u[q] = k == 0 ? double(pi[q]) : 0.0;
        v[q] = k == K - 1 ? 1.0 : 0.0;
    }
    if (mshape[0] != 0.0f) {
        const double sd = mshape[1], od = mshape[2];
        float nb[2][Q];
        double S[2] = {0.0, 0.0};
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int kk = h == 0 ? k - 1 : k + 1;
            if (kk >= 0 && kk < K)
#pragma unroll
                for (int q = 0; q < Q; ++q) nb[h][q] = Qp[size_t(kk) * Q + q];
            else
#pragma unroll
                for (int q = 0; q < Q; ++q) nb[h][q] = 0.0f;
#pragma unroll
            for (int q = 0; q < Q; ++q) S[h] += double(nb[h][q]);
        }
        if (k > 0)
#pragma unroll
            for (int q = 0; q < Q; ++q) u[q] = sd * double(nb[0][q]) + od * (S[0] - double(nb[0][q]));
        if (k < K - 1)
#pragma unroll
            for (int q = 0; q < Q; ++q) v[q] = sd * double(nb[1][q]) + od * (S[1] - double(nb[1][q]));
    } else {
        if (k > 0) {
            const float *qp = Qp + size_t(k - 1) * Q;
#pragma unroll 2
            for (int a = 0; a < Q; ++a) {
                const double qa = qp[a];
#pragma unroll
                for (int q = 0; q < Q; ++q) u[q] += qa * double(M[a * Q + q]);
            }
        }
        if (k < K - 1) {
            const float *qp = Qp + size_t(k + 1) * Q;
#pragma unroll 2
            for (int cc = 0; cc < Q; ++cc) {
                const double qc = qp[cc];
#pragma unroll
                for (int q = 0; q < Q; ++q) v[q] += double(M[q * Q + cc]) * qc;
            }
        }
    }
#pragma unroll
    for (int q = 0; q < Q; ++q) u[q] *= v[q];
    if (!normalise_q<Q>(u)) ++*g;
#pragma unroll
    for (int q = 0; q < Q; ++q) u[q] *= double(Lj[q]);
    if (!normalise_q<Q>(u)) ++*g;
#pragma unroll
    for (int q = 0; q < Q; ++q) pr[q] = float(u[q]);
}

template <int P, int DCM, int DVM>
__global__ __launch_bounds__(kThreads) void k_onchip(const Args a) {
    constexpr int Q = 1 << P;
    extern __shared__ __align__(16) unsigned char lds[];
    const DevCode &c = a.c;
    const Layout &ly = a.lay;
    const int tid = int(threadIdx.x);
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
            for (int x = tid; x < E * fw; x += kThreads) {
                const int w = x % fw, e = x / fw;
                if (!active[w]) continue;
                const uint32_t ge = eg[e];
                edge_r<P, DCM>(Qm(w), eg_rs(ge), eg_dc(ge), eg_self(ge), Zs(w)[erow[e]], mul, eg_hinv(ge),
                               Rr(w) + size_t(e) * Q);
            }
            __syncthreads();
            // A4: every column's pseudo-posterior, decision and q
            for (int x = tid; x < n * fw; x += kThreads) {
                const int w = x % fw, j = x / fw;
                if (!active[w]) continue;
                const uint32_t gc = cg[j];
                const int cs = int(gc & 0xffffu), dv = int(gc >> 16);
                const float *R = Rr(w);
                float rv[DVM][Q];
                int es[DVM];
#pragma unroll
                for (int d = 0; d < DVM; ++d)
                    if (d < dv) {
                        es[d] = cedge[cs + d];
                        lds_vec<Q>(R + size_t(es[d]) * Q, rv[d]);
                    }
                float pf[Q];
                lds_vec<Q>(prow(w, j), pf);
                double pv[Q];
#pragma unroll
                for (int q = 0; q < Q; ++q) pv[q] = pf[q];
                int g = 0;
                const int k1 = ck[j];
                posterior_step<P, DVM>(rv, dv, pv, a.wantQ && k1 > 0 ? Qp(w) + size_t(k1 - 1) * Q : nullptr,
                                       Xh(w) + j, &g);
#pragma unroll
                for (int d = 0; d < DVM; ++d)
                    if (d < dv) {
                        int hp[Q];
                        mul_row<Q>(mul, eg_h(eg[es[d]]), hp);
                        edge_q_step<P, DVM>(rv, dv, pv, d, Qm(w) + size_t(es[d]) * Q, hp, &g);
                    }
                if (g) atomicAdd(&gcount[w], g);
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
            const int cw = kThreads / per;
            const int col = tid / per, w = (tid % per) / a.rs, d = tid % a.rs;  // this thread's item
            for (int l = 0; l < a.nlev; ++l) {
                const int p0 = lptr[l], p1 = lptr[l + 1];
                for (int c0 = p0; c0 < p1; c0 += cw) {
                    const int nc = min(cw, p1 - c0);
                    const bool in = tid < nc * per;
                    const int p = c0 + (in ? col : 0);
                    const uint32_t pw = pe[size_t(p) * a.rs + d];
                    const int e = int(pw & 0xffffu), dv = int(pw >> 16);
                    const bool live = in && active[w] != 0;
                    if (live && d < dv) {
                        const uint32_t ge = eg[e];
                        edge_r<P, DCM>(Qm(w), eg_rs(ge), eg_dc(ge), eg_self(ge), Zs(w)[erow[e]], mul, eg_hinv(ge),
                                       rsh + size_t(tid) * Q);
                    }
                    __syncthreads();
                    if (live && (d < dv || d == 0)) {
                        const int j = lcol[p];
                        float rv[DVM][Q];
#pragma unroll
                        for (int d2 = 0; d2 < DVM; ++d2)
                            if (d2 < dv) lds_vec<Q>(rsh + size_t(tid - d + d2) * Q, rv[d2]);
                        float pf[Q];
                        lds_vec<Q>(prow(w, j), pf);
                        double pv[Q];
#pragma unroll
                        for (int q = 0; q < Q; ++q) pv[q] = pf[q];
                        int g = 0;
                        if (d == 0) {
                            const int k1 = ck[j];
                            posterior_step<P, DVM>(rv, dv, pv,
                                                   a.wantQ && k1 > 0 ? Qp(w) + size_t(k1 - 1) * Q : nullptr,
                                                   Xh(w) + j, &g);
                        }
                        if (d < dv) {
                            int hp[Q];
                            mul_row<Q>(mul, eg_h(eg[e]), hp);
                            edge_q_step<P, DVM>(rv, dv, pv, d, Qm(w) + size_t(e) * Q, hp, &g);
                        }
                        if (g) atomicAdd(&gcount[w], g);
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
            for (int x = tid; x < K * fw; x += kThreads) {
                const int w = x % fw, k = x / fw;
                if (!active[w]) continue;
                int g = 0;
                markov_row<P>(Qp(w), Lv(w) + size_t(kcol[k]) * Q, k, K, mk + 4 + Q, mk + 4, mk, Pr(w) + size_t(k) * Q,
                              &g);
                if (g) atomicAdd(&gcount[w], g);
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
