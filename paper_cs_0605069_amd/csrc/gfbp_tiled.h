// Decoder kernels for gfx950: one kernel family, tiled by (frames x lanes).
//
// Thread mapping.  A q-vector (q = 2^P) of one frame is spread over
// G = 2^LG consecutive lanes, each holding EL = q/G entries in registers:
// lane g of the frame holds entries y = g*EL + r, r = 0..EL-1.  A 64-lane
// wavefront therefore holds TF = 64/G frames, all working on the same graph
// node, so every index into the graph (and each edge coefficient h) is
// wavefront-uniform.  Walsh-Hadamard butterflies over the EL register bits
// are plain register arithmetic; only the LG lane bits need lane exchanges
// (DPP), and normalisation sums / decisions need LG exchange steps.
// G = 1 puts a whole vector in one lane (no exchanges at all); the kernels
// pick EL = 8 (4 for rows longer than 8) so that the register budget is the
// same for every q.
//
// Layout.  Every per-frame vector array is stored as
//   array[node][tile][a][fw]   (frame f = tile*TF + fw, frames padded to Fp)
// so that, for a fixed entry a, the TF frames of a wavefront are adjacent.
// Loads and stores of entry a for a wavefront touch G runs of TF*4 bytes.
//
// Check node (Eq. (3)).  With y = h x the weighted symbol of an edge, a
// check constrains the XOR-sum of the y's, so the sum over configurations is
// the XOR-convolution of the siblings' distributions q~(y) = q(h^-1 y).  The
// Walsh-Hadamard transform (WHT) turns that into a pointwise product.  The
// permutation by h^-1 is folded into the load address (entry h^-1 y is read
// for position y); the syndrome z is folded into the transform as the sign
// pattern (-1)^popcount(z & k), which shifts the result by z; the inverse
// transform gives T(y) = S(y + z) and r(a) = T(h a) is stored by writing
// position y to entry h^-1 y.  Transforms, products and normalisations run in
// float64 (a float32 transform loses every probability below ~1e-7 of the
// largest to cancellation); messages are stored as float32 probabilities.
#pragma once
#include "gfbp_kernels.h"

namespace gfbp {
namespace tiled {

template <int P, int LG>
struct Geo {
    static constexpr int Q = 1 << P;
    static constexpr int G = 1 << LG;        // lanes per frame
    static constexpr int LEL = P - LG;       // log2 entries per lane
    static constexpr int EL = 1 << LEL;      // entries per lane
    static constexpr int TF = kWave >> LG;   // frames per wavefront
};

struct Item {
    int node, tile, fw, g, f;
    bool ok;
};

// Wavefront w works on node w / nb and on entry w % nb of the list of tiles
// that still hold a running frame (entries past the list's current length,
// read on the device, do nothing).
template <int P, int LG>
__device__ __forceinline__ Item item(int nodes, const DevState &s) {
    using Gm = Geo<P, LG>;
    const int w = int(blockIdx.x) * (kBlock / kWave) + int(threadIdx.x) / kWave;
    const int lane = int(threadIdx.x) % kWave;
    Item it;
    it.node = w / s.nb;
    const int ti = w % s.nb;
    it.ok = it.node < nodes && ti < int(*s.nact);
    it.tile = it.ok ? s.act[ti] : 0;
    if (it.tile < 0 || it.tile >= s.Fp / Gm::TF) {  // the list only holds valid tiles; never index past it
        it.ok = false;
        it.tile = 0;
    }
    it.fw = lane >> LG;
    it.g = lane & (Gm::G - 1);
    it.f = it.tile * Gm::TF + it.fw;
    return it;
}

// Base of vector `node` for tile `tile`: entry a of frame fw is at
// base[a * TF + fw].
template <int P, int LG, typename T>
__device__ __forceinline__ T *vec_base(T *arr, size_t node, int tile, int ntiles) {
    using Gm = Geo<P, LG>;
    return arr + (node * size_t(ntiles) + size_t(tile)) * (Gm::Q * Gm::TF);
}

// Images under multiplication by h (basis images packed in `packed`) of the
// positions y = g*EL + r held by lane g: by linearity h y = h (g*EL) + h r,
// the second term being the same for every lane.
template <int P, int LG>
__device__ __forceinline__ void gf_positions(uint64_t packed, int g, int *out) {
    using Gm = Geo<P, LG>;
    const int hg = gf_apply<P>(packed, g * Gm::EL);
#pragma unroll
    for (int r = 0; r < Gm::EL; ++r) out[r] = hg ^ gf_apply<P>(packed, r);
}

// Index of entry a of vector `node` for frame (tile, fw).
template <int P, int LG>
__device__ __forceinline__ size_t at(size_t node, int tile, int a, int fw, int ntiles) {
    using Gm = Geo<P, LG>;
    return ((node * size_t(ntiles) + size_t(tile)) * Gm::Q + size_t(a)) * Gm::TF + size_t(fw);
}

// Unnormalised WHT of the distributed vector (positions y = g*EL + r).
template <int P, int LG, int S = 0>
__device__ __forceinline__ void wht(double *v, int g) {
    using Gm = Geo<P, LG>;
    if constexpr (S < P) {
        if constexpr (S < Gm::LEL) {
            constexpr int m = 1 << S;
#pragma unroll
            for (int r = 0; r < Gm::EL; ++r) {
                if (!(r & m)) {
                    const double a = v[r], b = v[r | m];
                    v[r] = a + b;
                    v[r | m] = a - b;
                }
            }
        } else {
            constexpr int mask = 1 << (S - Gm::LEL);
            const double sg = (g & mask) ? -1.0 : 1.0;
#pragma unroll
            for (int r = 0; r < Gm::EL; ++r) v[r] = fma(sg, v[r], xchg<mask>(v[r]));
        }
        wht<P, LG, S + 1>(v, g);
    }
}

// Sum over the G lanes of a frame (bitwise identical on each of them).
template <int LG, int S = 0>
__device__ __forceinline__ double lanes_sum(double v) {
    if constexpr (S < LG) {
        return lanes_sum<LG, S + 1>(v + xchg<(1 << S)>(v));
    } else {
        return v;
    }
}

template <int LG, int S = 0>
__device__ __forceinline__ int lanes_argmax(float v, int k) {
    if constexpr (S < LG) {
        const float ov = xchg<(1 << S)>(v);
        const int ok = xchg<(1 << S)>(k);
        const bool take = ov > v || (ov == v && ok < k);
        return lanes_argmax<LG, S + 1>(take ? ov : v, take ? ok : k);
    } else {
        return k;
    }
}

// Normalise the distributed vector to sum 1; uniform (and a guard event) when
// the sum is zero or not finite.
template <int P, int LG>
__device__ __forceinline__ void normalise(double *v, int32_t *guards, int f, int g) {
    using Gm = Geo<P, LG>;
    double s = 0.0;
#pragma unroll
    for (int r = 0; r < Gm::EL; ++r) s += v[r];
    s = lanes_sum<LG>(s);
    if (!(s > 0.0) || !isfinite(s)) {
        if (g == 0) atomicAdd(&guards[f], 1);
#pragma unroll
        for (int r = 0; r < Gm::EL; ++r) v[r] = 1.0 / double(Gm::Q);
        return;
    }
    const double inv = 1.0 / s;
#pragma unroll
    for (int r = 0; r < Gm::EL; ++r) v[r] *= inv;
}

template <int P, int LG>
__device__ __forceinline__ void syndrome_signs(int z, int g, double *v) {
    using Gm = Geo<P, LG>;
#pragma unroll
    for (int r = 0; r < Gm::EL; ++r) v[r] = (__popc(z & (g * Gm::EL + r)) & 1) ? -1.0 : 1.0;
}

// Edge e's weighted-symbol distribution q~(y) = q(h^-1 y) at this lane's
// positions (loads only; all the loads of a check are issued before any
// transform so that their latencies overlap).
template <int P, int LG>
__device__ __forceinline__ void load_permuted(const float *Qm, size_t e, const Item &it, int ntiles, uint64_t hinv,
                                              float *v) {
    using Gm = Geo<P, LG>;
    const float *base = vec_base<P, LG>(Qm, e, it.tile, ntiles);
    int pos[Gm::EL];
    gf_positions<P, LG>(hinv, it.g, pos);
#pragma unroll
    for (int r = 0; r < Gm::EL; ++r) v[r] = base[pos[r] * Gm::TF + it.fw];
}

template <int P, int LG>
__device__ __forceinline__ void transform(const float *raw, double *v, int g) {
    using Gm = Geo<P, LG>;
#pragma unroll
    for (int r = 0; r < Gm::EL; ++r) v[r] = double(raw[r]);
    wht<P, LG>(v, g);
}

struct Chan {
    int channel, markov;
    const uint8_t *rx, *erasure;
    const float *y, *lik, *param, *pi;
};

// A1 channel likelihood and A2 initialisation for column j of frame f:
// L_j(a) = P(received | x_j = a) as a product over the p transmitted bits;
// p_j = L_j (times the stationary Markov marginal pi for source symbols);
// every edge of column j starts with q_e = p_j.
template <int P, int LG>
__global__ __launch_bounds__(kBlock) void k_init(DevCode c, DevState s, Chan ch) {
    using Gm = Geo<P, LG>;
    const int ntiles = s.Fp / Gm::TF;
    const Item it = item<P, LG>(c.n, s);
    if (!it.ok || it.f >= s.F) return;
    if (s.fresh && !s.fresh[it.f]) return;
    const int j = it.node, f = it.f;
    const size_t fj = size_t(f) * c.n + j;
    const int channel = s.chan ? int(s.chan[f]) : ch.channel;
    const bool markov = s.mark ? s.mark[f] != 0 : ch.markov != 0;
    double L[Gm::EL];
    if (channel == GFBP_CH_BSC || channel == GFBP_CH_BEC) {
        const int rx = ch.rx[fj];
        const int er = channel == GFBP_CH_BEC ? ch.erasure[fj] : 0;
        const double fl = channel == GFBP_CH_BSC ? double(ch.param[f]) : 0.0;
#pragma unroll
        for (int r = 0; r < Gm::EL; ++r) {
            const int a = it.g * Gm::EL + r;
            double v = 1.0;
#pragma unroll
            for (int t = 0; t < P; ++t) {
                const bool flip = ((a ^ rx) >> t) & 1;
                if (channel == GFBP_CH_BSC) v *= flip ? fl : (1.0 - fl);
                else v *= ((er >> t) & 1) ? 0.5 : (flip ? 0.0 : 1.0);
            }
            L[r] = v;
        }
    } else if (channel == GFBP_CH_BIAWGN) {
        const double sg = ch.param[f];
        const double gain = 2.0 / (sg * sg);
        double p0[P], p1[P];
#pragma unroll
        for (int t = 0; t < P; ++t) {
            const double yb = ch.y[fj * P + t];
            p1[t] = 1.0 / (1.0 + exp(gain * yb));   // P(bit = 1 | y): bit 1 was sent as -1
            p0[t] = 1.0 / (1.0 + exp(-gain * yb));  // P(bit = 0 | y)
        }
#pragma unroll
        for (int r = 0; r < Gm::EL; ++r) {
            const int a = it.g * Gm::EL + r;
            double v = 1.0;
#pragma unroll
            for (int t = 0; t < P; ++t) v *= ((a >> t) & 1) ? p1[t] : p0[t];
            L[r] = v;
        }
    } else {
#pragma unroll
        for (int r = 0; r < Gm::EL; ++r) L[r] = ch.lik[fj * Gm::Q + it.g * Gm::EL + r];
    }
    normalise<P, LG>(L, s.guards, f, it.g);
    float pf[Gm::EL];
#pragma unroll
    for (int r = 0; r < Gm::EL; ++r) {
        pf[r] = float(L[r]);
        s.L[at<P, LG>(j, it.tile, it.g * Gm::EL + r, it.fw, ntiles)] = pf[r];
    }
    if (markov && j < c.n_info) {
        double pr[Gm::EL];
#pragma unroll
        for (int r = 0; r < Gm::EL; ++r) pr[r] = double(pf[r]) * double(ch.pi[it.g * Gm::EL + r]);
        normalise<P, LG>(pr, s.guards, f, it.g);
#pragma unroll
        for (int r = 0; r < Gm::EL; ++r) {
            pf[r] = float(pr[r]);
            s.Pr[at<P, LG>(j, it.tile, it.g * Gm::EL + r, it.fw, ntiles)] = pf[r];
        }
    }
    for (int t = c.col_ptr[j]; t < c.col_ptr[j + 1]; ++t) {
        const size_t e = size_t(c.col_edge[t]);
#pragma unroll
        for (int r = 0; r < Gm::EL; ++r) s.Qm[at<P, LG>(e, it.tile, it.g * Gm::EL + r, it.fw, ntiles)] = pf[r];
    }
}

// A3, parallel schedule: all r of check i from the previous iteration's q.
// DCM bounds the row degree: the siblings' transforms stay in registers.
template <int P, int LG, int DCM>
__global__ __launch_bounds__(kBlock) void k_check(DevCode c, DevState s, const uint8_t *z, Snap snap) {
    using Gm = Geo<P, LG>;
    const int ntiles = s.Fp / Gm::TF;
    const Item it = item<P, LG>(c.m, s);
    if (!it.ok || it.f >= s.F || !s.active[it.f]) return;
    const int i = it.node, f = it.f;
    const int rs = c.row_ptr[i], dc = c.row_ptr[i + 1] - rs;
    const int zi = z ? z[size_t(f) * c.m + i] : 0;
    float raw[DCM][Gm::EL];
#pragma unroll
    for (int d = 0; d < DCM; ++d)
        if (d < dc) load_permuted<P, LG>(s.Qm, size_t(rs + d), it, ntiles, c.emap[2 * (rs + d)], raw[d]);
    double W[DCM][Gm::EL];
#pragma unroll
    for (int d = 0; d < DCM; ++d)
        if (d < dc) transform<P, LG>(raw[d], W[d], it.g);
#pragma unroll
    for (int d = 0; d < DCM; ++d) {
        if (d < dc) {
            double T[Gm::EL];
            syndrome_signs<P, LG>(zi, it.g, T);
#pragma unroll
            for (int d2 = 0; d2 < DCM; ++d2)
                if (d2 < dc && d2 != d) {
#pragma unroll
                    for (int r = 0; r < Gm::EL; ++r) T[r] *= W[d2][r];
                }
            wht<P, LG>(T, it.g);
            const size_t e = size_t(rs + d);
            float *base = vec_base<P, LG>(s.R, e, it.tile, ntiles);
            int pos[Gm::EL];
            gf_positions<P, LG>(c.emap[2 * e], it.g, pos);
#pragma unroll
            for (int r = 0; r < Gm::EL; ++r) {
                const float rv = float(fmax(T[r] * (1.0 / double(Gm::Q)), 0.0));
                base[pos[r] * Gm::TF + it.fw] = rv;
                if (snap.r) snap.r[(size_t(f) * c.E + e) * Gm::Q + pos[r]] = rv;
            }
        }
    }
}

// A4 variable-node update of column j from its r-messages r[d][.]: the
// pseudo-posterior Q_j (Eq. (5)) and its decision, then each edge's q
// (Eq. (4)), normalised.
template <int P, int LG, int DVM>
__device__ __forceinline__ void variable_update(const DevCode &c, const DevState &s, const Item &it, int ntiles,
                                                int j, const float (*r)[Geo<P, LG>::EL], int cs, int dv, int markov,
                                                int wantQ, const Snap &snap) {
    using Gm = Geo<P, LG>;
    const int f = it.f;
    const bool mk = s.mark ? s.mark[f] != 0 : markov != 0;
    const float *pj = (mk && j < c.n_info) ? s.Pr : s.L;
    double pv[Gm::EL], acc[Gm::EL];
#pragma unroll
    for (int q = 0; q < Gm::EL; ++q) {
        pv[q] = pj[at<P, LG>(j, it.tile, it.g * Gm::EL + q, it.fw, ntiles)];
        acc[q] = pv[q];
    }
#pragma unroll
    for (int d = 0; d < DVM; ++d)
        if (d < dv) {
#pragma unroll
            for (int q = 0; q < Gm::EL; ++q) acc[q] *= double(r[d][q]);
        }
    normalise<P, LG>(acc, s.guards, f, it.g);
    int best = it.g * Gm::EL;
    float bv = float(acc[0]);
#pragma unroll
    for (int q = 0; q < Gm::EL; ++q) {
        const float v = float(acc[q]);
        if (wantQ) s.Qp[at<P, LG>(j, it.tile, it.g * Gm::EL + q, it.fw, ntiles)] = v;
        if (v > bv) { bv = v; best = it.g * Gm::EL + q; }
    }
    best = lanes_argmax<LG>(bv, best);
    if (it.g == 0) s.xh[size_t(j) * s.Fp + f] = uint8_t(best);
#pragma unroll
    for (int d = 0; d < DVM; ++d) {
        if (d < dv) {
            double qv[Gm::EL];
#pragma unroll
            for (int q = 0; q < Gm::EL; ++q) qv[q] = pv[q];
#pragma unroll
            for (int d2 = 0; d2 < DVM; ++d2)
                if (d2 < dv && d2 != d) {
#pragma unroll
                    for (int q = 0; q < Gm::EL; ++q) qv[q] *= double(r[d2][q]);
                }
            normalise<P, LG>(qv, s.guards, f, it.g);
            const size_t e = size_t(c.col_edge[cs + d]);
#pragma unroll
            for (int q = 0; q < Gm::EL; ++q) {
                const float qn = float(qv[q]);
                s.Qm[at<P, LG>(e, it.tile, it.g * Gm::EL + q, it.fw, ntiles)] = qn;
                if (snap.q) snap.q[(size_t(f) * c.E + e) * Gm::Q + it.g * Gm::EL + q] = qn;
            }
        }
    }
}

// A4, parallel schedule: every column from this iteration's r.
template <int P, int LG, int DVM>
__global__ __launch_bounds__(kBlock) void k_variable(DevCode c, DevState s, int markov, int wantQ, Snap snap) {
    using Gm = Geo<P, LG>;
    const int ntiles = s.Fp / Gm::TF;
    const Item it = item<P, LG>(c.n, s);
    if (!it.ok || it.f >= s.F || !s.active[it.f]) return;
    const int j = it.node;
    const int cs = c.col_ptr[j], dv = c.col_ptr[j + 1] - cs;
    float r[DVM][Gm::EL];
#pragma unroll
    for (int d = 0; d < DVM; ++d)
        if (d < dv) {
            const float *base = vec_base<P, LG>(s.R, size_t(c.col_edge[cs + d]), it.tile, ntiles);
#pragma unroll
            for (int q = 0; q < Gm::EL; ++q) r[d][q] = base[(it.g * Gm::EL + q) * Gm::TF + it.fw];
        }
    variable_update<P, LG, DVM>(c, s, it, ntiles, j, r, cs, dv, markov, wantQ, snap);
}

// A6 sequential schedule, the step of column j for one tile of frames, done
// by a workgroup: wavefront d (< column degree) computes the r of the
// column's d-th edge from the siblings' current q (partial horizontal pass);
// after a workgroup barrier, wavefront d combines the column's r into its
// edge's q and wavefront 0 into the pseudo-posterior and decision (partial
// vertical pass).  `live`: this lane's frame is still iterating.  perm is the
// wavefront's Q x TF buffer that applies r(a) = T(h a) (position y written to
// entry h^-1 y, entries read back in order); rsh holds the column's r as
// [d][register][lane].
template <int P, int LG, int DCM, int DVM>
__device__ __forceinline__ void sus_column(const DevCode &c, const DevState &s, const uint8_t *z, const Item &it,
                                           bool live, int ntiles, int j, int markov, int wantQ, const Snap &snap,
                                           float *perm, float *rsh) {
    using Gm = Geo<P, LG>;
    const int f = it.f;
    const int d = int(threadIdx.x) / kWave, lane = int(threadIdx.x) % kWave;
    const int cs = c.col_ptr[j], dv = c.col_ptr[j + 1] - cs;
    const bool mine = live && d < dv;
    size_t e = 0;
    if (d < dv) e = size_t(c.col_edge[cs + d]);
    if (mine) {
        const int i = c.edge_row[e];
        const int rs = c.row_ptr[i], dc = c.row_ptr[i + 1] - rs;
        const int self = int(e) - rs;
        float raw[DCM][Gm::EL];
#pragma unroll
        for (int t = 0; t < DCM; ++t)
            if (t < dc && t != self)
                load_permuted<P, LG>(s.Qm, size_t(rs + t), it, ntiles, c.emap[2 * (rs + t)], raw[t]);
        double acc[Gm::EL];
        syndrome_signs<P, LG>(z ? z[size_t(f) * c.m + i] : 0, it.g, acc);
#pragma unroll
        for (int t = 0; t < DCM; ++t) {
            if (t < dc && t != self) {
                double w[Gm::EL];
                transform<P, LG>(raw[t], w, it.g);
#pragma unroll
                for (int q = 0; q < Gm::EL; ++q) acc[q] *= w[q];
            }
        }
        wht<P, LG>(acc, it.g);
        int pos[Gm::EL];
        gf_positions<P, LG>(c.emap[2 * e], it.g, pos);
#pragma unroll
        for (int q = 0; q < Gm::EL; ++q) perm[pos[q] * Gm::TF + it.fw] = float(fmax(acc[q] * (1.0 / double(Gm::Q)), 0.0));
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
#pragma unroll
        for (int q = 0; q < Gm::EL; ++q) {
            const float rv = perm[(it.g * Gm::EL + q) * Gm::TF + it.fw];
            rsh[(d * Gm::EL + q) * kWave + lane] = rv;
            if (snap.r) snap.r[(size_t(f) * c.E + e) * Gm::Q + it.g * Gm::EL + q] = rv;
        }
    }
    __syncthreads();
    if (mine) {
        const bool mk = s.mark ? s.mark[f] != 0 : markov != 0;
        const float *pj = (mk && j < c.n_info) ? s.Pr : s.L;
        const float *pb = vec_base<P, LG>(pj, size_t(j), it.tile, ntiles);
        double pv[Gm::EL];
#pragma unroll
        for (int q = 0; q < Gm::EL; ++q) pv[q] = pb[(it.g * Gm::EL + q) * Gm::TF + it.fw];
        if (d == 0) {
            // A4/A5: pseudo-posterior (Eq. (5)) and decision
            double acc[Gm::EL];
#pragma unroll
            for (int q = 0; q < Gm::EL; ++q) acc[q] = pv[q];
#pragma unroll
            for (int d2 = 0; d2 < DVM; ++d2)
                if (d2 < dv) {
#pragma unroll
                    for (int q = 0; q < Gm::EL; ++q) acc[q] *= double(rsh[(d2 * Gm::EL + q) * kWave + lane]);
                }
            normalise<P, LG>(acc, s.guards, f, it.g);
            int best = it.g * Gm::EL;
            float bv = float(acc[0]);
#pragma unroll
            for (int q = 0; q < Gm::EL; ++q) {
                const float v = float(acc[q]);
                if (wantQ) s.Qp[at<P, LG>(j, it.tile, it.g * Gm::EL + q, it.fw, ntiles)] = v;
                if (v > bv) { bv = v; best = it.g * Gm::EL + q; }
            }
            best = lanes_argmax<LG>(bv, best);
            if (it.g == 0) s.xh[size_t(j) * s.Fp + f] = uint8_t(best);
        }
        // Eq. (4) for this wavefront's edge
        double qv[Gm::EL];
#pragma unroll
        for (int q = 0; q < Gm::EL; ++q) qv[q] = pv[q];
#pragma unroll
        for (int d2 = 0; d2 < DVM; ++d2)
            if (d2 < dv && d2 != d) {
#pragma unroll
                for (int q = 0; q < Gm::EL; ++q) qv[q] *= double(rsh[(d2 * Gm::EL + q) * kWave + lane]);
            }
        normalise<P, LG>(qv, s.guards, f, it.g);
        float *qb = vec_base<P, LG>(s.Qm, e, it.tile, ntiles);
#pragma unroll
        for (int q = 0; q < Gm::EL; ++q) {
            const float qn = float(qv[q]);
            qb[(it.g * Gm::EL + q) * Gm::TF + it.fw] = qn;
            if (snap.q) snap.q[(size_t(f) * c.E + e) * Gm::Q + it.g * Gm::EL + q] = qn;
        }
    }
    __syncthreads();
}

// Workgroup item: (node, tile) for the whole workgroup; each lane's frame.
template <int P, int LG>
__device__ __forceinline__ Item block_item(int nodes, const DevState &s) {
    using Gm = Geo<P, LG>;
    const int b = int(blockIdx.x);
    const int lane = int(threadIdx.x) % kWave;
    Item it;
    it.node = b / s.nb;
    const int ti = b % s.nb;
    it.ok = it.node < nodes && ti < int(*s.nact);
    it.tile = it.ok ? s.act[ti] : 0;
    if (it.tile < 0 || it.tile >= s.Fp / Gm::TF) {
        it.ok = false;
        it.tile = 0;
    }
    it.fw = lane >> LG;
    it.g = lane & (Gm::G - 1);
    it.f = it.tile * Gm::TF + it.fw;
    return it;
}

// A6, one dependency level: the columns cols[0..ncols) share no check, so
// their steps commute; each runs exactly as in the strict order.  One
// workgroup of DVM wavefronts per (column, tile).
template <int P, int LG, int DCM, int DVM>
__global__ __launch_bounds__(DVM *kWave) void k_sus_level(DevCode c, DevState s, const uint8_t *z, int markov,
                                                          int wantQ, Snap snap, const int32_t *cols, int ncols) {
    using Gm = Geo<P, LG>;
    __shared__ float perm[DVM * Gm::Q * Gm::TF];
    __shared__ float rsh[DVM * Gm::EL * kWave];
    const int ntiles = s.Fp / Gm::TF;
    const Item it = block_item<P, LG>(ncols, s);
    if (!it.ok) return;  // uniform over the workgroup
    const bool live = it.f < s.F && s.active[it.f];
    sus_column<P, LG, DCM, DVM>(c, s, z, it, live, ntiles, cols[it.node], markov, wantQ, snap,
                                perm + (int(threadIdx.x) / kWave) * Gm::Q * Gm::TF, rsh);
}

// A6, strict order: columns 0..n-1 one after the other for each tile.
template <int P, int LG, int DCM, int DVM>
__global__ __launch_bounds__(DVM *kWave) void k_sequential(DevCode c, DevState s, const uint8_t *z, int markov,
                                                           int wantQ, Snap snap) {
    using Gm = Geo<P, LG>;
    __shared__ float perm[DVM * Gm::Q * Gm::TF];
    __shared__ float rsh[DVM * Gm::EL * kWave];
    const int ntiles = s.Fp / Gm::TF;
    const Item it = block_item<P, LG>(1, s);
    if (!it.ok) return;  // uniform over the workgroup
    const bool live = it.f < s.F && s.active[it.f];
    float *mine = perm + (int(threadIdx.x) / kWave) * Gm::Q * Gm::TF;
    for (int j = 0; j < c.n; ++j) sus_column<P, LG, DCM, DVM>(c, s, z, it, live, ntiles, j, markov, wantQ, snap, mine, rsh);
}

// A7 dynamical block prior (Eq. (7)) for source symbol k: from this
// iteration's pseudo-posteriors of its chain neighbours, multiplied into the
// channel likelihood for the next iteration.
template <int P, int LG>
__global__ __launch_bounds__(kBlock) void k_markov(DevCode c, DevState s, const float *M, const float *pi) {
    using Gm = Geo<P, LG>;
    const int ntiles = s.Fp / Gm::TF;
    const Item it = item<P, LG>(c.n_info, s);
    if (!it.ok || it.f >= s.F || !s.active[it.f]) return;
    if (s.mark && !s.mark[it.f]) return;
    const int k = it.node, K = c.n_info;
    double u[Gm::EL], v[Gm::EL];
#pragma unroll
    for (int q = 0; q < Gm::EL; ++q) {
        const int b = it.g * Gm::EL + q;
        u[q] = k == 0 ? double(pi[b]) : 0.0;
        v[q] = k == K - 1 ? 1.0 : 0.0;
    }
    if (k > 0)
        for (int a = 0; a < Gm::Q; ++a) {
            const double qa = s.Qp[at<P, LG>(k - 1, it.tile, a, it.fw, ntiles)];
#pragma unroll
            for (int q = 0; q < Gm::EL; ++q) u[q] += qa * double(M[a * Gm::Q + it.g * Gm::EL + q]);
        }
    if (k < K - 1)
        for (int cc = 0; cc < Gm::Q; ++cc) {
            const double qc = s.Qp[at<P, LG>(k + 1, it.tile, cc, it.fw, ntiles)];
#pragma unroll
            for (int q = 0; q < Gm::EL; ++q) v[q] += double(M[(it.g * Gm::EL + q) * Gm::Q + cc]) * qc;
        }
#pragma unroll
    for (int q = 0; q < Gm::EL; ++q) u[q] *= v[q];
    normalise<P, LG>(u, s.guards, it.f, it.g);
#pragma unroll
    for (int q = 0; q < Gm::EL; ++q) u[q] *= double(s.L[at<P, LG>(k, it.tile, it.g * Gm::EL + q, it.fw, ntiles)]);
    normalise<P, LG>(u, s.guards, it.f, it.g);
#pragma unroll
    for (int q = 0; q < Gm::EL; ++q) s.Pr[at<P, LG>(k, it.tile, it.g * Gm::EL + q, it.fw, ntiles)] = float(u[q]);
}

// Ordered list of the tiles (of TF frames) holding a frame whose mask byte is
// set (frames still iterating; or frames just admitted), and its length.  One
// workgroup of 1024 threads; wavefront ballots and a workgroup scan keep the
// list in increasing tile order.
__global__ __launch_bounds__(1024) void k_tiles(const uint8_t *mask, int F, int Fp, int TF, int32_t *out,
                                                uint32_t *count) {
    __shared__ uint32_t wsum[1024 / kWave];
    __shared__ uint32_t base;
    const int ntiles = Fp / TF;
    const int lane = int(threadIdx.x) % kWave, wv = int(threadIdx.x) / kWave;
    if (threadIdx.x == 0) base = 0;
    __syncthreads();
    for (int t0 = 0; t0 < ntiles; t0 += 1024) {
        const int tile = t0 + int(threadIdx.x);
        bool any = false;
        if (tile < ntiles)
            for (int fw = 0; fw < TF; ++fw) {
                const int f = tile * TF + fw;
                any |= f < F && mask[f];
            }
        const uint64_t ballot = __ballot(any);
        if (lane == 0) wsum[wv] = uint32_t(__popcll(ballot));
        __syncthreads();
        uint32_t off = base;
        for (int w = 0; w < wv; ++w) off += wsum[w];
        if (any) out[off + uint32_t(__popcll(ballot & ((uint64_t(1) << lane) - 1)))] = tile;
        __syncthreads();
        if (threadIdx.x == 0) {
            uint32_t tot = 0;
            for (int w = 0; w < 1024 / kWave; ++w) tot += wsum[w];
            base += tot;
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) *count = base;
}

// [n][tile][Q][TF] -> [F][n][Q]
template <int P, int LG>
__global__ void k_out_vectors(const float *src, int n, int F, int Fp, float *out) {
    using Gm = Geo<P, LG>;
    const size_t t = size_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (t >= size_t(n) * F * Gm::Q) return;
    const int a = int(t % Gm::Q);
    const size_t fj = t / Gm::Q;
    const int f = int(fj / n), j = int(fj % n);
    out[t] = src[at<P, LG>(j, f / Gm::TF, a, f % Gm::TF, Fp / Gm::TF)];
}

}  // namespace tiled
}  // namespace gfbp
