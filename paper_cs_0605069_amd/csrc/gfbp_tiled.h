// Decoder kernels for gfx950: one kernel family, tiled by (frames x lanes).
//
// Thread mapping.  A q-vector (q = 2^P) of one frame is spread over
// G = 2^LG lanes, each holding EL = q/G consecutive entries in registers:
// lane g of the frame holds entries y = g*EL + r, r = 0..EL-1.  A 64-lane
// wavefront holds TF = 64/G frames, all working on the same graph node, so
// every index into the graph (and each edge coefficient h) is
// wavefront-uniform.  Lane = g*TF + fw: the frame index fills the low lane
// bits and g the high ones, so the lanes of one frame differ in the top LG
// lane bits (exchange masks TF, 2TF, ..., 32).
//
// Memory.  Arrays are [node][frame][a] (frames padded to whole 64-frame
// tiles), so a lane's EL entries are contiguous and the wavefront's TF
// frames form one contiguous run of TF*q floats: every load and store of a
// vector is a 16-byte-per-lane (or 8-byte) access covering whole cache lines.
// Where the field element multiplies the index (the weighted domain of the
// check side versus the symbol domain of the variable side), values pass
// through a per-wavefront LDS row buffer instead of scattered global accesses.
//
// Check node (Eq. (3)).  With y = h x the weighted symbol of an edge, a
// check constrains the XOR-sum of the y's, so the sum over configurations is
// the XOR-convolution of the siblings' distributions q~(y) = q(h^-1 y), which
// the q-messages store directly.  The Walsh-Hadamard transform (WHT) turns
// that into a pointwise product; the syndrome z is folded into the product as
// the sign pattern (-1)^popcount(z & k), which shifts the result by z; the
// inverse transform gives T(y) = S(y + z) and r(a) = T(h a).  Transforms,
// products and normalisations run in float64 (a float32 transform loses every
// probability below ~1e-7 of the largest to cancellation).
//
// Transform layout.  The WHT is a butterfly over each of the P index bits.
// Register bits are local.  The lane bits with masks 32 and 16 use the row
// swaps: one swap per pair of registers hands each lane the two operands of a
// butterfly, and afterwards that lane bit and the paired register bit have
// traded places.  So the forward transform leaves the entries in a
// transposed order (tindex gives the transform index of each register), the
// products are pointwise in that order, and the inverse transform, the same
// routine again, restores the natural order.  Lane bits with smaller masks
// (G > 4) exchange with DPP and combine in place.
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
    static constexpr int LTF = 6 - LG;       // log2 frames per wavefront
    static constexpr int TF = 1 << LTF;      // frames per wavefront
    static constexpr int QS = Q + 4;         // LDS row stride (floats): 16-byte aligned rows, banks staggered
    static constexpr int PERM = TF * QS;     // LDS floats per wavefront
    // lane bit of mask 32 (g bit LG-1) pairs with register bit LEL-1; mask 16
    // (g bit LG-2) with register bit LEL-2
    static constexpr bool S32 = LG >= 1 && LEL >= 1;
    static constexpr bool S16 = LG >= 2 && LEL >= 2;
    static constexpr int NSWAP = int(S32) + int(S16);
};

struct Item {
    int node, tile, fw, g, f;
    bool ok;
};

template <int P, int LG>
__device__ __forceinline__ void lane_of(Item &it) {
    using Gm = Geo<P, LG>;
    const int lane = int(threadIdx.x) % kWave;
    it.fw = lane & (Gm::TF - 1);
    it.g = lane >> Gm::LTF;
    it.f = it.tile * Gm::TF + it.fw;
}

// Wavefront w works on node w / nb and on entry w % nb of the list of tiles
// that still hold a running frame (entries past the list's current length,
// read on the device, do nothing).
template <int P, int LG>
__device__ __forceinline__ Item item(int nodes, const DevState &s) {
    using Gm = Geo<P, LG>;
    const int w = int(blockIdx.x) * (kBlock / kWave) + __builtin_amdgcn_readfirstlane(int(threadIdx.x) / kWave);
    Item it;
    it.node = w / s.nb;
    const int ti = w % s.nb;
    it.ok = it.node < nodes && ti < int(*s.nact);
    it.tile = it.ok ? s.act[ti] : 0;
    if (it.tile < 0 || it.tile >= s.Fp / Gm::TF) {  // the list only holds valid tiles; never index past it
        it.ok = false;
        it.tile = 0;
    }
    lane_of<P, LG>(it);
    return it;
}

// Workgroup item: (node, tile) for the whole workgroup; each lane's frame.
template <int P, int LG>
__device__ __forceinline__ Item block_item(int nodes, const DevState &s) {
    using Gm = Geo<P, LG>;
    const int b = int(blockIdx.x);
    Item it;
    it.node = b / s.nb;
    const int ti = b % s.nb;
    it.ok = it.node < nodes && ti < int(*s.nact);
    it.tile = it.ok ? s.act[ti] : 0;
    if (it.tile < 0 || it.tile >= s.Fp / Gm::TF) {
        it.ok = false;
        it.tile = 0;
    }
    lane_of<P, LG>(it);
    return it;
}

// This lane's EL entries of vector `node` of frame f.
template <int P, int LG, typename T>
__device__ __forceinline__ T *chunk(T *arr, size_t node, int Fp, const Item &it) {
    using Gm = Geo<P, LG>;
    return arr + (node * size_t(Fp) + size_t(it.f)) * Gm::Q + size_t(it.g * Gm::EL);
}

// Loads and stores of a lane's EL entries of a vector array.  Every such
// array is larger than the caches and each access streams (a vector is read
// again only after the whole family has passed), so the accesses carry the
// non-temporal hint, except the stores of 8 or more entries per lane: those
// take two or more instructions per lane, each covering every other 16 bytes
// of the wavefront's span, and with the hint the cache writes the partly
// filled lines out before the next instruction completes them (about 1.4x
// the written bytes at 8 entries per lane); plain stores let it merge them.
// The arrays live in global memory; the accesses name that address space, so
// that they compile to global (not generic) memory instructions also where
// the pointer was read from memory (the persistent kernels' per-code state),
// which the compiler cannot trace to a kernel argument.
typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
#define GFBP_GLOBAL __attribute__((address_space(1)))

template <int EL>
__device__ __forceinline__ void ld(const float *p, float *v) {
    if constexpr (EL == 1) {
        v[0] = __builtin_nontemporal_load((const GFBP_GLOBAL float *)p);
    } else if constexpr (EL == 2) {
        const f32x2 t = __builtin_nontemporal_load((const GFBP_GLOBAL f32x2 *)p);
        v[0] = t.x;
        v[1] = t.y;
    } else {
#pragma unroll
        for (int k = 0; k < EL / 4; ++k) {
            const f32x4 t = __builtin_nontemporal_load((const GFBP_GLOBAL f32x4 *)p + k);
            v[4 * k] = t.x;
            v[4 * k + 1] = t.y;
            v[4 * k + 2] = t.z;
            v[4 * k + 3] = t.w;
        }
    }
}

template <int EL>
__device__ __forceinline__ void st(float *p, const float *v) {
    if constexpr (EL == 1) {
        __builtin_nontemporal_store(v[0], (GFBP_GLOBAL float *)p);
    } else if constexpr (EL == 2) {
        const f32x2 t = {v[0], v[1]};
        __builtin_nontemporal_store(t, (GFBP_GLOBAL f32x2 *)p);
    } else {
#pragma unroll
        for (int k = 0; k < EL / 4; ++k) {
            const f32x4 t = {v[4 * k], v[4 * k + 1], v[4 * k + 2], v[4 * k + 3]};
            if constexpr (EL == 4)
                __builtin_nontemporal_store(t, (GFBP_GLOBAL f32x4 *)p + k);
            else
                ((GFBP_GLOBAL f32x4 *)p)[k] = t;
        }
    }
}

// Row degrees up to this bound load every slot of the degree class (the
// slots past the row's degree repeat an edge of the row, a cache hit whose
// value is not used): the loads then form one block and are all in flight
// before the first is used, where loads under a condition each wait for
// their own result.  Wider classes load only the row's edges.
constexpr int kAllSlots = 8;

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

// Permute one vector per frame through the wavefront's LDS rows: the value
// this lane holds for position g*EL + r goes to position pos[r]; afterwards
// the lane holds positions g*EL + r of the permuted vector.  Lanes of one
// frame only touch that frame's row.  Over GF(2) the only multiplier is 1:
// the permutation is the identity.
template <int P, int LG>
__device__ __forceinline__ void lds_permute(float *buf, const Item &it, const int *pos, const float *in,
                                            float *out) {
    using Gm = Geo<P, LG>;
    if constexpr (P == 1) {
#pragma unroll
        for (int r = 0; r < Gm::EL; ++r) out[r] = in[r];
        return;
    }
    float *row = buf + it.fw * Gm::QS;
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
#pragma unroll
    for (int r = 0; r < Gm::EL; ++r) row[pos[r]] = in[r];
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    const float *src = row + it.g * Gm::EL;  // 16-byte aligned rows of EL-entry chunks
    if constexpr (Gm::EL >= 4) {
#pragma unroll
        for (int k = 0; k < Gm::EL / 4; ++k) {
            const f32x4 t = reinterpret_cast<const f32x4 *>(src)[k];
            out[4 * k] = t.x;
            out[4 * k + 1] = t.y;
            out[4 * k + 2] = t.z;
            out[4 * k + 3] = t.w;
        }
    } else {
#pragma unroll
        for (int r = 0; r < Gm::EL; ++r) out[r] = src[r];
    }
}

// ------------------------------------------------------------- transforms
template <int EL, int S = 0>
__device__ __forceinline__ void wht_regs(double *v) {
    if constexpr ((1 << S) < EL) {
        constexpr int m = 1 << S;
#pragma unroll
        for (int r = 0; r < EL; ++r) {
            if (!(r & m)) {
                const double a = v[r], b = v[r | m];
                v[r] = a + b;
                v[r | m] = a - b;
            }
        }
        wht_regs<EL, S + 1>(v);
    }
}

// Butterflies over g bits B..LG-NSWAP-1 (lane masks below 16): exchange and
// combine in place.
template <int P, int LG, int B = 0>
__device__ __forceinline__ void wht_lanes(double *v, int g) {
    using Gm = Geo<P, LG>;
    if constexpr (B < LG - Gm::NSWAP) {
        constexpr int mask = Gm::TF << B;
        const double sg = ((g >> B) & 1) ? -1.0 : 1.0;
#pragma unroll
        for (int r = 0; r < Gm::EL; ++r) v[r] = fma(sg, v[r], xchg<mask>(v[r]));
        wht_lanes<P, LG, B + 1>(v, g);
    }
}

// Butterfly over the lane bit MASK (16 or 32) paired with register bit S:
// after the swap each lane holds both operands of a butterfly in registers
// r and r | 2^S; the sum goes to r and the difference to r | 2^S.
template <int MASK, int S, int EL>
__device__ __forceinline__ void wht_swap(double *v) {
    constexpr int m = 1 << S;
#pragma unroll
    for (int r = 0; r < EL; ++r) {
        if (!(r & m)) {
            double a = v[r], b = v[r | m];
            row_swap<MASK>(a, b);
            v[r] = a + b;
            v[r | m] = a - b;
        }
    }
}

// Unnormalised WHT: natural order in, transposed order out, and back.
template <int P, int LG>
__device__ __forceinline__ void wht(double *v, int g) {
    using Gm = Geo<P, LG>;
    wht_regs<Gm::EL>(v);
    wht_lanes<P, LG>(v, g);
    if constexpr (Gm::S32) wht_swap<32, Gm::LEL - 1, Gm::EL>(v);
    if constexpr (Gm::S16) wht_swap<16, Gm::LEL - 2, Gm::EL>(v);
}

__device__ __forceinline__ int swap_bits(int k, int i, int j) {
    const int d = ((k >> i) ^ (k >> j)) & 1;
    return k ^ ((d << i) | (d << j));
}

// Transform index held by register r of lane g in the transposed order.
template <int P, int LG>
__device__ __forceinline__ int tindex(int g, int r) {
    using Gm = Geo<P, LG>;
    int k = (g << Gm::LEL) | r;
    if constexpr (Gm::S32) k = swap_bits(k, Gm::LEL - 1, P - 1);
    if constexpr (Gm::S16) k = swap_bits(k, Gm::LEL - 2, P - 2);
    return k;
}

// Syndrome sign pattern (-1)^popcount(z & k) in the transposed order.
template <int P, int LG>
__device__ __forceinline__ void syndrome_signs(int z, int g, double *v) {
    using Gm = Geo<P, LG>;
#pragma unroll
    for (int r = 0; r < Gm::EL; ++r) v[r] = (__popc(z & tindex<P, LG>(g, r)) & 1) ? -1.0 : 1.0;
}

template <int P, int LG>
__device__ __forceinline__ void transform(const float *raw, double *v, int g) {
    using Gm = Geo<P, LG>;
#pragma unroll
    for (int r = 0; r < Gm::EL; ++r) v[r] = double(raw[r]);
    wht<P, LG>(v, g);
}

// ------------------------------------------------------------ reductions
// Sum over the G lanes of a frame (bitwise identical on each of them).
template <int P, int LG, int B = 0>
__device__ __forceinline__ double lanes_sum(double v) {
    using Gm = Geo<P, LG>;
    if constexpr (B < LG) {
        return lanes_sum<P, LG, B + 1>(v + xchg<(Gm::TF << B)>(v));
    } else {
        return v;
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
    s = lanes_sum<P, LG>(s);
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

// q-message of edge e from its natural-order values q(a): stored in the
// weighted domain, the value for a going to position h_e a.
template <int P, int LG>
__device__ __forceinline__ void store_q(const DevCode &c, const DevState &s, size_t e, const Item &it,
                                        const float *qa, float *perm) {
    using Gm = Geo<P, LG>;
    int pos[Gm::EL];
    gf_positions<P, LG>(c.emap[2 * e + 1], it.g, pos);
    float out[Gm::EL];
    lds_permute<P, LG>(perm, it, pos, qa, out);
    st<Gm::EL>(chunk<P, LG>(s.Qm, e, s.Fp, it), out);
}

// r-message of edge e from the inverse transform T (natural order, position
// y): r(a) = T(h_e a), so the value for y goes to entry h_e^-1 y.  Returns
// r in natural order in rv.
template <int P, int LG>
__device__ __forceinline__ void r_from_transform(const DevCode &c, size_t e, const Item &it, const double *T,
                                                 float *perm, float *rv) {
    using Gm = Geo<P, LG>;
    int pos[Gm::EL];
    gf_positions<P, LG>(c.emap[2 * e], it.g, pos);
    float tv[Gm::EL];
#pragma unroll
    for (int r = 0; r < Gm::EL; ++r) tv[r] = float(fmax(T[r] * (1.0 / double(Gm::Q)), 0.0));
    lds_permute<P, LG>(perm, it, pos, tv, rv);
}

// Where a frame's inputs are.  Batch-wide kinds, overridden per frame by
// chan_of (indexed by frame) or, in sessions, by DevState::chan (by slot).
// In a batch over several codes a slot f of one code's state holds frame
// gframe[f] of the batch, whose per-symbol inputs (rx, erasure: n entries)
// start at element off_n[frame], whose channel samples (y: n*p) start at
// off_np[frame] and whose likelihood vectors (n*q) start at off_nq[frame];
// null: slot f is frame f at f*n (f*n*p, f*n*q).
struct Chan {
    int channel;              // GFBP_CH_*
    int prior;                // GFBP_PRIOR_* of the source symbols
    int evidence;             // GFBP_EVIDENCE_*
    int static_per_symbol;    // static prior: one vector per source symbol
    const uint8_t *rx, *erasure;
    const float *y, *lik, *param, *pi, *static_P;
    const uint8_t *chan_of;   // [frames] channel kind of each frame, or null
    const int32_t *gframe;    // [F] frame held by slot f, or null
    const int64_t *off_n;     // [frames] or null
    const int64_t *off_np;    // [frames] or null
    const int64_t *off_nq;    // [frames] or null
};

// A1 channel evidence and A2 initialisation of column j for the lane's frame:
// L_j(a), the probability of what was received given x_j = a, as a product
// over the p transmitted bits; in the syndrome form of Section 2 (evidence
// GFBP_EVIDENCE_MN) a source column has no channel evidence (L_j = 1) and
// every other column is a noise symbol n_j, whose evidence is the
// probability of n_j = a given the channel output at column j: for the BSC
// the noise prior f^w (1-f)^(p-w), w the number of ones of a; for the BEC
// each unerased bit has noise 0 and an erased bit (read as 0) has noise equal
// to the unknown sent bit, 0 or 1 alike; for BI-AWGN the received bit is the
// sign of y, so noise bit 0 has probability 1/(1 + exp(-2|y|/sigma^2)).
// p_j = L_j, or for source symbol k = col_chain[j] with a prior
// p_j = norm(L_j P_k), P_k = pi (Markov, iteration 1) or the static prior;
// every edge of column j starts with q_e = p_j.
template <int P, int LG>
__device__ __forceinline__ void init_column(const DevCode &c, const DevState &s, const Chan &ch, const Item &it,
                                            float *perm) {
    using Gm = Geo<P, LG>;
    const int j = it.node, f = it.f;
    const int gf = ch.gframe ? ch.gframe[f] : f;
    const size_t fj = (ch.off_n ? size_t(ch.off_n[gf]) : size_t(gf) * c.n) + size_t(j);
    const int channel = s.chan ? int(s.chan[f]) : ch.chan_of ? int(ch.chan_of[gf]) : ch.channel;
    const int k = c.col_chain[j];
    const bool prior_on = (s.mark ? s.mark[f] != 0 : ch.prior != GFBP_PRIOR_UNIFORM) && k >= 0;
    double L[Gm::EL];
    if (ch.evidence == GFBP_EVIDENCE_MN && k >= 0) {
#pragma unroll
        for (int r = 0; r < Gm::EL; ++r) L[r] = 1.0;
    } else if (channel == GFBP_CH_BSC) {
        const double fl = double(ch.param[gf]);
        const int ref = ch.evidence == GFBP_EVIDENCE_MN ? 0 : int(ch.rx[fj]);  // noise: weight of a itself
#pragma unroll
        for (int r = 0; r < Gm::EL; ++r) {
            const int a = it.g * Gm::EL + r;
            double v = 1.0;
#pragma unroll
            for (int t = 0; t < P; ++t) v *= (((a ^ ref) >> t) & 1) ? fl : (1.0 - fl);
            L[r] = v;
        }
    } else if (channel == GFBP_CH_BEC) {
        const int ref = ch.evidence == GFBP_EVIDENCE_MN ? 0 : int(ch.rx[fj]);
        const int er = ch.erasure[fj];
#pragma unroll
        for (int r = 0; r < Gm::EL; ++r) {
            const int a = it.g * Gm::EL + r;
            double v = 1.0;
#pragma unroll
            for (int t = 0; t < P; ++t) v *= ((er >> t) & 1) ? 0.5 : ((((a ^ ref) >> t) & 1) ? 0.0 : 1.0);
            L[r] = v;
        }
    } else if (channel == GFBP_CH_BIAWGN) {
        const double sg = ch.param[gf];
        const double gain = 2.0 / (sg * sg);
        const size_t ys = (ch.off_np ? size_t(ch.off_np[gf]) : (fj - size_t(j)) * P) + size_t(j) * P;
        double p0[P], p1[P];
#pragma unroll
        for (int t = 0; t < P; ++t) {
            double yb = ch.y[ys + t];
            if (ch.evidence == GFBP_EVIDENCE_MN) yb = fabs(yb);  // bit 0 of the noise: y has the sent sign
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
        const size_t base = ch.off_nq ? size_t(ch.off_nq[gf]) + size_t(j) * Gm::Q : fj * Gm::Q;
#pragma unroll
        for (int r = 0; r < Gm::EL; ++r) L[r] = ch.lik[base + it.g * Gm::EL + r];
    }
    normalise<P, LG>(L, s.guards, f, it.g);
    float pf[Gm::EL];
#pragma unroll
    for (int r = 0; r < Gm::EL; ++r) pf[r] = float(L[r]);
    st<Gm::EL>(chunk<P, LG>(s.L, j, s.Fp, it), pf);
    if (prior_on) {
        const float *P0 = ch.prior == GFBP_PRIOR_MARKOV
                              ? ch.pi
                              : ch.static_P + (ch.static_per_symbol ? size_t(k) * Gm::Q : size_t(0));
        double pr[Gm::EL];
#pragma unroll
        for (int r = 0; r < Gm::EL; ++r) pr[r] = double(pf[r]) * double(P0[it.g * Gm::EL + r]);
        normalise<P, LG>(pr, s.guards, f, it.g);
#pragma unroll
        for (int r = 0; r < Gm::EL; ++r) pf[r] = float(pr[r]);
        st<Gm::EL>(chunk<P, LG>(s.Pr, size_t(k), s.Fp, it), pf);
    }
    for (int t = c.col_ptr[j]; t < c.col_ptr[j + 1]; ++t) store_q<P, LG>(c, s, size_t(c.col_edge[t]), it, pf, perm);
}

template <int P, int LG>
__global__ __launch_bounds__(kBlock) void k_init(DevCode c, DevState s, Chan ch) {
    using Gm = Geo<P, LG>;
    __shared__ __align__(16) float perm_all[(kBlock / kWave) * Gm::PERM];
    float *perm = perm_all + (int(threadIdx.x) / kWave) * Gm::PERM;
    const Item it = item<P, LG>(c.n, s);
    if (!it.ok || it.f >= s.F) return;
    if (s.fresh && !s.fresh[it.f]) return;
    init_column<P, LG>(c, s, ch, it, perm);
}

// A3, parallel schedule: all r of check i (it.node) from the previous
// iteration's q.  DCM bounds the row degree: the siblings' transforms stay in
// registers.
template <int P, int LG, int DCM>
__device__ __forceinline__ void check_node(const DevCode &c, const DevState &s, const uint8_t *z, const Snap &snap,
                                           const Item &it, float *perm) {
    using Gm = Geo<P, LG>;
    const int i = it.node, f = it.f;
    const int rs = c.row_ptr[i], dc = c.row_ptr[i + 1] - rs;
    if (dc == 0) return;
    const int zi = z ? z[size_t(f) * c.m + i] : 0;
    float raw[DCM][Gm::EL];
#pragma unroll
    for (int d = 0; d < DCM; ++d)
        if (DCM <= kAllSlots || d < dc)
            ld<Gm::EL>(chunk<P, LG>(s.Qm, size_t(rs + (d < dc ? d : dc - 1)), s.Fp, it), raw[d]);
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
            float rv[Gm::EL];
            r_from_transform<P, LG>(c, e, it, T, perm, rv);
            st<Gm::EL>(chunk<P, LG>(s.R, e, s.Fp, it), rv);
            if (snap.r)
#pragma unroll
                for (int r = 0; r < Gm::EL; ++r) snap.r[(size_t(f) * c.E + e) * Gm::Q + it.g * Gm::EL + r] = rv[r];
        }
    }
}

template <int P, int LG, int DCM>
__global__ __launch_bounds__(kBlock) void k_check(DevCode c, DevState s, const uint8_t *z, Snap snap) {
    using Gm = Geo<P, LG>;
    __shared__ __align__(16) float perm_all[(kBlock / kWave) * Gm::PERM];
    float *perm = perm_all + (int(threadIdx.x) / kWave) * Gm::PERM;
    const Item it = item<P, LG>(c.m, s);
    if (!it.ok || it.f >= s.F || !s.active[it.f]) return;
    check_node<P, LG, DCM>(c, s, z, snap, it, perm);
}

template <int P, int LG>
__device__ __forceinline__ void markov_prior(const DevCode &c, const DevState &s, const Item &it, int k,
                                             const float *M, const float *pi, const float *mshape,
                                             float (&pf)[Geo<P, LG>::EL]);

// The lane's entries of the prior-weighted evidence p_j of column j: the
// source symbol's prior row when the frame takes a prior, else L_j.
// frame_prior: the frame takes a prior (frame_prior_of).
__device__ __forceinline__ bool frame_prior_of(const DevState &s, int f, int prior_on) {
    return s.mark ? s.mark[f] != 0 : prior_on != 0;
}

template <int P, int LG>
__device__ __forceinline__ const float *prior_row(const DevCode &c, const DevState &s, const Item &it, int j,
                                                  bool frame_prior) {
    const int k = c.col_chain[j];
    return frame_prior && k >= 0 ? chunk<P, LG>(s.Pr, size_t(k), s.Fp, it) : chunk<P, LG>(s.L, size_t(j), s.Fp, it);
}

// Clipping (A5): the symbol of largest pseudo-posterior, the smallest one
// among exact maxima, from the frame's normalised double-precision vector
// distributed over its lanes.
template <int P, int LG, int B = 0>
__device__ __forceinline__ int lanes_argmax(double v, int k) {
    using Gm = Geo<P, LG>;
    if constexpr (B < LG) {
        constexpr int mask = Gm::TF << B;
        const double ov = xchg<mask>(v);
        const int ok = xchg<mask>(k);
        const bool take = ov > v || (ov == v && ok < k);
        return lanes_argmax<P, LG, B + 1>(take ? ov : v, take ? ok : k);
    } else {
        return k;
    }
}

template <int P, int LG>
__device__ __forceinline__ int clip(const double *acc, int g) {
    using Gm = Geo<P, LG>;
    int best = g * Gm::EL;
    double bv = acc[0];
#pragma unroll
    for (int q = 1; q < Gm::EL; ++q)
        if (acc[q] > bv) {
            bv = acc[q];
            best = g * Gm::EL + q;
        }
    return lanes_argmax<P, LG>(bv, best);
}

// A4 variable-node update of column j from its r-messages r[d][.] (natural
// order): the pseudo-posterior Q_j (Eq. (5)) and its decision, then each
// edge's q (Eq. (4)), normalised.
template <int P, int LG, int DVM>
__device__ __forceinline__ void variable_update(const DevCode &c, const DevState &s, const Item &it, int j,
                                                const float (*r)[Geo<P, LG>::EL], int cs, int dv, const float *pf,
                                                int wantQ, const Snap &snap, float *perm) {
    using Gm = Geo<P, LG>;
    const int f = it.f;
    double pv[Gm::EL], acc[Gm::EL];
#pragma unroll
    for (int q = 0; q < Gm::EL; ++q) {
        pv[q] = pf[q];
        acc[q] = pv[q];
    }
#pragma unroll
    for (int d = 0; d < DVM; ++d)
        if (d < dv) {
#pragma unroll
            for (int q = 0; q < Gm::EL; ++q) acc[q] *= double(r[d][q]);
        }
    normalise<P, LG>(acc, s.guards, f, it.g);
    if (wantQ) {
        float Qf[Gm::EL];
#pragma unroll
        for (int q = 0; q < Gm::EL; ++q) Qf[q] = float(acc[q]);
        st<Gm::EL>(chunk<P, LG>(s.Qp, size_t(j), s.Fp, it), Qf);
    }
    const int best = clip<P, LG>(acc, it.g);
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
            float qn[Gm::EL];
#pragma unroll
            for (int q = 0; q < Gm::EL; ++q) qn[q] = float(qv[q]);
            if (snap.q)
#pragma unroll
                for (int q = 0; q < Gm::EL; ++q) snap.q[(size_t(f) * c.E + e) * Gm::Q + it.g * Gm::EL + q] = qn[q];
            store_q<P, LG>(c, s, e, it, qn, perm);
        }
    }
}

// A4, parallel schedule: column it.node from this iteration's r.
template <int P, int LG, int DVM, bool MARKOV_PRIOR = false>
__device__ __forceinline__ void variable_node(const DevCode &c, const DevState &s, int prior_on, int wantQ,
                                              const Snap &snap, const Item &it, float *perm,
                                              const SweepPrior &sp = SweepPrior{}) {
    using Gm = Geo<P, LG>;
    const int j = it.node;
    const int cs = c.col_ptr[j], dv = c.col_ptr[j + 1] - cs;
    float r[DVM][Gm::EL];
#pragma unroll
    for (int d = 0; d < DVM; ++d)
        if (d < dv) ld<Gm::EL>(chunk<P, LG>(s.R, size_t(c.col_edge[cs + d]), s.Fp, it), r[d]);
    float pf[Gm::EL];
    bool assigned = false;
    if constexpr (MARKOV_PRIOR) {
        // A7 for source symbol k of this column from the previous iteration's
        // pseudo-posteriors (the values a separate refresh after that
        // iteration would have written to Pr)
        const int k = c.col_chain[j];
        if (sp.on && s.Qprev && frame_prior_of(s, it.f, prior_on) && k >= 0) {
            DevState sq = s;
            sq.Qp = const_cast<float *>(s.Qprev);
            markov_prior<P, LG>(c, sq, it, k, sp.M, sp.pi, sp.mshape, pf);
            assigned = true;
        }
    }
    if (!assigned) ld<Gm::EL>(prior_row<P, LG>(c, s, it, j, frame_prior_of(s, it.f, prior_on)), pf);
    variable_update<P, LG, DVM>(c, s, it, j, r, cs, dv, pf, wantQ, snap, perm);
}

template <int P, int LG, int DVM>
__global__ __launch_bounds__(kBlock) void k_variable(DevCode c, DevState s, int prior_on, int wantQ, Snap snap) {
    using Gm = Geo<P, LG>;
    __shared__ __align__(16) float perm_all[(kBlock / kWave) * Gm::PERM];
    float *perm = perm_all + (int(threadIdx.x) / kWave) * Gm::PERM;
    const Item it = item<P, LG>(c.n, s);
    if (!it.ok || it.f >= s.F || !s.active[it.f]) return;
    variable_node<P, LG, DVM>(c, s, prior_on, wantQ, snap, it, perm);
}

// A4 with the source symbols' Eq. (7) priors formed in the same step (PUS
// with a Markov source, from the second iteration on): one launch and 8 K q
// bytes per frame fewer than a separate refresh after each iteration.
template <int P, int LG, int DVM>
__global__ __launch_bounds__(kBlock) void k_variable_markov(DevCode c, DevState s, int prior_on, int wantQ,
                                                            Snap snap, SweepPrior sp) {
    using Gm = Geo<P, LG>;
    __shared__ __align__(16) float perm_all[(kBlock / kWave) * Gm::PERM];
    float *perm = perm_all + (int(threadIdx.x) / kWave) * Gm::PERM;
    const Item it = item<P, LG>(c.n, s);
    if (!it.ok || it.f >= s.F || !s.active[it.f]) return;
    variable_node<P, LG, DVM, true>(c, s, prior_on, wantQ, snap, it, perm, sp);
}

// The current q of the siblings of edge rec in its row, for the lane's frame:
// sibling u is edge u of the row below the edge itself, u + 1 from it on.
template <int P, int LG, int DCM>
__device__ __forceinline__ void sibling_loads(const DevState &s, const Item &it, const SusRec &rec,
                                              float (&raw)[DCM - 1][Geo<P, LG>::EL]) {
#pragma unroll
    for (int u = 0; u < DCM - 1; ++u) {
        const int t = u < rec.dc - 1 ? (u < rec.self ? u : u + 1) : rec.self;
        if (DCM <= kAllSlots || u < rec.dc - 1)
            ld<Geo<P, LG>::EL>(chunk<P, LG>(s.Qm, size_t(rec.rs + t), s.Fp, it), raw[u]);
    }
}

// The prior-weighted evidence of column j for the lane's frame (prior_row),
// or, in the variant that assigns source priors during the sweep, Eq. (7)
// from the chain neighbours' newest pseudo-posteriors: a neighbour visited
// earlier in the sweep sits on a lower level, one visited later on a higher
// level.
template <int P, int LG, bool SWEEP_PRIOR>
__device__ __forceinline__ void column_prior(const DevCode &c, const DevState &s, const Item &it, int j,
                                             bool frame_prior, const SweepPrior &sp,
                                             float (&pf)[Geo<P, LG>::EL]) {
    if constexpr (SWEEP_PRIOR) {
        const int k = c.col_chain[j];
        if (sp.on && frame_prior && k >= 0) {
            markov_prior<P, LG>(c, s, it, k, sp.M, sp.pi, sp.mshape, pf);
            return;
        }
    }
    ld<Geo<P, LG>::EL>(prior_row<P, LG>(c, s, it, j, frame_prior), pf);
}

// A6 sequential schedule, the step of one column for one tile of frames,
// done by a workgroup: wavefront d (< column degree) computes the r of the
// column's d-th edge (record rec) from the siblings' current q (partial
// horizontal pass); after a workgroup barrier, wavefront d combines the
// column's r into its edge's q and wavefront 0 into the pseudo-posterior and
// decision (partial vertical pass).  `live`: this lane's frame is still
// iterating.  perm is the wavefront's LDS rows; rsh holds the column's r as
// [d][register][lane].  The siblings' q and then the column's prior are
// requested before any of them is used.  SWEEP_PRIOR: the variant whose
// source-symbol priors are assigned during the sweep (a separate
// instantiation, so the default one carries none of its code or registers).
template <int P, int LG, int DCM, int DVM, bool SWEEP_PRIOR>
__device__ __forceinline__ void sus_column(const DevCode &c, const DevState &s, const uint8_t *z, const Item &it,
                                           bool live, const SusRec &rec, int prior_on, int wantQ, const Snap &snap,
                                           const SweepPrior &sp, float *perm, float *rsh) {
    using Gm = Geo<P, LG>;
    const int f = it.f;
    const int d = __builtin_amdgcn_readfirstlane(int(threadIdx.x) / kWave), lane = int(threadIdx.x) % kWave;
    const int j = rec.j, dv = rec.dv;
    const bool mine = live && d < dv;
    const bool post = live && d == 0;  // pseudo-posterior and decision (also for a column without edges)
    const size_t e = size_t(rec.e);
    const bool fprior = (mine || post) && frame_prior_of(s, f, prior_on);
    float pf[Gm::EL];
    if (mine) {
        // the siblings' q and the syndrome symbol, then the prior: all
        // requested before any is used
        const int dc = rec.dc;
        float raw[DCM - 1][Gm::EL];
        sibling_loads<P, LG, DCM>(s, it, rec, raw);
        const int zi = z ? z[size_t(f) * c.m + rec.i] : 0;
        column_prior<P, LG, SWEEP_PRIOR>(c, s, it, j, fprior, sp, pf);
        double acc[Gm::EL];
        syndrome_signs<P, LG>(zi, it.g, acc);
#pragma unroll
        for (int u = 0; u < DCM - 1; ++u) {
            if (u < dc - 1) {
                double w[Gm::EL];
                transform<P, LG>(raw[u], w, it.g);
#pragma unroll
                for (int q = 0; q < Gm::EL; ++q) acc[q] *= w[q];
            }
        }
        wht<P, LG>(acc, it.g);
        int pos[Gm::EL];
        gf_positions<P, LG>(rec.hinv, it.g, pos);
        float tv[Gm::EL], rv[Gm::EL];
#pragma unroll
        for (int q = 0; q < Gm::EL; ++q) tv[q] = float(fmax(acc[q] * (1.0 / double(Gm::Q)), 0.0));
        lds_permute<P, LG>(perm, it, pos, tv, rv);
#pragma unroll
        for (int q = 0; q < Gm::EL; ++q) {
            rsh[(d * Gm::EL + q) * kWave + lane] = rv[q];
            if (snap.r) snap.r[(size_t(f) * c.E + e) * Gm::Q + it.g * Gm::EL + q] = rv[q];
        }
    } else if (post) {
        column_prior<P, LG, SWEEP_PRIOR>(c, s, it, j, fprior, sp, pf);  // a column without edges
    }
    __syncthreads();
    double pv[Gm::EL];
#pragma unroll
    for (int q = 0; q < Gm::EL; ++q) pv[q] = pf[q];
    if (post) {
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
        if (wantQ) {
            float Qf[Gm::EL];
#pragma unroll
            for (int q = 0; q < Gm::EL; ++q) Qf[q] = float(acc[q]);
            st<Gm::EL>(chunk<P, LG>(s.Qp, size_t(j), s.Fp, it), Qf);
        }
        const int best = clip<P, LG>(acc, it.g);
        if (it.g == 0) s.xh[size_t(j) * s.Fp + f] = uint8_t(best);
    }
    if (mine) {
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
        float qn[Gm::EL];
#pragma unroll
        for (int q = 0; q < Gm::EL; ++q) qn[q] = float(qv[q]);
        if (snap.q)
#pragma unroll
            for (int q = 0; q < Gm::EL; ++q) snap.q[(size_t(f) * c.E + e) * Gm::Q + it.g * Gm::EL + q] = qn[q];
        int pos[Gm::EL];
        gf_positions<P, LG>(rec.h, it.g, pos);
        float out[Gm::EL];
        lds_permute<P, LG>(perm, it, pos, qn, out);
        st<Gm::EL>(chunk<P, LG>(s.Qm, e, s.Fp, it), out);
    }
}

// A6, one dependency level: the columns of recs[0..ncols) share no check, so
// their steps commute; each runs exactly as in the strict order.  One
// workgroup per (column, tile), one wavefront per edge of the column
// (blockDim = 64 x the largest column degree, at most DVM wavefronts; recs
// holds rstride >= that many slots per column).
template <int P, int LG, int DCM, int DVM, bool SWEEP_PRIOR>
__global__ __launch_bounds__(DVM *kWave) void k_sus_level(DevCode c, DevState s, const uint8_t *z, int prior_on,
                                                          int wantQ, Snap snap, SweepPrior sp, const SusRec *recs,
                                                          int rstride, int ncols) {
    using Gm = Geo<P, LG>;
    __shared__ __align__(16) float perm[DVM * Gm::PERM];
    __shared__ float rsh[DVM * Gm::EL * kWave];
    const Item it = block_item<P, LG>(ncols, s);
    if (!it.ok) return;  // uniform over the workgroup
    const int d = __builtin_amdgcn_readfirstlane(int(threadIdx.x) / kWave);
    const SusRec rec = recs[size_t(it.node) * rstride + d];
    const bool live = it.f < s.F && s.active[it.f];
    sus_column<P, LG, DCM, DVM, SWEEP_PRIOR>(c, s, z, it, live, rec, prior_on, wantQ, snap, sp, perm + d * Gm::PERM,
                                             rsh);
}

// A6, a run of thin dependency levels (a few columns each) in one launch:
// one workgroup per tile takes the columns of recs[0..ncols), in level order,
// one after the other as the strict sweep does; every column of the run
// depends only on columns of this frame at lower levels, which come earlier
// in the run or in an earlier launch.
template <int P, int LG, int DCM, int DVM, bool SWEEP_PRIOR>
__global__ __launch_bounds__(DVM *kWave) void k_sus_run(DevCode c, DevState s, const uint8_t *z, int prior_on,
                                                        int wantQ, Snap snap, SweepPrior sp, const SusRec *recs,
                                                        int rstride, int ncols) {
    using Gm = Geo<P, LG>;
    __shared__ __align__(16) float perm[DVM * Gm::PERM];
    __shared__ float rsh[DVM * Gm::EL * kWave];
    const Item it = block_item<P, LG>(1, s);
    if (!it.ok) return;  // uniform over the workgroup
    const bool live = it.f < s.F && s.active[it.f];
    const int d = __builtin_amdgcn_readfirstlane(int(threadIdx.x) / kWave);
    float *mine = perm + d * Gm::PERM;
    for (int p = 0; p < ncols; ++p) {
        const SusRec rec = recs[size_t(p) * rstride + d];
        sus_column<P, LG, DCM, DVM, SWEEP_PRIOR>(c, s, z, it, live, rec, prior_on, wantQ, snap, sp, mine, rsh);
        __syncthreads();  // rsh and the LDS rows are reused by the next column
    }
}

// A6, strict order: the columns in visiting order, one after the other, for
// each tile.
template <int P, int LG, int DCM, int DVM, bool SWEEP_PRIOR>
__global__ __launch_bounds__(DVM *kWave) void k_sequential(DevCode c, DevState s, const uint8_t *z, int prior_on,
                                                           int wantQ, Snap snap, SweepPrior sp) {
    using Gm = Geo<P, LG>;
    __shared__ __align__(16) float perm[DVM * Gm::PERM];
    __shared__ float rsh[DVM * Gm::EL * kWave];
    const Item it = block_item<P, LG>(1, s);
    if (!it.ok) return;  // uniform over the workgroup
    const bool live = it.f < s.F && s.active[it.f];
    const int d = __builtin_amdgcn_readfirstlane(int(threadIdx.x) / kWave);
    float *mine = perm + d * Gm::PERM;
    for (int t = 0; t < c.n; ++t) {
        const int j = c.visit[t];
        SusRec rec{};
        rec.j = j;
        const int cs = c.col_ptr[j];
        rec.dv = c.col_ptr[j + 1] - cs;
        if (d < rec.dv) {
            rec.e = c.col_edge[cs + d];
            rec.i = c.edge_row[rec.e];
            rec.rs = c.row_ptr[rec.i];
            rec.dc = c.row_ptr[rec.i + 1] - rec.rs;
            rec.self = rec.e - rec.rs;
            rec.hinv = c.emap[2 * size_t(rec.e)];
            rec.h = c.emap[2 * size_t(rec.e) + 1];
        }
        sus_column<P, LG, DCM, DVM, SWEEP_PRIOR>(c, s, z, it, live, rec, prior_on, wantQ, snap, sp, mine, rsh);
        __syncthreads();  // rsh and the LDS rows are reused by the next column
    }
}

// A7 dynamical block prior (Eq. (7)) for source symbol k of frame it.f,
// from the current pseudo-posteriors of its chain neighbours k-1 and k+1 (at
// columns chain_col[k -+ 1]) in Qp, times the evidence of its own column,
// into pf (both normalised).
//
// mshape (from k_markov_shape): when M = s I + o (J - I) (every diagonal entry
// s, every other entry o, as for a source that keeps its symbol or moves to
// any other one uniformly), the neighbour sums of Eq. (7) take O(q):
// sum_a Q(a) M(a, b) = sum_c M(b, c) Q(c) = s Q(b) + o (S - Q(b)), S = sum Q,
// and each lane needs only its own entries of the neighbours; any other M
// takes the O(q^2) sums.  Every lane of the frame takes part.
template <int P, int LG>
__device__ __forceinline__ void markov_prior(const DevCode &c, const DevState &s, const Item &it, int k,
                                             const float *M, const float *pi, const float *mshape,
                                             float (&pf)[Geo<P, LG>::EL]) {
    using Gm = Geo<P, LG>;
    const int K = c.n_info;
    double u[Gm::EL], v[Gm::EL];
#pragma unroll
    for (int q = 0; q < Gm::EL; ++q) {
        const int b = it.g * Gm::EL + q;
        u[q] = k == 0 ? double(pi[b]) : 0.0;
        v[q] = k == K - 1 ? 1.0 : 0.0;
    }
    const size_t fo = size_t(it.f) * Gm::Q;
    if (mshape[0] != 0.0f) {
        const double sd = mshape[1], od = mshape[2];
        // the two neighbours' sums, in the same order for both (lanes_sum
        // over the frame's lanes)
        float nb[2][Gm::EL];
        double S[2] = {0.0, 0.0};
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int kk = h == 0 ? k - 1 : k + 1;
            if (kk >= 0 && kk < K) ld<Gm::EL>(chunk<P, LG>(s.Qp, size_t(c.chain_col[kk]), s.Fp, it), nb[h]);
            else
#pragma unroll
                for (int q = 0; q < Gm::EL; ++q) nb[h][q] = 0.0f;
#pragma unroll
            for (int q = 0; q < Gm::EL; ++q) S[h] += double(nb[h][q]);
            S[h] = lanes_sum<P, LG>(S[h]);
        }
        if (k > 0)
#pragma unroll
            for (int q = 0; q < Gm::EL; ++q) u[q] = sd * double(nb[0][q]) + od * (S[0] - double(nb[0][q]));
        if (k < K - 1)
#pragma unroll
            for (int q = 0; q < Gm::EL; ++q) v[q] = sd * double(nb[1][q]) + od * (S[1] - double(nb[1][q]));
    } else {
        // the whole neighbour vectors (every lane of the frame reads all q entries)
        if (k > 0) {
            const float *qp = s.Qp + size_t(c.chain_col[k - 1]) * s.Fp * Gm::Q + fo;
#pragma unroll 2
            for (int a = 0; a < Gm::Q; ++a) {
                const double qa = qp[a];
#pragma unroll
                for (int q = 0; q < Gm::EL; ++q) u[q] += qa * double(M[a * Gm::Q + it.g * Gm::EL + q]);
            }
        }
        if (k < K - 1) {
            const float *qp = s.Qp + size_t(c.chain_col[k + 1]) * s.Fp * Gm::Q + fo;
#pragma unroll 2
            for (int cc = 0; cc < Gm::Q; ++cc) {
                const double qc = qp[cc];
#pragma unroll
                for (int q = 0; q < Gm::EL; ++q) v[q] += double(M[(it.g * Gm::EL + q) * Gm::Q + cc]) * qc;
            }
        }
    }
#pragma unroll
    for (int q = 0; q < Gm::EL; ++q) u[q] *= v[q];
    normalise<P, LG>(u, s.guards, it.f, it.g);
    float lf[Gm::EL];
    ld<Gm::EL>(chunk<P, LG>(s.L, size_t(c.chain_col[k]), s.Fp, it), lf);
#pragma unroll
    for (int q = 0; q < Gm::EL; ++q) u[q] *= double(lf[q]);
    normalise<P, LG>(u, s.guards, it.f, it.g);
#pragma unroll
    for (int q = 0; q < Gm::EL; ++q) pf[q] = float(u[q]);
}

// A7 after an iteration: every source symbol's prior for the next one.
template <int P, int LG>
__global__ __launch_bounds__(kBlock) void k_markov(DevCode c, DevState s, const float *M, const float *pi,
                                                   const float *mshape) {
    using Gm = Geo<P, LG>;
    const Item it = item<P, LG>(c.n_info, s);
    if (!it.ok || it.f >= s.F || !s.active[it.f]) return;
    if (s.mark && !s.mark[it.f]) return;
    float pf[Gm::EL];
    markov_prior<P, LG>(c, s, it, it.node, M, pi, mshape, pf);
    st<Gm::EL>(chunk<P, LG>(s.Pr, size_t(it.node), s.Fp, it), pf);
}

// Shape of the Markov matrix for k_markov: out = {1, s, o} when every
// diagonal entry of M (q x q) equals s and every other entry o, else {0, 0, 0}.
// One wavefront.
static __global__ __launch_bounds__(kWave) void k_markov_shape(const float *M, int q, float *out) {
    const float sd = M[0], od = q > 1 ? M[1] : 0.0f;
    bool ok = true;
    for (int t = int(threadIdx.x); t < q * q; t += kWave) ok &= M[t] == ((t / q == t % q) ? sd : od);
    const bool all = __ballot(!ok) == 0;
    if (threadIdx.x == 0) {
        out[0] = all ? 1.0f : 0.0f;
        out[1] = all ? sd : 0.0f;
        out[2] = all ? od : 0.0f;
        out[3] = 0.0f;
    }
}

// Ordered list of the tiles (of TF frames) holding a frame whose mask byte is
// set (frames still iterating; or frames just admitted), and its length.  One
// workgroup of 1024 threads; wavefront ballots and a workgroup scan keep the
// list in increasing tile order.
static __global__ __launch_bounds__(1024) void k_tiles(const uint8_t *mask, int F, int Fp, int TF, int32_t *out,
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

// [n][Fp][Q] -> [F][n][Q]
template <int P>
__global__ void k_out_vectors(const float *src, int n, int F, int Fp, float *out) {
    constexpr int Q = 1 << P;
    const size_t t = size_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (t >= size_t(n) * F * Q) return;
    const int a = int(t % Q);
    const size_t fj = t / Q;
    const int f = int(fj / n), j = int(fj % n);
    out[t] = src[(size_t(j) * Fp + f) * Q + a];
}

}  // namespace tiled
}  // namespace gfbp
