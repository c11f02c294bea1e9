// Persistent work-list decoding: one kernel launch decodes a batch whose
// frames may lie on many codes, over several fields.
//
// The work list holds tiles: the TF frames of one code that one wavefront's
// lanes cover (TF = 64 / lanes per frame).  A workgroup of W wavefronts takes
// the next tile from a device-side counter and decodes it from its channel
// outputs to its final decisions: initialisation, then each iteration's
// schedule with a workgroup barrier wherever a step reads what another
// wavefront wrote (between the PUS check and variable halves; between
// consecutive SUS dependency levels), the H x = z test of the tile's frames,
// their retirement and the Markov refresh; then it writes the decisions and
// takes the next tile.  Within a step the W wavefronts share the nodes (rows
// or columns, or the columns of one SUS level), one node at a time each.  The
// arithmetic of every node is that of the plain kernels (the same device
// functions; a SUS column's r-messages are formed by one wavefront in edge
// order instead of one wavefront per edge), so outputs are bitwise those of
// the plain decode.
//
// One kernel per field and degree class, its lanes per frame following from
// the entries per lane (2^LEL, at most q); the kernels of one batch run
// concurrently on forked streams, captured into one HIP graph.  Each list is
// ordered by the work of a tile (its code's edges times q times its frames),
// largest first, so that the long tiles start early.
#pragma once
#include "gfbp_tiled.h"

namespace gfbp {
namespace persist {

// One code's frames in a launch: slots 0..F-1 of its own message state.
struct Group {
    DevCode c;
    DevState s;             // F = frames of this code in the batch, stride Fp
    const SusRec *recs;     // SUS: the columns in level order, rs records each
    const int32_t *lvl;     // [nlev + 1] first position of each level in recs
    int nlev, rs, p;
    int32_t *iters;         // [F] first converged iteration (or max_iter)
    uint8_t *conv;          // [F]
    uint8_t *z;             // [F][m] syndromes by slot, or null for z = 0
    const int32_t *gframe;  // [F] the batch frame held by slot f
};

struct Work {
    int32_t group, tile;
};

// Batch-wide inputs and outputs.
struct Batch {
    int schedule, max_iter, early_stop, prior_on, markov;
    const float *M, *pi, *mshape;
    tiled::Chan ch;          // per-frame offsets in ch.off_n / ch.off_nq; gframe is per group
    const int64_t *off_m;    // [frames] start of each frame's syndrome in zin
    const uint8_t *zin;      // ragged syndromes, or null
    uint8_t *xhat;           // ragged decisions (at ch.off_n)
    int32_t *iters;          // [frames]
    uint8_t *conv;           // [frames]
    int32_t *guards;         // [frames] or null
};

template <int P, int LEL>
struct Pick {
    static constexpr int LG = P - (LEL < P ? LEL : P);
};

// A6, one SUS column step by one wavefront: the r-messages of the column's
// edges (records recs[0..dv)) in edge order from the siblings' current q,
// then the column's pseudo-posterior, decision and q-messages (A4).  Where
// registers allow (narrow rows, few entries per lane), the siblings of the
// next edge are requested before the current edge's arithmetic, so that one
// edge's loads are always in flight.
template <int P, int LG, int DCM, int DVM>
__device__ __forceinline__ void sus_column_wave(const DevCode &c, const DevState &s, const uint8_t *z,
                                                const tiled::Item &it, const SusRec *recs, int prior_on, int wantQ,
                                                float *perm) {
    using Gm = tiled::Geo<P, LG>;
    const int f = it.f;
    const int j = recs[0].j, dv = recs[0].dv;
    constexpr bool kAhead = (DCM - 1) * Gm::EL <= 24;
    constexpr int NB = kAhead ? 2 : 1;
    float r[DVM][Gm::EL];
    float raw[NB][DCM - 1][Gm::EL];
    if (kAhead && dv > 0) tiled::sibling_loads<P, LG, DCM>(s, it, recs[0], raw[0]);
    float pf[Gm::EL];  // the column's prior, requested early: used only at the end
    tiled::ld<Gm::EL>(tiled::prior_row<P, LG>(c, s, it, j, tiled::frame_prior_of(s, f, prior_on)), pf);
#pragma unroll
    for (int d = 0; d < DVM; ++d) {
        if (d < dv) {
            if (!kAhead)
                tiled::sibling_loads<P, LG, DCM>(s, it, recs[d], raw[0]);
            else if (d + 1 < DVM && d + 1 < dv)
                tiled::sibling_loads<P, LG, DCM>(s, it, recs[d + 1], raw[(d + 1) % NB]);
            const SusRec rec = recs[d];
            double acc[Gm::EL];
            tiled::syndrome_signs<P, LG>(z ? z[size_t(f) * c.m + rec.i] : 0, it.g, acc);
#pragma unroll
            for (int u = 0; u < DCM - 1; ++u) {
                if (u < rec.dc - 1) {
                    double w[Gm::EL];
                    tiled::transform<P, LG>(raw[d % NB][u], w, it.g);
#pragma unroll
                    for (int q = 0; q < Gm::EL; ++q) acc[q] *= w[q];
                }
            }
            tiled::wht<P, LG>(acc, it.g);
            int pos[Gm::EL];
            tiled::gf_positions<P, LG>(rec.hinv, it.g, pos);
            float tv[Gm::EL];
#pragma unroll
            for (int q = 0; q < Gm::EL; ++q) tv[q] = float(fmax(acc[q] * (1.0 / double(Gm::Q)), 0.0));
            tiled::lds_permute<P, LG>(perm, it, pos, tv, r[d]);
        }
    }
    tiled::variable_update<P, LG, DVM>(c, s, it, j, r, c.col_ptr[j], dv, pf, wantQ, Snap{nullptr, nullptr}, perm);
}

// Decode tile `tile` of group G to the end.  act/unsat: the tile's
// per-frame flags in LDS.
template <int P, int LG, int DCM, int DVM, int SCH>
__device__ __forceinline__ void decode_tile(const Group &G, const Batch &B, int tile, float *perm, uint32_t *act,
                                            uint32_t *unsat) {
    using Gm = tiled::Geo<P, LG>;
    constexpr int TF = Gm::TF;
    const DevCode &c = G.c;
    const DevState &s = G.s;
    const int F = s.F, f0 = tile * TF;
    const int tid = int(threadIdx.x);
    const int W = int(blockDim.x) / kWave, w = __builtin_amdgcn_readfirstlane(tid / kWave);
    tiled::Chan ch = B.ch;
    ch.gframe = G.gframe;
    if (tid < TF) {
        const int f = f0 + tid;
        act[tid] = f < F ? 1u : 0u;
        if (f < F) {
            s.guards[f] = 0;
            G.iters[f] = 0;
            G.conv[f] = 0;
        }
    }
    if (G.z)
        for (int k = tid; k < TF * c.m; k += int(blockDim.x)) {
            const int fw = k / c.m, i = k - fw * c.m, f = f0 + fw;
            if (f < F) G.z[size_t(f) * c.m + i] = B.zin[size_t(B.off_m[G.gframe[f]]) + size_t(i)];
        }
    __syncthreads();
    for (int j = w; j < c.n; j += W) {
        tiled::Item it;
        it.node = j;
        it.tile = tile;
        it.ok = true;
        tiled::lane_of<P, LG>(it);
        if (it.f < F) tiled::init_column<P, LG>(c, s, ch, it, perm);
    }
    __syncthreads();
    const uint8_t *z = G.z;
    const Snap nosnap{nullptr, nullptr};
    for (int t = 1; t <= B.max_iter; ++t) {
        if (tid < TF) unsat[tid] = 0u;
        if constexpr (SCH == GFBP_PUS) {
            for (int i = w; i < c.m; i += W) {
                tiled::Item it;
                it.node = i;
                it.tile = tile;
                it.ok = true;
                tiled::lane_of<P, LG>(it);
                if (it.f < F && act[it.fw]) tiled::check_node<P, LG, DCM>(c, s, z, nosnap, it, perm);
            }
            __syncthreads();
            for (int j = w; j < c.n; j += W) {
                tiled::Item it;
                it.node = j;
                it.tile = tile;
                it.ok = true;
                tiled::lane_of<P, LG>(it);
                if (it.f < F && act[it.fw]) tiled::variable_node<P, LG, DVM>(c, s, B.prior_on, B.markov, nosnap, it, perm);
            }
            __syncthreads();
        } else {
            for (int l = 0; l < G.nlev; ++l) {
                const int p1 = G.lvl[l + 1];
                for (int pos = G.lvl[l] + w; pos < p1; pos += W) {
                    const SusRec *rr = G.recs + size_t(pos) * G.rs;
                    tiled::Item it;
                    it.node = rr->j;
                    it.tile = tile;
                    it.ok = true;
                    tiled::lane_of<P, LG>(it);
                    if (it.f < F && act[it.fw])
                        sus_column_wave<P, LG, DCM, DVM>(c, s, z, it, rr, B.prior_on, B.markov, perm);
                }
                __syncthreads();
            }
        }
        // A5: H x = z for the tile's frames, 64 / TF rows per wavefront pass
        {
            constexpr int RPW = kWave / TF;
            const int lane = tid % kWave, ro = lane / TF, fw = lane % TF, f = f0 + fw;
            const bool run = f < F && act[fw];
            for (int i0 = w * RPW; i0 < c.m; i0 += W * RPW) {
                const int i = i0 + ro;
                if (run && i < c.m) {
                    int acc = 0;
                    for (int e = c.row_ptr[i]; e < c.row_ptr[i + 1]; ++e)
                        acc ^= c.mul[int(c.coef[e]) * c.q + s.xh[size_t(c.col[e]) * s.Fp + f]];
                    if (acc != (z ? int(z[size_t(f) * c.m + i]) : 0)) unsat[fw] = 1u;
                }
            }
        }
        __syncthreads();
        int alive = 0;
        if (tid < TF && act[tid]) {
            const int f = f0 + tid;
            const bool ok = unsat[tid] == 0u;
            if (ok && !G.conv[f]) {
                G.conv[f] = 1;
                G.iters[f] = t;
            }
            if ((ok && B.early_stop) || t >= B.max_iter) {
                act[tid] = 0u;
                if (!G.conv[f]) G.iters[f] = B.max_iter;
                const int gf = G.gframe[f];
                B.iters[gf] = G.iters[f];
                B.conv[gf] = G.conv[f];
                if (B.guards) B.guards[gf] = s.guards[f];
            } else {
                alive = 1;
            }
        }
        if (!__syncthreads_or(alive)) break;
        if (B.markov) {
            for (int k = w; k < c.n_info; k += W) {
                tiled::Item it;
                it.node = k;
                it.tile = tile;
                it.ok = true;
                tiled::lane_of<P, LG>(it);
                if (it.f < F && act[it.fw]) {
                    float pf[Gm::EL];
                    tiled::markov_prior<P, LG>(c, s, it, k, B.M, B.pi, B.mshape, pf);
                    tiled::st<Gm::EL>(tiled::chunk<P, LG>(s.Pr, size_t(k), s.Fp, it), pf);
                }
            }
            __syncthreads();
        }
    }
    for (int k = tid; k < TF * c.n; k += int(blockDim.x)) {
        const int fw = k / c.n, j = k - fw * c.n, f = f0 + fw;
        if (f < F) B.xhat[size_t(B.ch.off_n[G.gframe[f]]) + size_t(j)] = s.xh[size_t(j) * s.Fp + f];
    }
}

// The persistent kernel of one field (P), degree class (DCM, DVM) and
// schedule (SCH): workgroups take tiles until the list is exhausted.
// blockDim = W x 64 (W <= 8); dynamic LDS = W x Geo::PERM floats.
template <int P, int LEL, int DCM, int DVM, int SCH>
__global__ __launch_bounds__(512) void k_persist(const Group *groups, const Work *work, int n_work, uint32_t *next,
                                                 Batch B) {
    constexpr int LG = Pick<P, LEL>::LG;
    extern __shared__ __align__(16) float lds[];
    __shared__ int sh_item;
    __shared__ uint32_t act[kWave], unsat[kWave];
    float *perm = lds + __builtin_amdgcn_readfirstlane(int(threadIdx.x) / kWave) * tiled::Geo<P, LG>::PERM;
    for (;;) {
        if (threadIdx.x == 0) sh_item = int(atomicAdd(next, 1u));
        __syncthreads();
        const int idx = __builtin_amdgcn_readfirstlane(sh_item);
        __syncthreads();  // sh_item is read before the next round writes it
        if (idx >= n_work) return;
        const Work wk = work[idx];
        const Group &G = groups[__builtin_amdgcn_readfirstlane(wk.group)];
        decode_tile<P, LG, DCM, DVM, SCH>(G, B, __builtin_amdgcn_readfirstlane(wk.tile), perm, act, unsat);
        __syncthreads();  // the tile's LDS flags are free for the next one
    }
}

// Host side (gfbp_persist.hip): launch the persistent kernel of field p,
// entries per lane 2^lel, degree class small (rows <= 6, columns <= 4) or
// general, schedule sch, with `waves` wavefronts per workgroup and a grid
// that fills the device (at most n_work workgroups); with events a and b, the
// launch records its start and end in them.  Returns hipSuccess or the
// failing call's error; hipErrorInvalidValue for a shape without a kernel.
hipError_t launch_persistent(int p, int lel, bool small, int sch, const Group *groups, const Work *work, int n_work,
                             uint32_t *next, const Batch &B, int waves, hipStream_t st, hipEvent_t a, hipEvent_t b);

}  // namespace persist
}  // namespace gfbp
