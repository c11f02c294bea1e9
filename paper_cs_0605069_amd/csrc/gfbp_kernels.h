// Device-side building blocks of the GF(2^p) belief-propagation decoder:
// the graph and state views passed to every kernel, multiplication by a
// fixed field element, and lane exchanges inside a 64-lane wavefront.
//
// Every per-frame vector array (messages, likelihoods, posteriors) is stored
// as array[node][frame][a]: the q entries of one frame's vector are
// contiguous and consecutive frames follow each other, frames padded to a
// whole number of 64-frame tiles.  Messages are float32 probabilities (which
// keep small probabilities to full relative precision).  The variable-to-
// check messages of edge e are stored in the weighted domain,
// q~_e(y) = q_e(h_e^-1 y) (entry y holds the probability that h_e x = y),
// which is what the check update consumes; every other array is indexed by
// the field element a itself.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "gfbp_plan.h"

namespace gfbp {

constexpr int kWave = 64;
constexpr int kBlock = 256;
constexpr int kDcMax = 16;  // GFBP_MAX_ROW_DEGREE
constexpr int kDvMax = 8;   // GFBP_MAX_COL_DEGREE

struct DevCode {
    int n, m, E, q, p, n_info;
    int max_dv;               // largest column degree
    const int32_t *row_ptr;   // [m+1]
    const int32_t *col;       // [E]
    const uint8_t *coef;      // [E]
    const int32_t *col_ptr;   // [n+1]
    const int32_t *col_edge;  // [E] edges of each column, increasing edge index
    const int32_t *edge_row;  // [E]
    const uint8_t *mul;       // [q][q] field multiplication
    const uint64_t *emap;     // [E][2] images of x^b under h^-1 (word 0) and h (word 1), 6 bits each
    const int32_t *visit;     // [n] SUS visiting order of the columns
    const int32_t *chain_col; // [n_info] column of source symbol k (the Markov chain's order)
    const int32_t *col_chain; // [n] source symbol held by column j, or -1
};

struct DevState {
    float *Qm;        // [E][F][Q] variable-to-check messages, weighted domain q~(y) = q(h^-1 y)
    float *R;         // [E][F][Q] check-to-variable messages r (PUS only)
    float *L;         // [n][F][Q] normalised channel likelihoods
    float *Pr;        // [K][F][Q] normalised likelihood x Markov prior (Markov only)
    float *Qp;        // [n][F][Q] pseudo-posteriors (when needed)
    const float *Qprev;  // PUS with a Markov source: the previous iteration's pseudo-posteriors, read by
                         // the variable step for Eq. (7) (null: the source priors in Pr are used as they are)
    uint8_t *xh;      // [n][F] decisions
    uint32_t *unsat;  // [F] some check unsatisfied in this iteration
    uint8_t *active;  // [F] frame still iterating
    uint32_t *count;  // [2][2] by iteration parity: frames still iterating, tiles holding them
    int32_t *guards;  // [F]
    int32_t *tiles;   // [2][ntiles] tiles with a running frame, by iteration parity
    int F;            // frames (slots)
    int Fp;           // frame stride (whole 64-frame tiles)
    int nb;           // launch bound on the current tile list (grid = nodes x nb)
    const int32_t *act;      // current tile list
    const uint32_t *nact;    // its length, read on the device (<= nb)
    // per-frame overrides, used by sessions (null: the batch-wide value)
    const uint8_t *fresh;    // only these frames initialise
    const uint8_t *chan;     // channel kind of each frame
    const uint8_t *mark;     // 1 if the frame's source symbols take the Markov prior
};

// Markov source for priors assigned during a SUS sweep: the transition
// matrix M [q][q], the first symbol's distribution pi [q], the matrix shape
// from k_markov_shape, and whether this sweep assigns them (0: the priors in
// Pr are used as they are).
struct SweepPrior {
    const float *M;
    const float *pi;
    const float *mshape;
    int on;
};

struct Snap {
    float *q;  // [F][E][Q] or null
    float *r;  // [F][E][Q] or null
};

// Multiplication by a fixed field element h, applied to y through the images
// of the basis vectors x^b (packed 6 bits each): h y = XOR over set bits b of
// y of h x^b.
template <int P>
__device__ __forceinline__ int gf_apply(uint64_t packed, int y) {
    int r = 0;
#pragma unroll
    for (int b = 0; b < P; ++b) r ^= ((y >> b) & 1) ? int((packed >> (6 * b)) & 63u) : 0;
    return r;
}

// ---------------------------------------------------------------- group ops
// Exchange with lane (lane ^ MASK), each in one step that reads the partner
// lane directly (the lanes of one frame may be the only active ones): DPP
// quad permutes for masks 1 and 2, an xor swizzle for 4, a 16-lane row
// rotation by 8 for 8, and the gfx950 row swaps v_permlane16_swap /
// v_permlane32_swap for 16 and 32.
template <int MASK>
__device__ __forceinline__ uint32_t xchg_u32(uint32_t v) {
    const int x = int(v);
    if constexpr (MASK == 1) {
        return uint32_t(__builtin_amdgcn_mov_dpp(x, 0xB1, 0xF, 0xF, false));   // quad_perm [1,0,3,2]
    } else if constexpr (MASK == 2) {
        return uint32_t(__builtin_amdgcn_mov_dpp(x, 0x4E, 0xF, 0xF, false));   // quad_perm [2,3,0,1]
    } else if constexpr (MASK == 4) {
        // swizzle in bit-mask mode: and 0x1F, or 0, xor 4 (one step: the value
        // comes straight from the partner lane, whatever the other lanes do)
        return uint32_t(__builtin_amdgcn_ds_swizzle(x, 0x101F));
    } else if constexpr (MASK == 8) {
        return uint32_t(__builtin_amdgcn_mov_dpp(x, 0x128, 0xF, 0xF, false));  // row_ror:8
    } else if constexpr (MASK == 16) {
        const auto r = __builtin_amdgcn_permlane16_swap(v, v, false, false);
        return (threadIdx.x & 16) ? r[0] : r[1];
    } else {
        static_assert(MASK == 32, "exchange mask");
        const auto r = __builtin_amdgcn_permlane32_swap(v, v, false, false);
        return (threadIdx.x & 32) ? r[0] : r[1];
    }
}

template <int MASK>
__device__ __forceinline__ float xchg(float v) {
    return __uint_as_float(xchg_u32<MASK>(__float_as_uint(v)));
}

template <int MASK>
__device__ __forceinline__ int xchg(int v) {
    return int(xchg_u32<MASK>(uint32_t(v)));
}

template <int MASK>
__device__ __forceinline__ double xchg(double v) {
    const uint64_t u = uint64_t(__double_as_longlong(v));
    const uint32_t lo = xchg_u32<MASK>(uint32_t(u)), hi = xchg_u32<MASK>(uint32_t(u >> 32));
    return __longlong_as_double((long long)((uint64_t(hi) << 32) | lo));
}

// Row swap of two registers (gfx950 v_permlane16_swap / v_permlane32_swap):
// for MASK = 32 the upper half-wave (lanes 32..63) of `a` trades places with
// the lower half-wave of `b`; for MASK = 16 the odd 16-lane rows of `a` with
// the even rows of `b`.  Afterwards a lane whose MASK bit is 0 holds its own
// a and its partner's a (in b); a lane whose bit is 1 holds its partner's b
// (in a) and its own b.
template <int MASK>
__device__ __forceinline__ void row_swap(uint32_t &a, uint32_t &b) {
    if constexpr (MASK == 16) {
        const auto r = __builtin_amdgcn_permlane16_swap(a, b, false, false);
        a = r[0];
        b = r[1];
    } else {
        static_assert(MASK == 32, "row swap mask");
        const auto r = __builtin_amdgcn_permlane32_swap(a, b, false, false);
        a = r[0];
        b = r[1];
    }
}

template <int MASK>
__device__ __forceinline__ void row_swap(double &a, double &b) {
    const uint64_t ua = uint64_t(__double_as_longlong(a)), ub = uint64_t(__double_as_longlong(b));
    uint32_t al = uint32_t(ua), ah = uint32_t(ua >> 32), bl = uint32_t(ub), bh = uint32_t(ub >> 32);
    row_swap<MASK>(al, bl);
    row_swap<MASK>(ah, bh);
    a = __longlong_as_double((long long)((uint64_t(ah) << 32) | al));
    b = __longlong_as_double((long long)((uint64_t(bh) << 32) | bl));
}

}  // namespace gfbp
