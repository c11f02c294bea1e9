// Device-side building blocks of the GF(2^p) belief-propagation decoder.
//
// Thread mapping: one "group" of Q = 2^P consecutive lanes holds one q-vector
// of one frame, lane k holding entry k; a 64-lane wavefront holds 64/Q frames
// that all work on the same graph node, so every index into the graph is
// wavefront-uniform and every message access stays inside one contiguous
// 256-byte run.
//
// Message layout (frame-interleaved, edge-major): message[e][f][a] with f the
// frame and a the field element, messages kept as probabilities in float32
// (which holds small probabilities to full relative precision).
//
// Check-node arithmetic (Eq. (3)): with y = h x the weighted symbol of an
// edge, the check constraint is an XOR-sum of the y's, so the sum over
// configurations is an XOR-convolution of the siblings' distributions of y,
// q~(y) = q(h^-1 y).  The Walsh-Hadamard transform (WHT) turns XOR-convolution
// into a pointwise product.  The permutation by h^-1 is folded into the load
// address (lane y reads entry h^-1 y), the transforms and products run in
// float64 registers (a float32 transform loses every probability below ~1e-7
// of the largest one to cancellation), and the result S(y) goes back to
// r(a) = S(z + h a) by the store address a = h^-1 (y + z).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace gfbp {

constexpr int kWave = 64;
constexpr int kBlock = 256;
constexpr int kDcMax = 16;  // GFBP_MAX_ROW_DEGREE
constexpr int kDvMax = 8;   // GFBP_MAX_COL_DEGREE

struct DevCode {
    int n, m, E, q, p, n_info;
    const int32_t *row_ptr;   // [m+1]
    const int32_t *col;       // [E]
    const uint8_t *coef;      // [E]
    const int32_t *col_ptr;   // [n+1]
    const int32_t *col_edge;  // [E] edges of each column, increasing edge index
    const int32_t *edge_row;  // [E]
    const uint8_t *mul;       // [q][q] field multiplication
    const uint64_t *emap;     // [E][2] images of x^b under h^-1 (word 0) and h (word 1), 6 bits each
};

struct DevState {
    float *Qm;        // [E][F][Q] variable-to-check messages q
    float *R;         // [E][F][Q] check-to-variable messages r (PUS only)
    float *L;         // [n][F][Q] normalised channel likelihoods
    float *Pr;        // [K][F][Q] normalised likelihood x Markov prior (Markov only)
    float *Qp;        // [n][F][Q] pseudo-posteriors (when needed)
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
// Exchange with lane (lane ^ MASK) without the LDS crossbar: DPP quad
// permutes for masks 1 and 2, half-row mirror followed by a quad reversal for
// 4, a 16-lane row rotation by 8 for 8, and the gfx950 row swaps
// v_permlane16_swap / v_permlane32_swap for 16 and 32.
template <int MASK>
__device__ __forceinline__ uint32_t xchg_u32(uint32_t v) {
    const int x = int(v);
    if constexpr (MASK == 1) {
        return uint32_t(__builtin_amdgcn_mov_dpp(x, 0xB1, 0xF, 0xF, false));   // quad_perm [1,0,3,2]
    } else if constexpr (MASK == 2) {
        return uint32_t(__builtin_amdgcn_mov_dpp(x, 0x4E, 0xF, 0xF, false));   // quad_perm [2,3,0,1]
    } else if constexpr (MASK == 4) {
        const int t = __builtin_amdgcn_mov_dpp(x, 0x141, 0xF, 0xF, false);      // row_half_mirror: i -> 7-i
        return uint32_t(__builtin_amdgcn_mov_dpp(t, 0x1B, 0xF, 0xF, false));   // quad_perm [3,2,1,0]
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

template <int P, typename T>
__device__ __forceinline__ T grp_gather(T v, int src_in_group) {
    return __shfl(v, src_in_group, 1 << P);
}

// Unnormalised Walsh-Hadamard transform across the Q lanes of a group:
// out(k) = sum_y v(y) (-1)^popcount(k & y).  Stage S pairs lanes that differ
// in bit S.
template <int P, int S = 0, typename T>
__device__ __forceinline__ T wht(T v, int k) {
    if constexpr (S < P) {
        const T o = xchg<(1 << S)>(v);
        v = (k & (1 << S)) ? (o - v) : (v + o);
        return wht<P, S + 1>(v, k);
    } else {
        return v;
    }
}

// Sum over the group, bitwise identical on every lane.
template <int P, int S = 0, typename T>
__device__ __forceinline__ T grp_sum(T v) {
    if constexpr (S < P) {
        return grp_sum<P, S + 1>(v + xchg<(1 << S)>(v));
    } else {
        return v;
    }
}

// Index of the largest entry, the smallest index among equal maxima.
template <int P, int S = 0>
__device__ __forceinline__ int grp_argmax(float v, int k) {
    if constexpr (S < P) {
        const float ov = xchg<(1 << S)>(v);
        const int oi = xchg<(1 << S)>(k);
        const bool take = ov > v || (ov == v && oi < k);
        return grp_argmax<P, S + 1>(take ? ov : v, take ? oi : k);
    } else {
        return k;
    }
}

// v / sum over the group; uniform 1/Q (and a guard event) when the sum is
// zero or not finite.
template <int P>
__device__ __forceinline__ double grp_normalise(double v, int32_t *guards, int f, int k) {
    const double s = grp_sum<P>(v);
    if (!(s > 0.0) || !isfinite(s)) {
        if (k == 0) atomicAdd(&guards[f], 1);
        return 1.0 / double(1 << P);
    }
    return v / s;
}

}  // namespace gfbp
