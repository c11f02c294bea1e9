/*
 * Systematic encoder for LDPC codes over GF(2^p), used only to synthesise
 * test and benchmark workloads (codewords whose information symbols follow a
 * chosen source).  It is not part of the decoding path and shares nothing
 * with the decoder library or the reference decoder.
 *
 * Method: the code  { x : H x = 0 }  over GF(2^p) is also a binary linear code
 * once every symbol is written as p bits in the polynomial basis (bit b of a
 * symbol is the coefficient of x^b).  Its binary image is reduced to row
 * echelon form by plain GF(2) Gaussian elimination, taking pivot columns
 * greedily in increasing order.  Because the span of the p bit-columns of one
 * symbol column is a GF(2^p)-subspace, a symbol column is either entirely
 * pivotal or entirely free, so the free symbols are the information symbols
 * and the pivotal ones the parity symbols.  Each pivot row then expresses one
 * parity bit as a GF(2) sum of information bits.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    int p;
    int n_info;          /* K, information symbols                         */
    int rank;            /* parity symbols                                  */
    int wpar;            /* 64-bit words per parity-bit mask                */
    uint64_t *genc;      /* [p*K][wpar]: parity bits flipped by each info bit */
} synth_encoder;

static unsigned gf_mul_poly(unsigned a, unsigned b, int p, unsigned poly)
{
    unsigned r = 0;
    for (int i = 0; i < p; ++i) {
        if (b & 1u) r ^= a;
        b >>= 1;
        a <<= 1;
        if (a & (1u << p)) a ^= poly;
    }
    return r;
}

/*
 * Build the encoder.  col_order receives N column indices: the information
 * columns in increasing order, then the parity columns in increasing order.
 * Returns NULL on allocation failure or if the symbol-level pivot structure is
 * violated (which would indicate a bad field polynomial).
 */
synth_encoder *synth_encoder_build(int p, unsigned poly, int M, int N,
                                   const int32_t *row_ptr, const int32_t *col,
                                   const uint8_t *coef, int32_t *col_order)
{
    const int R = p * M, C = p * N;
    const int W = (C + 63) / 64;
    uint64_t *A = (uint64_t *)calloc((size_t)R * W, sizeof(uint64_t));
    int *pivcol = (int *)malloc(sizeof(int) * (size_t)(R > 0 ? R : 1));
    int *sym_piv = (int *)calloc((size_t)N, sizeof(int));
    if (!A || !pivcol || !sym_piv) { free(A); free(pivcol); free(sym_piv); return NULL; }

    for (int i = 0; i < M; ++i) {
        for (int e = row_ptr[i]; e < row_ptr[i + 1]; ++e) {
            const int j = col[e];
            const unsigned h = coef[e];
            for (int b = 0; b < p; ++b) {
                const unsigned img = gf_mul_poly(h, 1u << b, p, poly);
                for (int r = 0; r < p; ++r) {
                    if ((img >> r) & 1u) {
                        const int rr = i * p + r, cc = j * p + b;
                        A[(size_t)rr * W + cc / 64] ^= (uint64_t)1 << (cc % 64);
                    }
                }
            }
        }
    }

    int rank = 0;
    for (int c = 0; c < C && rank < R; ++c) {
        const int w = c / 64;
        const uint64_t bit = (uint64_t)1 << (c % 64);
        int piv = -1;
        for (int r = rank; r < R; ++r)
            if (A[(size_t)r * W + w] & bit) { piv = r; break; }
        if (piv < 0) continue;
        if (piv != rank) {
            uint64_t *a = A + (size_t)piv * W, *b = A + (size_t)rank * W;
            for (int k = w; k < W; ++k) { uint64_t t = a[k]; a[k] = b[k]; b[k] = t; }
        }
        const uint64_t *pr = A + (size_t)rank * W;
        for (int r = 0; r < R; ++r) {
            if (r == rank) continue;
            uint64_t *rw = A + (size_t)r * W;
            if (rw[w] & bit)
                for (int k = w; k < W; ++k) rw[k] ^= pr[k];
        }
        pivcol[rank] = c;
        sym_piv[c / p]++;
        ++rank;
    }

    int K = 0, nparity = 0;
    for (int j = 0; j < N; ++j) {
        if (sym_piv[j] != 0 && sym_piv[j] != p) { free(A); free(pivcol); free(sym_piv); return NULL; }
        if (sym_piv[j] == 0) ++K; else ++nparity;
    }
    /* info index of each symbol column, parity index of each symbol column */
    int *idx = (int *)malloc(sizeof(int) * (size_t)(N > 0 ? N : 1));
    int ki = 0, pi = 0;
    for (int j = 0; j < N; ++j) if (sym_piv[j] == 0) { idx[j] = ki; col_order[ki++] = j; }
    for (int j = 0; j < N; ++j) if (sym_piv[j] != 0) { idx[j] = pi; col_order[K + pi++] = j; }

    synth_encoder *enc = (synth_encoder *)calloc(1, sizeof(synth_encoder));
    const int wpar = (p * nparity + 63) / 64;
    enc->p = p; enc->n_info = K; enc->rank = nparity; enc->wpar = wpar > 0 ? wpar : 1;
    enc->genc = (uint64_t *)calloc((size_t)p * (K > 0 ? K : 1) * enc->wpar, sizeof(uint64_t));
    if (!enc->genc) { free(enc); free(A); free(pivcol); free(sym_piv); free(idx); return NULL; }

    /* pivot row r:  x[pivcol] = sum over free bit-columns c with A[r][c] = 1 of x[c] */
    for (int r = 0; r < rank; ++r) {
        const int pc = pivcol[r];
        const int pbit = idx[pc / p] * p + (pc % p);           /* parity-bit index */
        const uint64_t *rw = A + (size_t)r * W;
        for (int c = pc + 1; c < C; ++c) {
            if (!((rw[c / 64] >> (c % 64)) & 1u)) continue;
            const int j = c / p;
            if (sym_piv[j] != 0) continue;                     /* zero in RREF anyway */
            const int ibit = idx[j] * p + (c % p);
            enc->genc[(size_t)ibit * enc->wpar + pbit / 64] ^= (uint64_t)1 << (pbit % 64);
        }
    }
    free(A); free(pivcol); free(sym_piv); free(idx);
    return enc;
}

int synth_encoder_info(const synth_encoder *e, int32_t *out_k, int32_t *out_rank)
{
    *out_k = e->n_info; *out_rank = e->rank; return 0;
}

/* parity[f][m] for F frames of information symbols s[f][k]. */
void synth_encoder_encode(const synth_encoder *e, int F, const uint8_t *s, uint8_t *parity)
{
    const int p = e->p, K = e->n_info, Rk = e->rank, wp = e->wpar;
    uint64_t *acc = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)wp);
    for (int f = 0; f < F; ++f) {
        memset(acc, 0, sizeof(uint64_t) * (size_t)wp);
        const uint8_t *sf = s + (size_t)f * K;
        for (int k = 0; k < K; ++k) {
            unsigned v = sf[k];
            for (int b = 0; b < p; ++b) {
                if (!((v >> b) & 1u)) continue;
                const uint64_t *g = e->genc + (size_t)(k * p + b) * wp;
                for (int w = 0; w < wp; ++w) acc[w] ^= g[w];
            }
        }
        uint8_t *pf = parity + (size_t)f * Rk;
        for (int m = 0; m < Rk; ++m) {
            unsigned v = 0;
            for (int b = 0; b < p; ++b) {
                const int bit = m * p + b;
                v |= (unsigned)((acc[bit / 64] >> (bit % 64)) & 1u) << b;
            }
            pf[m] = (uint8_t)v;
        }
    }
    free(acc);
}

void synth_encoder_free(synth_encoder *e)
{
    if (!e) return;
    free(e->genc);
    free(e);
}
