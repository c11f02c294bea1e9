/*
 * Reference decoder: belief-propagation decoding of LDPC codes over GF(2^p),
 * written plainly in double precision.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing on the decoding product path may call,
 * link or load this file; it is used by the test suite, by the smoke check and
 * by the benchmark's CPU-baseline leg.  It shares no source with the GPU
 * decoder: its field tables, channel models, message updates, schedules and
 * prior updates are all written here, from the paper (Yacov, Efraim, Kfir,
 * Kanter, Shental, "Parallel vs. Sequential Belief Propagation Decoding of
 * LDPC Codes over GF(q) and Markov Sources", Section 2).
 *
 * What each function follows:
 *   field arithmetic ........ GF(2^p), polynomial basis (Section 2: q-ary
 *                             symbols sent as their binary representation,
 *                             noise added bit-wise)
 *   ref_likelihood .......... BSC noise prior f^L (1-f)^(p-L) of Section 2,
 *                             taken about the received symbol; BEC and BI-AWGN
 *                             as bit-wise products (Section 3 channels)
 *   ref_noise_evidence ...... MacKay-Neal syndrome form (Section 2, Eqs. (1),
 *                             (2)): the decoder sees z = B r and, for each
 *                             noise symbol, the probability of each noise
 *                             value given the channel output; for the BSC
 *                             the paper's noise prior f^L (1-f)^(p-L), for
 *                             the BEC and BI-AWGN the bit-wise analogues
 *   static prior ............ Section 2: source symbols carry a prior that is
 *                             multiplied into their evidence (fixed here; the
 *                             Markov prior below re-estimates it)
 *   check update ............ Eq. (3): sum, over sibling configurations
 *                             that satisfy check i with x_j = a, of the
 *                             product of sibling q-messages, accumulated one
 *                             sibling at a time (distributivity only)
 *   variable update ......... Eq. (4), normalised
 *   pseudo-posterior ........ Eq. (5), normalised, then clipped (argmax)
 *   parallel schedule ....... Section 2, PUS: all r from the previous
 *                             iteration's q, then all q
 *   sequential schedule ..... Section 2, SUS steps 1-4: per column, partial
 *                             horizontal pass then partial vertical pass
 *   stopping ................ Section 2: test H x = z after each iteration
 *   Markov prior ............ Eq. (7), the paper's O(q) form of
 *                             Eq. (6), refreshed after each iteration
 *
 * Readings taken where the paper is silent (also listed in the design notes):
 *   - all sums over symbols run over the q field elements 0..q-1;
 *   - r is left unnormalised, as Eq. (3) states it;
 *   - a zero or non-finite normaliser makes the vector uniform and counts a
 *     guard event;
 *   - the clipping decision is the argmax of the double-precision
 *     pseudo-posterior, exact ties going to the smallest symbol;
 *   - the iteration count is the first iteration whose decision satisfies
 *     H x = z (max_iter if none);
 *   - Markov priors: iteration 1 uses the stationary marginal pi; after every
 *     iteration that does not end decoding, all source symbols are refreshed
 *     from that iteration's pseudo-posteriors; chain ends use pi on the left
 *     and a vector of ones on the right; the prior is normalised and
 *     multiplied into the channel evidence;
 *   - the source symbols form a chain in a given order of columns (by
 *     default columns 0..n_info-1), and SUS visits the columns in a given
 *     order (by default 0..n-1);
 *   - in SUS the pseudo-posterior is computed after the sweep from the
 *     r-messages of that sweep;
 *   - SUS variant with the prior assigned during the vertical pass (Section
 *     2, priors paragraph): from iteration 2 on, source symbol k takes, when
 *     its column is visited, the Eq. (7) prior from the newest pseudo-
 *     posteriors of its chain neighbours k-1 and k+1 (of the current sweep
 *     for a neighbour visited earlier in it, else of the previous sweep;
 *     iteration 1 uses pi, as above), and no refresh follows the iteration.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define REF_QMAX 64

typedef struct {
    int p, q;
    unsigned poly;
    int expt[2 * REF_QMAX];
    int logt[REF_QMAX];
} ref_field;

static void field_init(ref_field *F, int p, unsigned poly)
{
    F->p = p;
    F->q = 1 << p;
    F->poly = poly;
    memset(F->logt, 0, sizeof F->logt);
    int v = 1;
    for (int i = 0; i < F->q - 1; ++i) {
        F->expt[i] = v;
        F->expt[i + F->q - 1] = v;
        F->logt[v] = i;
        v <<= 1;                       /* multiply by the primitive element x */
        if (v & F->q) v ^= (int)poly;
    }
}

static inline int fmul(const ref_field *F, int a, int b)
{
    if (a == 0 || b == 0) return 0;
    return F->expt[F->logt[a] + F->logt[b]];
}

static inline int finv(const ref_field *F, int a)
{
    return F->expt[(F->q - 1 - F->logt[a]) % (F->q - 1)];
}

/* ---------------------------------------------------------------- exports */

int ref_gf_mul(int p, unsigned poly, int a, int b)
{
    ref_field F; field_init(&F, p, poly); return fmul(&F, a, b);
}

int ref_gf_inv(int p, unsigned poly, int a)
{
    ref_field F; field_init(&F, p, poly); return a ? finv(&F, a) : -1;
}

/* L[a] = P(received | x = a) for one symbol. channel: 0 BSC (rx, f),
 * 1 BEC (rx, erased-bit mask, unused param), 2 BI-AWGN (y[p], sigma). */
void ref_likelihood(int p, int channel, double param, int rx, int er, const float *y, double *L)
{
    const int q = 1 << p;
    for (int a = 0; a < q; ++a) {
        double v = 1.0;
        for (int b = 0; b < p; ++b) {
            const int ab = (a >> b) & 1;
            if (channel == 0) {
                v *= (ab == ((rx >> b) & 1)) ? (1.0 - param) : param;
            } else if (channel == 1) {
                if ((er >> b) & 1) v *= 0.5;
                else v *= (ab == ((rx >> b) & 1)) ? 1.0 : 0.0;
            } else {
                const double s2 = param * param;
                const double yb = (double)y[b];
                /* P(bit = 0 | y) = 1 / (1 + exp(-2y/s2)),  P(1 | y) = 1 / (1 + exp(2y/s2)) */
                v *= ab ? 1.0 / (1.0 + exp(2.0 * yb / s2)) : 1.0 / (1.0 + exp(-2.0 * yb / s2));
            }
        }
        L[a] = v;
    }
}

/* Channel likelihoods of F frames of n symbols: L[f][j][a]. */
void ref_frame_likelihoods(int p, int channel, int F, int n, const double *param, const uint8_t *rx,
                           const uint8_t *er, const float *y, double *L)
{
    const int q = 1 << p;
    for (int f = 0; f < F; ++f)
        for (int j = 0; j < n; ++j) {
            const size_t fj = (size_t)f * n + j;
            ref_likelihood(p, channel, param[f], rx ? rx[fj] : 0, er ? er[fj] : 0, y ? y + fj * p : NULL,
                           L + fj * q);
        }
}

/* MacKay-Neal syndrome form (Section 2): the decoder is given z = B r, r
 * the received word, so the unknowns are the source symbols and the noise
 * symbols n = r - t.  N[a] = P(noise symbol = a | channel output) for one
 * noise symbol.  BSC (param f): the paper's noise prior f^L (1-f)^(p-L), L the
 * number of ones of a (the BSC flips bits independently of what was sent).
 * BEC (er: erased-bit mask): an unerased bit was received as sent, so its
 * noise bit is 0; an erased bit was read as 0, so its noise bit equals the
 * unknown sent bit, 0 or 1 alike.  BI-AWGN (y[p], sigma): r takes the sign
 * of y, and the noise bit is 0 when the sent bit has that sign, which has
 * probability exp(|y|/s2) / (exp(|y|/s2) + exp(-|y|/s2)) for BPSK +-1 in
 * Gaussian noise of variance s2. */
void ref_noise_evidence(int p, int channel, double param, int er, const float *y, double *N)
{
    const int q = 1 << p;
    for (int a = 0; a < q; ++a) {
        if (channel == 0) {
            int L = 0;
            for (int b = 0; b < p; ++b) L += (a >> b) & 1;
            N[a] = pow(param, L) * pow(1.0 - param, p - L);
        } else if (channel == 1) {
            double v = 1.0;
            for (int b = 0; b < p; ++b) {
                if ((er >> b) & 1) v *= 0.5;
                else if ((a >> b) & 1) v = 0.0;
            }
            N[a] = v;
        } else {
            const double s2 = param * param;
            double v = 1.0;
            for (int b = 0; b < p; ++b) {
                const double u = fabs((double)y[b]) / s2;
                const double same = 1.0 / (1.0 + exp(-2.0 * u));  /* noise bit 0 */
                v *= ((a >> b) & 1) ? 1.0 - same : same;
            }
            N[a] = v;
        }
    }
}

/* Eq. (3) for edge d of a check with dc edges (coefficients h, syndrome z),
 * from the q-messages qin[dc][q]: sum over configurations of the other dc-1
 * symbols such that  h_d a + sum_{d' != d} h_d' x_d' = z.  The sum is taken
 * one sibling at a time: D(y) is the total weight of the siblings handled so
 * far whose weighted sum is y. */
static void check_edge(const ref_field *F, int dc, const uint8_t *h, int z, const double *qin, int d,
                       double *rout)
{
    const int q = F->q;
    double D[REF_QMAX], Dn[REF_QMAX];
    for (int y = 0; y < q; ++y) D[y] = (y == 0) ? 1.0 : 0.0;
    for (int s = 0; s < dc; ++s) {
        if (s == d) continue;
        const double *qs = qin + (size_t)s * q;
        int hx[REF_QMAX];
        for (int x = 0; x < q; ++x) hx[x] = fmul(F, h[s], x);
        for (int y = 0; y < q; ++y) Dn[y] = 0.0;
        for (int y = 0; y < q; ++y)
            for (int x = 0; x < q; ++x) Dn[y ^ hx[x]] += D[y] * qs[x];
        memcpy(D, Dn, sizeof(double) * (size_t)q);
    }
    for (int a = 0; a < q; ++a) rout[a] = D[z ^ fmul(F, h[d], a)];
}

void ref_check_update(int p, unsigned poly, int dc, const uint8_t *h, int z, const double *qin,
                      double *rout)
{
    ref_field F; field_init(&F, p, poly);
    for (int d = 0; d < dc; ++d) check_edge(&F, dc, h, z, qin, d, rout + (size_t)d * F.q);
}

/* normalise v[q] to sum 1; uniform (and a guard event) if that is impossible */
static int normalise(double *v, int q)
{
    double s = 0.0;
    for (int a = 0; a < q; ++a) s += v[a];
    if (!(s > 0.0) || !isfinite(s)) {
        for (int a = 0; a < q; ++a) v[a] = 1.0 / q;
        return 1;
    }
    for (int a = 0; a < q; ++a) v[a] /= s;
    return 0;
}

/* Eq. (7) for source symbol k of a chain of K: P_k(b) is proportional to
 * [sum_a Q_{k-1}(a) M(a,b)] [sum_c M(b,c) Q_{k+1}(c)], with pi in place of the
 * left factor at k = 0 (Qprev NULL) and 1 in place of the right factor at
 * k = K-1 (Qnext NULL). */
static int markov_prior_at(int q, const double *Qprev, const double *Qnext, const double *M, const double *pi,
                           double *Pk)
{
    for (int b = 0; b < q; ++b) {
        double u = 0.0, v = 0.0;
        if (!Qprev) u = pi[b];
        else for (int a = 0; a < q; ++a) u += Qprev[a] * M[a * q + b];
        if (!Qnext) v = 1.0;
        else for (int c = 0; c < q; ++c) v += M[b * q + c] * Qnext[c];
        Pk[b] = u * v;
    }
    return normalise(Pk, q);
}

/* Eq. (7) for every source symbol of a chain, all from the same Q [K][q] */
int ref_markov_prior(int q, int K, const double *Q, const double *M, const double *pi, double *P)
{
    int guards = 0;
    for (int k = 0; k < K; ++k)
        guards += markov_prior_at(q, k > 0 ? Q + (size_t)(k - 1) * q : NULL, k < K - 1 ? Q + (size_t)(k + 1) * q : NULL,
                                  M, pi, P + (size_t)k * q);
    return guards;
}

/* ------------------------------------------------------------------ decode */

typedef struct {
    int p;
    unsigned poly;
    int n, m, n_info;
    const int32_t *row_ptr;   /* [m+1] */
    const int32_t *col;       /* [E] column of each edge; edges numbered row by row */
    const uint8_t *coef;      /* [E] nonzero coefficient of each edge */
    const int32_t *visit;     /* [n] order in which SUS visits the columns, or NULL for 0..n-1 */
    const int32_t *source;    /* [n_info] columns of the source symbols in chain order, or NULL for 0..n_info-1 */
} ref_code;

typedef struct {
    int n_frames;
    int schedule;             /* 0 = PUS (parallel), 1 = SUS (sequential) */
    int max_iter;
    int early_stop;           /* 0: always run max_iter iterations */
    int channel;              /* 0 BSC, 1 BEC, 2 BI-AWGN, 3 given likelihoods */
    int evidence;             /* 0: the channel output of every column is about that column's symbol;
                                 1: MacKay-Neal syndrome form, source columns carry no channel
                                 evidence and every other column is a noise symbol (ref_noise_evidence) */
    const double *param;      /* [F] f, eps or sigma */
    const uint8_t *rx;        /* [F][n] */
    const uint8_t *erasure;   /* [F][n] */
    const float *y;           /* [F][n][p] */
    const double *likelihood; /* [F][n][q] */
    const uint8_t *syndrome;  /* [F][m] or NULL for z = 0 */
    int prior;                /* 0 uniform, 1 Markov, 2 static, over the source symbols */
    const double *markov_M;   /* [q][q] row-stochastic, M[a][b] = P(next b | a) */
    const double *markov_pi;  /* [q] */
    const double *static_P;   /* [q], or [n_info][q] in chain order when static_per_symbol */
    int static_per_symbol;
    int snap_iter;            /* 1-based iteration after which messages are copied out; 0 = none */
    int n_threads;            /* 0 = OpenMP default */
    int prior_in_sweep;       /* SUS with the Markov prior: 0, priors refreshed after each
                                 iteration; 1, assigned during the sweep (see decode_frame) */
} ref_batch;

typedef struct {
    uint8_t *xhat;            /* [F][n] */
    int32_t *iters;           /* [F] */
    uint8_t *converged;       /* [F] */
    double *posterior;        /* [F][n][q] or NULL: final pseudo-posteriors */
    double *snap_q;           /* [F][E][q] or NULL */
    double *snap_r;           /* [F][E][q] or NULL */
    double *snap_Q;           /* [F][n][q] or NULL */
    uint8_t *xhat_trace;      /* [F][max_iter][n] or NULL: decision after each iteration */
    double *gap_trace;        /* [F][max_iter] or NULL: after each iteration, the smallest gap over
                                 the columns between the two largest pseudo-posterior entries */
    int32_t *guards;          /* [F] or NULL */
} ref_result;

typedef struct {
    int *col_ptr;             /* [n+1] */
    int *col_edge;            /* [E] edges of each column, increasing edge id */
    int *edge_row;            /* [E] */
    int *visit;               /* [n] SUS visiting order */
    int *source;              /* [K] source columns in chain order */
    int *chain;               /* [n] chain position of a source column, -1 for the others */
} ref_graph;

static void graph_free(ref_graph *G)
{
    free(G->col_ptr); free(G->col_edge); free(G->edge_row); free(G->visit); free(G->source); free(G->chain);
}

static int graph_build(const ref_code *C, ref_graph *G)
{
    const int n = C->n, m = C->m, E = C->row_ptr[m], K = C->n_info;
    memset(G, 0, sizeof *G);
    G->col_ptr = (int *)calloc((size_t)n + 1, sizeof(int));
    G->col_edge = (int *)malloc(sizeof(int) * (size_t)(E > 0 ? E : 1));
    G->edge_row = (int *)malloc(sizeof(int) * (size_t)(E > 0 ? E : 1));
    G->visit = (int *)malloc(sizeof(int) * (size_t)(n > 0 ? n : 1));
    G->source = (int *)malloc(sizeof(int) * (size_t)(K > 0 ? K : 1));
    G->chain = (int *)malloc(sizeof(int) * (size_t)(n > 0 ? n : 1));
    int *fill = (int *)calloc((size_t)n + 1, sizeof(int));
    if (!G->col_ptr || !G->col_edge || !G->edge_row || !G->visit || !G->source || !G->chain || !fill) {
        free(fill);
        return -1;
    }
    for (int e = 0; e < E; ++e) G->col_ptr[C->col[e] + 1]++;
    for (int j = 0; j < n; ++j) G->col_ptr[j + 1] += G->col_ptr[j];
    for (int i = 0; i < m; ++i)
        for (int e = C->row_ptr[i]; e < C->row_ptr[i + 1]; ++e) {
            G->edge_row[e] = i;
            const int j = C->col[e];
            G->col_edge[G->col_ptr[j] + fill[j]++] = e;
        }
    /* the visiting order and the chain must be permutations / distinct columns */
    memset(fill, 0, sizeof(int) * ((size_t)n + 1));
    for (int t = 0; t < n; ++t) {
        const int j = C->visit ? C->visit[t] : t;
        if (j < 0 || j >= n || fill[j]) { free(fill); return -3; }
        fill[j] = 1;
        G->visit[t] = j;
    }
    for (int j = 0; j < n; ++j) G->chain[j] = -1;
    for (int k = 0; k < K; ++k) {
        const int j = C->source ? C->source[k] : k;
        if (j < 0 || j >= n || G->chain[j] >= 0) { free(fill); return -3; }
        G->source[k] = j;
        G->chain[j] = k;
    }
    free(fill);
    return 0;
}

/* r-message of edge e from the current q-messages of its siblings */
static void update_r(const ref_field *F, const ref_code *C, const ref_graph *G, const uint8_t *z,
                     const double *qm, double *rm, int e, double *scratch_q, uint8_t *scratch_h)
{
    const int q = F->q;
    const int i = G->edge_row[e];
    const int rs = C->row_ptr[i], dc = C->row_ptr[i + 1] - rs;
    for (int s = 0; s < dc; ++s) {
        scratch_h[s] = C->coef[rs + s];
        memcpy(scratch_q + (size_t)s * q, qm + (size_t)(rs + s) * q, sizeof(double) * (size_t)q);
    }
    check_edge(F, dc, scratch_h, z ? z[i] : 0, scratch_q, e - rs, rm + (size_t)e * q);
}

/* q-message of edge e, Eq. (4) */
static int update_q(int q, const ref_graph *G, int j, int e, const double *pj, const double *rm, double *qm)
{
    double *out = qm + (size_t)e * q;
    for (int a = 0; a < q; ++a) {
        double v = pj[(size_t)j * q + a];
        for (int t = G->col_ptr[j]; t < G->col_ptr[j + 1]; ++t) {
            const int e2 = G->col_edge[t];
            if (e2 != e) v *= rm[(size_t)e2 * q + a];
        }
        out[a] = v;
    }
    return normalise(out, q);
}

/* pseudo-posterior of column j, Eq. (5) */
static int posterior(int q, const ref_graph *G, int j, const double *pj, const double *rm, double *Q)
{
    double *out = Q + (size_t)j * q;
    for (int a = 0; a < q; ++a) {
        double v = pj[(size_t)j * q + a];
        for (int t = G->col_ptr[j]; t < G->col_ptr[j + 1]; ++t) v *= rm[(size_t)G->col_edge[t] * q + a];
        out[a] = v;
    }
    return normalise(out, q);
}

/* the decision for one column: the symbol of largest pseudo-posterior, the
 * smallest such symbol when several share the maximum exactly */
static int clip(const double *Qj, int q)
{
    int best = 0;
    for (int a = 1; a < q; ++a)
        if (Qj[a] > Qj[best]) best = a;
    return best;
}

/* gap between the two largest entries of Qj */
static double top_gap(const double *Qj, int q)
{
    double m1 = -1.0, m2 = -1.0;
    for (int a = 0; a < q; ++a) {
        if (Qj[a] > m1) { m2 = m1; m1 = Qj[a]; }
        else if (Qj[a] > m2) m2 = Qj[a];
    }
    return m1 - m2;
}

static int satisfied(const ref_field *F, const ref_code *C, const uint8_t *z, const uint8_t *x)
{
    for (int i = 0; i < C->m; ++i) {
        int s = 0;
        for (int e = C->row_ptr[i]; e < C->row_ptr[i + 1]; ++e) s ^= fmul(F, C->coef[e], x[C->col[e]]);
        if (s != (z ? z[i] : 0)) return 0;
    }
    return 1;
}

/* Eq. (7) prior of chain symbol k from the current pseudo-posteriors of its
 * chain neighbours (columns G->source[k-1], G->source[k+1]) */
static int markov_prior_of(int q, int K, const ref_graph *G, int k, const double *Q, const double *M,
                           const double *pi, double *Pk)
{
    const double *prev = k > 0 ? Q + (size_t)G->source[k - 1] * q : NULL;
    const double *next = k < K - 1 ? Q + (size_t)G->source[k + 1] * q : NULL;
    return markov_prior_at(q, prev, next, M, pi, Pk);
}

/* p_j = norm(L_j * P_k) for the source symbol k at column j */
static int source_prior(int q, const double *Lj, const double *Pk, double *pj)
{
    for (int a = 0; a < q; ++a) pj[a] = Lj[a] * Pk[a];
    return normalise(pj, q);
}

static void decode_frame(const ref_field *F, const ref_code *C, const ref_graph *G, const ref_batch *B,
                         int f, ref_result *R)
{
    const int q = F->q, p = F->p, n = C->n, E = C->row_ptr[C->m], K = C->n_info;
    const int markov = (B->prior == 1) && K > 0;
    const int prior_on = (B->prior == 1 || B->prior == 2) && K > 0;
    const int in_sweep = markov && B->schedule == 1 && B->prior_in_sweep;
    double *L = (double *)malloc(sizeof(double) * (size_t)n * q);
    double *pj = (double *)malloc(sizeof(double) * (size_t)n * q);
    double *Pk = (double *)malloc(sizeof(double) * (size_t)(K > 0 ? K : 1) * q);
    double *qm = (double *)malloc(sizeof(double) * (size_t)(E > 0 ? E : 1) * q);
    double *rm = (double *)calloc((size_t)(E > 0 ? E : 1) * q, sizeof(double));
    double *Q = (double *)malloc(sizeof(double) * (size_t)n * q);
    double *sq = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1) * q);
    uint8_t *sh = (uint8_t *)malloc((size_t)(n > 0 ? n : 1));
    uint8_t *x = (uint8_t *)malloc((size_t)(n > 0 ? n : 1));
    const uint8_t *z = B->syndrome ? B->syndrome + (size_t)f * C->m : NULL;
    int guards = 0;

    /* evidence of every column */
    for (int j = 0; j < n; ++j) {
        double *Lj = L + (size_t)j * q;
        const size_t fj = (size_t)f * n + j;
        if (B->channel == 3) {
            for (int a = 0; a < q; ++a) Lj[a] = B->likelihood[fj * q + a];
        } else if (B->evidence == 1) {
            if (G->chain[j] >= 0) {
                for (int a = 0; a < q; ++a) Lj[a] = 1.0;  /* a source symbol: no channel evidence */
            } else {
                ref_noise_evidence(p, B->channel, B->param[f], B->erasure ? B->erasure[fj] : 0,
                                   B->y ? B->y + fj * p : NULL, Lj);
            }
        } else {
            ref_likelihood(p, B->channel, B->param[f], B->rx ? B->rx[fj] : 0, B->erasure ? B->erasure[fj] : 0,
                           B->y ? B->y + fj * p : NULL, Lj);
        }
    }
    /* the source symbols' priors for iteration 1: pi (Markov) or the static prior */
    if (prior_on)
        for (int k = 0; k < K; ++k) {
            const double *src = B->prior == 1 ? B->markov_pi
                                              : B->static_P + (B->static_per_symbol ? (size_t)k * q : 0);
            memcpy(Pk + (size_t)k * q, src, sizeof(double) * (size_t)q);
        }
    for (int j = 0; j < n; ++j) {
        const int k = G->chain[j];
        if (prior_on && k >= 0) {
            guards += source_prior(q, L + (size_t)j * q, Pk + (size_t)k * q, pj + (size_t)j * q);
        } else {
            memcpy(pj + (size_t)j * q, L + (size_t)j * q, sizeof(double) * (size_t)q);
            guards += normalise(pj + (size_t)j * q, q);
        }
    }
    for (int e = 0; e < E; ++e) memcpy(qm + (size_t)e * q, pj + (size_t)C->col[e] * q, sizeof(double) * (size_t)q);

    int first_ok = 0, last_ok = 0;
    for (int t = 1; t <= B->max_iter; ++t) {
        if (B->schedule == 0) {
            for (int e = 0; e < E; ++e) update_r(F, C, G, z, qm, rm, e, sq, sh);
            for (int j = 0; j < n; ++j)
                for (int s = G->col_ptr[j]; s < G->col_ptr[j + 1]; ++s)
                    guards += update_q(q, G, j, G->col_edge[s], pj, rm, qm);
        } else {
            for (int v = 0; v < n; ++v) {
                const int j = G->visit[v];
                const int k = G->chain[j];
                for (int s = G->col_ptr[j]; s < G->col_ptr[j + 1]; ++s)
                    update_r(F, C, G, z, qm, rm, G->col_edge[s], sq, sh);
                if (in_sweep && k >= 0 && t >= 2) {
                    /* the prior of source symbol k, assigned at its vertical
                     * pass from the newest pseudo-posteriors of its chain
                     * neighbours (of this sweep if visited already, else of
                     * the last) */
                    guards += markov_prior_of(q, K, G, k, Q, B->markov_M, B->markov_pi, Pk + (size_t)k * q);
                    guards += source_prior(q, L + (size_t)j * q, Pk + (size_t)k * q, pj + (size_t)j * q);
                }
                for (int s = G->col_ptr[j]; s < G->col_ptr[j + 1]; ++s)
                    guards += update_q(q, G, j, G->col_edge[s], pj, rm, qm);
                if (in_sweep && k >= 0) {
                    /* Q_j now, for its chain neighbours' priors (the same value
                     * the pass after the sweep computes: neither p_j nor the r
                     * of column j change later in the sweep) */
                    (void)posterior(q, G, j, pj, rm, Q);
                }
            }
        }
        double gap = 2.0;
        for (int j = 0; j < n; ++j) {
            guards += posterior(q, G, j, pj, rm, Q);
            x[j] = (uint8_t)clip(Q + (size_t)j * q, q);
            if (R->gap_trace) {
                const double g = top_gap(Q + (size_t)j * q, q);
                gap = g < gap ? g : gap;
            }
        }
        if (R->xhat_trace) memcpy(R->xhat_trace + ((size_t)f * B->max_iter + (t - 1)) * n, x, (size_t)n);
        if (R->gap_trace) R->gap_trace[(size_t)f * B->max_iter + (t - 1)] = gap;
        if (t == B->snap_iter) {
            if (R->snap_q) memcpy(R->snap_q + (size_t)f * E * q, qm, sizeof(double) * (size_t)E * q);
            if (R->snap_r) memcpy(R->snap_r + (size_t)f * E * q, rm, sizeof(double) * (size_t)E * q);
            if (R->snap_Q) memcpy(R->snap_Q + (size_t)f * n * q, Q, sizeof(double) * (size_t)n * q);
        }
        last_ok = satisfied(F, C, z, x);
        if (last_ok && !first_ok) first_ok = t;
        if (last_ok && B->early_stop) break;
        if (t == B->max_iter) break;
        if (markov && !in_sweep) {
            /* Eq. (7) for every source symbol from this iteration's Q */
            for (int k = 0; k < K; ++k)
                guards += markov_prior_of(q, K, G, k, Q, B->markov_M, B->markov_pi, Pk + (size_t)k * q);
            for (int k = 0; k < K; ++k) {
                const int j = G->source[k];
                guards += source_prior(q, L + (size_t)j * q, Pk + (size_t)k * q, pj + (size_t)j * q);
            }
        }
    }
    memcpy(R->xhat + (size_t)f * n, x, (size_t)n);
    R->iters[f] = first_ok ? first_ok : B->max_iter;
    R->converged[f] = (uint8_t)(first_ok != 0);
    if (R->posterior) memcpy(R->posterior + (size_t)f * n * q, Q, sizeof(double) * (size_t)n * q);
    if (R->guards) R->guards[f] = guards;
    free(L); free(pj); free(Pk); free(qm); free(rm); free(Q); free(sq); free(sh); free(x);
}

int ref_decode(const ref_code *C, const ref_batch *B, ref_result *R)
{
    if (C->p < 1 || C->p > 6 || B->n_frames < 0 || B->max_iter < 1) return -1;
    if (B->prior < 0 || B->prior > 2 || (B->prior == 1 && (!B->markov_M || !B->markov_pi)) ||
        (B->prior == 2 && !B->static_P))
        return -1;
    if (B->evidence == 1 && B->channel == 3) return -1;
    ref_field F;
    field_init(&F, C->p, C->poly);
    ref_graph G;
    const int gs = graph_build(C, &G);
    if (gs) { graph_free(&G); return gs == -3 ? -3 : -2; }
#ifdef _OPENMP
    if (B->n_threads > 0) omp_set_num_threads(B->n_threads);
#pragma omp parallel for schedule(dynamic, 1)
#endif
    for (int f = 0; f < B->n_frames; ++f) decode_frame(&F, C, &G, B, f, R);
    graph_free(&G);
    return 0;
}

int ref_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
