/*
 * gfbp — belief-propagation decoding of LDPC codes over GF(q = 2^p) on
 * AMD Instinct MI355X (gfx950).
 *
 * Method: Yacov, Efraim, Kfir, Kanter, Shental, "Parallel vs. Sequential
 * Belief Propagation Decoding of LDPC Codes over GF(q) and Markov Sources",
 * Section 2.  The decoder solves H x = z for x over GF(q) given per-symbol
 * channel evidence and priors, by the message passing of Eqs. (3)
 * (check-to-variable r), (4) (variable-to-check q) and (5)
 * (pseudo-posterior Q, clipped to a decision), under either
 *   - the parallel updating scheme (PUS): all r from the previous
 *     iteration's q, then all q; or
 *   - the sequential updating scheme (SUS): for each column j in order, the
 *     r of column j's edges from the current q, then column j's q.
 * After each iteration the decision is tested against H x = z.  With a Markov
 * source, the priors of the information symbols are re-estimated after every
 * iteration by the dynamical block prior of Eq. (7) (or, for SUS on request,
 * during the sweep: GFBP_OPT_PRIOR_IN_SWEEP).
 *
 * Conventions shared by every call:
 *   - GF(2^p) in the polynomial basis of a primitive polynomial (bit b of a
 *     symbol is the coefficient of x^b and is the b-th transmitted bit);
 *   - BPSK maps bit 0 to +1 and bit 1 to -1;
 *   - all sums over symbols run over the q field elements 0..q-1;
 *   - messages are stored as IEEE binary32 probabilities; transforms,
 *     products and normalisations are computed in binary64; symbols and
 *     syndromes are bytes.
 *
 * Errors: every call returns a gfbp_status; 0 is success, negative values are
 * errors, and gfbp_last_error() returns a message for the calling thread's
 * last failure.  No C++ exception crosses this interface.
 *
 * Threads and streams: decodes only read a code handle, so one handle may be
 * shared by concurrent decode calls on different streams, each with its own
 * workspace; gfbp_code_set_shape and gfbp_tune change the handle and must not
 * run concurrently with decodes on it.  A session is used by one thread at a
 * time.
 */
#ifndef GFBP_H
#define GFBP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t gfbp_status;
#define GFBP_OK 0
#define GFBP_EINVAL (-1)       /* bad argument (null pointer, bad size, bad enum) */
#define GFBP_EUNSUPPORTED (-2) /* q not 2^p with 1 <= p <= 6, or a degree beyond the kernels' limits */
#define GFBP_ENOMEM (-3)       /* device or host allocation failed (code build only) */
#define GFBP_EHIP (-4)         /* a HIP runtime call failed */
#define GFBP_ESMALL (-5)       /* workspace smaller than gfbp_workspace_size() */

/* schedules (Section 2) */
#define GFBP_PUS 0
#define GFBP_SUS 1

/* channels */
#define GFBP_CH_BSC 0        /* rx: received hard symbols; param: crossover f      */
#define GFBP_CH_BEC 1        /* rx + erasure: erased-bit masks; param unused      */
#define GFBP_CH_BIAWGN 2     /* y: p samples per symbol; param: noise std sigma   */
#define GFBP_CH_LIKELIHOOD 3 /* likelihood: P(received | x = a) for every a       */

/* priors of the source symbols (Section 2: a source symbol's prior multiplies
 * its channel evidence; the chain of source symbols is gfbp_code_desc's
 * source_cols) */
#define GFBP_PRIOR_UNIFORM 0 /* i.i.d. uniform source: prior 1/q                            */
#define GFBP_PRIOR_MARKOV 1  /* first-order Markov source: pi at iteration 1, then the
                                dynamical block prior of Eq. (7) after every iteration   */
#define GFBP_PRIOR_STATIC 2  /* a fixed prior: one vector for every source symbol, or one
                                per source symbol (gfbp_batch.static_prior)              */

/* What the channel output of a column is evidence about. */
#define GFBP_EVIDENCE_SYMBOL 0 /* the symbol x_j itself (codeword sent over the channel)   */
#define GFBP_EVIDENCE_MN 1     /* MacKay-Neal syndrome form (Section 2, Eqs. (1)-(2)): H = [A B],
                                  x = (source s, noise n), z = B r for the received word r.
                                  Source columns carry no channel evidence; every other
                                  column j is a noise symbol, with evidence
                                  P(n_j = a | channel output at j):
                                    BSC: f^w (1-f)^(p-w), w the number of ones of a (the
                                         paper's noise prior; rx is not read);
                                    BEC: 2^-e over the a with no one at an unerased bit
                                         (erased bits were read as 0), else 0;
                                    BI-AWGN: per bit, noise 0 with probability
                                         1 / (1 + exp(-2|y|/sigma^2)) (the received bit is
                                         the sign of y).
                                  GFBP_CH_LIKELIHOOD is refused with this mode.          */

/* Limits of the decoding kernels. */
#define GFBP_MAX_Q 64
#define GFBP_MAX_ROW_DEGREE 16
#define GFBP_MAX_COL_DEGREE 8

typedef struct gfbp_code gfbp_code; /* opaque, device-resident Tanner graph */

/* A parity-check matrix H (m x n) over GF(q) in compressed-row form.  All
 * pointers are host memory, read during gfbp_code_build only (the library
 * copies them).  Edges (nonzeros) are numbered row by row in the given
 * order; that numbering is the "edge index" used by message snapshots. */
typedef struct {
    int32_t q;               /* field size 2^p, 2 <= q <= 64                        */
    int32_t poly;            /* primitive polynomial incl. x^p (e.g. 0x13 for q=16); 0 = default */
    int32_t n;               /* columns (code symbols)                                */
    int32_t m;               /* rows (checks)                                        */
    int32_t n_info;          /* number of source symbols (see source_cols)           */
    const int32_t *row_ptr;  /* [m+1], row_ptr[0] = 0, nondecreasing                */
    const int32_t *col;      /* [E] column of each edge, 0 <= col < n, no repeats in a row */
    const uint8_t *coef;     /* [E] nonzero field element of each edge, < q          */
    const int32_t *visit_order; /* [n] the order in which SUS visits the columns (Section 2,
                                   SUS steps: column by column), a permutation of 0..n-1;
                                   NULL = 0..n-1                                          */
    const int32_t *source_cols; /* [n_info] the columns of the source symbols in chain order
                                   (the Markov chain of Eq. (7) runs over them), distinct;
                                   NULL = 0..n_info-1                                     */
} gfbp_code_desc;

typedef struct {
    int32_t q, p, n, m, n_info, n_edges;
    int32_t max_row_degree, max_col_degree;
    int32_t poly;
    int32_t sus_levels;      /* dependency levels of one SUS sweep (see GFBP_OPT_SUS_STRICT) */
    int32_t sus_levels_in_sweep; /* the same when source symbol k also waits for k-1
                                    (GFBP_OPT_PRIOR_IN_SWEEP): at least n_info */
} gfbp_code_info;

/* Build the device-resident Tanner graph of the parity-check matrix H of
 * Section 2 (Eq. (2): H x = z) on the current HIP device, with its SUS
 * dependency levels.  Rejects: null pointers, q not a power of two in
 * [2, 64], a polynomial that is not primitive of degree p, column/coefficient
 * out of range, a column repeated in a row, row degree > GFBP_MAX_ROW_DEGREE,
 * column degree > GFBP_MAX_COL_DEGREE, a visit_order that is not a
 * permutation, source_cols out of range or repeated.  Synchronous.  The
 * library copies every input; the handle owns its device memory and is freed
 * by gfbp_code_free. */
gfbp_status gfbp_code_build(const gfbp_code_desc *desc, gfbp_code **out);
gfbp_status gfbp_code_free(gfbp_code *code);
gfbp_status gfbp_code_info_get(const gfbp_code *code, gfbp_code_info *out);

/* One batch of frames.  All pointers are device memory owned by the caller
 * and only read, except code_index (host memory, read during the call).
 * Frames of one code: arrays are frame-major with the code's sizes ([F][n],
 * [F][m], ...).  Frames of several codes (n_codes > 1): each frame's entries
 * follow the previous frame's ("ragged"), with the sizes of the frame's own
 * code: frame f's rx and erasure start at the sum over earlier frames g of
 * n(g), its y at the sum of n(g) p(g), its likelihoods at the sum of n(g) q(g),
 * its syndrome at the sum of m(g), its decisions (xhat) at the sum of n(g);
 * per-frame scalars (param, channel_of) are [F]. */
typedef struct {
    int32_t n_frames;        /* F >= 0                                                */
    int32_t schedule;        /* GFBP_PUS or GFBP_SUS                                  */
    int32_t max_iter;        /* >= 1                                                  */
    int32_t early_stop;      /* 1: a frame stops at the first iteration with H x = z;
                                0: every frame runs max_iter iterations              */
    int32_t channel;         /* GFBP_CH_* of every frame (unless channel_of)          */
    const float *param;      /* [F] crossover f (BSC) or sigma (BI-AWGN); may be NULL when
                                no frame is BSC or BI-AWGN                            */
    const uint8_t *rx;       /* received symbols (BSC, BEC; erased bits 0)            */
    const uint8_t *erasure;  /* erased-bit masks (BEC)                                */
    const float *y;          /* p channel outputs per symbol (BI-AWGN)                */
    const float *likelihood; /* q values P(received | a) per symbol (LIKELIHOOD), need not
                                be normalised                                         */
    const uint8_t *syndrome; /* z, or NULL for z = 0                                  */
    int32_t prior;           /* GFBP_PRIOR_*                                          */
    const float *markov_M;   /* [q][q] M[a][b] = P(next = b | current = a) (MARKOV)   */
    const float *markov_pi;  /* [q] distribution of the first source symbol (MARKOV)  */
    int32_t options;         /* bit set of GFBP_OPT_*                                 */
    const uint8_t *truth;    /* [F][n] true symbols, for gfbp_result.trace, or NULL   */
    int32_t evidence;        /* GFBP_EVIDENCE_*                                       */
    const uint8_t *channel_of; /* [F] channel kind of each frame (GFBP_CH_*), or NULL: every
                                frame is `channel`.  Read back to the host to check that the
                                inputs each kind needs are given.                     */
    const float *static_prior; /* STATIC: [q], or [n_info][q] in chain order           */
    int32_t static_per_symbol; /* STATIC: 1 if static_prior holds one vector per source symbol */
    int32_t n_codes;         /* entries of codes[] (0 is taken as 1)                  */
    const int32_t *code_index; /* HOST [F] code of each frame (index into codes[]), or NULL:
                                every frame is on codes[0]                            */
    int32_t persist_el;      /* persistent path: entries per lane (2, 4 or 8), 0 = 4; per
                                field taken down to max(2, q/4) (a tile then holds at
                                most 16 frames), to 4 outside the narrow degree class
                                (rows <= 6, columns <= 4) and to q                    */
    int32_t persist_waves;   /* persistent path: wavefronts per workgroup (1..8), 0 = 8 */
} gfbp_batch;

/* SUS runs, by default, in dependency levels: two columns that share no check
 * commute, so columns are grouped into levels (a column's level is one more
 * than the highest level of the earlier columns it shares a check with) and
 * the columns of one level are updated concurrently.  Every column still sees
 * exactly the messages it would see in the strict column order, and its
 * arithmetic is the same, so results are bitwise identical to the strict
 * sweep.  This option runs the strict sweep instead (one column after the
 * other within each frame). */
#define GFBP_OPT_SUS_STRICT 1

/* Frames are processed in tiles of up to 64 frames that share every kernel
 * launch, and a tile keeps running while any of its frames does.  When, after
 * an iteration, the running frames fill less than 31/32 of the running tiles,
 * the decoder by default moves running frames (their messages, likelihoods,
 * priors and counters) into the slots of finished frames so that the running
 * frames form whole tiles again; each frame's arithmetic, and so every output,
 * is unchanged (results are written per frame when it finishes).  Not done
 * when posteriors, snapshots or a trace are requested.  This option turns it
 * off. */
#define GFBP_OPT_NO_COMPACT 2

/* Sessions: gfbp_session_step with an even number of iterations on a created
 * (non-default) stream replays a HIP graph of those iterations, captured on
 * first use and kept by the session for each (iterations, launch bound)
 * pair, the launch bound being the smallest power of two of tiles covering
 * the running frames.  The work and the results are those of the eager step;
 * only the host's launch cost changes.  The graphs are freed with the
 * session. */
#define GFBP_OPT_STEP_GRAPHS 4

/* Decode through the persistent work-list kernel (the no-allocation entry
 * takes it for every batch over several codes): one launch per kernel shape
 * class, sized to fill the
 * GPU, in which each workgroup takes the next tile of frames of one code from
 * a device-side list (largest codes first), decodes it through every
 * iteration to convergence or max_iter (initialisation, the schedule's
 * sweeps with a workgroup barrier between dependent steps, the H x = z test,
 * retirement and Markov refreshes all inside the kernel) and writes its
 * results, then takes the next tile.  No host work between iterations.  One
 * launch serves every field; codes beyond the small degree class (rows of
 * more than 6 or columns of more than 4 entries) take a second launch after
 * the first.  Outputs equal those of the plain decode bitwise.  Not with
 * posteriors, snapshots, traces or GFBP_OPT_PRIOR_IN_SWEEP
 * (GFBP_EUNSUPPORTED). */
#define GFBP_OPT_PERSISTENT 16

/* Batch decode of one code: decode through the tiled kernels even where the
 * frames' state fits in LDS.  By default a one-code batch over GF(2), GF(4)
 * or GF(8) whose frame state (messages, evidence, priors, decisions:
 * 4 q (E (1 + PUS) + n + K (prior) + K (Markov)) + n + m bytes) fits in the
 * LDS of a workgroup is decoded in one launch with each workgroup holding up
 * to four frames in LDS through every iteration (Section 2's schedules, the
 * H x = z test, retirement and Markov refreshes inside the kernel; HBM only
 * for the initial state and the results), unless posteriors, snapshots,
 * traces, GFBP_OPT_SUS_STRICT or GFBP_OPT_PRIOR_IN_SWEEP are asked for.  Its
 * outputs equal bitwise those of the tiled decode at q entries per lane (PUS)
 * or two entries per lane (SUS). */
#define GFBP_OPT_NO_ONCHIP 32

/* Batch decode, SUS with the Markov prior: the prior of each source symbol is
 * assigned during the sweep, at its column's vertical pass (Section 2, the
 * paragraph on priors), instead of after each iteration.  From iteration 2 on,
 * source symbol k takes the Eq. (7) prior from the pseudo-posterior of symbol
 * k-1 computed earlier in the same sweep and that of symbol k+1 from the
 * previous sweep; iteration 1 uses pi as usual.  Symbol k then depends on
 * symbol k-1 within a sweep, so the sweep has at least n_info dependency
 * levels (gfbp_code_info.sus_levels_in_sweep).  GFBP_EINVAL with PUS; no
 * effect with the uniform prior; sessions return GFBP_EUNSUPPORTED. */
#define GFBP_OPT_PRIOR_IN_SWEEP 8

/* Outputs, device memory owned by the caller. */
typedef struct {
    uint8_t *xhat;           /* [F][n] (ragged for several codes) decision after the frame's
                                last iteration                                        */
    int32_t *iters;          /* [F] first iteration with H x = z, else max_iter       */
    uint8_t *converged;      /* [F] 1 if some iteration satisfied H x = z             */
    float *posterior;        /* [F][n][q] final pseudo-posteriors, or NULL            */
    int32_t *guards;         /* [F] count of zero/non-finite normalisers met, or NULL */
    int32_t snap_iter;       /* 1-based iteration after which messages are copied; 0 = none */
    float *snap_q;           /* [F][E][q] q-messages (probability domain), or NULL   */
    float *snap_r;           /* [F][E][q] r-messages, or NULL                         */
    float *snap_Q;           /* [F][n][q] pseudo-posteriors, or NULL                  */
    int32_t *trace;          /* [F][max_iter] or NULL (needs batch->truth): after each
                                iteration t the frame ran, entry t-1 counts the bits of
                                its source symbols (columns 0..n_info-1; all columns when
                                n_info = 0) whose decision equals the truth; entries after
                                its last iteration are 0 (the Fig. 1 diagnostic)        */
} gfbp_result;

/* Bytes of device workspace gfbp_decode_batch needs for F frames of one code
 * decoded by the plain kernels. */
size_t gfbp_workspace_size(const gfbp_code *code, int32_t n_frames, int32_t schedule, int32_t prior);
/* Bytes of device workspace gfbp_decode_batch needs for this batch (any
 * number of codes, any options); 0 on a bad argument. */
size_t gfbp_batch_workspace_size(const gfbp_code *const *codes, const gfbp_batch *batch);

/* Decode a batch: solve H x = z for every frame by belief propagation
 * (Section 2: Eq. (3) check-to-variable messages, Eq. (4) variable-to-check
 * messages, Eq. (5) pseudo-posteriors clipped to the decision, the stopping
 * test H x = z after each iteration) under the parallel (PUS) or sequential
 * (SUS) schedule, with the Eq. (7) Markov prior or a static prior on the
 * source symbols when asked.  codes[0..n_codes): the codes the frames are on
 * (batch->code_index); with one code the plain kernels run (several launches
 * per iteration over the frames still iterating).  With several codes,
 * unless GFBP_OPT_PERSISTENT is set, each code's frames are gathered from the
 * ragged inputs into contiguous buffers in the workspace, decoded with the
 * plain kernels as a one-code batch (the code's kernel shape) and their
 * results scattered back, the codes running concurrently on the library's
 * four worker threads (created on the first such call and kept for the
 * process), each with a stream of its own; the results equal, bitwise, each
 * code's frames decoded alone.  With GFBP_OPT_PERSISTENT the persistent
 * kernel runs.  workspace: device memory of at least
 * gfbp_batch_workspace_size() bytes, 256-byte aligned, owned by the caller,
 * clobbered.  stream: a hipStream_t (NULL = default stream).  All work is
 * enqueued on the stream (several codes: the caller's stream is synchronised
 * first, then the workers' streams run the codes); the call returns after the
 * frames have finished, with the results complete in the output buffers.  No
 * device memory is allocated; a thread's first plain decode allocates 64
 * bytes of pinned host memory and four events, kept for the life of the
 * thread.  Errors: EINVAL
 * for a null or inconsistent argument (a missing input a frame's channel
 * needs, a code index out of range, LIKELIHOOD with the MN evidence mode),
 * ESMALL for a small workspace, EUNSUPPORTED for options the path lacks,
 * EHIP when a HIP call fails. */
gfbp_status gfbp_decode_batch(const gfbp_code *const *codes, const gfbp_batch *batch, gfbp_result *out,
                              void *workspace, size_t ws_bytes, void *stream);

/* For callers that cannot allocate (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc): gfbp_decode_batch with the
 * library's own static device scratch as its workspace instead of a caller's.
 * The scratch is one array of 256 MiB per GPU the library runs on, held until
 * the process ends; a batch whose gfbp_batch_workspace_size() exceeds it is
 * refused with GFBP_ESMALL (and a message giving both sizes).  The call makes
 * no device, pinned-host, event or stream allocation: the first call on a
 * device looks up the scratch's address there (hipGetSymbolAddress, not an
 * allocation); the plain path reads its iteration counts back through
 * thread-local host memory after a stream synchronisation; the persistent path
 * runs its kernels one after the other on `stream` (no forked streams, no
 * graph); tracing is off for the call; the batch plan itself lives in host
 * heap memory.  Results equal gfbp_decode_batch's.  Every call on a GPU uses
 * the same scratch, which keeps the last call's contents (each decode
 * initialises what it reads): calls that overlap on one GPU (other threads,
 * other streams) race and must not be made. */
gfbp_status gfbp_decode_batch_noalloc(const gfbp_code *const *codes, const gfbp_batch *batch, gfbp_result *out,
                                      void *stream);

/* ---- Sessions: continuous batching with resident frame state. ----
 * A session holds n_slots frame slots of one code on the device (message
 * state, staged channel inputs, per-slot iteration counters).  Frames are
 * admitted into free slots as they arrive; every step advances each running
 * slot by a number of iterations of the session's schedule; a slot whose
 * decision satisfies H x = z, or that reaches max_iter, finishes; poll hands
 * back finished frames (decision, iterations, converged) and frees their
 * slots.  A frame's arithmetic does not depend on the other frames, so its
 * result is the same alone or in any mix (and equal to gfbp_decode_batch).
 * Channel kind and prior are per frame.  The kernel shape is the code's shape
 * for the schedule when the session is created.  Calls on one session must
 * not overlap; different sessions may run on different streams. */
typedef struct gfbp_session gfbp_session;

typedef struct {
    int32_t n_slots;         /* resident frames (rounded up to a multiple of 64); 0: as many
                                as device_bytes allows (GFBP_ENOMEM if not even 64)        */
    int32_t schedule;        /* GFBP_PUS or GFBP_SUS                                      */
    int32_t max_iter;        /* >= 1                                                      */
    int32_t has_syndrome;    /* 1: frames may carry z (else z = 0)                        */
    const float *markov_M;   /* host [q][q], or NULL: no frame uses a Markov prior        */
    const float *markov_pi;  /* host [q] (with markov_M)                                  */
    int32_t options;         /* GFBP_OPT_SUS_STRICT, GFBP_OPT_STEP_GRAPHS (PRIOR_IN_SWEEP:
                                GFBP_EUNSUPPORTED)                                        */
    int64_t device_bytes;    /* with n_slots = 0: the session's device-memory budget       */
} gfbp_session_desc;

/* n frames to admit: device pointers, frame-major, read during the call. */
typedef struct {
    const uint8_t *channel;  /* [n] GFBP_CH_BSC, GFBP_CH_BEC or GFBP_CH_BIAWGN (required) */
    const uint8_t *markov;   /* [n] 1: Markov prior on the source symbols, or NULL        */
    const float *param;      /* [n] crossover f or sigma (unused for BEC)                  */
    const uint8_t *rx;       /* [n][code n] received symbols, or NULL if no BSC/BEC frame  */
    const uint8_t *erasure;  /* [n][code n] erased-bit masks, or NULL if no BEC frame      */
    const float *y;          /* [n][code n][p] samples, or NULL if no BI-AWGN frame        */
    const uint8_t *syndrome; /* [n][m], or NULL (z = 0)                                    */
} gfbp_frames;

typedef struct {
    int64_t id;              /* the caller's id of the frame                               */
    int32_t iters;           /* iterations run                                             */
    int32_t converged;       /* 1 if the decision satisfies H x = z                        */
    uint64_t t_admit;        /* device clock when the frame's state was initialised        */
    uint64_t t_retire;       /* device clock when the frame finished (retirement kernel)   */
} gfbp_retired;

/* Rate of the device clock of gfbp_retired's timestamps, in ticks per second
 * (the current device's constant-rate wall clock); 0 on failure. */
uint64_t gfbp_device_clock_hz(void);

/* Device bytes a session would allocate (for admission by memory budget;
 * with n_slots = 0, for the slots device_bytes allows). */
size_t gfbp_session_bytes(const gfbp_code *code, const gfbp_session_desc *desc);
/* Allocates the session's device memory (synchronous). */
gfbp_status gfbp_session_create(const gfbp_code *code, const gfbp_session_desc *desc, gfbp_session **out);
gfbp_status gfbp_session_destroy(gfbp_session *session);
/* Admits the first *n_admitted of the n frames (as many as there are free
 * slots; the caller offers the rest later) and initialises them on stream. */
gfbp_status gfbp_session_admit(gfbp_session *session, int32_t n, const int64_t *ids, const gfbp_frames *frames,
                               int32_t *n_admitted, void *stream);
/* Enqueues `iters` iterations of every running slot; no host synchronisation
 * (with GFBP_OPT_STEP_GRAPHS, an even `iters` on a non-null stream replays a
 * captured graph; the first use of a key captures and instantiates it). */
gfbp_status gfbp_session_step(gfbp_session *session, int32_t iters, void *stream);
/* Collects up to cap finished frames: out[0..*n_out) and, if xhat (host) is
 * not NULL, their decisions xhat[r][code n]; frees their slots.  Synchronises
 * the stream. */
gfbp_status gfbp_session_poll(gfbp_session *session, gfbp_retired *out, uint8_t *xhat, int32_t cap, int32_t *n_out,
                              void *stream);
int32_t gfbp_session_free_slots(const gfbp_session *session);
/* Frames admitted and not yet collected by poll. */
int32_t gfbp_session_running(const gfbp_session *session);

/* ---- Batches of sessions as one HIP graph. ----
 * gfbp_graph_capture records `iters` iterations (even, >= 2) of every session
 * in sessions[0..n) -- possibly of different codes, fields and schedules --
 * into one HIP graph, with launch grids covering every slot, so that the graph
 * stays valid while frames finish and while new frames are admitted between
 * launches.  gfbp_graph_launch replays it on a stream (no host
 * synchronisation); gfbp_session_poll collects finished frames as usual.
 * stream must be a created stream (not the default stream).  The sessions
 * must outlive the graph; do not call gfbp_session_step on them between
 * capture and destroy. */
typedef struct gfbp_graph gfbp_graph;
gfbp_status gfbp_graph_capture(gfbp_session *const *sessions, int32_t n, int32_t iters, void *stream,
                               gfbp_graph **out);
gfbp_status gfbp_graph_launch(gfbp_graph *graph, void *stream);
gfbp_status gfbp_graph_destroy(gfbp_graph *graph);

/* ---- Kernel shape and its autotuner. ----
 * The decoding kernels spread one frame's q-vector over G lanes with
 * q/G "entries per lane" in registers (EL): a larger EL makes more of the
 * Walsh-Hadamard butterflies register arithmetic, a smaller EL uses fewer
 * registers (more wavefronts per compute unit).  EL in {2, 4, 8} (at most q;
 * at most 4 for codes with rows longer than 6 or columns longer than 4).
 * gfbp_code_set_shape fixes EL for one schedule (0 = default: 4, or 2 when
 * q = 2); gfbp_code_get_shape returns the EL in use.  gfbp_tune times
 * trial_iters fixed iterations of `batch` (same buffers and workspace as a
 * decode; outputs are overwritten) with every allowed EL (one warm-up run
 * each, then three rounds over them, each keeping its fastest run) and keeps
 * the fastest for batch->schedule, returned in *chosen.  These calls change the
 * code handle: do not run them concurrently with decodes on the same code. */
gfbp_status gfbp_code_set_shape(gfbp_code *code, int32_t schedule, int32_t entries_per_lane);
int32_t gfbp_code_get_shape(const gfbp_code *code, int32_t schedule);
gfbp_status gfbp_tune(gfbp_code *code, const gfbp_batch *batch, gfbp_result *out, void *workspace, size_t ws_bytes,
                      void *stream, int32_t trial_iters, int32_t *chosen);
/* The persistent path's tile shape: times trial_iters fixed iterations of the
 * batch (any codes; outputs overwritten) with entries per lane 4 and 8
 * (frames per tile 64 x EL / q) and 4 and 8 wavefronts per workgroup (one
 * warm-up run each, then three rounds keeping each shape's fastest run),
 * skipping shapes whose workspace exceeds ws_bytes, and returns the fastest in
 * *el and *waves for batch->persist_el / persist_waves.  Changes no handle. */
gfbp_status gfbp_tune_persistent(const gfbp_code *const *codes, const gfbp_batch *batch, gfbp_result *out,
                                 void *workspace, size_t ws_bytes, void *stream, int32_t trial_iters, int32_t *el,
                                 int32_t *waves);

/* ---- Tracing: per-kernel timing with HIP events on the decode stream. ----
 * Off by default.  When on, every kernel launch of gfbp_decode_batch is
 * bracketed by two HIP events on the caller's stream; after the decode's final
 * synchronisation the elapsed times are added to process-wide totals per
 * kernel kind ("init", "check", "variable", "sequential", "sus_level",
 * "sus_run" (runs of thin SUS levels), "syndrome", "retire", "markov", "output",
 * "compact"), together with the launch's algorithmic HBM bytes
 * (float32 messages read and written once, as the method defines them; frames
 * that have stopped iterating are not counted) and its edge-q updates (E*q per
 * running frame for one iteration). */
typedef struct {
    char name[32];
    int64_t launches;
    double total_ms;      /* sum of event-measured launch durations */
    double algo_bytes;    /* sum of algorithmic bytes of those launches */
    double edge_q;        /* sum of edge-q updates of those launches */
} gfbp_kernel_stats;

gfbp_status gfbp_profile_enable(int32_t on);
gfbp_status gfbp_profile_reset(void);
/* Copies up to cap entries (kinds with at least one launch) and returns how
 * many kinds have data. */
int32_t gfbp_profile_read(gfbp_kernel_stats *out, int32_t cap);

/* Measurement: the HBM bandwidth a plain streaming kernel reaches on this
 * device, to state beside the nominal peak.  Copies `bytes` (> 0, a multiple
 * of 16) from src to dst (device pointers, 16-byte aligned, not overlapping)
 * `reps` times (>= 1) on `stream` (a hipStream_t, null for the default
 * stream) with 16-byte non-temporal loads and stores, four in flight per
 * lane, and writes the best read + write rate in bytes per second to *rate.
 * Synchronises the stream; GFBP_EINVAL for bad arguments. */
gfbp_status gfbp_stream_copy_rate(void *dst, const void *src, size_t bytes, int32_t reps, void *stream, double *rate);

/* Thread-local description of the last error on this thread ("" if none). */
const char *gfbp_last_error(void);

/* Library version string. */
const char *gfbp_version(void);

#ifdef __cplusplus
}
#endif
#endif /* GFBP_H */
