// GF(2^p) LDPC belief-propagation decoder for gfx950: kernels and C ABI.
//
// Paper: Yacov, Efraim, Kfir, Kanter, Shental, "Parallel vs. Sequential Belief
// Propagation Decoding of LDPC Codes over GF(q) and Markov Sources", Section 2.
// The public contract is include/gfbp.h.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <algorithm>
#include <chrono>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "../../include/gfbp.h"
#include "gfbp_kernels.h"
#include "gfbp_tiled.h"

using namespace gfbp;

namespace {

thread_local std::string g_err;

gfbp_status fail(gfbp_status s, const std::string &msg) {
    g_err = msg;
    return s;
}

#define HIP_TRY(expr)                                                                       \
    do {                                                                                    \
        hipError_t e_ = (expr);                                                             \
        if (e_ != hipSuccess)                                                               \
            return fail(GFBP_EHIP, std::string(#expr) + ": " + hipGetErrorString(e_));      \
    } while (0)

inline size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

}  // namespace

struct gfbp_code {
    gfbp_code_info info;
    DevCode dev;
    double sum_dc2;       // sum over checks of d_c (d_c - 1): sibling vectors read by one SUS sweep
    // SUS dependency levels: columns level_ptr[l]..level_ptr[l+1]-1 of level_cols
    std::vector<int32_t> level_ptr;
    std::vector<double> level_sibs;   // per level: sibling vectors read (sum over its edges of d_c - 1)
    std::vector<double> level_edges;  // per level: edges
    const int32_t *level_cols = nullptr;  // device [n]
    int el[2] = {0, 0};   // entries per lane chosen for PUS / SUS (0 = default)
    void *mem = nullptr;  // one device allocation holding every array of dev
};

// ======================================================================= tracing
// Optional per-kernel timing with HIP events recorded on the decode stream
// around each launch, with the algorithmic bytes and edge-q updates of the
// launch attached.  Read back after the decode's final synchronisation.
namespace {

enum Kind { K_INIT, K_CHECK, K_VARIABLE, K_SEQUENTIAL, K_SUS_LEVEL, K_SYNDROME, K_RETIRE, K_MARKOV, K_OUTPUT, K_COUNT };
const char *kKindName[K_COUNT] = {"init",     "check",   "variable", "sequential", "sus_level",
                                  "syndrome", "retire",  "markov",   "output"};

struct Totals {
    int64_t launches = 0;
    double ms = 0, bytes = 0, edgeq = 0;
};

std::mutex g_prof_mu;
bool g_prof_on = false;
Totals g_prof[K_COUNT];

struct Tracer {
    struct Rec {
        int kind;
        hipEvent_t a, b;
        double bytes, edgeq;
    };
    bool on;
    hipStream_t st;
    std::vector<Rec> recs;
    hipEvent_t pending = nullptr;
    static thread_local std::vector<hipEvent_t> pool;

    explicit Tracer(hipStream_t s) : st(s) {
        std::lock_guard<std::mutex> g(g_prof_mu);
        on = g_prof_on;
    }
    hipEvent_t get() {
        if (!pool.empty()) {
            hipEvent_t e = pool.back();
            pool.pop_back();
            return e;
        }
        hipEvent_t e = nullptr;
        if (hipEventCreate(&e) != hipSuccess) return nullptr;
        return e;
    }
    void begin() {
        if (!on) return;
        pending = get();
        if (pending) (void)hipEventRecord(pending, st);
    }
    void end(int kind, double bytes, double edgeq) {
        if (!on || !pending) return;
        hipEvent_t b = get();
        if (!b) return;
        (void)hipEventRecord(b, st);
        recs.push_back(Rec{kind, pending, b, bytes, edgeq});
        pending = nullptr;
    }
    // call after the stream has been synchronised
    void flush() {
        if (!on) return;
        std::lock_guard<std::mutex> g(g_prof_mu);
        for (auto &r : recs) {
            float ms = 0;
            if (hipEventElapsedTime(&ms, r.a, r.b) == hipSuccess) {
                Totals &t = g_prof[r.kind];
                t.launches++;
                t.ms += ms;
                t.bytes += r.bytes;
                t.edgeq += r.edgeq;
            }
            pool.push_back(r.a);
            pool.push_back(r.b);
        }
        recs.clear();
    }
};
thread_local std::vector<hipEvent_t> Tracer::pool;

}  // namespace

// ======================================================================= kernels
namespace {

__global__ void k_state_init(DevState s, int32_t *iters, uint8_t *conv) {
    const int f = blockIdx.x * blockDim.x + threadIdx.x;
    if (f < 4 && blockIdx.x == 0) s.count[f] = 0;
    if (f >= s.F) return;
    s.active[f] = 1;
    s.unsat[f] = 0;
    iters[f] = 0;
    conv[f] = 0;
    s.guards[f] = 0;
}

// A5 convergence test: check i of frame f against z_i.
__global__ __launch_bounds__(kBlock) void k_syndrome(DevCode c, DevState s, const uint8_t *z) {
    const int F = s.F;
    const int nchunk = (F + kBlock - 1) / kBlock;
    const int i = blockIdx.x / nchunk;
    const int f = (blockIdx.x % nchunk) * kBlock + threadIdx.x;
    if (f >= F || !s.active[f]) return;
    int acc = 0;
    for (int e = c.row_ptr[i]; e < c.row_ptr[i + 1]; ++e)
        acc ^= c.mul[c.coef[e] * c.q + s.xh[size_t(c.col[e]) * s.Fp + f]];
    if (acc != (z ? z[size_t(f) * c.m + i] : 0)) s.unsat[f] = 1;
}

// A5 retirement after iteration t.
__global__ void k_retire(DevState s, int t, int max_iter, int early_stop, int32_t *iters, uint8_t *conv) {
    const int f = blockIdx.x * blockDim.x + threadIdx.x;
    if (f == 0) s.count[2 * ((t + 1) & 1)] = 0;
    if (f >= s.F) return;
    if (s.active[f]) {
        const bool ok = s.unsat[f] == 0;
        if (ok && !conv[f]) { conv[f] = 1; iters[f] = t; }
        if ((ok && early_stop) || t >= max_iter) {
            s.active[f] = 0;
            if (!conv[f]) iters[f] = max_iter;
        } else {
            atomicAdd(&s.count[2 * (t & 1)], 1u);
        }
    }
    s.unsat[f] = 0;
}

__global__ void k_out_xhat(const uint8_t *xh, int n, int F, int Fp, uint8_t *out) {
    const size_t t = size_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (t >= size_t(n) * F) return;
    const int f = int(t / n), j = int(t % n);
    out[t] = xh[size_t(j) * Fp + f];
}

// ---------------------------------------------------------------- dispatch
// Algorithmic HBM bytes per frame of each iteration kernel (float32 messages).
struct Bytes {
    double check, variable, sequential, syndrome, markov;
};

Bytes bytes_per_frame(const gfbp_code *code, int needQ, int has_z) {
    const double E = code->info.n_edges, n = code->info.n, m = code->info.m, K = code->info.n_info,
                 Q = code->info.q;
    Bytes b;
    b.check = 8.0 * E * Q + (has_z ? m : 0);
    b.variable = 8.0 * E * Q + 4.0 * n * Q * (1 + needQ) + n;
    b.sequential = 4.0 * Q * (code->sum_dc2 + E) + 4.0 * n * Q * (1 + needQ) + n + (has_z ? E : 0);
    b.syndrome = E + (has_z ? m : 0);
    b.markov = 16.0 * K * Q;
    return b;
}

// Kernel shape for a code and schedule.  Degree class "small" (rows <= 6,
// columns <= 4) keeps up to 6 siblings' transforms in registers and allows
// EL = 2, 4 or 8 entries per lane; the general class (rows <= 16, columns <= 8)
// allows EL = 2 or 4.  The default is the largest allowed EL (at most q);
// gfbp_code_set_shape / gfbp_tune choose another.
struct Shape {
    bool small;
    int lel;  // log2 of entries per lane
};

inline bool small_class(const gfbp_code *code) {
    return code->info.max_row_degree <= 6 && code->info.max_col_degree <= 4;
}

inline int max_lel(const gfbp_code *code) { return std::min(code->info.p, small_class(code) ? 3 : 2); }

inline bool allowed_el(const gfbp_code *code, int el) {
    if (el == 0) return true;
    for (int l = 1; l <= max_lel(code); ++l)
        if (el == (1 << l)) return true;
    return false;
}

inline Shape shape_of(const gfbp_code *code, int schedule) {
    Shape sh;
    sh.small = small_class(code);
    const int el = code->el[schedule == GFBP_SUS ? 1 : 0];
    int lel = max_lel(code);
    if (el > 0)
        for (int l = 1; l <= max_lel(code); ++l)
            if (el == (1 << l)) lel = l;
    sh.lel = lel;
    return sh;
}

// Frame stride of the workspace arrays: whole 64-frame tiles.
inline int frame_stride(int F) { return (F + kWave - 1) / kWave * kWave; }

inline unsigned tiled_blocks(int nodes, const DevState &s) {
    const long long waves = (long long)nodes * s.nact;
    return unsigned(std::max<long long>(1, (waves + (kBlock / kWave) - 1) / (kBlock / kWave)));
}

template <int P, int LG, int DCM, int DVM>
struct TiledLaunch {
    static void init(hipStream_t st, const DevCode &c, const DevState &s, const gfbp_batch *b) {
        tiled::Chan ch{b->channel, b->prior == GFBP_PRIOR_MARKOV, b->rx, b->erasure, b->y, b->likelihood, b->param,
                       b->markov_pi};
        hipLaunchKernelGGL((tiled::k_init<P, LG>), dim3(tiled_blocks(c.n, s)), dim3(kBlock), 0, st, c, s, ch);
    }
    static void check(hipStream_t st, const DevCode &c, const DevState &s, const uint8_t *z, Snap sn) {
        hipLaunchKernelGGL((tiled::k_check<P, LG, DCM>), dim3(tiled_blocks(c.m, s)), dim3(kBlock), 0, st, c, s,
                           z, sn);
    }
    static void variable(hipStream_t st, const DevCode &c, const DevState &s, int markov, int wantQ, Snap sn) {
        hipLaunchKernelGGL((tiled::k_variable<P, LG, DVM>), dim3(tiled_blocks(c.n, s)), dim3(kBlock), 0, st, c,
                           s, markov, wantQ, sn);
    }
    static void sus_level(hipStream_t st, const DevCode &c, const DevState &s, const uint8_t *z, int markov, int wantQ,
                          Snap sn, const int32_t *cols, int nc) {
        hipLaunchKernelGGL((tiled::k_sus_level<P, LG, DCM, DVM>), dim3(unsigned(nc) * unsigned(s.nact)),
                           dim3(DVM * kWave), 0, st, c, s, z, markov, wantQ, sn, cols, nc);
    }
    static void sequential(hipStream_t st, const DevCode &c, const DevState &s, const uint8_t *z, int markov,
                           int wantQ, Snap sn) {
        hipLaunchKernelGGL((tiled::k_sequential<P, LG, DCM, DVM>), dim3(unsigned(s.nact)), dim3(DVM * kWave), 0, st, c,
                           s, z, markov, wantQ, sn);
    }
    static void markov(hipStream_t st, const DevCode &c, const DevState &s, const float *M, const float *pi) {
        hipLaunchKernelGGL((tiled::k_markov<P, LG>), dim3(tiled_blocks(c.n_info, s)), dim3(kBlock), 0, st, c, s,
                           M, pi);
    }
    static constexpr int TF = kWave >> LG;
    static void tiles(hipStream_t st, const DevState &s, int t) {
        hipLaunchKernelGGL(tiled::k_tiles, dim3(1), dim3(1024), 0, st, s, TF, t);
    }
    static void vectors(hipStream_t st, const float *src, int n, const DevState &s, float *out) {
        const size_t tot = size_t(n) * s.F * (1 << P);
        hipLaunchKernelGGL((tiled::k_out_vectors<P, LG>), dim3(unsigned((tot + 255) / 256)), dim3(256), 0, st, src, n,
                           s.F, s.Fp, out);
    }
};

template <int P, class K>
gfbp_status run_batch(const gfbp_code *code, const gfbp_batch *b, gfbp_result *out, DevState &s,
                      hipStream_t st, int needQ) {
    constexpr int Q = 1 << P;
    const DevCode &c = code->dev;
    const int F = s.F;
    const unsigned fb = unsigned((F + kBlock - 1) / kBlock);
    const Bytes bpf = bytes_per_frame(code, needQ, b->syndrome != nullptr);
    const double eq_frame = double(c.E) * Q;
    Tracer tr(st);
    hipLaunchKernelGGL(k_state_init, dim3(fb), dim3(kBlock), 0, st, s, out->iters, out->converged);
    const int ntiles = s.Fp / K::TF;
    K::tiles(st, s, 0);
    // k_tiles(0) lists exactly the tiles holding a frame: ceil(F / TF) of them
    // (ntiles can be larger: the stride is padded to whole 64-frame tiles).
    s.act = s.tiles;
    s.nact = (F + K::TF - 1) / K::TF;
    tr.begin();
    K::init(st, c, s, b);
    tr.end(K_INIT, double(F) * (4.0 * Q * (c.n + c.E) + c.n * 4.0 * P), 0);
    HIP_TRY(hipGetLastError());
    const int markov = (b->prior == GFBP_PRIOR_MARKOV) && c.n_info > 0;
    uint32_t running = uint32_t(F);
    for (int t = 1; t <= b->max_iter; ++t) {
        const bool snap_now = (t == out->snap_iter);
        Snap sn{snap_now ? out->snap_q : nullptr, snap_now ? out->snap_r : nullptr};
        const int wantQ = needQ || (snap_now && out->snap_Q);
        const double Fa = running;
        if (b->schedule == GFBP_PUS) {
            tr.begin();
            K::check(st, c, s, b->syndrome, sn);
            tr.end(K_CHECK, Fa * bpf.check, Fa * eq_frame);
            tr.begin();
            K::variable(st, c, s, markov, wantQ, sn);
            tr.end(K_VARIABLE, Fa * bpf.variable, Fa * eq_frame);
        } else if (b->options & GFBP_OPT_SUS_STRICT) {
            tr.begin();
            K::sequential(st, c, s, b->syndrome, markov, wantQ, sn);
            tr.end(K_SEQUENTIAL, Fa * bpf.sequential, Fa * eq_frame);
        } else {
            const int nlev = int(code->level_ptr.size()) - 1;
            for (int l = 0; l < nlev; ++l) {
                const int c0 = code->level_ptr[l], nc = code->level_ptr[l + 1] - c0;
                tr.begin();
                K::sus_level(st, c, s, b->syndrome, markov, wantQ, sn, code->level_cols + c0, nc);
                tr.end(K_SUS_LEVEL,
                       Fa * (4.0 * Q * (code->level_sibs[l] + code->level_edges[l]) + nc * (4.0 * Q * (1 + needQ) + 1)),
                       Fa * code->level_edges[l] * Q);
            }
        }
        if (snap_now && out->snap_Q) K::vectors(st, s.Qp, c.n, s, out->snap_Q);
        tr.begin();
        hipLaunchKernelGGL(k_syndrome, dim3(unsigned(c.m) * fb), dim3(kBlock), 0, st, c, s, b->syndrome);
        tr.end(K_SYNDROME, Fa * bpf.syndrome, 0);
        hipLaunchKernelGGL(k_retire, dim3(fb), dim3(kBlock), 0, st, s, t, b->max_iter, b->early_stop, out->iters,
                           out->converged);
        HIP_TRY(hipGetLastError());
        if (t == b->max_iter) break;
        K::tiles(st, s, t);
        uint32_t cnt[2] = {0, 0};
        HIP_TRY(hipMemcpyAsync(cnt, s.count + 2 * (t & 1), sizeof cnt, hipMemcpyDeviceToHost, st));
        HIP_TRY(hipStreamSynchronize(st));
        const uint32_t left = cnt[0];
        running = left;
        if (left == 0) break;
        s.act = s.tiles + size_t(t & 1) * ntiles;
        s.nact = int(cnt[1]);
        if (markov) {
            tr.begin();
            K::markov(st, c, s, b->markov_M, b->markov_pi);
            tr.end(K_MARKOV, double(left) * bpf.markov, 0);
        }
    }
    tr.begin();
    {
        const size_t tot = size_t(c.n) * F;
        hipLaunchKernelGGL(k_out_xhat, dim3(unsigned((tot + 255) / 256)), dim3(256), 0, st, s.xh, c.n, F, s.Fp,
                           out->xhat);
    }
    if (out->posterior) K::vectors(st, s.Qp, c.n, s, out->posterior);
    tr.end(K_OUTPUT, double(F) * c.n * (2.0 + (out->posterior ? 8.0 * Q : 0.0)), 0);
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipStreamSynchronize(st));
    tr.flush();
    return GFBP_OK;
}

template <int P, int LEL>
gfbp_status run_lel(const gfbp_code *code, const gfbp_batch *b, gfbp_result *out, DevState &s, hipStream_t st,
                    int needQ, bool small) {
    if constexpr (LEL <= 3 && LEL <= P) {
        if (small) return run_batch<P, TiledLaunch<P, P - LEL, 6, 4>>(code, b, out, s, st, needQ);
    }
    if constexpr (LEL <= 2 && LEL <= P) {
        if (!small) return run_batch<P, TiledLaunch<P, P - LEL, 16, 8>>(code, b, out, s, st, needQ);
    }
    return fail(GFBP_EUNSUPPORTED, "no kernel for this shape");
}

template <int P>
gfbp_status run_any(const gfbp_code *code, const gfbp_batch *b, gfbp_result *out, DevState &s, hipStream_t st,
                    int needQ) {
    const Shape sh = shape_of(code, b->schedule);
    switch (sh.lel) {
        case 1: return run_lel<P, 1>(code, b, out, s, st, needQ, sh.small);
        case 2: return run_lel<P, 2>(code, b, out, s, st, needQ, sh.small);
        case 3: return run_lel<P, 3>(code, b, out, s, st, needQ, sh.small);
        default: return fail(GFBP_EUNSUPPORTED, "bad shape");
    }
}

// Workspace carving, shared by size query and decode.
struct Carve {
    size_t Qm, R, L, Pr, Qp, xh, unsat, active, count, tiles, guards, total;
};

Carve carve(const gfbp_code *code, int F_, int schedule, int prior) {
    const size_t E = code->info.n_edges, n = code->info.n, K = code->info.n_info, Q = code->info.q;
    const size_t F = size_t(frame_stride(F_));
    Carve c{};
    size_t off = 0;
    auto take = [&](size_t bytes) { size_t o = off; off += align256(bytes); return o; };
    c.Qm = take(E * F * Q * 4);
    c.R = take(schedule == GFBP_PUS ? E * F * Q * 4 : 0);
    c.L = take(n * F * Q * 4);
    c.Pr = take(prior == GFBP_PRIOR_MARKOV ? K * F * Q * 4 : 0);
    c.Qp = take(n * F * Q * 4);
    c.xh = take(n * F);
    c.unsat = take(size_t(F_) * 4);
    c.active = take(size_t(F_));
    c.count = take(16);
    c.tiles = take(2 * F * 4);
    c.guards = take(size_t(F_) * 4);
    c.total = off;
    return c;
}

// ---------------------------------------------------------------- host GF
bool field_tables(int p, unsigned poly, std::vector<uint8_t> &mul, std::vector<uint8_t> &inv) {
    const int q = 1 << p;
    if (poly >> p != 1u) return false;
    std::vector<int> ex(2 * q), lg(q, -1);
    int v = 1;
    for (int i = 0; i < q - 1; ++i) {
        if (lg[v] != -1) return false;  // x is not primitive
        ex[i] = ex[i + q - 1] = v;
        lg[v] = i;
        v <<= 1;
        if (v & q) v ^= int(poly);
    }
    if (v != 1) return false;
    mul.assign(size_t(q) * q, 0);
    inv.assign(q, 0);
    for (int a = 1; a < q; ++a) {
        for (int b = 1; b < q; ++b) mul[a * q + b] = uint8_t(ex[lg[a] + lg[b]]);
        inv[a] = uint8_t(ex[(q - 1 - lg[a]) % (q - 1)]);
    }
    return true;
}

const unsigned kDefaultPoly[7] = {0, 0x3, 0x7, 0xB, 0x13, 0x25, 0x43};

}  // namespace

// ======================================================================= C ABI
extern "C" {

const char *gfbp_last_error(void) { return g_err.c_str(); }

const char *gfbp_version(void) { return "gfbp 0.4 (gfx950)"; }

gfbp_status gfbp_code_build(const gfbp_code_desc *d, gfbp_code **out) {
    if (!d || !out) return fail(GFBP_EINVAL, "null argument");
    *out = nullptr;
    const int q = d->q;
    int p = 0;
    while ((1 << p) < q) ++p;
    if (q < 2 || q > GFBP_MAX_Q || (1 << p) != q) return fail(GFBP_EUNSUPPORTED, "q must be 2^p with 1 <= p <= 6");
    if (d->n <= 0 || d->m <= 0 || d->n_info < 0 || d->n_info > d->n)
        return fail(GFBP_EINVAL, "bad n, m or n_info");
    if (!d->row_ptr || !d->col || !d->coef) return fail(GFBP_EINVAL, "null row_ptr/col/coef");
    const unsigned poly = d->poly ? unsigned(d->poly) : kDefaultPoly[p];
    std::vector<uint8_t> mul, inv;
    if (!field_tables(p, poly, mul, inv)) return fail(GFBP_EINVAL, "polynomial is not primitive of degree p");
    const int n = d->n, m = d->m;
    if (d->row_ptr[0] != 0) return fail(GFBP_EINVAL, "row_ptr[0] must be 0");
    for (int i = 0; i < m; ++i)
        if (d->row_ptr[i + 1] < d->row_ptr[i]) return fail(GFBP_EINVAL, "row_ptr not nondecreasing");
    const int E = d->row_ptr[m];
    int max_dc = 0;
    double sum_dc2 = 0;
    std::vector<int> col_deg(n, 0), seen(n, -1);
    for (int i = 0; i < m; ++i) {
        const int dc = d->row_ptr[i + 1] - d->row_ptr[i];
        max_dc = dc > max_dc ? dc : max_dc;
        sum_dc2 += double(dc) * (dc - 1);
        for (int e = d->row_ptr[i]; e < d->row_ptr[i + 1]; ++e) {
            const int j = d->col[e];
            if (j < 0 || j >= n) return fail(GFBP_EINVAL, "column index out of range");
            if (d->coef[e] == 0 || d->coef[e] >= q) return fail(GFBP_EINVAL, "coefficient not in GF(q)\\{0}");
            if (seen[j] == i) return fail(GFBP_EINVAL, "column repeated in a row");
            seen[j] = i;
            col_deg[j]++;
        }
    }
    int max_dv = 0;
    for (int j = 0; j < n; ++j) max_dv = col_deg[j] > max_dv ? col_deg[j] : max_dv;
    if (max_dc > GFBP_MAX_ROW_DEGREE) return fail(GFBP_EUNSUPPORTED, "row degree above GFBP_MAX_ROW_DEGREE");
    if (max_dv > GFBP_MAX_COL_DEGREE) return fail(GFBP_EUNSUPPORTED, "column degree above GFBP_MAX_COL_DEGREE");

    std::vector<int32_t> col_ptr(n + 1, 0), col_edge(E), edge_row(E), fill(n, 0);
    for (int j = 0; j < n; ++j) col_ptr[j + 1] = col_ptr[j] + col_deg[j];
    for (int i = 0; i < m; ++i)
        for (int e = d->row_ptr[i]; e < d->row_ptr[i + 1]; ++e) {
            edge_row[e] = i;
            const int j = d->col[e];
            col_edge[col_ptr[j] + fill[j]++] = e;
        }
    // SUS dependency levels: level(j) = 1 + the highest level among earlier
    // columns sharing a check with j (0 if none).
    std::vector<int32_t> level(n, 0), row_top(m, -1);
    int nlev = 0;
    for (int j = 0; j < n; ++j) {
        int lv = 0;
        for (int t = col_ptr[j]; t < col_ptr[j + 1]; ++t) lv = std::max(lv, row_top[edge_row[col_edge[t]]] + 1);
        for (int t = col_ptr[j]; t < col_ptr[j + 1]; ++t) row_top[edge_row[col_edge[t]]] = lv;
        level[j] = lv;
        nlev = std::max(nlev, lv + 1);
    }
    std::vector<int32_t> level_ptr(nlev + 1, 0), level_cols(n);
    std::vector<double> level_sibs(nlev, 0.0), level_edges(nlev, 0.0);
    for (int j = 0; j < n; ++j) level_ptr[level[j] + 1]++;
    for (int l = 0; l < nlev; ++l) level_ptr[l + 1] += level_ptr[l];
    {
        std::vector<int32_t> fillp(level_ptr.begin(), level_ptr.end() - 1);
        for (int j = 0; j < n; ++j) {
            const int l = level[j];
            level_cols[fillp[l]++] = j;
            for (int t = col_ptr[j]; t < col_ptr[j + 1]; ++t) {
                const int i = edge_row[col_edge[t]];
                level_sibs[l] += d->row_ptr[i + 1] - d->row_ptr[i] - 1;
                level_edges[l] += 1;
            }
        }
    }
    // per-edge images of the basis x^b under multiplication by h^-1 and h
    std::vector<uint64_t> emap(2 * size_t(E));
    for (int e = 0; e < E; ++e) {
        const int h = d->coef[e], hi = inv[h];
        uint64_t wi = 0, wm = 0;
        for (int b = 0; b < p; ++b) {
            wi |= uint64_t(mul[hi * q + (1 << b)]) << (6 * b);
            wm |= uint64_t(mul[h * q + (1 << b)]) << (6 * b);
        }
        emap[2 * size_t(e)] = wi;
        emap[2 * size_t(e) + 1] = wm;
    }

    gfbp_code *c = new (std::nothrow) gfbp_code();
    if (!c) return fail(GFBP_ENOMEM, "host allocation");
    size_t off = 0;
    auto take = [&](size_t bytes) { size_t o = off; off += align256(bytes ? bytes : 1); return o; };
    const size_t o_rp = take(4 * size_t(m + 1)), o_col = take(4 * size_t(E)), o_coef = take(size_t(E)),
                 o_cp = take(4 * size_t(n + 1)), o_ce = take(4 * size_t(E)), o_er = take(4 * size_t(E)),
                 o_mul = take(size_t(q) * q), o_em = take(16 * size_t(E)), o_lc = take(4 * size_t(n));
    if (hipMalloc(&c->mem, off) != hipSuccess) {
        delete c;
        return fail(GFBP_ENOMEM, "device allocation for the code");
    }
    char *base = static_cast<char *>(c->mem);
    auto up = [&](size_t o, const void *src, size_t bytes) {
        return bytes ? hipMemcpy(base + o, src, bytes, hipMemcpyHostToDevice) : hipSuccess;
    };
    hipError_t err = hipSuccess;
    if (err == hipSuccess) err = up(o_rp, d->row_ptr, 4 * size_t(m + 1));
    if (err == hipSuccess) err = up(o_col, d->col, 4 * size_t(E));
    if (err == hipSuccess) err = up(o_coef, d->coef, size_t(E));
    if (err == hipSuccess) err = up(o_cp, col_ptr.data(), 4 * size_t(n + 1));
    if (err == hipSuccess) err = up(o_ce, col_edge.data(), 4 * size_t(E));
    if (err == hipSuccess) err = up(o_er, edge_row.data(), 4 * size_t(E));
    if (err == hipSuccess) err = up(o_mul, mul.data(), mul.size());
    if (err == hipSuccess) err = up(o_em, emap.data(), 16 * size_t(E));
    if (err == hipSuccess) err = up(o_lc, level_cols.data(), 4 * size_t(n));
    if (err != hipSuccess) {
        (void)hipFree(c->mem);
        delete c;
        return fail(GFBP_EHIP, std::string("copying the code to the device: ") + hipGetErrorString(err));
    }
    c->info = gfbp_code_info{q, p, n, m, d->n_info, E, max_dc, max_dv, int32_t(poly), nlev};
    c->sum_dc2 = sum_dc2;
    c->level_ptr = std::move(level_ptr);
    c->level_sibs = std::move(level_sibs);
    c->level_edges = std::move(level_edges);
    c->level_cols = reinterpret_cast<const int32_t *>(base + o_lc);
    c->dev = DevCode{n, m, E, q, p, d->n_info,
                     reinterpret_cast<const int32_t *>(base + o_rp), reinterpret_cast<const int32_t *>(base + o_col),
                     reinterpret_cast<const uint8_t *>(base + o_coef), reinterpret_cast<const int32_t *>(base + o_cp),
                     reinterpret_cast<const int32_t *>(base + o_ce), reinterpret_cast<const int32_t *>(base + o_er),
                     reinterpret_cast<const uint8_t *>(base + o_mul), reinterpret_cast<const uint64_t *>(base + o_em)};
    *out = c;
    return GFBP_OK;
}

gfbp_status gfbp_code_free(gfbp_code *c) {
    if (!c) return GFBP_OK;
    hipError_t e = hipFree(c->mem);
    delete c;
    if (e != hipSuccess) return fail(GFBP_EHIP, std::string("hipFree: ") + hipGetErrorString(e));
    return GFBP_OK;
}

gfbp_status gfbp_code_info_get(const gfbp_code *c, gfbp_code_info *out) {
    if (!c || !out) return fail(GFBP_EINVAL, "null argument");
    *out = c->info;
    return GFBP_OK;
}

size_t gfbp_workspace_size(const gfbp_code *code, int32_t n_frames, int32_t schedule, int32_t prior) {
    if (!code || n_frames < 0) return 0;
    return carve(code, n_frames, schedule, prior).total;
}

gfbp_status gfbp_decode_batch(const gfbp_code *code, const gfbp_batch *b, gfbp_result *out, void *workspace,
                              size_t ws_bytes, void *stream) {
    if (!code || !b || !out) return fail(GFBP_EINVAL, "null argument");
    const int F = b->n_frames;
    if (F < 0) return fail(GFBP_EINVAL, "n_frames < 0");
    if (b->schedule != GFBP_PUS && b->schedule != GFBP_SUS) return fail(GFBP_EINVAL, "bad schedule");
    if (b->max_iter < 1) return fail(GFBP_EINVAL, "max_iter < 1");
    if (b->prior != GFBP_PRIOR_UNIFORM && b->prior != GFBP_PRIOR_MARKOV) return fail(GFBP_EINVAL, "bad prior");
    if (F == 0) return GFBP_OK;
    switch (b->channel) {
        case GFBP_CH_BSC:
            if (!b->rx || !b->param) return fail(GFBP_EINVAL, "BSC needs rx and param");
            break;
        case GFBP_CH_BEC:
            if (!b->rx || !b->erasure) return fail(GFBP_EINVAL, "BEC needs rx and erasure");
            break;
        case GFBP_CH_BIAWGN:
            if (!b->y || !b->param) return fail(GFBP_EINVAL, "BI-AWGN needs y and param");
            break;
        case GFBP_CH_LIKELIHOOD:
            if (!b->likelihood) return fail(GFBP_EINVAL, "LIKELIHOOD needs likelihood");
            break;
        default:
            return fail(GFBP_EINVAL, "bad channel");
    }
    if (b->prior == GFBP_PRIOR_MARKOV && (!b->markov_M || !b->markov_pi))
        return fail(GFBP_EINVAL, "Markov prior needs markov_M and markov_pi");
    if (!out->xhat || !out->iters || !out->converged) return fail(GFBP_EINVAL, "null output buffer");
    if (!workspace) return fail(GFBP_EINVAL, "null workspace");
    if (reinterpret_cast<uintptr_t>(workspace) % 256) return fail(GFBP_EINVAL, "workspace not 256-byte aligned");
    const Carve cv = carve(code, F, b->schedule, b->prior);
    if (ws_bytes < cv.total) return fail(GFBP_ESMALL, "workspace too small");
    char *w = static_cast<char *>(workspace);
    DevState s{};
    s.Qm = reinterpret_cast<float *>(w + cv.Qm);
    s.R = reinterpret_cast<float *>(w + cv.R);
    s.L = reinterpret_cast<float *>(w + cv.L);
    s.Pr = reinterpret_cast<float *>(w + cv.Pr);
    s.Qp = reinterpret_cast<float *>(w + cv.Qp);
    s.xh = reinterpret_cast<uint8_t *>(w + cv.xh);
    s.unsat = reinterpret_cast<uint32_t *>(w + cv.unsat);
    s.active = reinterpret_cast<uint8_t *>(w + cv.active);
    s.count = reinterpret_cast<uint32_t *>(w + cv.count);
    s.tiles = reinterpret_cast<int32_t *>(w + cv.tiles);
    s.guards = out->guards ? out->guards : reinterpret_cast<int32_t *>(w + cv.guards);
    s.F = F;
    s.Fp = frame_stride(F);
    const int needQ = (b->prior == GFBP_PRIOR_MARKOV) || out->posterior != nullptr;
    hipStream_t st = static_cast<hipStream_t>(stream);
    switch (code->info.p) {
        case 1: return run_any<1>(code, b, out, s, st, needQ);
        case 2: return run_any<2>(code, b, out, s, st, needQ);
        case 3: return run_any<3>(code, b, out, s, st, needQ);
        case 4: return run_any<4>(code, b, out, s, st, needQ);
        case 5: return run_any<5>(code, b, out, s, st, needQ);
        case 6: return run_any<6>(code, b, out, s, st, needQ);
        default: return fail(GFBP_EUNSUPPORTED, "bad field");
    }
}

gfbp_status gfbp_code_set_shape(gfbp_code *c, int32_t schedule, int32_t entries_per_lane) {
    if (!c) return fail(GFBP_EINVAL, "null code");
    if (schedule != GFBP_PUS && schedule != GFBP_SUS) return fail(GFBP_EINVAL, "bad schedule");
    if (!allowed_el(c, entries_per_lane)) return fail(GFBP_EUNSUPPORTED, "entries per lane not available for this code");
    c->el[schedule == GFBP_SUS ? 1 : 0] = entries_per_lane;
    return GFBP_OK;
}

int32_t gfbp_code_get_shape(const gfbp_code *c, int32_t schedule) {
    if (!c || (schedule != GFBP_PUS && schedule != GFBP_SUS)) return 0;
    return 1 << shape_of(c, schedule).lel;
}

gfbp_status gfbp_tune(gfbp_code *c, const gfbp_batch *b, gfbp_result *out, void *workspace, size_t ws_bytes,
                      void *stream, int32_t trial_iters, int32_t *chosen) {
    if (!c || !b || !out) return fail(GFBP_EINVAL, "null argument");
    if (trial_iters < 1) return fail(GFBP_EINVAL, "trial_iters < 1");
    const int slot = b->schedule == GFBP_SUS ? 1 : 0;
    const int keep = c->el[slot];
    gfbp_batch tb = *b;
    tb.max_iter = trial_iters;
    tb.early_stop = 0;
    gfbp_result to = *out;
    to.posterior = nullptr;
    to.snap_iter = 0;
    to.snap_q = to.snap_r = to.snap_Q = nullptr;
    double best_t = 1e300;
    int best = 0;
    for (int l = 1; l <= max_lel(c); ++l) {
        c->el[slot] = 1 << l;
        double t = 0;
        for (int rep = 0; rep < 2; ++rep) {  // the first run warms up, the second is timed
            const auto t0 = std::chrono::steady_clock::now();
            const gfbp_status st = gfbp_decode_batch(c, &tb, &to, workspace, ws_bytes, stream);
            if (st != GFBP_OK) {
                c->el[slot] = keep;
                return st;
            }
            t = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
        }
        if (t < best_t) {
            best_t = t;
            best = 1 << l;
        }
    }
    c->el[slot] = best;
    if (chosen) *chosen = best;
    return GFBP_OK;
}

gfbp_status gfbp_profile_enable(int32_t on) {
    std::lock_guard<std::mutex> g(g_prof_mu);
    g_prof_on = on != 0;
    return GFBP_OK;
}

gfbp_status gfbp_profile_reset(void) {
    std::lock_guard<std::mutex> g(g_prof_mu);
    for (auto &t : g_prof) t = Totals{};
    return GFBP_OK;
}

int32_t gfbp_profile_read(gfbp_kernel_stats *out, int32_t cap) {
    std::lock_guard<std::mutex> g(g_prof_mu);
    int32_t n = 0;
    for (int k = 0; k < K_COUNT; ++k) {
        if (g_prof[k].launches == 0) continue;
        if (out && n < cap) {
            gfbp_kernel_stats &o = out[n];
            std::memset(&o, 0, sizeof o);
            std::strncpy(o.name, kKindName[k], sizeof(o.name) - 1);
            o.launches = g_prof[k].launches;
            o.total_ms = g_prof[k].ms;
            o.algo_bytes = g_prof[k].bytes;
            o.edge_q = g_prof[k].edgeq;
        }
        ++n;
    }
    return n;
}

}  // extern "C"
