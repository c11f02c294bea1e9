// GF(2^p) LDPC belief-propagation decoder for gfx950: kernels and C ABI.
//
// Paper: Yacov, Efraim, Kfir, Kanter, Shental, "Parallel vs. Sequential Belief
// Propagation Decoding of LDPC Codes over GF(q) and Markov Sources", Section 2.
// The public contract is include/gfbp.h.
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <functional>
#include <mutex>
#include <thread>
#include <new>
#include <string>
#include <vector>

#include "../../include/gfbp.h"
#include "gfbp_kernels.h"
#include "gfbp_plan.h"
#include "gfbp_tiled.h"
#include "gfbp_persist.h"
#include "gfbp_onchip.h"

using namespace gfbp;

namespace {

thread_local std::string g_err;

// Set while gfbp_decode_batch_noalloc runs on this thread: the decode then
// takes no pinned memory, events or streams of its own (see that entry point).
thread_local bool g_no_alloc = false;

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
    // SUS dependency levels (host plan, gfbp_plan.h) with their device
    // records: [0] from shared checks; [1] also along the source chain
    struct Levels : LevelPlan {
        const SusRec *recs = nullptr;  // device [n][max column degree], columns in level order
        const int32_t *dptr = nullptr; // device copy of ptr
    } lv[2];
    int el[2] = {0, 0};   // entries per lane chosen for PUS / SUS (0 = default)
    void *mem = nullptr;  // one device allocation holding every array of dev
};

// ======================================================================= tracing
// Optional per-kernel timing with HIP events recorded on the decode stream
// around each launch, with the algorithmic bytes and edge-q updates of the
// launch attached.  Read back after the decode's final synchronisation.
namespace {

enum Kind {
    K_INIT, K_CHECK, K_VARIABLE, K_SEQUENTIAL, K_SUS_LEVEL, K_SYNDROME, K_RETIRE, K_MARKOV, K_OUTPUT, K_COMPACT,
    K_SUS_RUN, K_PERSIST, K_ONCHIP, K_COUNT
};
const char *kKindName[K_COUNT] = {"init",     "check",  "variable", "sequential", "sus_level", "syndrome",
                                  "retire",   "markov", "output",   "compact",    "sus_run",   "persistent",
                                  "onchip"};

struct Totals {
    int64_t launches = 0;
    double ms = 0, bytes = 0, edgeq = 0;
};

std::mutex g_prof_mu;
bool g_prof_on = false;
Totals g_prof[K_COUNT];

// Events handed to the next kernel launch (see launch()): the kernel's own
// start and end timestamps, so a traced duration is the kernel's alone.
thread_local hipEvent_t g_launch_ev[2] = {nullptr, nullptr};

struct Tracer {
    struct Rec {
        int kind;
        hipEvent_t a, b;
        double bytes, edgeq;  // absolute, or per running frame when iter > 0
        int iter;
    };
    bool on;
    hipStream_t st;
    std::vector<Rec> recs;
    static thread_local std::vector<hipEvent_t> pool;

    explicit Tracer(hipStream_t s) : st(s) {
        std::lock_guard<std::mutex> g(g_prof_mu);
        on = g_prof_on && !g_no_alloc;
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
    // the next launch() on this thread carries a pair of events
    void begin() {
        if (!on) return;
        hipEvent_t a = get(), b = get();
        if (!a || !b) {
            if (a) pool.push_back(a);
            if (b) pool.push_back(b);
            return;
        }
        g_launch_ev[0] = a;
        g_launch_ev[1] = b;
    }
    // the launch since begin() took the events (else nothing is recorded)
    void end(int kind, double bytes, double edgeq) {
        if (!on) return;
        if (g_launch_ev[0]) {  // no launch happened
            pool.push_back(g_launch_ev[0]);
            pool.push_back(g_launch_ev[1]);
            g_launch_ev[0] = g_launch_ev[1] = nullptr;
            return;
        }
        recs.push_back(Rec{kind, last_[0], last_[1], bytes, edgeq, 0});
    }
    // as end(), with bytes and updates per running frame of iteration `iter`
    // (multiplied at flush by the number of frames that iteration ran)
    void end_iter(int kind, double bytes_per_frame, double edgeq_per_frame, int iter) {
        end(kind, bytes_per_frame, edgeq_per_frame);
        if (on && !recs.empty() && recs.back().a == last_[0]) recs.back().iter = iter;
    }
    static thread_local hipEvent_t last_[2];
    // call after the stream has been synchronised; running[t] = frames that
    // iteration t ran
    void flush(const std::vector<double> &running = {}) {
        if (!on) return;
        std::lock_guard<std::mutex> g(g_prof_mu);
        for (auto &r : recs) {
            float ms = 0;
            if (hipEventElapsedTime(&ms, r.a, r.b) == hipSuccess) {
                const double mult = r.iter > 0 && size_t(r.iter) < running.size() ? running[size_t(r.iter)] : 1.0;
                Totals &t = g_prof[r.kind];
                t.launches++;
                t.ms += ms;
                t.bytes += r.bytes * mult;
                t.edgeq += r.edgeq * mult;
            }
            pool.push_back(r.a);
            pool.push_back(r.b);
        }
        recs.clear();
    }
};
thread_local hipEvent_t Tracer::last_[2] = {nullptr, nullptr};
thread_local std::vector<hipEvent_t> Tracer::pool;

// Kernel launch; when a tracer has handed out events, they are attached to
// this launch (hipExtLaunchKernelGGL) and then belong to the tracer.
template <typename F, typename... Args>
inline void launch(F kernel, dim3 grid, dim3 block, uint32_t shmem, hipStream_t st, Args... args) {
    if (g_launch_ev[0]) {
        hipExtLaunchKernelGGL(kernel, grid, block, shmem, st, g_launch_ev[0], g_launch_ev[1], 0, args...);
        Tracer::last_[0] = g_launch_ev[0];
        Tracer::last_[1] = g_launch_ev[1];
        g_launch_ev[0] = g_launch_ev[1] = nullptr;
    } else {
        hipLaunchKernelGGL(kernel, grid, block, shmem, st, args...);
    }
}

}  // namespace

// ======================================================================= kernels
namespace {

// Per-slot state of a batch decode that is not in DevState.  A slot holds
// frame orig[slot]; running frames may move to other slots (compaction), so
// every per-frame result is written through orig when the frame finishes.
struct BatchAux {
    int32_t *orig;    // [Fp] frame held by each slot
    int32_t *iters;   // [Fp] first converged iteration (or max_iter)
    uint8_t *conv;    // [Fp] converged at some iteration
    uint8_t *z;       // [Fp][m] syndromes by slot (null when z = 0)
    int32_t *holes;   // [Fp] compaction: finished slots below the running count
    int32_t *movers;  // [Fp] compaction: running slots at or above it
    uint8_t *pending; // [Fp] finished frame whose decision is not yet written out
    float *mshape;    // [4] shape of the Markov matrix (k_markov_shape)
    float *qp2;       // PUS with a Markov source: the second pseudo-posterior buffer (iterations alternate)
};

__global__ void k_state_init(DevState s, BatchAux a) {
    const int f = blockIdx.x * blockDim.x + threadIdx.x;
    if (f < 16 && blockIdx.x == 0) s.count[f] = 0;
    if (f >= s.F) return;
    s.active[f] = 1;
    s.unsat[f] = 0;
    s.guards[f] = 0;
    a.iters[f] = 0;
    a.conv[f] = 0;
    a.orig[f] = f;
    a.pending[f] = 0;
}

// A5 convergence test: check i of frames 8k..8k+7 against z_i (one 8-byte
// load of each column's decisions for the eight frames; the frame stride is a
// multiple of 64 and every per-frame byte array is padded to 256 bytes, so the
// loads are aligned and stay inside their arrays).
constexpr int kSynFrames = 8;

__global__ __launch_bounds__(kBlock) void k_syndrome(DevCode c, DevState s, const uint8_t *z) {
    __shared__ uint8_t mul[64 * 64];  // the field's multiplication table
    for (int t = int(threadIdx.x); t < c.q * c.q; t += kBlock) mul[t] = c.mul[t];
    __syncthreads();
    const int F = s.F;
    const int groups = (F + kSynFrames - 1) / kSynFrames;
    const int nchunk = (groups + kBlock - 1) / kBlock;
    const int i = blockIdx.x / nchunk;
    const int k = (blockIdx.x % nchunk) * kBlock + threadIdx.x;
    if (k >= groups) return;
    const int f0 = k * kSynFrames;
    uint64_t act = *reinterpret_cast<const uint64_t *>(s.active + f0);
    if (F - f0 < kSynFrames) act &= (uint64_t(1) << (8 * (F - f0))) - 1;  // frames past F
    if (!act) return;
    int acc[kSynFrames];
#pragma unroll
    for (int u = 0; u < kSynFrames; ++u) acc[u] = 0;
    for (int e = c.row_ptr[i]; e < c.row_ptr[i + 1]; ++e) {
        const uint8_t *m = mul + c.coef[e] * c.q;
        const uint64_t x = *reinterpret_cast<const uint64_t *>(s.xh + size_t(c.col[e]) * s.Fp + f0);
#pragma unroll
        for (int u = 0; u < kSynFrames; ++u) acc[u] ^= m[(x >> (8 * u)) & 0xffu];
    }
#pragma unroll
    for (int u = 0; u < kSynFrames; ++u)
        if (((act >> (8 * u)) & 0xffu) && acc[u] != (z ? z[size_t(f0 + u) * c.m + i] : 0)) s.unsat[f0 + u] = 1;
}

inline unsigned syndrome_blocks(int m, int F) {
    const int groups = (F + kSynFrames - 1) / kSynFrames;
    return unsigned(m) * unsigned((groups + kBlock - 1) / kBlock);
}

// A5 retirement after iteration t: a frame whose decision satisfies H x = z
// (with early stopping) or that has run max_iter iterations stops; its
// iteration count, convergence flag and guard count are written to the
// outputs of frame orig[f], its decision later (k_emit) from the slot.
// Running frames are counted for this iteration's parity; the other parity's
// counter is cleared for the next.
__global__ void k_retire(DevState s, BatchAux a, int t, int max_iter, int early_stop, int32_t *out_iters,
                         uint8_t *out_conv, int32_t *out_guards) {
    const int f = blockIdx.x * blockDim.x + threadIdx.x;
    if (f == 0) s.count[2 * ((t + 1) & 1)] = 0;
    if (f >= s.F) return;
    if (s.active[f]) {
        const bool ok = s.unsat[f] == 0;
        if (ok && !a.conv[f]) {
            a.conv[f] = 1;
            a.iters[f] = t;
        }
        if ((ok && early_stop) || t >= max_iter) {
            s.active[f] = 0;
            if (!a.conv[f]) a.iters[f] = max_iter;
            const size_t o = size_t(a.orig[f]);
            out_iters[o] = a.iters[f];
            out_conv[o] = a.conv[f];
            if (out_guards) out_guards[o] = s.guards[f];
            a.pending[f] = 1;
        } else {
            atomicAdd(&s.count[2 * (t & 1)], 1u);
        }
    }
    s.unsat[f] = 0;
}

// Fig. 1 diagnostic: correct bits of the K source symbols (columns
// cols[0..K), or columns 0..K-1 when cols is null) of running frame f after
// iteration t, added to trace[f][t-1] (slot = frame: frames do not move when
// a trace is asked for).  Threads over frames, blockIdx.y over chunks of 128
// symbols.
__global__ void k_trace(DevState s, const uint8_t *truth, int n, int K, int p, int t, int max_iter,
                        int32_t *trace, const int32_t *cols) {
    const int f = blockIdx.x * blockDim.x + threadIdx.x;
    const int k0 = int(blockIdx.y) * 128, k1 = min(K, k0 + 128);
    if (f >= s.F || !s.active[f]) return;
    int c = 0;
    for (int k = k0; k < k1; ++k) {
        const int j = cols ? cols[k] : k;
        c += p - __popc(unsigned(s.xh[size_t(j) * s.Fp + f] ^ truth[size_t(f) * n + j]));
    }
    if (c) atomicAdd(&trace[size_t(f) * max_iter + (t - 1)], c);
}

__global__ void k_fill_i32(int32_t *p, size_t count, int32_t v) {
    const size_t t = size_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (t < count) p[t] = v;
}

// Decisions of finished frames to their rows of out: the frames in slots
// list[0..k) (before those slots are reused), or with list null every slot
// r < k still flagged pending.
__global__ void k_emit(DevState s, BatchAux a, const int32_t *list, int k, int n, uint8_t *out) {
    const size_t t = size_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (t >= size_t(k) * n) return;
    const int r = int(t / n), j = int(t % n);
    const int f = list ? list[r] : r;
    if (!list && !a.pending[f]) return;
    out[size_t(a.orig[f]) * n + j] = s.xh[size_t(j) * s.Fp + f];
}

// Compaction plan with R = *running frames running: the finished slots below R (holes)
// and the running slots at or above R (movers), both in increasing order;
// there are as many of each, written to *count.  One workgroup of 1024.
__global__ __launch_bounds__(1024) void k_plan_moves(const uint8_t *active, int F, const uint32_t *running,
                                                     int32_t *holes, int32_t *movers, uint32_t *count) {
    const int R = int(*running);
    __shared__ uint32_t hs[1024 / kWave], ms[1024 / kWave];
    __shared__ uint32_t hb, mb;
    const int lane = int(threadIdx.x) % kWave, wv = int(threadIdx.x) / kWave;
    if (threadIdx.x == 0) hb = mb = 0;
    __syncthreads();
    for (int c0 = 0; c0 < F; c0 += 1024) {
        const int f = c0 + int(threadIdx.x);
        const bool act = f < F && active[f];
        const bool hole = f < F && f < R && !act, mover = f >= R && act;
        const uint64_t bh = __ballot(hole), bm = __ballot(mover);
        if (lane == 0) {
            hs[wv] = uint32_t(__popcll(bh));
            ms[wv] = uint32_t(__popcll(bm));
        }
        __syncthreads();
        uint32_t oh = hb, om = mb;
        for (int w = 0; w < wv; ++w) {
            oh += hs[w];
            om += ms[w];
        }
        const uint64_t below = (uint64_t(1) << lane) - 1;
        if (hole) holes[oh + uint32_t(__popcll(bh & below))] = f;
        if (mover) movers[om + uint32_t(__popcll(bm & below))] = f;
        __syncthreads();
        if (threadIdx.x == 0) {
            for (int w = 0; w < 1024 / kWave; ++w) {
                hb += hs[w];
                mb += ms[w];
            }
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) *count = mb;
}

// Move running frame movers[k] into finished slot holes[k] (k = blockIdx.x):
// its q-messages, likelihoods and Markov-weighted likelihoods (the vectors
// that carry over between iterations), W floats per thread over
// blockIdx.y; block y = 0 also moves the per-slot scalars and the syndrome.
// Holes and movers are disjoint, so the copies never overlap.
__global__ __launch_bounds__(256) void k_move_frames(DevState s, BatchAux a, int E, int n, int K, int Kq, int Q,
                                                     int W, int m) {
    const int k = blockIdx.x;
    const int src = a.movers[k], dst = a.holes[k];
    const size_t o = (size_t(blockIdx.y) * blockDim.x + threadIdx.x) * W;
    const size_t per = size_t(E + n + K + Kq) * Q;
    if (o < per) {
        const size_t v = o / Q, e = o % Q;
        float *arr;
        size_t node;
        if (v < size_t(E)) {
            arr = s.Qm;
            node = v;
        } else if (v < size_t(E + n)) {
            arr = s.L;
            node = v - E;
        } else if (v < size_t(E + n + K)) {
            arr = s.Pr;
            node = v - E - n;
        } else {
            arr = s.Qp;
            node = v - E - n - K;
        }
        const float *from = arr + (node * s.Fp + src) * Q + e;
        float *to = arr + (node * s.Fp + dst) * Q + e;
        if (W == 4) *reinterpret_cast<float4 *>(to) = *reinterpret_cast<const float4 *>(from);
        else *reinterpret_cast<float2 *>(to) = *reinterpret_cast<const float2 *>(from);
    }
    if (blockIdx.y == 0) {
        if (a.z)
            for (int i = threadIdx.x; i < m; i += blockDim.x) a.z[size_t(dst) * m + i] = a.z[size_t(src) * m + i];
        if (threadIdx.x == 0) {
            a.orig[dst] = a.orig[src];
            a.iters[dst] = a.iters[src];
            a.conv[dst] = a.conv[src];
            a.pending[dst] = 0;
            s.guards[dst] = s.guards[src];
            s.active[dst] = 1;
            s.active[src] = 0;
        }
    }
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
// EL = 2, 4 or 8 entries per lane; the general class (rows <= 16, columns <=
// 8) allows EL = 2 or 4.  EL never exceeds q.  The default is EL = 4 (2 for
// q = 2), the fastest on every field measured; gfbp_code_set_shape /
// gfbp_tune choose another.
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
    int lel = std::min(2, max_lel(code));
    if (el > 0)
        for (int l = 1; l <= max_lel(code); ++l)
            if (el == (1 << l)) lel = l;
    sh.lel = lel;
    return sh;
}

// Frame stride of the workspace arrays: whole 64-frame tiles.
inline int frame_stride(int F) { return (F + kWave - 1) / kWave * kWave; }

inline unsigned tiled_blocks(int nodes, const DevState &s) {
    const long long waves = (long long)nodes * s.nb;
    return unsigned(std::max<long long>(1, (waves + (kBlock / kWave) - 1) / (kBlock / kWave)));
}

template <int P, int LG, int DCM, int DVM>
struct TiledLaunch {
    static void init(hipStream_t st, const DevCode &c, const DevState &s, const tiled::Chan &ch) {
        launch((tiled::k_init<P, LG>), dim3(tiled_blocks(c.n, s)), dim3(kBlock), 0, st, c, s, ch);
    }
    static void check(hipStream_t st, const DevCode &c, const DevState &s, const uint8_t *z, Snap sn) {
        launch((tiled::k_check<P, LG, DCM>), dim3(tiled_blocks(c.m, s)), dim3(kBlock), 0, st, c, s,
                           z, sn);
    }
    static void variable(hipStream_t st, const DevCode &c, const DevState &s, int prior_on, int wantQ, Snap sn) {
        launch((tiled::k_variable<P, LG, DVM>), dim3(tiled_blocks(c.n, s)), dim3(kBlock), 0, st, c,
                           s, prior_on, wantQ, sn);
    }
    static void variable_markov(hipStream_t st, const DevCode &c, const DevState &s, int prior_on, int wantQ,
                                Snap sn, const SweepPrior &sp) {
        launch((tiled::k_variable_markov<P, LG, DVM>), dim3(tiled_blocks(c.n, s)), dim3(kBlock), 0, st, c, s,
               prior_on, wantQ, sn, sp);
    }
    static void sus_level(hipStream_t st, const DevCode &c, const DevState &s, const uint8_t *z, int prior_on, int wantQ,
                          Snap sn, const SweepPrior &sp, const SusRec *recs, int nc) {
        const dim3 g(std::max(1u, unsigned(nc) * unsigned(s.nb)));
        const dim3 b(unsigned(std::max(1, std::min(c.max_dv, DVM))) * kWave);
        if (sp.on)
            launch((tiled::k_sus_level<P, LG, DCM, DVM, true>), g, b, 0, st, c, s, z, prior_on, wantQ, sn, sp, recs,
                   std::max(1, c.max_dv), nc);
        else
            launch((tiled::k_sus_level<P, LG, DCM, DVM, false>), g, b, 0, st, c, s, z, prior_on, wantQ, sn, sp, recs,
                   std::max(1, c.max_dv), nc);
    }
    static void sus_run(hipStream_t st, const DevCode &c, const DevState &s, const uint8_t *z, int prior_on, int wantQ,
                        Snap sn, const SweepPrior &sp, const SusRec *recs, int nc) {
        const dim3 g(std::max(1u, unsigned(s.nb)));
        const dim3 b(unsigned(std::max(1, std::min(c.max_dv, DVM))) * kWave);
        if (sp.on)
            launch((tiled::k_sus_run<P, LG, DCM, DVM, true>), g, b, 0, st, c, s, z, prior_on, wantQ, sn, sp, recs,
                   std::max(1, c.max_dv), nc);
        else
            launch((tiled::k_sus_run<P, LG, DCM, DVM, false>), g, b, 0, st, c, s, z, prior_on, wantQ, sn, sp, recs,
                   std::max(1, c.max_dv), nc);
    }
    // one sweep of levels (lv.segs)
    static void sweep(hipStream_t st, const DevCode &c, const DevState &s, const uint8_t *z, int prior_on, int wantQ,
                      Snap sn, const SweepPrior &sp, const gfbp_code::Levels &lv, Tracer *tr, int needQ, int t) {
        const int RS = std::max(1, c.max_dv);
        for (const auto &g : lv.segs) {
            if (tr) tr->begin();
            if (g.run) sus_run(st, c, s, z, prior_on, wantQ, sn, sp, lv.recs + size_t(g.c0) * RS, g.nc);
            else sus_level(st, c, s, z, prior_on, wantQ, sn, sp, lv.recs + size_t(g.c0) * RS, g.nc);
            // an assigned prior reads two neighbours' Q and L in place of Pr
            if (tr)
                tr->end_iter(g.run ? K_SUS_RUN : K_SUS_LEVEL,
                             4.0 * (1 << P) * (g.sibs + g.edges) + g.nc * (4.0 * (1 << P) * (1 + needQ) + 1) +
                                 (sp.on ? 8.0 * (1 << P) * g.src : 0.0),
                             g.edges * (1 << P), t);
        }
    }
    static void sequential(hipStream_t st, const DevCode &c, const DevState &s, const uint8_t *z, int prior_on,
                           int wantQ, Snap sn, const SweepPrior &sp) {
        const dim3 g(std::max(1u, unsigned(s.nb)));
        const dim3 b(unsigned(std::max(1, std::min(c.max_dv, DVM))) * kWave);
        if (sp.on)
            launch((tiled::k_sequential<P, LG, DCM, DVM, true>), g, b, 0, st, c, s, z, prior_on, wantQ, sn, sp);
        else
            launch((tiled::k_sequential<P, LG, DCM, DVM, false>), g, b, 0, st, c, s, z, prior_on, wantQ, sn, sp);
    }
    static void markov(hipStream_t st, const DevCode &c, const DevState &s, const float *M, const float *pi,
                       const float *mshape) {
        launch((tiled::k_markov<P, LG>), dim3(tiled_blocks(c.n_info, s)), dim3(kBlock), 0, st, c, s,
                           M, pi, mshape);
    }
    static constexpr int TF = kWave >> LG;
    static void tiles(hipStream_t st, const uint8_t *mask, int F, int Fp, int32_t *out, uint32_t *count) {
        launch(tiled::k_tiles, dim3(1), dim3(1024), 0, st, mask, F, Fp, TF, out, count);
    }
    static void vectors(hipStream_t st, const float *src, int n, const DevState &s, float *out) {
        const size_t tot = size_t(n) * s.F * (1 << P);
        launch((tiled::k_out_vectors<P>), dim3(unsigned((tot + 255) / 256)), dim3(256), 0, st, src, n,
                           s.F, s.Fp, out);
    }
};

// Per-thread pinned host slots for the iteration counts (4 iterations x 2,
// plus one for compaction) and their events; allocated once, kept for the
// life of the thread.
uint32_t *pinned_counts() {
    static thread_local uint32_t *p = nullptr;
    if (!p) {
        void *q = nullptr;
        if (hipHostMalloc(&q, 16 * sizeof(uint32_t), hipHostMallocDefault) != hipSuccess) return nullptr;
        p = static_cast<uint32_t *>(q);
    }
    return p;
}

hipEvent_t *count_events() {
    static thread_local hipEvent_t e[4] = {nullptr, nullptr, nullptr, nullptr};
    for (auto &x : e)
        if (!x && hipEventCreateWithFlags(&x, hipEventDisableTiming) != hipSuccess) return nullptr;
    return e;
}

template <int P, class K>
gfbp_status run_batch(const gfbp_code *code, const gfbp_batch *b, gfbp_result *out, DevState &s, BatchAux &a,
                      hipStream_t st, int needQ) {
    constexpr int Q = 1 << P;
    const DevCode &c = code->dev;
    const int F = s.F;
    const unsigned fb = unsigned((F + kBlock - 1) / kBlock);
    const Bytes bpf = bytes_per_frame(code, needQ, b->syndrome != nullptr);
    const double eq_frame = double(c.E) * Q;
    const uint8_t *z = b->syndrome ? a.z : nullptr;  // syndromes by slot
    const int prior_on = (b->prior != GFBP_PRIOR_UNIFORM) && c.n_info > 0;  // source columns read Pr
    const int markov = (b->prior == GFBP_PRIOR_MARKOV) && c.n_info > 0;     // ... refreshed by Eq. (7)
    // SUS priors assigned during the sweep (from iteration 2)
    const int insweep = markov && b->schedule == GFBP_SUS && (b->options & GFBP_OPT_PRIOR_IN_SWEEP);
    // PUS: the priors formed in the next iteration's variable step from the
    // previous iteration's pseudo-posteriors, the two buffers alternating;
    // not where posteriors or snapshots are read back (a frame that stopped
    // earlier keeps its last ones in the buffer of that iteration).  (For SUS
    // the same inside the level kernels made them slower than the separate
    // refresh they replaced: GF(8) N = 3000, 1.43e11 -> 1.33e11 edge-q/s.)
    const bool fused = markov && b->schedule == GFBP_PUS && !out->posterior && out->snap_iter <= 0;
    float *const qbuf[2] = {s.Qp, a.qp2};
    // moving frames keeps running frames in whole tiles; posteriors and
    // snapshots are read by slot at the end, so they keep frames in place
    const bool tracing = out->trace && b->truth;
    const bool compact = !(b->options & GFBP_OPT_NO_COMPACT) && !out->posterior && out->snap_iter <= 0 &&
                         !tracing && F > K::TF;
    const int Kp = prior_on ? c.n_info : 0;  // prior-weighted evidence moves with the frame
    Tracer tr(st);
    launch(k_state_init, dim3(fb), dim3(kBlock), 0, st, s, a);
    if (tracing) {
        const size_t cnt = size_t(F) * b->max_iter;
        launch(k_fill_i32, dim3(unsigned((cnt + 255) / 256)), dim3(256), 0, st, out->trace, cnt, 0);
    }
    if (b->syndrome) HIP_TRY(hipMemcpyAsync(a.z, b->syndrome, size_t(F) * c.m, hipMemcpyDeviceToDevice, st));
    const int ntiles = s.Fp / K::TF;
    K::tiles(st, s.active, F, s.Fp, s.tiles, s.count + 1);
    // the first list holds exactly the tiles holding a frame: ceil(F / TF) of
    // them (ntiles can be larger: the stride is padded to whole 64-frame tiles).
    s.act = s.tiles;
    s.nact = s.count + 1;
    s.nb = (F + K::TF - 1) / K::TF;
    if (markov) hipLaunchKernelGGL(tiled::k_markov_shape, dim3(1), dim3(kWave), 0, st, b->markov_M, Q, a.mshape);
    tiled::Chan ch{};
    ch.channel = b->channel;
    ch.prior = prior_on ? b->prior : GFBP_PRIOR_UNIFORM;
    ch.evidence = b->evidence;
    ch.static_per_symbol = b->static_per_symbol;
    ch.rx = b->rx;
    ch.erasure = b->erasure;
    ch.y = b->y;
    ch.lik = b->likelihood;
    ch.param = b->param;
    ch.pi = b->markov_pi;
    ch.static_P = b->static_prior;
    ch.chan_of = b->channel_of;
    tr.begin();
    K::init(st, c, s, ch);
    tr.end(K_INIT, double(F) * (4.0 * Q * (c.n + c.E) + c.n * 4.0 * P), 0);
    HIP_TRY(hipGetLastError());
    // The host stays one iteration ahead of the device: iteration t+1 is
    // launched with a grid bound taken from the counts of iteration t-1 (tile
    // lists only shrink, so that bound covers the list the kernels read on the
    // device), while the counts of iteration t come back asynchronously.
    std::vector<double> ran(size_t(b->max_iter) + 2, 0.0);  // frames iteration t ran
    ran[1] = F;
    // without allocations (gfbp_decode_batch_noalloc) the counts come back
    // into thread-local pageable memory, read after a stream synchronisation
    static thread_local uint32_t tls_counts[16];
    uint32_t *pin = g_no_alloc ? tls_counts : pinned_counts();
    if (!pin) return fail(GFBP_ENOMEM, "pinned host memory for the iteration counts");
    hipEvent_t *ev = g_no_alloc ? nullptr : count_events();
    if (!g_no_alloc && !ev) return fail(GFBP_EHIP, "events for the iteration counts");
    int last_read = 0;  // the latest iteration whose counts the host has read
    uint32_t known_running = uint32_t(F), known_tiles = uint32_t(s.nb);
    auto read_counts = [&](int t) -> gfbp_status {  // counts after iteration t
        if (ev) HIP_TRY(hipEventSynchronize(ev[t & 3]));
        else HIP_TRY(hipStreamSynchronize(st));
        known_running = pin[2 * (t & 3)];
        known_tiles = pin[2 * (t & 3) + 1];
        ran[size_t(t) + 1 < ran.size() ? size_t(t) + 1 : ran.size() - 1] = known_running;
        last_read = t;
        return GFBP_OK;
    };
    int t_end = 0;
    for (int t = 1; t <= b->max_iter; ++t) {
        t_end = t;
        const bool snap_now = (t == out->snap_iter);
        Snap sn{snap_now ? out->snap_q : nullptr, snap_now ? out->snap_r : nullptr};
        const int wantQ = needQ || (snap_now && out->snap_Q);
        if (fused) {
            s.Qp = qbuf[t & 1];
            s.Qprev = t >= 2 ? qbuf[(t - 1) & 1] : nullptr;
        }
        if (b->schedule == GFBP_PUS) {
            tr.begin();
            K::check(st, c, s, z, sn);
            tr.end_iter(K_CHECK, bpf.check, eq_frame, t);
            tr.begin();
            if (fused) {
                const SweepPrior sp{b->markov_M, b->markov_pi, a.mshape, t >= 2};
                K::variable_markov(st, c, s, prior_on, wantQ, sn, sp);
            } else {
                K::variable(st, c, s, prior_on, wantQ, sn);
            }
            // with the priors formed here: two neighbours' Q and L in place of Pr
            tr.end_iter(K_VARIABLE, bpf.variable + (fused && t >= 2 ? 8.0 * Q * c.n_info : 0.0), eq_frame, t);
        } else if (b->options & GFBP_OPT_SUS_STRICT) {
            const SweepPrior sp{b->markov_M, b->markov_pi, a.mshape, insweep && t >= 2};
            tr.begin();
            K::sequential(st, c, s, z, prior_on, wantQ, sn, sp);
            tr.end_iter(K_SEQUENTIAL, bpf.sequential + (sp.on ? 8.0 * Q * c.n_info : 0.0), eq_frame, t);
        } else {
            const SweepPrior sp{b->markov_M, b->markov_pi, a.mshape, insweep && t >= 2};
            K::sweep(st, c, s, z, prior_on, wantQ, sn, sp, code->lv[insweep ? 1 : 0], &tr, needQ, t);
        }
        if (snap_now && out->snap_Q) K::vectors(st, s.Qp, c.n, s, out->snap_Q);
        if (tracing) {
            const int Kt = c.n_info > 0 ? c.n_info : c.n;
            launch(k_trace, dim3(fb, unsigned((Kt + 127) / 128)), dim3(kBlock), 0, st, s, b->truth, c.n, Kt, P, t,
                   b->max_iter, out->trace, c.n_info > 0 ? c.chain_col : nullptr);
        }
        tr.begin();
        launch(k_syndrome, dim3(syndrome_blocks(c.m, F)), dim3(kBlock), 0, st, c, s, z);
        tr.end_iter(K_SYNDROME, bpf.syndrome, 0, t);
        tr.begin();
        launch(k_retire, dim3(fb), dim3(kBlock), 0, st, s, a, t, b->max_iter, b->early_stop,
               out->iters, out->converged, out->guards);
        tr.end_iter(K_RETIRE, 8.0, 0, t);
        HIP_TRY(hipGetLastError());
        if (t == b->max_iter) break;
        uint32_t *cnt_dev = s.count + 2 * (t & 1);  // [running after t, tiles listed]
        K::tiles(st, s.active, F, s.Fp, s.tiles + size_t(t & 1) * ntiles, cnt_dev + 1);
        HIP_TRY(hipMemcpyAsync(pin + 2 * (t & 3), cnt_dev, 2 * sizeof(uint32_t), hipMemcpyDeviceToHost, st));
        if (ev) HIP_TRY(hipEventRecord(ev[t & 3], st));
        if (t >= 2) {
            const gfbp_status rs = read_counts(t - 1);
            if (rs != GFBP_OK) return rs;
            if (known_running == 0) break;  // every frame finished by iteration t-1
        }
        s.act = s.tiles + size_t(t & 1) * ntiles;
        s.nact = cnt_dev + 1;
        s.nb = int(known_tiles);  // counts of iteration t-1 (or the first list): a bound on the list of t
        if (markov && !insweep && !fused) {
            tr.begin();
            K::markov(st, c, s, b->markov_M, b->markov_pi, a.mshape);
            tr.end_iter(K_MARKOV, bpf.markov, 0, t + 1);
        }
        if (compact && t >= 2 && uint64_t(known_running) * 32 < uint64_t(known_tiles) * K::TF * 31) {
            // running frames filled less than 31/32 of their tiles: move the
            // frames still running after iteration t into the finished slots
            // below their count, then list the (now whole) tiles
            launch(k_plan_moves, dim3(1), dim3(1024), 0, st, s.active, F, cnt_dev, a.holes, a.movers, s.count + 8);
            HIP_TRY(hipMemcpyAsync(pin + 8, s.count + 8, sizeof(uint32_t), hipMemcpyDeviceToHost, st));
            HIP_TRY(hipMemcpyAsync(pin + 2 * (t & 3), cnt_dev, 2 * sizeof(uint32_t), hipMemcpyDeviceToHost, st));
            HIP_TRY(hipStreamSynchronize(st));
            const uint32_t nm = pin[8];
            known_running = pin[2 * (t & 3)];
            known_tiles = pin[2 * (t & 3) + 1];
            ran[size_t(t) + 1] = known_running;
            last_read = t;
            if (known_running == 0) break;
            if (nm > 0) {
                const size_t ne = size_t(nm) * c.n;
                launch(k_emit, dim3(unsigned((ne + 255) / 256)), dim3(256), 0, st, s, a, a.holes, int(nm), c.n,
                       out->xhat);
                const int W = Q >= 4 ? 4 : 2;
                const int Kq = insweep || fused ? c.n : 0;  // the next step's priors read the source columns' Q
                const size_t per = size_t(c.E + c.n + Kp + Kq) * Q;
                const unsigned chunks = unsigned((per / W + 255) / 256);
                tr.begin();
                launch(k_move_frames, dim3(nm, chunks), dim3(256), 0, st, s, a, c.E, c.n, Kp, Kq, Q, W, c.m);
                tr.end(K_COMPACT, double(nm) * (8.0 * per + 2.0 * c.m), 0);
                K::tiles(st, s.active, F, s.Fp, s.tiles + size_t(t & 1) * ntiles, cnt_dev + 1);
                known_tiles = (known_running + K::TF - 1) / K::TF;
                s.nb = int(known_tiles);
                HIP_TRY(hipGetLastError());
            } else {
                s.nb = int(known_tiles);
            }
        }
    }
    (void)t_end;
    tr.begin();
    {
        const size_t ne = size_t(F) * c.n;
        launch(k_emit, dim3(unsigned((ne + 255) / 256)), dim3(256), 0, st, s, a, nullptr, F, c.n,
                           out->xhat);
    }
    tr.end(K_OUTPUT, double(F) * c.n * 2.0, 0);
    if (out->posterior) {
        tr.begin();
        K::vectors(st, s.Qp, c.n, s, out->posterior);
        tr.end(K_OUTPUT, double(F) * c.n * 8.0 * Q, 0);
    }
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipStreamSynchronize(st));
    if (tr.on) {
        // iterations whose counts were not read: the frames they ran
        for (int t = last_read + 1; t < t_end; ++t) ran[size_t(t) + 1] = pin[2 * (t & 3)];
    }
    tr.flush(ran);
    return GFBP_OK;
}

template <int P, int LEL>
gfbp_status run_lel(const gfbp_code *code, const gfbp_batch *b, gfbp_result *out, DevState &s, BatchAux &a,
                    hipStream_t st, int needQ, bool small) {
    if constexpr (LEL <= 3 && LEL <= P) {
        if (small) return run_batch<P, TiledLaunch<P, P - LEL, 6, 4>>(code, b, out, s, a, st, needQ);
    }
    if constexpr (LEL <= 2 && LEL <= P) {
        if (!small) return run_batch<P, TiledLaunch<P, P - LEL, 16, 8>>(code, b, out, s, a, st, needQ);
    }
    return fail(GFBP_EUNSUPPORTED, "no kernel for this shape");
}

template <int P>
gfbp_status run_any(const gfbp_code *code, const gfbp_batch *b, gfbp_result *out, DevState &s, BatchAux &a,
                    hipStream_t st, int needQ) {
    const Shape sh = shape_of(code, b->schedule);
    switch (sh.lel) {
        case 1: return run_lel<P, 1>(code, b, out, s, a, st, needQ, sh.small);
        case 2: return run_lel<P, 2>(code, b, out, s, a, st, needQ, sh.small);
        case 3: return run_lel<P, 3>(code, b, out, s, a, st, needQ, sh.small);
        default: return fail(GFBP_EUNSUPPORTED, "bad shape");
    }
}

// ------------------------------------------------------ whole decodes in LDS
// LDS a workgroup may use on the current device (queried once per device).
int lds_limit() {
    static std::mutex mu;
    static std::vector<int> per_dev;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0) return 0;
    std::lock_guard<std::mutex> g(mu);
    if (size_t(dev) >= per_dev.size()) per_dev.resize(size_t(dev) + 1, -1);
    if (per_dev[size_t(dev)] < 0) {
        int v = 0;
        if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess) v = 0;
        per_dev[size_t(dev)] = std::max(0, v);
    }
    return per_dev[size_t(dev)];
}

// Whether a one-code batch may be decoded in LDS: q <= 8, outputs no more
// than decisions, iterations, convergence and guards, the level sweep for SUS
// with priors from the previous iteration.
bool onchip_allowed(const gfbp_code *code, const gfbp_batch *b, const gfbp_result *out) {
    if (b->options & GFBP_OPT_NO_ONCHIP) return false;
    if (code->info.p > onchip::kMaxP) return false;
    // the packed graph: 16-bit edge, column and row indices
    if (code->info.n_edges >= 65536 || code->info.n >= 65536 || code->info.m >= 65536) return false;
    if (out->posterior || out->snap_iter > 0 || (out->trace && b->truth)) return false;
    if (b->schedule == GFBP_SUS && (b->options & (GFBP_OPT_SUS_STRICT | GFBP_OPT_PRIOR_IN_SWEEP))) return false;
    return true;
}

// LDS layout of the in-LDS decode of this batch (fw = 0: a frame does not
// fit).  Frames per workgroup: as many as fit in half the limit (two
// workgroups per compute unit), at least one if one fits in all of it.  A
// decode's time is mostly that of its slowest frames (those that run to
// max_iter), which more frames per workgroup only delay: on GF(4) N = 504,
// SUS, 2000 frames, the whole LDS (four frames per workgroup) took 15.6 ms
// and half of it (one) 11.0 ms; with every frame running 200 iterations
// the four frames per workgroup were faster (137 against 220 us per
// iteration).
onchip::Layout onchip_layout(const gfbp_code *code, const gfbp_batch *b, int limit) {
    const bool pus = b->schedule == GFBP_PUS;
    const int K = code->info.n_info;
    return onchip_layout_for(code->info.q, code->info.n_edges, code->info.n, code->info.m, K,
                             code->info.max_col_degree, int(code->lv[0].ptr.size()) - 1, pus,
                             b->prior != GFBP_PRIOR_UNIFORM && K > 0, b->prior == GFBP_PRIOR_MARKOV && K > 0,
                             b->n_frames, limit);
}

// Allows the in-LDS kernel of this code's degree class `bytes` of dynamic
// LDS (beyond the default bound this must be set per kernel); false (the
// runtime's error cleared) when the runtime refuses.
template <int P, int LG>
bool onchip_allow_lds(const gfbp_code *code, int bytes) {
    const void *kern = small_class(code) ? reinterpret_cast<const void *>(&onchip::k_onchip<P, LG, 6, 4>)
                                         : reinterpret_cast<const void *>(&onchip::k_onchip<P, LG, kDcMax, kDvMax>);
    if (hipFuncSetAttribute(kern, hipFuncAttributeMaxDynamicSharedMemorySize, bytes) == hipSuccess) return true;
    (void)hipGetLastError();
    return false;
}

// The whole decode in LDS; *ran false (nothing launched) when the runtime
// does not allow the kernel its LDS, and the caller takes the tiled kernels.
template <int P, int LG>
gfbp_status run_onchip(const gfbp_code *code, const gfbp_batch *b, gfbp_result *out, DevState &s, BatchAux &a,
                       hipStream_t st, int needQ, const onchip::Layout &ly, bool *ran) {
    constexpr int Q = 1 << P;
    const DevCode &c = code->dev;
    const int F = s.F;
    *ran = onchip_allow_lds<P, LG>(code, ly.total);
    if (!*ran) return GFBP_OK;
    const unsigned fb = unsigned((F + kBlock - 1) / kBlock);
    const int prior_on = (b->prior != GFBP_PRIOR_UNIFORM) && c.n_info > 0;
    const int markov = (b->prior == GFBP_PRIOR_MARKOV) && c.n_info > 0;
    Tracer tr(st);
    constexpr int TF = kWave >> LG;
    launch(k_state_init, dim3(fb), dim3(kBlock), 0, st, s, a);
    // the initialisation kernel's tile list (every frame), at the in-LDS
    // kernel's lanes per vector
    launch(tiled::k_tiles, dim3(1), dim3(1024), 0, st, s.active, F, s.Fp, TF, s.tiles, s.count + 1);
    s.act = s.tiles;
    s.nact = s.count + 1;
    s.nb = (F + TF - 1) / TF;
    if (markov) hipLaunchKernelGGL(tiled::k_markov_shape, dim3(1), dim3(kWave), 0, st, b->markov_M, Q, a.mshape);
    tiled::Chan ch{};
    ch.channel = b->channel;
    ch.prior = prior_on ? b->prior : GFBP_PRIOR_UNIFORM;
    ch.evidence = b->evidence;
    ch.static_per_symbol = b->static_per_symbol;
    ch.rx = b->rx;
    ch.erasure = b->erasure;
    ch.y = b->y;
    ch.lik = b->likelihood;
    ch.param = b->param;
    ch.pi = b->markov_pi;
    ch.static_P = b->static_prior;
    ch.chan_of = b->channel_of;
    tr.begin();
    launch((tiled::k_init<P, LG>), dim3(tiled_blocks(c.n, s)), dim3(kBlock), 0, st, c, s, ch);
    tr.end(K_INIT, double(F) * (4.0 * Q * (c.n + c.E) + c.n * 4.0 * P), 0);
    onchip::Args oa{};
    oa.c = c;
    oa.Qm = s.Qm;
    oa.L = s.L;
    oa.Pr = s.Pr;
    oa.guards0 = s.guards;
    oa.F = F;
    oa.Fp = s.Fp;
    oa.z = b->syndrome;
    oa.schedule = b->schedule;
    oa.max_iter = b->max_iter;
    oa.early_stop = b->early_stop;
    oa.prior_on = prior_on;
    oa.markov = markov;
    oa.wantQ = markov ? needQ : 0;  // (posteriors are not decoded in LDS)
    oa.M = b->markov_M;
    oa.pi = b->markov_pi;
    oa.mshape = a.mshape;
    oa.recs = code->lv[0].recs;
    oa.lvl = code->lv[0].dptr;
    oa.nlev = int(code->lv[0].ptr.size()) - 1;
    oa.rs = std::max(1, c.max_dv);
    oa.xhat = out->xhat;
    oa.iters = out->iters;
    oa.conv = out->converged;
    oa.guards = out->guards;
    oa.lay = ly;
    // HBM: the initial state and syndromes in, the results out
    const double hbm = double(F) * (4.0 * Q * (c.E + c.n + (prior_on ? c.n_info : 0)) + 4.0 +
                                    (b->syndrome ? c.m : 0) + c.n + 9.0);
    // the degree class bounds the rows' siblings and the columns' r-vectors
    // held in registers
    auto go = [&](auto kern) {
        tr.begin();
        launch(kern, dim3(unsigned((F + ly.fw - 1) / ly.fw)), dim3(onchip::kThreads), size_t(ly.total), st, oa);
    };
    if (small_class(code)) go(onchip::k_onchip<P, LG, 6, 4>);
    else go(onchip::k_onchip<P, LG, kDcMax, kDvMax>);
    tr.end(K_ONCHIP, hbm, 0);
    HIP_TRY(hipGetLastError());
    if (tr.on) {
        HIP_TRY(hipStreamSynchronize(st));
        tr.flush();
    }
    return GFBP_OK;
}

// ======================================================================= sessions
// Continuous batching: a session holds S resident frame slots of one code;
// frames are admitted into free slots as they arrive, every step advances all
// running slots, finished slots are collected by poll and reused.
}  // namespace

struct gfbp_graph {
    hipGraph_t graph;
    hipGraphExec_t exec;
    int iters;
};

// Device view of a session (trivially copyable: passed to kernels).
struct SessDev {
    DevState st;  // message state for S slots (F = S)
    int S, max_iter;
    uint8_t *rx, *er, *z, *chan, *mark;
    float *y, *param;
    int32_t *iters;
    uint8_t *conv, *fresh, *done, *xout;
    int32_t *pairs, *list, *res;
    uint64_t *t_admit, *t_done, *ts;  // [S] device clock at admission / retirement; [2][S] of listed slots
};

struct gfbp_session {
    const gfbp_code *code = nullptr;
    int S = 0, schedule = 0, max_iter = 0, has_z = 0, options = 0, markov = 0;
    int tf = 0, ntiles = 0;
    void *mem = nullptr;
    size_t bytes = 0;
    SessDev dv{};
    float *M = nullptr, *pi = nullptr, *mshape = nullptr;
    int32_t *ftiles = nullptr;
    uint32_t *aux = nullptr;  // [0] fresh tiles, [1] finished slots, [2..3] running tiles by parity
    int parity = 0;
    // host
    std::vector<int64_t> id;
    std::vector<int32_t> free_slots;  // sorted descending: back() is the lowest free slot
    int running = 0;                  // admitted and not yet collected
    void *pin = nullptr;              // pinned host staging
    size_t pin_bytes = 0;
    gfbp_status (*init_fn)(gfbp_session *, int, hipStream_t) = nullptr;
    gfbp_status (*step_fn)(gfbp_session *, int, hipStream_t, int) = nullptr;
    // GFBP_OPT_STEP_GRAPHS: captured steps by (iterations, launch bound, parity)
    struct StepGraph {
        int iters, nb, parity;
        hipGraph_t graph;
        hipGraphExec_t exec;
    };
    std::vector<StepGraph> graphs;
};

namespace {

struct AdmitIn {
    const float *param;
    const uint8_t *rx, *erasure, *syndrome, *channel, *markov;
    const float *y;
};

// Copy admitted frames' inputs into their slots and reset the slots' state.
__global__ void k_admit(SessDev s, AdmitIn in, int n, int m, int p) {
    const int k = blockIdx.x;
    const int slot = s.pairs[2 * k], src = s.pairs[2 * k + 1];
    for (int j = threadIdx.x; j < n; j += blockDim.x) {
        if (in.rx) s.rx[size_t(slot) * n + j] = in.rx[size_t(src) * n + j];
        if (in.erasure) s.er[size_t(slot) * n + j] = in.erasure[size_t(src) * n + j];
    }
    if (in.y)
        for (int t = threadIdx.x; t < n * p; t += blockDim.x) s.y[size_t(slot) * n * p + t] = in.y[size_t(src) * n * p + t];
    if (s.z)
        for (int i = threadIdx.x; i < m; i += blockDim.x)
            s.z[size_t(slot) * m + i] = in.syndrome ? in.syndrome[size_t(src) * m + i] : 0;
    if (threadIdx.x == 0) {
        s.param[slot] = in.param ? in.param[src] : 0.0f;
        s.chan[slot] = in.channel[src];
        s.mark[slot] = in.markov ? in.markov[src] : 0;
        s.fresh[slot] = 1;
        s.st.active[slot] = 1;
        s.st.unsat[slot] = 0;
        s.st.guards[slot] = 0;
        s.iters[slot] = 0;
        s.conv[slot] = 0;
        s.done[slot] = 0;
        s.t_admit[slot] = uint64_t(wall_clock64());
    }
}

__global__ void k_clear_fresh(SessDev s, int k) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < k) s.fresh[s.pairs[2 * t]] = 0;
}

// Per-slot retirement after one more iteration of that slot.
__global__ void k_session_retire(SessDev s) {
    const int f = blockIdx.x * blockDim.x + threadIdx.x;
    if (f >= s.S) return;
    if (s.st.active[f]) {
        const int t = ++s.iters[f];
        const bool ok = s.st.unsat[f] == 0;
        if (ok) s.conv[f] = 1;
        if (ok || t >= s.max_iter) {
            s.st.active[f] = 0;
            s.done[f] = 1;
            s.t_done[f] = uint64_t(wall_clock64());
        }
    }
    s.st.unsat[f] = 0;
}

// Gather the decisions [k][n] and (iterations, converged) of listed slots.
__global__ void k_collect(SessDev s, int k, int n) {
    const size_t t = size_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (t >= size_t(k) * n) return;
    const int r = int(t / n), j = int(t % n);
    const int slot = s.list[r];
    s.xout[t] = s.st.xh[size_t(j) * s.st.Fp + slot];
    if (j == 0) {
        s.res[2 * r] = s.iters[slot];
        s.res[2 * r + 1] = s.conv[slot];
        s.ts[2 * r] = s.t_admit[slot];
        s.ts[2 * r + 1] = s.t_done[slot];
        s.done[slot] = 0;
    }
}

template <int P, class K>
struct SessionRun {
    // initialise the slots flagged fresh (k_admit), then rebuild the running list
    static gfbp_status init(gfbp_session *ss, int nadm, hipStream_t st) {
        const DevCode &c = ss->code->dev;
        DevState s = ss->dv.st;
        K::tiles(st, ss->dv.fresh, s.F, s.Fp, ss->ftiles, ss->aux + 0);
        s.act = ss->ftiles;
        s.nact = ss->aux + 0;
        s.nb = std::min(ss->ntiles, nadm);
        s.fresh = ss->dv.fresh;
        tiled::Chan ch{};
        ch.channel = GFBP_CH_BSC;  // per-slot channel kinds override this
        ch.param = ss->dv.param;
        ch.rx = ss->dv.rx;
        ch.erasure = ss->dv.er;
        ch.y = ss->dv.y;
        ch.prior = ss->markov ? GFBP_PRIOR_MARKOV : GFBP_PRIOR_UNIFORM;  // per-slot flags in s.mark
        ch.pi = ss->pi;
        K::init(st, c, s, ch);
        hipLaunchKernelGGL(k_clear_fresh, dim3((nadm + 255) / 256), dim3(256), 0, st, ss->dv, nadm);
        K::tiles(st, s.active, s.F, s.Fp, ss->dv.st.tiles + size_t(ss->parity) * ss->ntiles, ss->aux + 2 + ss->parity);
        HIP_TRY(hipGetLastError());
        return GFBP_OK;
    }
    // `iters` iterations of every running slot, no host synchronisation.
    // nb: the launch bound in tiles (at least the tiles holding a running
    // frame; every slot's tile for a graph that must outlive admissions).
    static gfbp_status step(gfbp_session *ss, int iters, hipStream_t st, int nb) {
        const gfbp_code *code = ss->code;
        const DevCode &c = code->dev;
        DevState s = ss->dv.st;
        s.nb = std::min(ss->ntiles, nb);
        if (s.nb == 0) return GFBP_OK;
        const Snap sn{nullptr, nullptr};
        const SweepPrior sp{ss->M, ss->pi, ss->mshape, 0};  // sessions refresh priors after each iteration
        const int needQ = ss->markov;
        const uint8_t *z = ss->has_z ? ss->dv.z : nullptr;
        const unsigned fb = unsigned((s.F + kBlock - 1) / kBlock);
        for (int it = 0; it < iters; ++it) {
            s.act = ss->dv.st.tiles + size_t(ss->parity) * ss->ntiles;
            s.nact = ss->aux + 2 + ss->parity;
            if (ss->schedule == GFBP_PUS) {
                K::check(st, c, s, z, sn);
                K::variable(st, c, s, ss->markov, needQ, sn);
            } else if (ss->options & GFBP_OPT_SUS_STRICT) {
                K::sequential(st, c, s, z, ss->markov, needQ, sn, sp);
            } else {
                K::sweep(st, c, s, z, ss->markov, needQ, sn, sp, code->lv[0], nullptr, needQ, 0);
            }
            hipLaunchKernelGGL(k_syndrome, dim3(syndrome_blocks(c.m, s.F)), dim3(kBlock), 0, st, c, s, z);
            hipLaunchKernelGGL(k_session_retire, dim3(fb), dim3(kBlock), 0, st, ss->dv);
            ss->parity ^= 1;
            K::tiles(st, s.active, s.F, s.Fp, ss->dv.st.tiles + size_t(ss->parity) * ss->ntiles, ss->aux + 2 + ss->parity);
            if (ss->markov) {
                s.act = ss->dv.st.tiles + size_t(ss->parity) * ss->ntiles;
                s.nact = ss->aux + 2 + ss->parity;
                K::markov(st, c, s, ss->M, ss->pi, ss->mshape);
            }
        }
        HIP_TRY(hipGetLastError());
        return GFBP_OK;
    }
};

template <int P, int LEL>
bool session_bind_lel(gfbp_session *ss, bool small) {
    if constexpr (LEL <= 3 && LEL <= P) {
        if (small) {
            using K = TiledLaunch<P, P - LEL, 6, 4>;
            ss->init_fn = &SessionRun<P, K>::init;
            ss->step_fn = &SessionRun<P, K>::step;
            ss->tf = K::TF;
            return true;
        }
    }
    if constexpr (LEL <= 2 && LEL <= P) {
        if (!small) {
            using K = TiledLaunch<P, P - LEL, 16, 8>;
            ss->init_fn = &SessionRun<P, K>::init;
            ss->step_fn = &SessionRun<P, K>::step;
            ss->tf = K::TF;
            return true;
        }
    }
    return false;
}

template <int P>
bool session_bind(gfbp_session *ss) {
    const Shape sh = shape_of(ss->code, ss->schedule);
    switch (sh.lel) {
        case 1: return session_bind_lel<P, 1>(ss, sh.small);
        case 2: return session_bind_lel<P, 2>(ss, sh.small);
        case 3: return session_bind_lel<P, 3>(ss, sh.small);
        default: return false;
    }
}

// Workspace carving, shared by size query and decode.
struct Carve {
    size_t Qm, R, L, Pr, Qp, Qp2, xh, unsat, active, count, tiles, guards, orig, iters, conv, z, holes, movers,
        pending, mshape, total;
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
    c.Pr = take(prior != GFBP_PRIOR_UNIFORM ? K * F * Q * 4 : 0);
    c.Qp = take(n * F * Q * 4);
    c.Qp2 = take(schedule == GFBP_PUS && prior == GFBP_PRIOR_MARKOV ? n * F * Q * 4 : 0);
    c.xh = take(n * F);
    c.unsat = take(size_t(F_) * 4);
    c.active = take(size_t(F_));
    c.count = take(64);
    c.tiles = take(2 * F * 4);
    c.guards = take(F * 4);
    c.orig = take(F * 4);
    c.iters = take(F * 4);
    c.conv = take(F);
    c.z = take(F * size_t(code->info.m));
    c.holes = take(F * 4);
    c.movers = take(F * 4);
    c.pending = take(F);
    c.mshape = take(16);
    c.total = off;
    return c;
}

// Device memory of a session, carved from one allocation.
struct SessCarve {
    size_t Qm, R, L, Pr, Qp, xh, unsat, active, count, tiles, guards;
    size_t rx, er, y, param, z, chan, mark, iters, conv, fresh, done, xout, pairs, list, res, ftiles, aux, M, pi, mshape;
    size_t t_admit, t_done, ts;
    size_t total;
};

SessCarve session_carve(const gfbp_code *code, int S, int schedule, int markov, int has_z) {
    const size_t E = code->info.n_edges, n = code->info.n, m = code->info.m, K = code->info.n_info,
                 Q = code->info.q, p = code->info.p, F = size_t(S);
    SessCarve c{};
    size_t off = 0;
    auto take = [&](size_t bytes) { size_t o = off; off += align256(bytes ? bytes : 1); return o; };
    c.Qm = take(E * Q * F * 4);
    c.R = take(schedule == GFBP_PUS ? E * Q * F * 4 : 0);
    c.L = take(n * Q * F * 4);
    c.Pr = take(markov ? K * Q * F * 4 : 0);
    c.Qp = take(markov ? n * Q * F * 4 : 0);
    c.xh = take(n * F);
    c.unsat = take(F * 4);
    c.active = take(F);
    c.count = take(16);
    c.tiles = take(2 * F * 4);
    c.guards = take(F * 4);
    c.rx = take(n * F);
    c.er = take(n * F);
    c.y = take(n * p * F * 4);
    c.param = take(F * 4);
    c.z = take(has_z ? m * F : 0);
    c.chan = take(F);
    c.mark = take(F);
    c.iters = take(F * 4);
    c.conv = take(F);
    c.fresh = take(F);
    c.done = take(F);
    c.xout = take(n * F);
    c.pairs = take(2 * F * 4);
    c.list = take(F * 4);
    c.res = take(2 * F * 4);
    c.ftiles = take(F * 4);
    c.aux = take(64);
    c.M = take(Q * Q * 4);
    c.pi = take(Q * 4);
    c.mshape = take(16);
    c.t_admit = take(F * 8);
    c.t_done = take(F * 8);
    c.ts = take(2 * F * 8);
    c.total = off;
    return c;
}

// Slots of a session: n_slots rounded up to whole 64-slot tiles, or with
// n_slots = 0 the most whole tiles whose state fits device_bytes (0 if none).
int session_slots(const gfbp_code *code, const gfbp_session_desc *d) {
    if (d->n_slots > 0) return (d->n_slots + kWave - 1) / kWave * kWave;
    if (d->device_bytes <= 0) return 0;
    const int mk = d->markov_M != nullptr;
    auto fits = [&](long long tiles) {
        return session_carve(code, int(tiles * kWave), d->schedule, mk, d->has_syndrome).total <=
               size_t(d->device_bytes);
    };
    long long lo = 0, hi = 1;
    while (hi < (1 << 24) && fits(hi)) hi *= 2;  // the largest fitting count lies in [lo, hi)
    lo = hi / 2;
    if (!fits(std::max(1LL, lo))) return 0;
    while (hi - lo > 1) {
        const long long mid = (lo + hi) / 2;
        if (fits(mid)) lo = mid;
        else hi = mid;
    }
    return int(lo * kWave);
}




// ---------------------------------------------------------------- persistent path
// Plan of a batch for the persistent kernel: the codes with frames (groups),
// the frames of each in batch order, every frame's input offsets, the work
// list of each degree class, and the workspace layout.
struct PersistPlan {
    int F = 0, lel = 2, waves = 8;
    std::vector<int> gcode;                       // code index of each group
    std::vector<std::vector<int32_t>> gframe;     // frames of each group
    std::vector<int64_t> off_n, off_np, off_nq, off_m;  // [F]
    // work lists by (degree class, field): list 6 * cls + p - 1
    std::vector<persist::Work> work[12];
    std::vector<double> top;                      // largest tile's work of each list
    // workspace
    size_t o_off_n = 0, o_off_np = 0, o_off_nq = 0, o_off_m = 0, o_groups = 0, o_work[12] = {}, o_next = 0, o_mshape = 0;
    struct G {
        size_t gframe, Qm, R, L, Pr, Qp, xh, unsat, active, guards, iters, conv, z;
        int Fp;
    };
    std::vector<G> g;
    size_t total = 0;
};

inline int persist_tf(int p, int lel) {  // frames per tile: 64 x entries per lane / q
    const int l = std::min(lel, p);
    return kWave >> (p - l);
}

// log2 entries per lane of field 2^p's tiles in degree class cls (0: narrow)
// for the batch's shape lel: at most 2 in the general class, and small fields
// taken down so that a tile holds at most 16 frames (at least 2 entries per
// lane).  A tile is decoded by one workgroup, so tiles of 64 frames of a long
// low-order code would set the running time of a whole uneven batch alone.
inline int persist_lel(int p, int lel, int cls) {
    const int l = std::min(cls == 0 ? lel : std::min(lel, 2), std::max(1, p - 2));
    return std::min(l, p);
}

gfbp_status persist_plan(const gfbp_code *const *codes, int nc, const gfbp_batch *b, PersistPlan &pl) {
    const int F = b->n_frames;
    pl.F = F;
    pl.lel = 2;
    if (b->persist_el) {
        if (b->persist_el != 2 && b->persist_el != 4 && b->persist_el != 8)
            return fail(GFBP_EUNSUPPORTED, "persist_el must be 2, 4 or 8");
        pl.lel = b->persist_el == 2 ? 1 : b->persist_el == 4 ? 2 : 3;
    }
    if (pl.lel == 1) pl.lel = 2;  // entries per lane 2 runs as 4 (the q = 2 field takes 2 in every shape)
    pl.waves = b->persist_waves ? b->persist_waves : 8;
    if (pl.waves < 1 || pl.waves > 8) return fail(GFBP_EINVAL, "persist_waves must be 1..8");
    std::vector<int> count(size_t(nc), 0), gid(size_t(nc), -1);
    for (int f = 0; f < F; ++f) {
        const int k = b->code_index ? b->code_index[f] : 0;
        if (k < 0 || k >= nc) return fail(GFBP_EINVAL, "code_index out of range");
        count[size_t(k)]++;
    }
    for (int k = 0; k < nc; ++k)
        if (count[size_t(k)]) {
            gid[size_t(k)] = int(pl.gcode.size());
            pl.gcode.push_back(k);
            pl.gframe.emplace_back();
            pl.gframe.back().reserve(size_t(count[size_t(k)]));
        }
    pl.off_n.resize(size_t(F));
    pl.off_np.resize(size_t(F));
    pl.off_nq.resize(size_t(F));
    pl.off_m.resize(size_t(F));
    int64_t on = 0, onp = 0, onq = 0, om = 0;
    for (int f = 0; f < F; ++f) {
        const int k = b->code_index ? b->code_index[f] : 0;
        const gfbp_code_info &ci = codes[k]->info;
        pl.off_n[size_t(f)] = on;
        pl.off_np[size_t(f)] = onp;
        pl.off_nq[size_t(f)] = onq;
        pl.off_m[size_t(f)] = om;
        on += ci.n;
        onp += int64_t(ci.n) * ci.p;
        onq += int64_t(ci.n) * ci.q;
        om += ci.m;
        pl.gframe[size_t(gid[size_t(k)])].push_back(f);
    }
    if ((b->options & GFBP_OPT_PRIOR_IN_SWEEP))
        return fail(GFBP_EUNSUPPORTED, "the persistent path refreshes priors after each iteration");
    // work lists, largest tile first
    struct Cand {
        double cost;
        persist::Work w;
    };
    std::vector<Cand> cand[12];
    for (size_t g = 0; g < pl.gcode.size(); ++g) {
        const gfbp_code *code = codes[pl.gcode[g]];
        const int cls = small_class(code) ? 0 : 1;
        const int TF = persist_tf(code->info.p, persist_lel(code->info.p, pl.lel, cls));
        const int Fg = int(pl.gframe[g].size());
        const int list = 6 * cls + code->info.p - 1;
        for (int t = 0; t * TF < Fg; ++t) {
            const int nf = std::min(TF, Fg - t * TF);
            cand[list].push_back({double(code->info.n_edges) * code->info.q * nf, {int32_t(g), int32_t(t)}});
        }
    }
    pl.top.assign(12, 0.0);
    for (int l = 0; l < 12; ++l) {
        std::stable_sort(cand[l].begin(), cand[l].end(), [](const Cand &x, const Cand &y) { return x.cost > y.cost; });
        pl.work[l].clear();
        for (const auto &c : cand[l]) pl.work[l].push_back(c.w);
        if (!cand[l].empty()) pl.top[size_t(l)] = cand[l].front().cost;
    }
    // workspace layout
    size_t off = 0;
    auto take = [&](size_t bytes) { size_t o = off; off += align256(bytes ? bytes : 1); return o; };
    pl.o_off_n = take(8 * size_t(F));
    pl.o_off_np = take(8 * size_t(F));
    pl.o_off_nq = take(8 * size_t(F));
    pl.o_off_m = take(8 * size_t(F));
    pl.o_groups = take(sizeof(persist::Group) * pl.gcode.size());
    for (int l = 0; l < 12; ++l) pl.o_work[l] = take(sizeof(persist::Work) * pl.work[l].size());
    pl.o_next = take(4 * 12);
    pl.o_mshape = take(16);
    const int prior_on = b->prior != GFBP_PRIOR_UNIFORM, markov = b->prior == GFBP_PRIOR_MARKOV;
    pl.g.resize(pl.gcode.size());
    for (size_t g = 0; g < pl.gcode.size(); ++g) {
        const gfbp_code_info &ci = codes[pl.gcode[g]]->info;
        const size_t E = ci.n_edges, n = ci.n, K = ci.n_info, Q = ci.q, m = ci.m;
        const size_t Fg = pl.gframe[g].size(), Fp = size_t(frame_stride(int(Fg)));
        PersistPlan::G &G = pl.g[g];
        G.Fp = int(Fp);
        G.gframe = take(4 * Fg);
        G.Qm = take(E * Fp * Q * 4);
        G.R = take(b->schedule == GFBP_PUS ? E * Fp * Q * 4 : 0);
        G.L = take(n * Fp * Q * 4);
        G.Pr = take(prior_on ? K * Fp * Q * 4 : 0);
        G.Qp = take(markov ? n * Fp * Q * 4 : 0);
        G.xh = take(n * Fp);
        G.unsat = take(Fp * 4);
        G.active = take(Fp);
        G.guards = take(Fp * 4);
        G.iters = take(Fp * 4);
        G.conv = take(Fp);
        G.z = take(b->syndrome ? Fp * m : 0);
    }
    pl.total = off;
    return GFBP_OK;
}

// Side streams and events of the calling thread for forking the persistent
// launches of one batch (created on first use, kept for the thread's life).
struct ForkSet {
    hipStream_t side[11] = {};
    hipEvent_t ev[12] = {};
};

ForkSet *fork_set() {
    static thread_local ForkSet fs;
    static thread_local bool ready = false;
    if (!ready) {
        for (auto &x : fs.side)
            if (hipStreamCreateWithFlags(&x, hipStreamNonBlocking) != hipSuccess) return nullptr;
        for (auto &e : fs.ev)
            if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) return nullptr;
        ready = true;
    }
    return &fs;
}

gfbp_status decode_persistent(const gfbp_code *const *codes, int nc, const gfbp_batch *b, gfbp_result *out,
                              void *workspace, size_t ws_bytes, hipStream_t st) {
    if (out->posterior || out->snap_iter > 0 || (out->trace && b->truth))
        return fail(GFBP_EUNSUPPORTED, "the persistent path returns decisions, iterations, convergence and guards only");
    PersistPlan pl;
    const gfbp_status ps = persist_plan(codes, nc, b, pl);
    if (ps != GFBP_OK) return ps;
    if (ws_bytes < pl.total) return fail(GFBP_ESMALL, "workspace too small");
    char *w = static_cast<char *>(workspace);
    const int prior_on = b->prior != GFBP_PRIOR_UNIFORM, markov = b->prior == GFBP_PRIOR_MARKOV;
    std::vector<persist::Group> groups(pl.gcode.size());
    for (size_t g = 0; g < pl.gcode.size(); ++g) {
        const gfbp_code *code = codes[pl.gcode[g]];
        const PersistPlan::G &o = pl.g[g];
        persist::Group &G = groups[g];
        G.c = code->dev;
        DevState &s = G.s;
        s = DevState{};
        s.Qm = reinterpret_cast<float *>(w + o.Qm);
        s.R = reinterpret_cast<float *>(w + o.R);
        s.L = reinterpret_cast<float *>(w + o.L);
        s.Pr = reinterpret_cast<float *>(w + o.Pr);
        s.Qp = reinterpret_cast<float *>(w + o.Qp);
        s.xh = reinterpret_cast<uint8_t *>(w + o.xh);
        s.unsat = reinterpret_cast<uint32_t *>(w + o.unsat);
        s.active = reinterpret_cast<uint8_t *>(w + o.active);
        s.guards = reinterpret_cast<int32_t *>(w + o.guards);
        s.F = int(pl.gframe[g].size());
        s.Fp = o.Fp;
        G.recs = code->lv[0].recs;
        G.lvl = code->lv[0].dptr;
        G.nlev = code->info.sus_levels;
        G.rs = std::max(1, code->info.max_col_degree);
        G.p = code->info.p;
        G.iters = reinterpret_cast<int32_t *>(w + o.iters);
        G.conv = reinterpret_cast<uint8_t *>(w + o.conv);
        G.z = b->syndrome ? reinterpret_cast<uint8_t *>(w + o.z) : nullptr;
        G.gframe = reinterpret_cast<const int32_t *>(w + o.gframe);
        HIP_TRY(hipMemcpyAsync(w + o.gframe, pl.gframe[g].data(), 4 * pl.gframe[g].size(), hipMemcpyHostToDevice, st));
    }
    const size_t F = size_t(pl.F);
    HIP_TRY(hipMemcpyAsync(w + pl.o_off_n, pl.off_n.data(), 8 * F, hipMemcpyHostToDevice, st));
    HIP_TRY(hipMemcpyAsync(w + pl.o_off_np, pl.off_np.data(), 8 * F, hipMemcpyHostToDevice, st));
    HIP_TRY(hipMemcpyAsync(w + pl.o_off_nq, pl.off_nq.data(), 8 * F, hipMemcpyHostToDevice, st));
    HIP_TRY(hipMemcpyAsync(w + pl.o_off_m, pl.off_m.data(), 8 * F, hipMemcpyHostToDevice, st));
    HIP_TRY(hipMemcpyAsync(w + pl.o_groups, groups.data(), sizeof(persist::Group) * groups.size(),
                           hipMemcpyHostToDevice, st));
    for (int l = 0; l < 12; ++l)
        if (!pl.work[l].empty())
            HIP_TRY(hipMemcpyAsync(w + pl.o_work[l], pl.work[l].data(), sizeof(persist::Work) * pl.work[l].size(),
                                   hipMemcpyHostToDevice, st));
    uint32_t *next = reinterpret_cast<uint32_t *>(w + pl.o_next);
    float *mshape = reinterpret_cast<float *>(w + pl.o_mshape);
    launch(k_fill_i32, dim3(1), dim3(64), 0, st, reinterpret_cast<int32_t *>(next), size_t(12), 0);
    if (markov)  // the matrix is batch-wide (every code on its field)
        hipLaunchKernelGGL(tiled::k_markov_shape, dim3(1), dim3(kWave), 0, st, b->markov_M, codes[pl.gcode[0]]->info.q,
                           mshape);
    persist::Batch B{};
    B.schedule = b->schedule;
    B.max_iter = b->max_iter;
    B.early_stop = b->early_stop;
    B.prior_on = prior_on;
    B.markov = markov;
    B.M = b->markov_M;
    B.pi = b->markov_pi;
    B.mshape = mshape;
    B.ch.channel = b->channel;
    B.ch.prior = b->prior;
    B.ch.evidence = b->evidence;
    B.ch.static_per_symbol = b->static_per_symbol;
    B.ch.rx = b->rx;
    B.ch.erasure = b->erasure;
    B.ch.y = b->y;
    B.ch.lik = b->likelihood;
    B.ch.param = b->param;
    B.ch.pi = b->markov_pi;
    B.ch.static_P = b->static_prior;
    B.ch.chan_of = b->channel_of;
    B.ch.off_n = reinterpret_cast<const int64_t *>(w + pl.o_off_n);
    B.ch.off_np = reinterpret_cast<const int64_t *>(w + pl.o_off_np);
    B.ch.off_nq = reinterpret_cast<const int64_t *>(w + pl.o_off_nq);
    B.off_m = reinterpret_cast<const int64_t *>(w + pl.o_off_m);
    B.zin = b->syndrome;
    B.xhat = out->xhat;
    B.iters = out->iters;
    B.conv = out->converged;
    B.guards = out->guards;
    const persist::Group *dg = reinterpret_cast<const persist::Group *>(w + pl.o_groups);
    // the lists present, the one with the largest tile first: it runs on the
    // caller's stream, the others on forked streams joined back into it
    std::vector<int> lists;
    for (int l = 0; l < 12; ++l)
        if (!pl.work[l].empty()) lists.push_back(l);
    std::stable_sort(lists.begin(), lists.end(), [&](int x, int y) { return pl.top[size_t(x)] > pl.top[size_t(y)]; });
    Tracer tr(st);
    // without allocations the lists run one after the other on the stream
    ForkSet *fs = lists.size() > 1 && !g_no_alloc ? fork_set() : nullptr;
    if (lists.size() > 1 && !g_no_alloc && !fs) return fail(GFBP_EHIP, "creating the streams for the persistent launches");
    // several launches: captured into one HIP graph on a created stream
    const bool graph = fs != nullptr && st != nullptr && !tr.on;
    if (graph) HIP_TRY(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
    hipError_t he = hipSuccess;
    if (fs) he = hipEventRecord(fs->ev[11], st);
    for (size_t k = 0; k < lists.size() && he == hipSuccess; ++k) {
        const int l = lists[k];
        hipStream_t ls = k == 0 || !fs ? st : fs->side[k - 1];
        if (k > 0 && fs) he = hipStreamWaitEvent(ls, fs->ev[11], 0);
        if (he != hipSuccess) break;
        tr.begin();
        hipEvent_t ea = g_launch_ev[0], eb = g_launch_ev[1];
        g_launch_ev[0] = g_launch_ev[1] = nullptr;
        const int lp = l % 6 + 1;
        he = persist::launch_persistent(lp, persist_lel(lp, pl.lel, l / 6), l < 6, b->schedule, dg,
                                        reinterpret_cast<const persist::Work *>(w + pl.o_work[l]),
                                        int(pl.work[l].size()), next + l, B, pl.waves, ls, ea, eb);
        if (ea) {
            Tracer::last_[0] = ea;
            Tracer::last_[1] = eb;
        }
        tr.end(K_PERSIST, 0, 0);
        if (he == hipSuccess && k > 0 && fs) he = hipEventRecord(fs->ev[k - 1], ls);
        if (he == hipSuccess && k > 0 && fs) he = hipStreamWaitEvent(st, fs->ev[k - 1], 0);
    }
    if (graph) {
        hipGraph_t gr = nullptr;
        const hipError_t ec = hipStreamEndCapture(st, &gr);
        if (he == hipSuccess) he = ec;
        hipGraphExec_t ex = nullptr;
        if (he == hipSuccess) he = hipGraphInstantiate(&ex, gr, nullptr, nullptr, 0);
        if (he == hipSuccess) he = hipGraphLaunch(ex, st);
        if (he == hipSuccess) he = hipStreamSynchronize(st);
        if (ex) (void)hipGraphExecDestroy(ex);
        if (gr) (void)hipGraphDestroy(gr);
    }
    if (he != hipSuccess) return fail(GFBP_EHIP, std::string("persistent launch: ") + hipGetErrorString(he));
    HIP_TRY(hipStreamSynchronize(st));
    if (tr.on) {
        // algorithmic bytes and updates of the iterations the frames ran
        std::vector<int32_t> it(F);
        HIP_TRY(hipMemcpy(it.data(), out->iters, 4 * F, hipMemcpyDeviceToHost));
        double bytes = 0, eq = 0;
        for (size_t g = 0; g < pl.gcode.size(); ++g) {
            const gfbp_code *code = codes[pl.gcode[g]];
            const Bytes bp = bytes_per_frame(code, markov, b->syndrome != nullptr);
            const double per = b->schedule == GFBP_PUS ? bp.check + bp.variable : bp.sequential;
            for (int32_t f : pl.gframe[g]) {
                bytes += double(it[size_t(f)]) * (per + bp.syndrome + (markov ? bp.markov : 0.0));
                eq += double(it[size_t(f)]) * code->info.n_edges * code->info.q;
            }
        }
        for (auto &r : tr.recs) {
            r.bytes = bytes / double(tr.recs.size());
            r.edgeq = eq / double(tr.recs.size());
        }
    }
    tr.flush();
    return GFBP_OK;
}

// Checks shared by both paths: the inputs each channel kind present needs.
gfbp_status check_inputs(const gfbp_batch *b, hipStream_t st) {
    bool kind[4] = {false, false, false, false};
    if (b->channel_of) {
        std::vector<uint8_t> ch(size_t(b->n_frames));
        HIP_TRY(hipMemcpyAsync(ch.data(), b->channel_of, ch.size(), hipMemcpyDeviceToHost, st));
        HIP_TRY(hipStreamSynchronize(st));
        for (uint8_t v : ch) {
            if (v > GFBP_CH_LIKELIHOOD) return fail(GFBP_EINVAL, "bad channel kind in channel_of");
            kind[v] = true;
        }
    } else {
        if (b->channel < 0 || b->channel > GFBP_CH_LIKELIHOOD) return fail(GFBP_EINVAL, "bad channel");
        kind[b->channel] = true;
    }
    const bool mn = b->evidence == GFBP_EVIDENCE_MN;
    if (b->evidence != GFBP_EVIDENCE_SYMBOL && !mn) return fail(GFBP_EINVAL, "bad evidence mode");
    if (kind[GFBP_CH_BSC] && ((!mn && !b->rx) || !b->param)) return fail(GFBP_EINVAL, "BSC needs rx and param");
    if (kind[GFBP_CH_BEC] && ((!mn && !b->rx) || !b->erasure)) return fail(GFBP_EINVAL, "BEC needs rx and erasure");
    if (kind[GFBP_CH_BIAWGN] && (!b->y || !b->param)) return fail(GFBP_EINVAL, "BI-AWGN needs y and param");
    if (kind[GFBP_CH_LIKELIHOOD] && (!b->likelihood || mn))
        return fail(GFBP_EINVAL, "LIKELIHOOD needs likelihood, and is not an MN evidence mode");
    if (b->prior == GFBP_PRIOR_MARKOV && (!b->markov_M || !b->markov_pi))
        return fail(GFBP_EINVAL, "Markov prior needs markov_M and markov_pi");
    if (b->prior == GFBP_PRIOR_STATIC && !b->static_prior) return fail(GFBP_EINVAL, "static prior needs static_prior");
    return GFBP_OK;
}

inline bool persistent_batch(const gfbp_batch *b) {
    return b->n_codes > 1 || b->code_index != nullptr || (b->options & GFBP_OPT_PERSISTENT);
}

// One code's batch through the plain kernels (inputs already checked).
gfbp_status decode_plain(const gfbp_code *code, const gfbp_batch *b, gfbp_result *out, void *workspace,
                         size_t ws_bytes, hipStream_t st) {
    const int F = b->n_frames;
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
    s.guards = reinterpret_cast<int32_t *>(w + cv.guards);
    BatchAux a{};
    a.orig = reinterpret_cast<int32_t *>(w + cv.orig);
    a.iters = reinterpret_cast<int32_t *>(w + cv.iters);
    a.conv = reinterpret_cast<uint8_t *>(w + cv.conv);
    a.z = reinterpret_cast<uint8_t *>(w + cv.z);
    a.holes = reinterpret_cast<int32_t *>(w + cv.holes);
    a.movers = reinterpret_cast<int32_t *>(w + cv.movers);
    a.pending = reinterpret_cast<uint8_t *>(w + cv.pending);
    a.mshape = reinterpret_cast<float *>(w + cv.mshape);
    a.qp2 = reinterpret_cast<float *>(w + cv.Qp2);
    s.F = F;
    s.Fp = frame_stride(F);
    const int needQ = (b->prior == GFBP_PRIOR_MARKOV) || out->posterior != nullptr;
    if (F > 0 && onchip_allowed(code, b, out)) {
        const onchip::Layout ly = onchip_layout(code, b, lds_limit());
        bool ran = false;
        gfbp_status rs = GFBP_OK;
        const bool sus = b->schedule == GFBP_SUS;
        if (ly.fw > 0) switch (code->info.p) {
                case 1: rs = run_onchip<1, onchip::lanes_log<1>(GFBP_PUS)>(code, b, out, s, a, st, needQ, ly, &ran);
                    break;  // (one lane per vector either way)
                case 2:
                    rs = sus ? run_onchip<2, onchip::lanes_log<2>(GFBP_SUS)>(code, b, out, s, a, st, needQ, ly, &ran)
                             : run_onchip<2, onchip::lanes_log<2>(GFBP_PUS)>(code, b, out, s, a, st, needQ, ly, &ran);
                    break;
                case 3:
                    rs = sus ? run_onchip<3, onchip::lanes_log<3>(GFBP_SUS)>(code, b, out, s, a, st, needQ, ly, &ran)
                             : run_onchip<3, onchip::lanes_log<3>(GFBP_PUS)>(code, b, out, s, a, st, needQ, ly, &ran);
                    break;
                default: break;
            }
        if (ran || rs != GFBP_OK) return rs;
    }
    switch (code->info.p) {
        case 1: return run_any<1>(code, b, out, s, a, st, needQ);
        case 2: return run_any<2>(code, b, out, s, a, st, needQ);
        case 3: return run_any<3>(code, b, out, s, a, st, needQ);
        case 4: return run_any<4>(code, b, out, s, a, st, needQ);
        case 5: return run_any<5>(code, b, out, s, a, st, needQ);
        case 6: return run_any<6>(code, b, out, s, a, st, needQ);
        default: return fail(GFBP_EUNSUPPORTED, "bad field");
    }
}

// ------------------------------------------------------ several codes, code by code
// A batch over several codes (without GFBP_OPT_PERSISTENT) is decoded code by
// code with the plain kernels: each code's frames are gathered into
// contiguous inputs, decoded as a one-code batch, and their results
// scattered back to the batch's places.  The codes run concurrently on the
// library's worker threads, each with a stream of its own (a code with few
// frames leaves most of the device idle; several together fill it).

// dst[k len + i] = src[off[k] + i] (k < nf, i < len): a frame's ragged segment.
template <typename T>
__global__ void k_gather(const T *src, const int64_t *off, int64_t len, int nf, T *dst) {
    const int64_t total = int64_t(nf) * len;
    for (int64_t x = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; x < total; x += int64_t(gridDim.x) * blockDim.x) {
        const int64_t k = x / len, i = x - k * len;
        dst[x] = src[off[k] + i];
    }
}

// dst[off[k] + i] = src[k len + i]: the inverse, for the decisions.
template <typename T>
__global__ void k_scatter(const T *src, const int64_t *off, int64_t len, int nf, T *dst) {
    const int64_t total = int64_t(nf) * len;
    for (int64_t x = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; x < total; x += int64_t(gridDim.x) * blockDim.x) {
        const int64_t k = x / len, i = x - k * len;
        dst[off[k] + i] = src[x];
    }
}

inline unsigned copy_blocks(int64_t total) {
    return unsigned(std::max<int64_t>(1, std::min<int64_t>(4096, (total + 255) / 256)));
}

// The library's worker threads: created on first use and kept for the
// process (their streams, pinned count buffers and events are thread-local
// and live as long).  run() hands out tasks 0..n-1 and blocks until all end.
class Workers {
public:
    static constexpr int kThreads = 4;  // streams beyond the device's hardware queues add nothing
    using Task = std::function<gfbp_status(int, hipStream_t, std::string &)>;

    static Workers &get() {
        static Workers *w = new Workers();  // never destroyed: its threads stay parked until the process ends
        return *w;
    }

    gfbp_status run(int n, int dev, const Task &task, std::string &err) {
        std::unique_lock<std::mutex> lk(mu_);
        busy_.wait(lk, [&] { return job_ == nullptr; });  // one batch at a time
        Job job{&task, n, dev};
        job.status.assign(size_t(n), GFBP_OK);
        job.errs.assign(size_t(n), std::string());
        job.left = n;
        job_ = &job;
        wake_.notify_all();
        done_.wait(lk, [&] { return job.left == 0 && job.active == 0; });
        job_ = nullptr;
        busy_.notify_all();
        for (int i = 0; i < n; ++i)
            if (job.status[size_t(i)] != GFBP_OK) {
                err = job.errs[size_t(i)];
                return job.status[size_t(i)];
            }
        return GFBP_OK;
    }

private:
    struct Job {
        const Task *task;
        int n, dev;
        int next = 0, left = 0, active = 0;
        std::vector<gfbp_status> status;
        std::vector<std::string> errs;
    };

    Workers() {
        for (int t = 0; t < kThreads; ++t) std::thread([this] { loop(); }).detach();
    }

    static hipStream_t stream_for(int dev) {
        static thread_local std::vector<hipStream_t> per_dev;
        if (size_t(dev) >= per_dev.size()) per_dev.resize(size_t(dev) + 1, nullptr);
        if (!per_dev[size_t(dev)] && hipStreamCreateWithFlags(&per_dev[size_t(dev)], hipStreamNonBlocking) != hipSuccess)
            per_dev[size_t(dev)] = nullptr;
        return per_dev[size_t(dev)];
    }

    void loop() {
        std::unique_lock<std::mutex> lk(mu_);
        for (;;) {
            wake_.wait(lk, [&] { return job_ != nullptr && job_->next < job_->n; });
            Job &j = *job_;
            const int i = j.next++;
            j.active++;
            lk.unlock();
            gfbp_status st = GFBP_OK;
            std::string e;
            if (hipSetDevice(j.dev) != hipSuccess) {
                st = GFBP_EHIP;
                e = "worker: hipSetDevice";
            } else if (hipStream_t s = stream_for(j.dev)) {
                st = (*j.task)(i, s, e);
            } else {
                st = GFBP_EHIP;
                e = "worker: creating its stream";
            }
            lk.lock();
            j.status[size_t(i)] = st;
            j.errs[size_t(i)] = e;
            j.active--;
            j.left--;
            if (j.left == 0 && j.active == 0) done_.notify_all();
        }
    }

    std::mutex mu_;
    std::condition_variable wake_, done_, busy_;
    Job *job_ = nullptr;
};

// Workspace of the code-by-code path: per code, its frames' source offsets
// and batch indices, the gathered inputs, the results before the scatter and
// the one-code decode's own workspace.
struct PartPlan {
    int code = 0;
    std::vector<int32_t> frames;  // batch frames of this code, in batch order
    std::vector<int64_t> src_n, src_np, src_nq, src_m, src_one;  // element offsets of each frame's inputs
    size_t o_src_n = 0, o_src_np = 0, o_src_nq = 0, o_src_m = 0, o_src_one = 0;
    size_t o_rx = 0, o_er = 0, o_y = 0, o_lik = 0, o_z = 0, o_param = 0, o_chan = 0;
    size_t o_xhat = 0, o_iters = 0, o_conv = 0, o_guards = 0, o_ws = 0, ws_bytes = 0;
};

gfbp_status percode_plan(const gfbp_code *const *codes, int nc, const gfbp_batch *b, std::vector<PartPlan> &parts,
                         size_t &total) {
    const int F = b->n_frames;
    std::vector<int> part_of(size_t(nc), -1);
    parts.clear();
    int64_t on = 0, onp = 0, onq = 0, om = 0;
    for (int f = 0; f < F; ++f) {
        const int k = b->code_index ? b->code_index[f] : 0;
        if (k < 0 || k >= nc) return fail(GFBP_EINVAL, "code_index out of range");
        if (part_of[size_t(k)] < 0) {
            part_of[size_t(k)] = int(parts.size());
            parts.emplace_back();
            parts.back().code = k;
        }
        PartPlan &pp = parts[size_t(part_of[size_t(k)])];
        const gfbp_code_info &ci = codes[k]->info;
        pp.frames.push_back(f);
        pp.src_n.push_back(on);
        pp.src_np.push_back(onp);
        pp.src_nq.push_back(onq);
        pp.src_m.push_back(om);
        pp.src_one.push_back(f);
        on += ci.n;
        onp += int64_t(ci.n) * ci.p;
        onq += int64_t(ci.n) * ci.q;
        om += ci.m;
    }
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t at = off;
        off += (bytes + 255) / 256 * 256;
        return at;
    };
    for (PartPlan &pp : parts) {
        const gfbp_code_info &ci = codes[pp.code]->info;
        const size_t Fg = pp.frames.size(), n = size_t(ci.n);
        pp.o_src_n = take(8 * Fg);
        pp.o_src_np = take(8 * Fg);
        pp.o_src_nq = take(8 * Fg);
        pp.o_src_m = take(8 * Fg);
        pp.o_src_one = take(8 * Fg);
        pp.o_rx = take(b->rx ? Fg * n : 0);
        pp.o_er = take(b->erasure ? Fg * n : 0);
        pp.o_y = take(b->y ? Fg * n * size_t(ci.p) * 4 : 0);
        pp.o_lik = take(b->likelihood ? Fg * n * size_t(ci.q) * 4 : 0);
        pp.o_z = take(b->syndrome ? Fg * size_t(ci.m) : 0);
        pp.o_param = take(b->param ? Fg * 4 : 0);
        pp.o_chan = take(b->channel_of ? Fg : 0);
        pp.o_xhat = take(Fg * n);
        pp.o_iters = take(Fg * 4);
        pp.o_conv = take(Fg);
        pp.o_guards = take(Fg * 4);
        pp.ws_bytes = carve(codes[pp.code], int(Fg), b->schedule, b->prior).total;
        pp.o_ws = take(pp.ws_bytes);
    }
    total = off;
    return GFBP_OK;
}

gfbp_status decode_percode(const gfbp_code *const *codes, int nc, const gfbp_batch *b, gfbp_result *out,
                           void *workspace, size_t ws_bytes, hipStream_t st) {
    if (out->posterior || out->snap_iter > 0 || (out->trace && b->truth))
        return fail(GFBP_EUNSUPPORTED, "a batch over several codes returns decisions, iterations, convergence and "
                                       "guards only");
    std::vector<PartPlan> parts;
    size_t total = 0;
    const gfbp_status ps = percode_plan(codes, nc, b, parts, total);
    if (ps != GFBP_OK) return ps;
    if (ws_bytes < total) return fail(GFBP_ESMALL, "workspace too small");
    char *w = static_cast<char *>(workspace);
    for (const PartPlan &pp : parts) {
        const size_t Fg = pp.frames.size();
        HIP_TRY(hipMemcpyAsync(w + pp.o_src_n, pp.src_n.data(), 8 * Fg, hipMemcpyHostToDevice, st));
        HIP_TRY(hipMemcpyAsync(w + pp.o_src_np, pp.src_np.data(), 8 * Fg, hipMemcpyHostToDevice, st));
        HIP_TRY(hipMemcpyAsync(w + pp.o_src_nq, pp.src_nq.data(), 8 * Fg, hipMemcpyHostToDevice, st));
        HIP_TRY(hipMemcpyAsync(w + pp.o_src_m, pp.src_m.data(), 8 * Fg, hipMemcpyHostToDevice, st));
        HIP_TRY(hipMemcpyAsync(w + pp.o_src_one, pp.src_one.data(), 8 * Fg, hipMemcpyHostToDevice, st));
    }
    HIP_TRY(hipStreamSynchronize(st));  // the offsets, and the caller's inputs, are in place
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    // the largest code first: it runs longest
    std::vector<int> order(parts.size());
    for (size_t i = 0; i < order.size(); ++i) order[i] = int(i);
    std::stable_sort(order.begin(), order.end(), [&](int x, int y) {
        const auto &a = codes[parts[size_t(x)].code]->info, &c = codes[parts[size_t(y)].code]->info;
        return double(a.n_edges) * a.q * double(parts[size_t(x)].frames.size()) >
               double(c.n_edges) * c.q * double(parts[size_t(y)].frames.size());
    });
    const Workers::Task task = [&](int t, hipStream_t ws, std::string &err) -> gfbp_status {
        const PartPlan &pp = parts[size_t(order[size_t(t)])];
        const gfbp_code *code = codes[pp.code];
        const gfbp_code_info &ci = code->info;
        const int Fg = int(pp.frames.size());
        const int64_t n = ci.n;
        auto at = [&](size_t o) { return w + o; };
        auto fail_here = [&](const char *what, hipError_t e) {
            err = std::string(what) + ": " + hipGetErrorString(e);
            return GFBP_EHIP;
        };
        const int64_t *sn = reinterpret_cast<const int64_t *>(at(pp.o_src_n));
        const int64_t *snp = reinterpret_cast<const int64_t *>(at(pp.o_src_np));
        const int64_t *snq = reinterpret_cast<const int64_t *>(at(pp.o_src_nq));
        const int64_t *sm = reinterpret_cast<const int64_t *>(at(pp.o_src_m));
        const int64_t *s1 = reinterpret_cast<const int64_t *>(at(pp.o_src_one));
        gfbp_batch bg = *b;
        bg.n_frames = Fg;
        bg.n_codes = 1;
        bg.code_index = nullptr;
        bg.truth = nullptr;
        bg.options &= ~GFBP_OPT_PERSISTENT;
        if (b->rx) {
            hipLaunchKernelGGL(k_gather<uint8_t>, dim3(copy_blocks(Fg * n)), dim3(256), 0, ws, b->rx, sn, n, Fg,
                               reinterpret_cast<uint8_t *>(at(pp.o_rx)));
            bg.rx = reinterpret_cast<const uint8_t *>(at(pp.o_rx));
        }
        if (b->erasure) {
            hipLaunchKernelGGL(k_gather<uint8_t>, dim3(copy_blocks(Fg * n)), dim3(256), 0, ws, b->erasure, sn, n, Fg,
                               reinterpret_cast<uint8_t *>(at(pp.o_er)));
            bg.erasure = reinterpret_cast<const uint8_t *>(at(pp.o_er));
        }
        if (b->y) {
            const int64_t len = n * ci.p;
            hipLaunchKernelGGL(k_gather<float>, dim3(copy_blocks(Fg * len)), dim3(256), 0, ws, b->y, snp, len, Fg,
                               reinterpret_cast<float *>(at(pp.o_y)));
            bg.y = reinterpret_cast<const float *>(at(pp.o_y));
        }
        if (b->likelihood) {
            const int64_t len = n * ci.q;
            hipLaunchKernelGGL(k_gather<float>, dim3(copy_blocks(Fg * len)), dim3(256), 0, ws, b->likelihood, snq, len,
                               Fg, reinterpret_cast<float *>(at(pp.o_lik)));
            bg.likelihood = reinterpret_cast<const float *>(at(pp.o_lik));
        }
        if (b->syndrome) {
            hipLaunchKernelGGL(k_gather<uint8_t>, dim3(copy_blocks(Fg * int64_t(ci.m))), dim3(256), 0, ws, b->syndrome,
                               sm, int64_t(ci.m), Fg, reinterpret_cast<uint8_t *>(at(pp.o_z)));
            bg.syndrome = reinterpret_cast<const uint8_t *>(at(pp.o_z));
        }
        if (b->param) {
            hipLaunchKernelGGL(k_gather<float>, dim3(copy_blocks(Fg)), dim3(256), 0, ws, b->param, s1, int64_t(1), Fg,
                               reinterpret_cast<float *>(at(pp.o_param)));
            bg.param = reinterpret_cast<const float *>(at(pp.o_param));
        }
        if (b->channel_of) {
            hipLaunchKernelGGL(k_gather<uint8_t>, dim3(copy_blocks(Fg)), dim3(256), 0, ws, b->channel_of, s1,
                               int64_t(1), Fg, reinterpret_cast<uint8_t *>(at(pp.o_chan)));
            bg.channel_of = reinterpret_cast<const uint8_t *>(at(pp.o_chan));
        }
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return fail_here("gathering a code's inputs", e);
        gfbp_result og{};
        og.xhat = reinterpret_cast<uint8_t *>(at(pp.o_xhat));
        og.iters = reinterpret_cast<int32_t *>(at(pp.o_iters));
        og.converged = reinterpret_cast<uint8_t *>(at(pp.o_conv));
        og.guards = out->guards ? reinterpret_cast<int32_t *>(at(pp.o_guards)) : nullptr;
        const gfbp_status rs = decode_plain(code, &bg, &og, at(pp.o_ws), pp.ws_bytes, ws);
        if (rs != GFBP_OK) {
            err = g_err;
            return rs;
        }
        // results back to the batch's places: decisions at the frame's ragged
        // offset, the per-frame scalars at its index
        hipLaunchKernelGGL(k_scatter<uint8_t>, dim3(copy_blocks(Fg * n)), dim3(256), 0, ws, og.xhat, sn, n, Fg,
                           out->xhat);
        hipLaunchKernelGGL(k_scatter<int32_t>, dim3(copy_blocks(Fg)), dim3(256), 0, ws, og.iters, s1, int64_t(1), Fg,
                           out->iters);
        hipLaunchKernelGGL(k_scatter<uint8_t>, dim3(copy_blocks(Fg)), dim3(256), 0, ws, og.converged, s1, int64_t(1),
                           Fg, out->converged);
        if (out->guards)
            hipLaunchKernelGGL(k_scatter<int32_t>, dim3(copy_blocks(Fg)), dim3(256), 0, ws, og.guards, s1, int64_t(1),
                               Fg, out->guards);
        e = hipGetLastError();
        if (e == hipSuccess) e = hipStreamSynchronize(ws);
        if (e != hipSuccess) return fail_here("scattering a code's results", e);
        return GFBP_OK;
    };
    std::string err;
    const gfbp_status rs = Workers::get().run(int(parts.size()), dev, task, err);
    if (rs != GFBP_OK) return fail(rs, err);
    return GFBP_OK;
}

// Streaming copy of n 16-byte vectors, four loads in flight per lane (the
// measurement behind gfbp_stream_copy_rate).
constexpr int kCopyUnroll = 4;
__global__ __launch_bounds__(256) void k_stream_copy(const tiled::f32x4 *__restrict__ src,
                                                     tiled::f32x4 *__restrict__ dst, size_t n) {
    const size_t stride = size_t(gridDim.x) * 256 * kCopyUnroll;
    for (size_t base = size_t(blockIdx.x) * 256 * kCopyUnroll + threadIdx.x; base < n; base += stride) {
        tiled::f32x4 t[kCopyUnroll];
#pragma unroll
        for (int u = 0; u < kCopyUnroll; ++u)
            if (base + size_t(u) * 256 < n) t[u] = __builtin_nontemporal_load(src + base + size_t(u) * 256);
#pragma unroll
        for (int u = 0; u < kCopyUnroll; ++u)
            if (base + size_t(u) * 256 < n) __builtin_nontemporal_store(t[u], dst + base + size_t(u) * 256);
    }
}

}  // namespace

// ======================================================================= C ABI
extern "C" {

const char *gfbp_last_error(void) { return g_err.c_str(); }

const char *gfbp_version(void) { return "gfbp 0.6 (gfx950)"; }

gfbp_status gfbp_stream_copy_rate(void *dst, const void *src, size_t bytes, int32_t reps, void *stream, double *rate) {
    if (!dst || !src || !rate) return fail(GFBP_EINVAL, "null argument");
    if (bytes == 0 || bytes % 16 != 0 || reps < 1)
        return fail(GFBP_EINVAL, "bytes must be a positive multiple of 16, reps >= 1");
    if ((reinterpret_cast<uintptr_t>(dst) | reinterpret_cast<uintptr_t>(src)) % 16 != 0)
        return fail(GFBP_EINVAL, "buffers must be 16-byte aligned");
    const auto d = reinterpret_cast<uintptr_t>(dst), sr = reinterpret_cast<uintptr_t>(src);
    if (d < sr + bytes && sr < d + bytes) return fail(GFBP_EINVAL, "buffers overlap");
    hipStream_t st = static_cast<hipStream_t>(stream);
    const size_t n = bytes / 16;
    const size_t per_block = size_t(256) * kCopyUnroll;
    const unsigned grid = unsigned(std::min<size_t>(32768, (n + per_block - 1) / per_block));
    hipEvent_t a = nullptr, b = nullptr;
    HIP_TRY(hipEventCreate(&a));
    if (hipEventCreate(&b) != hipSuccess) {
        (void)hipEventDestroy(a);
        return fail(GFBP_EHIP, "hipEventCreate");
    }
    float best = 0.0f;
    hipError_t e = hipSuccess;
    for (int r = -1; r < reps && e == hipSuccess; ++r) {  // r = -1: warm-up
        e = hipEventRecord(a, st);
        if (e == hipSuccess) {
            hipLaunchKernelGGL(k_stream_copy, dim3(grid), dim3(256), 0, st,
                               static_cast<const tiled::f32x4 *>(src), static_cast<tiled::f32x4 *>(dst), n);
            e = hipGetLastError();
        }
        if (e == hipSuccess) e = hipEventRecord(b, st);
        if (e == hipSuccess) e = hipEventSynchronize(b);
        float ms = 0.0f;
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, a, b);
        if (e == hipSuccess && r >= 0 && (best == 0.0f || ms < best)) best = ms;
    }
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    if (e != hipSuccess) return fail(GFBP_EHIP, std::string("stream copy: ") + hipGetErrorString(e));
    *rate = best > 0.0f ? 2.0 * double(bytes) / (double(best) * 1e-3) : 0.0;
    return GFBP_OK;
}

gfbp_status gfbp_code_build(const gfbp_code_desc *d, gfbp_code **out) {
    if (!d || !out) return fail(GFBP_EINVAL, "null argument");
    *out = nullptr;
    CodePlan pl;
    std::string perr;
    const gfbp_status ps = build_plan(d, pl, perr);
    if (ps != GFBP_OK) return fail(ps, perr);
    const int q = pl.q, p = pl.p, n = pl.n, m = pl.m, E = pl.E, max_dc = pl.max_dc, max_dv = pl.max_dv;
    const unsigned poly = pl.poly;
    const double sum_dc2 = pl.sum_dc2;
    const std::vector<uint8_t> &mul = pl.mul;
    const std::vector<int32_t> &col_ptr = pl.col_ptr, &col_edge = pl.col_edge, &edge_row = pl.edge_row,
                               &visit = pl.visit, &chain_col = pl.chain_col, &col_chain = pl.col_chain;
    const std::vector<uint64_t> &emap = pl.emap;
    std::vector<SusRec> *recs = pl.recs;
    LevelPlan *lvs = pl.lv;
    gfbp_code *c = new (std::nothrow) gfbp_code();
    if (!c) return fail(GFBP_ENOMEM, "host allocation");
    size_t off = 0;
    auto take = [&](size_t bytes) { size_t o = off; off += align256(bytes ? bytes : 1); return o; };
    const size_t o_rp = take(4 * size_t(m + 1)), o_col = take(4 * size_t(E)), o_coef = take(size_t(E)),
                 o_cp = take(4 * size_t(n + 1)), o_ce = take(4 * size_t(E)), o_er = take(4 * size_t(E)),
                 o_mul = take(size_t(q) * q), o_em = take(16 * size_t(E)),
                 o_sr0 = take(sizeof(SusRec) * recs[0].size()), o_sr1 = take(sizeof(SusRec) * recs[1].size()),
                 o_vis = take(4 * size_t(n)), o_cc = take(4 * chain_col.size()), o_colc = take(4 * size_t(n)),
                 o_lp0 = take(4 * lvs[0].ptr.size()), o_lp1 = take(4 * lvs[1].ptr.size());
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
    if (err == hipSuccess) err = up(o_sr0, recs[0].data(), sizeof(SusRec) * recs[0].size());
    if (err == hipSuccess) err = up(o_sr1, recs[1].data(), sizeof(SusRec) * recs[1].size());
    if (err == hipSuccess) err = up(o_vis, visit.data(), 4 * size_t(n));
    if (err == hipSuccess) err = up(o_cc, chain_col.data(), 4 * chain_col.size());
    if (err == hipSuccess) err = up(o_colc, col_chain.data(), 4 * size_t(n));
    if (err == hipSuccess) err = up(o_lp0, lvs[0].ptr.data(), 4 * lvs[0].ptr.size());
    if (err == hipSuccess) err = up(o_lp1, lvs[1].ptr.data(), 4 * lvs[1].ptr.size());
    if (err != hipSuccess) {
        (void)hipFree(c->mem);
        delete c;
        return fail(GFBP_EHIP, std::string("copying the code to the device: ") + hipGetErrorString(err));
    }
    c->info = gfbp_code_info{q, p, n, m, d->n_info, E, max_dc, max_dv, int32_t(poly),
                             int32_t(lvs[0].ptr.size()) - 1, int32_t(lvs[1].ptr.size()) - 1};
    c->sum_dc2 = sum_dc2;
    static_cast<LevelPlan &>(c->lv[0]) = std::move(lvs[0]);
    static_cast<LevelPlan &>(c->lv[1]) = std::move(lvs[1]);
    c->lv[0].recs = reinterpret_cast<const SusRec *>(base + o_sr0);
    c->lv[1].recs = reinterpret_cast<const SusRec *>(base + o_sr1);
    c->lv[0].dptr = reinterpret_cast<const int32_t *>(base + o_lp0);
    c->lv[1].dptr = reinterpret_cast<const int32_t *>(base + o_lp1);
    c->dev = DevCode{n, m, E, q, p, d->n_info, max_dv,
                     reinterpret_cast<const int32_t *>(base + o_rp), reinterpret_cast<const int32_t *>(base + o_col),
                     reinterpret_cast<const uint8_t *>(base + o_coef), reinterpret_cast<const int32_t *>(base + o_cp),
                     reinterpret_cast<const int32_t *>(base + o_ce), reinterpret_cast<const int32_t *>(base + o_er),
                     reinterpret_cast<const uint8_t *>(base + o_mul), reinterpret_cast<const uint64_t *>(base + o_em),
                     reinterpret_cast<const int32_t *>(base + o_vis), reinterpret_cast<const int32_t *>(base + o_cc),
                     reinterpret_cast<const int32_t *>(base + o_colc)};
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

size_t gfbp_batch_workspace_size(const gfbp_code *const *codes, const gfbp_batch *b) {
    if (!codes || !b || b->n_frames < 0) return 0;
    const int nc = b->n_codes > 0 ? b->n_codes : 1;
    for (int k = 0; k < nc; ++k)
        if (!codes[k]) return 0;
    if (!persistent_batch(b)) return carve(codes[0], b->n_frames, b->schedule, b->prior).total;
    if (!(b->options & GFBP_OPT_PERSISTENT)) {  // several codes, code by code
        std::vector<PartPlan> parts;
        size_t total = 0;
        if (percode_plan(codes, nc, b, parts, total) != GFBP_OK) return 0;
        return total;
    }
    PersistPlan pl;
    if (persist_plan(codes, nc, b, pl) != GFBP_OK) return 0;
    return pl.total;
}

gfbp_status gfbp_decode_batch(const gfbp_code *const *codes, const gfbp_batch *b, gfbp_result *out, void *workspace,
                              size_t ws_bytes, void *stream) {
    if (!codes || !b || !out) return fail(GFBP_EINVAL, "null argument");
    const int nc = b->n_codes > 0 ? b->n_codes : 1;
    for (int k = 0; k < nc; ++k)
        if (!codes[k]) return fail(GFBP_EINVAL, "null code");
    const gfbp_code *code = codes[0];
    const int F = b->n_frames;
    if (F < 0) return fail(GFBP_EINVAL, "n_frames < 0");
    if (b->schedule != GFBP_PUS && b->schedule != GFBP_SUS) return fail(GFBP_EINVAL, "bad schedule");
    if (b->max_iter < 1) return fail(GFBP_EINVAL, "max_iter < 1");
    if (b->prior != GFBP_PRIOR_UNIFORM && b->prior != GFBP_PRIOR_MARKOV && b->prior != GFBP_PRIOR_STATIC)
        return fail(GFBP_EINVAL, "bad prior");
    if (F == 0) return GFBP_OK;
    if (b->prior == GFBP_PRIOR_MARKOV)
        for (int k = 1; k < nc; ++k)
            if (codes[k]->info.q != code->info.q)
                return fail(GFBP_EINVAL, "a Markov prior's matrix is over one field: every code needs its q");
    if (b->prior == GFBP_PRIOR_STATIC && nc > 1)
        for (int k = 1; k < nc; ++k)
            if (codes[k]->info.q != code->info.q || (b->static_per_symbol && codes[k]->info.n_info != code->info.n_info))
                return fail(GFBP_EINVAL, "a static prior is over one field and chain length");
    if ((b->options & GFBP_OPT_PRIOR_IN_SWEEP) && b->schedule != GFBP_SUS)
        return fail(GFBP_EINVAL, "priors assigned during the sweep need the sequential schedule");
    if (!out->xhat || !out->iters || !out->converged) return fail(GFBP_EINVAL, "null output buffer");
    if (!workspace) return fail(GFBP_EINVAL, "null workspace");
    if (reinterpret_cast<uintptr_t>(workspace) % 256) return fail(GFBP_EINVAL, "workspace not 256-byte aligned");
    hipStream_t st = static_cast<hipStream_t>(stream);
    const gfbp_status ci = check_inputs(b, st);
    if (ci != GFBP_OK) return ci;
    if (persistent_batch(b)) {
        if ((b->options & GFBP_OPT_PERSISTENT) || g_no_alloc)
            return decode_persistent(codes, nc, b, out, workspace, ws_bytes, st);
        return decode_percode(codes, nc, b, out, workspace, ws_bytes, st);
    }
    return decode_plain(code, b, out, workspace, ws_bytes, st);
}

// ---- decoding without allocations: the library's static device scratch.
// One array per GPU, held until the process ends.  In host code its name is
// a host-side stand-in, not a device address: the address comes from
// hipGetSymbolAddress, once per device, and only that address is used.
}  // extern "C"

namespace {
constexpr size_t kScratchBytes = size_t(256) << 20;
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};
}  // namespace

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

extern "C" {

gfbp_status gfbp_decode_batch_noalloc(const gfbp_code *const *codes, const gfbp_batch *b, gfbp_result *out,
                                      void *stream) {
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return fail(GFBP_EUNSUPPORTED, "device index beyond the scratch table");
    void *ptr = nullptr;
    {
        std::lock_guard<std::mutex> g(g_scratch_mu);
        if (!g_scratch_ptr[dev]) {  // set-up on this device's first call (the device is current)
            void *p = nullptr;
            const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
            if (e != hipSuccess || !p)
                return fail(GFBP_EHIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
            g_scratch_ptr[dev] = p;
        }
        ptr = g_scratch_ptr[dev];
    }
    if (!codes || !b || !out) return fail(GFBP_EINVAL, "null argument");
    // a batch over several codes runs through the persistent kernels here (the
    // code-by-code path's worker threads and their streams are allocations)
    gfbp_batch pb = *b;
    if (persistent_batch(b)) pb.options |= GFBP_OPT_PERSISTENT;
    const size_t need = gfbp_batch_workspace_size(codes, &pb);
    if (pb.n_frames > 0 && need == 0) return fail(GFBP_EINVAL, "bad batch (workspace size 0)");
    if (need > kScratchBytes)
        return fail(GFBP_ESMALL, "the batch needs " + std::to_string(need) + " bytes of scratch; the static scratch holds " +
                                     std::to_string(kScratchBytes));
    g_no_alloc = true;
    const gfbp_status rs = gfbp_decode_batch(codes, &pb, out, ptr, kScratchBytes, stream);
    g_no_alloc = false;
    return rs;
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
    tb.n_codes = 1;
    tb.code_index = nullptr;
    tb.options &= ~GFBP_OPT_PERSISTENT;
    tb.options |= GFBP_OPT_NO_ONCHIP;  // the shapes are those of the tiled kernels
    gfbp_result to = *out;
    to.posterior = nullptr;
    to.snap_iter = 0;
    to.snap_q = to.snap_r = to.snap_Q = nullptr;
    to.trace = nullptr;
    // one warm-up run per candidate, then kRounds rounds over the candidates
    // in turn (so that drift hits all alike); each keeps its fastest run
    constexpr int kRounds = 3;
    const int nl = max_lel(c);
    std::vector<double> best_of(size_t(nl) + 1, 1e300);
    for (int round = -1; round < kRounds; ++round)
        for (int l = 1; l <= nl; ++l) {
            c->el[slot] = 1 << l;
            const auto t0 = std::chrono::steady_clock::now();
            const gfbp_code *cc[1] = {c};
            const gfbp_status st = gfbp_decode_batch(cc, &tb, &to, workspace, ws_bytes, stream);
            if (st != GFBP_OK) {
                c->el[slot] = keep;
                return st;
            }
            const double t = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
            if (round >= 0) best_of[size_t(l)] = std::min(best_of[size_t(l)], t);
        }
    double best_t = 1e300;
    int best = 0;
    for (int l = 1; l <= nl; ++l)
        if (best_of[size_t(l)] < best_t) {
            best_t = best_of[size_t(l)];
            best = 1 << l;
        }
    c->el[slot] = best;
    if (chosen) *chosen = best;
    return GFBP_OK;
}

gfbp_status gfbp_tune_persistent(const gfbp_code *const *codes, const gfbp_batch *b, gfbp_result *out,
                                 void *workspace, size_t ws_bytes, void *stream, int32_t trial_iters, int32_t *el,
                                 int32_t *waves) {
    if (!codes || !b || !out) return fail(GFBP_EINVAL, "null argument");
    if (trial_iters < 1) return fail(GFBP_EINVAL, "trial_iters < 1");
    gfbp_batch tb = *b;
    tb.max_iter = trial_iters;
    tb.early_stop = 0;
    tb.options |= GFBP_OPT_PERSISTENT;
    struct Cand {
        int el, waves;
    };
    std::vector<Cand> cands;
    for (int e : {4, 8})
        for (int wv : {4, 8}) cands.push_back({e, wv});
    constexpr int kRounds = 3;
    std::vector<double> best_of(cands.size(), 1e300);
    for (int round = -1; round < kRounds; ++round)
        for (size_t k = 0; k < cands.size(); ++k) {
            tb.persist_el = cands[k].el;
            tb.persist_waves = cands[k].waves;
            if (gfbp_batch_workspace_size(codes, &tb) > ws_bytes) continue;
            const auto t0 = std::chrono::steady_clock::now();
            const gfbp_status st = gfbp_decode_batch(codes, &tb, out, workspace, ws_bytes, stream);
            if (st != GFBP_OK) return st;
            const double t = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
            if (round >= 0) best_of[k] = std::min(best_of[k], t);
        }
    size_t best = 0;
    for (size_t k = 1; k < cands.size(); ++k)
        if (best_of[k] < best_of[best]) best = k;
    if (best_of[best] >= 1e300) return fail(GFBP_ESMALL, "workspace too small for every candidate shape");
    if (el) *el = cands[best].el;
    if (waves) *waves = cands[best].waves;
    return GFBP_OK;
}

size_t gfbp_session_bytes(const gfbp_code *code, const gfbp_session_desc *d) {
    if (!code || !d || d->n_slots < 0) return 0;
    const int S = session_slots(code, d);
    if (S < 1) return 0;
    return session_carve(code, S, d->schedule, d->markov_M != nullptr, d->has_syndrome).total;
}

uint64_t gfbp_device_clock_hz(void) {
    int dev = 0, khz = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev) != hipSuccess || khz <= 0) return 0;
    return uint64_t(khz) * 1000u;
}

gfbp_status gfbp_session_create(const gfbp_code *code, const gfbp_session_desc *d, gfbp_session **out) {
    if (!code || !d || !out) return fail(GFBP_EINVAL, "null argument");
    *out = nullptr;
    if (d->n_slots < 0 || (d->n_slots == 0 && d->device_bytes <= 0))
        return fail(GFBP_EINVAL, "n_slots < 1 and no device_bytes budget");
    if (d->schedule != GFBP_PUS && d->schedule != GFBP_SUS) return fail(GFBP_EINVAL, "bad schedule");
    if (d->max_iter < 1) return fail(GFBP_EINVAL, "max_iter < 1");
    if ((d->markov_M == nullptr) != (d->markov_pi == nullptr)) return fail(GFBP_EINVAL, "markov_M and markov_pi go together");
    if (d->options & GFBP_OPT_PRIOR_IN_SWEEP)
        return fail(GFBP_EUNSUPPORTED, "sessions refresh priors after each iteration");
    gfbp_session *ss = new (std::nothrow) gfbp_session();
    if (!ss) return fail(GFBP_ENOMEM, "host allocation");
    ss->code = code;
    ss->S = session_slots(code, d);
    if (ss->S < 1) {
        delete ss;
        return fail(GFBP_ENOMEM, "device_bytes holds no 64-slot tile of this code's state");
    }
    ss->schedule = d->schedule;
    ss->max_iter = d->max_iter;
    ss->has_z = d->has_syndrome != 0;
    ss->options = d->options;
    ss->markov = d->markov_M != nullptr;
    bool bound = false;
    switch (code->info.p) {
        case 1: bound = session_bind<1>(ss); break;
        case 2: bound = session_bind<2>(ss); break;
        case 3: bound = session_bind<3>(ss); break;
        case 4: bound = session_bind<4>(ss); break;
        case 5: bound = session_bind<5>(ss); break;
        case 6: bound = session_bind<6>(ss); break;
    }
    if (!bound) {
        delete ss;
        return fail(GFBP_EUNSUPPORTED, "no kernel for this code's shape");
    }
    ss->ntiles = ss->S / ss->tf;
    const SessCarve cv = session_carve(code, ss->S, ss->schedule, ss->markov, ss->has_z);
    if (hipMalloc(&ss->mem, cv.total) != hipSuccess) {
        delete ss;
        return fail(GFBP_ENOMEM, "device allocation for the session");
    }
    ss->bytes = cv.total;
    const size_t pin_bytes = size_t(ss->S) * 6 * 4 + size_t(ss->S) * 16 + 256;
    if (hipHostMalloc(&ss->pin, pin_bytes, hipHostMallocDefault) != hipSuccess) {
        (void)hipFree(ss->mem);
        delete ss;
        return fail(GFBP_ENOMEM, "pinned host allocation for the session");
    }
    ss->pin_bytes = pin_bytes;
    if (hipMemset(ss->mem, 0, cv.total) != hipSuccess) {
        (void)hipFree(ss->mem);
        (void)hipHostFree(ss->pin);
        delete ss;
        return fail(GFBP_EHIP, "clearing session memory");
    }
    char *w = static_cast<char *>(ss->mem);
    SessDev &v = ss->dv;
    DevState &st = v.st;
    st.Qm = reinterpret_cast<float *>(w + cv.Qm);
    st.R = reinterpret_cast<float *>(w + cv.R);
    st.L = reinterpret_cast<float *>(w + cv.L);
    st.Pr = reinterpret_cast<float *>(w + cv.Pr);
    st.Qp = reinterpret_cast<float *>(w + cv.Qp);
    st.xh = reinterpret_cast<uint8_t *>(w + cv.xh);
    st.unsat = reinterpret_cast<uint32_t *>(w + cv.unsat);
    st.active = reinterpret_cast<uint8_t *>(w + cv.active);
    st.count = reinterpret_cast<uint32_t *>(w + cv.count);
    st.tiles = reinterpret_cast<int32_t *>(w + cv.tiles);
    st.guards = reinterpret_cast<int32_t *>(w + cv.guards);
    st.F = ss->S;
    st.Fp = ss->S;
    v.S = ss->S;
    v.max_iter = ss->max_iter;
    v.rx = reinterpret_cast<uint8_t *>(w + cv.rx);
    v.er = reinterpret_cast<uint8_t *>(w + cv.er);
    v.y = reinterpret_cast<float *>(w + cv.y);
    v.param = reinterpret_cast<float *>(w + cv.param);
    v.z = ss->has_z ? reinterpret_cast<uint8_t *>(w + cv.z) : nullptr;
    v.chan = reinterpret_cast<uint8_t *>(w + cv.chan);
    v.mark = reinterpret_cast<uint8_t *>(w + cv.mark);
    v.iters = reinterpret_cast<int32_t *>(w + cv.iters);
    v.conv = reinterpret_cast<uint8_t *>(w + cv.conv);
    v.fresh = reinterpret_cast<uint8_t *>(w + cv.fresh);
    v.done = reinterpret_cast<uint8_t *>(w + cv.done);
    v.xout = reinterpret_cast<uint8_t *>(w + cv.xout);
    v.pairs = reinterpret_cast<int32_t *>(w + cv.pairs);
    v.list = reinterpret_cast<int32_t *>(w + cv.list);
    v.res = reinterpret_cast<int32_t *>(w + cv.res);
    v.t_admit = reinterpret_cast<uint64_t *>(w + cv.t_admit);
    v.t_done = reinterpret_cast<uint64_t *>(w + cv.t_done);
    v.ts = reinterpret_cast<uint64_t *>(w + cv.ts);
    st.chan = v.chan;
    st.mark = v.mark;
    ss->ftiles = reinterpret_cast<int32_t *>(w + cv.ftiles);
    ss->aux = reinterpret_cast<uint32_t *>(w + cv.aux);
    ss->M = reinterpret_cast<float *>(w + cv.M);
    ss->pi = reinterpret_cast<float *>(w + cv.pi);
    ss->mshape = reinterpret_cast<float *>(w + cv.mshape);
    if (ss->markov) {
        const int q = code->info.q;
        bool ok = hipMemcpy(ss->M, d->markov_M, sizeof(float) * q * q, hipMemcpyHostToDevice) == hipSuccess &&
                  hipMemcpy(ss->pi, d->markov_pi, sizeof(float) * q, hipMemcpyHostToDevice) == hipSuccess;
        if (ok) {
            hipLaunchKernelGGL(tiled::k_markov_shape, dim3(1), dim3(kWave), 0, nullptr, ss->M, q, ss->mshape);
            ok = hipGetLastError() == hipSuccess && hipDeviceSynchronize() == hipSuccess;
        }
        if (!ok) {
            (void)hipFree(ss->mem);
            (void)hipHostFree(ss->pin);
            delete ss;
            return fail(GFBP_EHIP, "copying the Markov source to the device");
        }
    }
    ss->id.assign(ss->S, -1);
    ss->free_slots.resize(ss->S);
    for (int k = 0; k < ss->S; ++k) ss->free_slots[k] = ss->S - 1 - k;
    *out = ss;
    return GFBP_OK;
}

gfbp_status gfbp_session_destroy(gfbp_session *ss) {
    if (!ss) return GFBP_OK;
    for (auto &g : ss->graphs) {
        (void)hipGraphExecDestroy(g.exec);
        (void)hipGraphDestroy(g.graph);
    }
    hipError_t e1 = hipFree(ss->mem), e2 = hipHostFree(ss->pin);
    delete ss;
    if (e1 != hipSuccess || e2 != hipSuccess) return fail(GFBP_EHIP, "freeing the session");
    return GFBP_OK;
}

int32_t gfbp_session_free_slots(const gfbp_session *ss) { return ss ? int32_t(ss->free_slots.size()) : 0; }

int32_t gfbp_session_running(const gfbp_session *ss) { return ss ? ss->running : 0; }

gfbp_status gfbp_session_admit(gfbp_session *ss, int32_t n, const int64_t *ids, const gfbp_frames *fr,
                               int32_t *n_admitted, void *stream) {
    if (!ss || !fr || (n > 0 && !ids)) return fail(GFBP_EINVAL, "null argument");
    if (n_admitted) *n_admitted = 0;
    if (n <= 0) return GFBP_OK;
    if (!fr->channel) return fail(GFBP_EINVAL, "frames need per-frame channel kinds");
    if (fr->markov && !ss->markov) return fail(GFBP_EINVAL, "Markov frames need a session created with a Markov source");
    if (fr->syndrome && !ss->has_z) return fail(GFBP_EINVAL, "syndromes need a session created with has_syndrome");
    hipStream_t st = static_cast<hipStream_t>(stream);
    const int k = std::min<int>(n, int(ss->free_slots.size()));
    if (k == 0) return GFBP_OK;
    int32_t *pairs = static_cast<int32_t *>(ss->pin);
    for (int r = 0; r < k; ++r) {
        const int slot = ss->free_slots.back();
        ss->free_slots.pop_back();
        pairs[2 * r] = slot;
        pairs[2 * r + 1] = r;
        ss->id[slot] = ids[r];
    }
    HIP_TRY(hipMemcpyAsync(ss->dv.pairs, pairs, sizeof(int32_t) * 2 * k, hipMemcpyHostToDevice, st));
    HIP_TRY(hipStreamSynchronize(st));  // the pinned staging is reused by the next call
    AdmitIn in{fr->param, fr->rx, fr->erasure, fr->syndrome, fr->channel, fr->markov, fr->y};
    hipLaunchKernelGGL(k_admit, dim3(k), dim3(256), 0, st, ss->dv, in, ss->code->info.n, ss->code->info.m,
                       ss->code->info.p);
    HIP_TRY(hipGetLastError());
    ss->running += k;
    const gfbp_status rs = ss->init_fn(ss, k, st);
    if (rs != GFBP_OK) return rs;
    if (n_admitted) *n_admitted = k;
    return GFBP_OK;
}

gfbp_status gfbp_session_step(gfbp_session *ss, int32_t iters, void *stream) {
    if (!ss) return fail(GFBP_EINVAL, "null session");
    if (iters < 1) return fail(GFBP_EINVAL, "iters < 1");
    hipStream_t st = static_cast<hipStream_t>(stream);
    const int need = std::min(ss->ntiles, ss->running);  // tiles holding a running frame, at most
    if (need == 0) return GFBP_OK;
    if (!(ss->options & GFBP_OPT_STEP_GRAPHS) || iters % 2 || !st) return ss->step_fn(ss, iters, st, need);
    int nb = 1;
    while (nb < need) nb <<= 1;
    nb = std::min(nb, ss->ntiles);
    for (const auto &g : ss->graphs)
        if (g.iters == iters && g.nb == nb && g.parity == ss->parity) {
            HIP_TRY(hipGraphLaunch(g.exec, st));
            return GFBP_OK;
        }
    // capture: an even number of iterations leaves the parity as it was
    const int parity = ss->parity;
    HIP_TRY(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
    const gfbp_status rs = ss->step_fn(ss, iters, st, nb);
    hipGraph_t graph = nullptr;
    const hipError_t ec = hipStreamEndCapture(st, &graph);
    if (rs != GFBP_OK) {
        if (graph) (void)hipGraphDestroy(graph);
        return rs;
    }
    if (ec != hipSuccess) return fail(GFBP_EHIP, std::string("hipStreamEndCapture: ") + hipGetErrorString(ec));
    hipGraphExec_t exec = nullptr;
    const hipError_t ei = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    if (ei != hipSuccess) {
        (void)hipGraphDestroy(graph);
        return fail(GFBP_EHIP, std::string("hipGraphInstantiate: ") + hipGetErrorString(ei));
    }
    ss->graphs.push_back(gfbp_session::StepGraph{iters, nb, parity, graph, exec});
    HIP_TRY(hipGraphLaunch(exec, st));
    return GFBP_OK;
}

gfbp_status gfbp_session_poll(gfbp_session *ss, gfbp_retired *out, uint8_t *xhat, int32_t cap, int32_t *n_out,
                              void *stream) {
    if (!ss || !out || !n_out) return fail(GFBP_EINVAL, "null argument");
    *n_out = 0;
    if (cap <= 0) return GFBP_OK;
    hipStream_t st = static_cast<hipStream_t>(stream);
    const int n = ss->code->info.n;
    hipLaunchKernelGGL(tiled::k_tiles, dim3(1), dim3(1024), 0, st, ss->dv.done, ss->S, ss->S, 1, ss->dv.list, ss->aux + 1);
    uint32_t *hcount = static_cast<uint32_t *>(ss->pin);
    HIP_TRY(hipMemcpyAsync(hcount, ss->aux + 1, sizeof(uint32_t), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    const int k = std::min<int>(int(*hcount), cap);
    if (k == 0) return GFBP_OK;
    const size_t tot = size_t(k) * n;
    hipLaunchKernelGGL(k_collect, dim3(unsigned((tot + 255) / 256)), dim3(256), 0, st, ss->dv, k, n);
    int32_t *hlist = static_cast<int32_t *>(ss->pin);
    int32_t *hres = hlist + ss->S;
    uint64_t *hts = reinterpret_cast<uint64_t *>(hres + 2 * size_t(ss->S));  // 12 S bytes in: 8-byte aligned
    HIP_TRY(hipMemcpyAsync(hlist, ss->dv.list, sizeof(int32_t) * k, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipMemcpyAsync(hres, ss->dv.res, sizeof(int32_t) * 2 * k, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipMemcpyAsync(hts, ss->dv.ts, sizeof(uint64_t) * 2 * k, hipMemcpyDeviceToHost, st));
    if (xhat) HIP_TRY(hipMemcpyAsync(xhat, ss->dv.xout, tot, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    for (int r = 0; r < k; ++r) {
        const int slot = hlist[r];
        out[r].id = ss->id[slot];
        out[r].iters = hres[2 * r];
        out[r].converged = hres[2 * r + 1];
        out[r].t_admit = hts[2 * r];
        out[r].t_retire = hts[2 * r + 1];
        ss->id[slot] = -1;
        ss->free_slots.push_back(slot);
    }
    std::sort(ss->free_slots.begin(), ss->free_slots.end(), std::greater<int32_t>());
    ss->running -= k;
    *n_out = k;
    return GFBP_OK;
}

gfbp_status gfbp_graph_capture(gfbp_session *const *sessions, int32_t n, int32_t iters, void *stream,
                               gfbp_graph **out) {
    if (!sessions || n < 1 || !out) return fail(GFBP_EINVAL, "null argument");
    *out = nullptr;
    if (iters < 2 || iters % 2) return fail(GFBP_EINVAL, "iters must be even and >= 2");
    hipStream_t st = static_cast<hipStream_t>(stream);
    if (!st) return fail(GFBP_EINVAL, "graph capture needs a created stream, not the default stream");
    for (int k = 0; k < n; ++k)
        if (!sessions[k]) return fail(GFBP_EINVAL, "null session");
    // each session's iterations on a stream of its own, forked from and joined
    // back into the capturing stream, so the graph's session branches are
    // independent and may run concurrently
    std::vector<hipStream_t> ws(size_t(n), nullptr);
    std::vector<hipEvent_t> ev(size_t(n) + 1, nullptr);
    auto release = [&]() {
        for (auto &x : ws)
            if (x) (void)hipStreamDestroy(x);
        for (auto &e : ev)
            if (e) (void)hipEventDestroy(e);
    };
    for (int k = 0; k < n; ++k)
        if (hipStreamCreateWithFlags(&ws[k], hipStreamNonBlocking) != hipSuccess) {
            release();
            return fail(GFBP_EHIP, "creating capture streams");
        }
    for (auto &e : ev)
        if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) {
            release();
            return fail(GFBP_EHIP, "creating capture events");
        }
    if (hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal) != hipSuccess) {
        release();
        return fail(GFBP_EHIP, "hipStreamBeginCapture");
    }
    gfbp_status rs = GFBP_OK;
    hipError_t he = hipEventRecord(ev[n], st);
    for (int k = 0; k < n && rs == GFBP_OK && he == hipSuccess; ++k) {
        he = hipStreamWaitEvent(ws[k], ev[n], 0);
        if (he == hipSuccess) rs = sessions[k]->step_fn(sessions[k], iters, ws[k], sessions[k]->ntiles);
        if (rs == GFBP_OK && he == hipSuccess) he = hipEventRecord(ev[k], ws[k]);
        if (rs == GFBP_OK && he == hipSuccess) he = hipStreamWaitEvent(st, ev[k], 0);
    }
    hipGraph_t graph = nullptr;
    const hipError_t ec = hipStreamEndCapture(st, &graph);
    release();
    if (rs != GFBP_OK || he != hipSuccess) {
        if (graph) (void)hipGraphDestroy(graph);
        return rs != GFBP_OK ? rs : fail(GFBP_EHIP, std::string("graph capture: ") + hipGetErrorString(he));
    }
    if (ec != hipSuccess) return fail(GFBP_EHIP, std::string("hipStreamEndCapture: ") + hipGetErrorString(ec));
    hipGraphExec_t exec = nullptr;
    const hipError_t ei = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    if (ei != hipSuccess) {
        (void)hipGraphDestroy(graph);
        return fail(GFBP_EHIP, std::string("hipGraphInstantiate: ") + hipGetErrorString(ei));
    }
    gfbp_graph *gr = new (std::nothrow) gfbp_graph{graph, exec, iters};
    if (!gr) {
        (void)hipGraphExecDestroy(exec);
        (void)hipGraphDestroy(graph);
        return fail(GFBP_ENOMEM, "host allocation");
    }
    *out = gr;
    return GFBP_OK;
}

gfbp_status gfbp_graph_launch(gfbp_graph *g, void *stream) {
    if (!g) return fail(GFBP_EINVAL, "null graph");
    HIP_TRY(hipGraphLaunch(g->exec, static_cast<hipStream_t>(stream)));
    return GFBP_OK;
}

gfbp_status gfbp_graph_destroy(gfbp_graph *g) {
    if (!g) return GFBP_OK;
    const hipError_t e1 = hipGraphExecDestroy(g->exec), e2 = hipGraphDestroy(g->graph);
    delete g;
    if (e1 != hipSuccess || e2 != hipSuccess) return fail(GFBP_EHIP, "destroying the graph");
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
