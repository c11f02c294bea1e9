"""GPU decoder against the reference decoder, through the C ABI, at sizes the
reference finishes in seconds (the workload-size checks are in
test_gpu_configs.py).

Same seeded inputs on both sides.  Bars (tests/_parity.py):
  * messages (q, r, Q) after the first iterations within 1e-4 absolute;
  * BEC with an i.i.d. source: messages bit-identical (every value is dyadic);
  * decisions and iteration counts identical on >= 99.9% of frames, the only
    excused (logged) frames being reference near-ties before the two sides
    diverge and frames neither side decoded;
  * FER and mean iterations within each other's 95% confidence intervals.
"""
import numpy as np
import pytest

import oracle
from paper_cs_0605069_amd import workloads as wl
from tests._parity import MSG_TOL, classify, gpu_decode, messages_close, sched

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gfbp():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_cs_0605069_amd as g

    g.lib()
    return g


def _gpu(gfbp, code, fr, schedule, **kw):
    return gpu_decode(gfbp, code, gfbp.frames_to_device(fr), schedule, **kw)


def _ref(code, fr, schedule, **kw):
    return oracle.decode(code, fr, schedule=sched(schedule), **kw)


def _small_code(q, n, seed, d_v=3, d_c=6):
    m = n * d_v // d_c
    return wl.systematic(wl.make_code(n, m, d_v, q, seed, reject_4cycles=False))


def _decide(gfbp, code, fr, schedule, label, budget=0.001, **kw):
    g = _gpu(gfbp, code, fr, schedule, **kw)
    r = _ref(code, fr, schedule, **{k: v for k, v in kw.items() if k not in ("sus_strict", "persistent")})
    return classify(gfbp, code, fr, g, r, schedule, label, budget=budget, **kw), g, r


# --------------------------------------------------------------- messages
@pytest.mark.parametrize("q", [2, 4, 8, 16, 32, 64])
@pytest.mark.parametrize("schedule", ["pus", "sus"])
def test_messages_after_first_iterations(gfbp, q, schedule):
    code, enc = _small_code(q, 72, seed=100 + q)
    fr = wl.make_frames(code, enc, 13, 200 + q, "bsc", 0.09)  # 13 frames: a ragged tile
    messages_close(gfbp, code, fr, schedule, iters=(1, 2, 3), label=f"q={q}")


@pytest.mark.parametrize("q", [2, 8])
@pytest.mark.parametrize("schedule", ["pus", "sus"])
def test_bec_messages_bit_identical(gfbp, schedule, q):
    """Every BEC message value is dyadic, so it is exact in float32."""
    code, enc = _small_code(q, 96, seed=7)
    fr = wl.make_frames(code, enc, 10, 8, "bec", 0.3)
    for it in (1, 2, 4):
        g = _gpu(gfbp, code, fr, schedule, max_iter=it, early_stop=False, snap_iter=it)
        r = _ref(code, fr, schedule, max_iter=it, early_stop=False, snap_iter=it)
        for key in ("snap_q", "snap_r", "snap_Q"):
            assert np.array_equal(g[key], r[key].astype(np.float32)), f"{schedule} iter {it} {key} not bit-identical"


# --------------------------------------------------------------- decisions, small codes
@pytest.mark.parametrize("channel,param", [("bec", 0.42), ("biawgn", 0.85)])
@pytest.mark.parametrize("schedule", ["pus", "sus"])
def test_other_channels(gfbp, channel, param, schedule):
    code, enc = wl.regular_code(240, 3, 6, 8, seed=9)
    fr = wl.make_frames(code, enc, 150, 10, channel, param)
    _decide(gfbp, code, fr, schedule, f"{channel} {schedule}", max_iter=60)
    messages_close(gfbp, code, fr.subset(range(64)), schedule, iters=(1, 3), label=channel)


@pytest.mark.parametrize("q,kind", [(8, "self"), (8, "general"), (64, "self")])
@pytest.mark.parametrize("schedule", ["pus", "sus"])
def test_markov_prior(gfbp, schedule, q, kind):
    """Eq. (7) priors: a self-transition source (the device takes the O(q)
    neighbour sums) and a general transition matrix (O(q^2) sums)."""
    code, enc = wl.regular_code(300, 3, 6, q, seed=11)
    M = wl.self_transition_matrix(q, 0.7)
    if kind == "general":
        D = np.random.default_rng(0x3A7).dirichlet(np.ones(q), size=q)
        M = 0.5 * M + 0.5 * D
    pi = wl.stationary(M)
    fr = wl.make_frames(code, enc, 120, 12, "bsc", 0.1, source="markov", markov=M)
    kw = dict(prior="markov", markov_M=M, markov_pi=pi)
    messages_close(gfbp, code, fr.subset(range(64)), schedule, iters=(1, 2, 4), label=f"markov {kind}", **kw)
    _decide(gfbp, code, fr, schedule, f"markov {kind} q={q} {schedule}", max_iter=100, **kw)


@pytest.mark.parametrize("per_symbol", [False, True])
@pytest.mark.parametrize("schedule", ["pus", "sus"])
def test_static_prior(gfbp, schedule, per_symbol):
    """A fixed source prior (Section 2: a source symbol's prior multiplies its
    evidence): one vector for every source symbol, or one per symbol."""
    q = 16
    code, enc = wl.regular_code(240, 3, 6, q, seed=15)
    rng = np.random.default_rng(0x57A7)
    K, F = code.n_info, 120
    P = rng.dirichlet(np.full(q, 0.6), size=K if per_symbol else None)
    cdf = np.cumsum(np.broadcast_to(P, (K, q)), axis=1)
    u = rng.random((F, K, 1))
    s = np.minimum((u > cdf[None]).sum(axis=2), q - 1).astype(np.uint8)  # s[f][k] drawn from P_k
    cw = enc.encode(s)
    fr = wl.Frames("bsc", np.full(F, 0.11), cw, rx=wl.bsc(cw, code.p, 0.11, 16))
    kw = dict(prior="static", static_prior=P)
    messages_close(gfbp, code, fr.subset(range(64)), schedule, iters=(1, 2), label="static", **kw)
    _, g, r = _decide(gfbp, code, fr, schedule, f"static per_symbol={per_symbol} {schedule}", max_iter=60, **kw)
    u = _ref(code, fr, schedule, max_iter=60)
    assert r["converged"].mean() >= u["converged"].mean()  # the prior helps


@pytest.mark.parametrize("kind", ["self", "general"])
@pytest.mark.parametrize("strict", [False, True])
def test_prior_in_sweep(gfbp, strict, kind):
    """SUS with each source symbol's prior assigned at its column's vertical
    pass (Section 2, priors paragraph), against the reference's in-sweep
    timing: messages after iterations 1, 2 and 4, then the decisions; in the
    levelled sweep (source symbols on increasing levels) and the strict one."""
    q = 8
    code, enc = wl.regular_code(300, 3, 6, q, seed=11)
    M = wl.self_transition_matrix(q, 0.7)
    if kind == "general":
        M = 0.5 * M + 0.5 * np.random.default_rng(0x3A9).dirichlet(np.ones(q), size=q)
    pi = wl.stationary(M)
    fr = wl.make_frames(code, enc, 120, 13, "bsc", 0.11 if kind == "self" else 0.07, source="markov", markov=M)
    kw = dict(prior="markov", markov_M=M, markov_pi=pi, prior_in_sweep=True)
    dcode = gfbp.DeviceCode(code)
    assert dcode.info.sus_levels_in_sweep >= code.n_info > dcode.info.sus_levels
    messages_close(gfbp, code, fr.subset(range(64)), "sus", iters=(1, 2, 4), label="in-sweep", sus_strict=strict, **kw)
    d = _gpu(gfbp, code, fr, "sus", max_iter=2, early_stop=False, snap_iter=2, prior="markov", markov_M=M,
             markov_pi=pi)
    g = _gpu(gfbp, code, fr, "sus", max_iter=2, early_stop=False, snap_iter=2, **kw)
    assert np.abs(d["snap_Q"] - g["snap_Q"]).max() > 1e-3  # the timing matters from iteration 2 on
    _decide(gfbp, code, fr, "sus", f"in-sweep {kind} strict={strict}", max_iter=100, sus_strict=strict, **kw)


def test_prior_in_sweep_levelled_is_bitwise_strict_and_errors(gfbp):
    import ctypes

    q = 16
    code, enc = wl.regular_code(256, 3, 6, q, seed=14)
    M = wl.self_transition_matrix(q, 0.8)
    pi = wl.stationary(M)
    fr = wl.make_frames(code, enc, 70, 15, "biawgn", 0.75, source="markov", markov=M)
    kw = dict(prior="markov", markov_M=M, markov_pi=pi, prior_in_sweep=True, max_iter=50, posterior=True)
    a = _gpu(gfbp, code, fr, "sus", **kw)
    b = _gpu(gfbp, code, fr, "sus", sus_strict=True, **kw)
    for k in ("xhat", "iters", "converged", "posterior"):
        assert np.array_equal(a[k], b[k]), k
    with pytest.raises(gfbp.GfbpError):
        _gpu(gfbp, code, fr, "pus", **kw)
    dcode = gfbp.DeviceCode(code)
    d = gfbp.SessionDesc(64, gfbp.SCHEDULES["sus"], 10, 0, None, None, gfbp.OPT_PRIOR_IN_SWEEP, 0)
    h = ctypes.c_void_p()
    assert gfbp.lib().gfbp_session_create(dcode.handle, ctypes.byref(d), ctypes.byref(h)) != 0 and not h.value


@pytest.mark.parametrize("schedule", ["pus", "sus"])
def test_nonzero_syndrome_and_given_likelihoods(gfbp, schedule):
    """Coset decoding (H x = z with z != 0) from raw likelihood vectors."""
    import torch

    q = 16
    code, enc = _small_code(q, 120, seed=13)
    rng = np.random.default_rng(14)
    F = 40
    x = rng.integers(0, q, size=(F, code.n)).astype(np.uint8)
    z = wl.syndromes(code, x)
    noisy = wl.bsc(x, code.p, 0.05, 15)
    L = np.stack([oracle.likelihood(code.p, "bsc", 0.05, rx=int(v)) for v in noisy.ravel()]).reshape(F, code.n, q)
    L32 = L.astype(np.float32)
    dcode = gfbp.DeviceCode(code)
    dfr = {"channel": "likelihood", "F": F, "likelihood": torch.from_numpy(L32).cuda(),
           "syndrome": torch.from_numpy(z).cuda()}
    out = gfbp.decode_batch(dcode, dfr, schedule=schedule, max_iter=50)
    g = {k: v.cpu().numpy() for k, v in out.items()}
    fr = wl.Frames("likelihood", np.zeros(F), x)
    fr.lik = L32
    fr.syndrome = z
    r = oracle.decode(code, likelihoods=L32.astype(np.float64), syndrome=z, schedule=sched(schedule), max_iter=50)
    classify(gfbp, code, fr, g, r, schedule, f"coset {schedule}", max_iter=50)
    assert (g["xhat"][g["converged"] == 1] == x[g["converged"] == 1]).mean() > 0.99


# --------------------------------------------------------------- readings R13 and R14
@pytest.mark.parametrize("schedule", ["pus", "sus"])
def test_zero_evidence_row_is_uniform_with_one_guard(gfbp, schedule):
    """Reading R13: a likelihood row of zeros normalises to the uniform vector
    and counts one guard event, on both sides; the frames still decode."""
    import torch

    q = 8
    code, enc = _small_code(q, 96, seed=51)
    fr = wl.make_frames(code, enc, 20, 52, "bsc", 0.03)
    L = oracle.frame_likelihoods(code, fr)
    zero_cols = [3, 40, 77]
    L[:, zero_cols, :] = 0.0
    L32 = L.astype(np.float32)
    dcode = gfbp.DeviceCode(code)
    dfr = {"channel": "likelihood", "F": fr.F, "likelihood": torch.from_numpy(L32).cuda()}
    out = gfbp.decode_batch(dcode, dfr, schedule=schedule, max_iter=1, early_stop=False, snap_iter=1)
    r = oracle.decode(code, likelihoods=L32.astype(np.float64), schedule=sched(schedule), max_iter=1,
                      early_stop=False, snap_iter=1)
    g = {k: v.cpu().numpy() for k, v in out.items()}
    assert (r["guards"] == len(zero_cols)).all()
    assert np.array_equal(g["guards"], r["guards"])
    assert np.abs(g["snap_q"] - r["snap_q"]).max() <= MSG_TOL
    # the q-messages of a zero row's edges start uniform: after one
    # iteration they carry the other edges' r only, so they are not zero
    out = gfbp.decode_batch(dcode, dfr, schedule=schedule, max_iter=40)
    torch.cuda.synchronize()
    assert out["converged"].float().mean().item() > 0.9


@pytest.mark.parametrize("schedule", ["pus", "sus"])
def test_exact_tie_takes_the_smallest_symbol(gfbp, schedule):
    """Reading R14: a column whose pseudo-posterior is exactly flat (uniform
    evidence, in no check) and a column whose evidence ties two symbols
    exactly are decided as the smallest tied symbol on both sides."""
    import torch

    q = 8
    code, enc = _small_code(q, 48, seed=23)
    ext = wl.Code(code.q, code.n + 2, code.m, code.row_ptr, code.col, code.coef, poly=code.poly,
                  n_info=code.n_info)
    fr = wl.make_frames(code, enc, 12, 24, "bsc", 0.02)
    L = oracle.frame_likelihoods(code, fr)
    flat = np.full((fr.F, 1, q), 1.0 / q)
    two = np.zeros((fr.F, 1, q))
    two[:, 0, 5] = two[:, 0, 3] = 0.5  # symbols 3 and 5 tie exactly
    Lx = np.concatenate([L, flat, two], axis=1).astype(np.float32)
    dfr = {"channel": "likelihood", "F": fr.F, "likelihood": torch.from_numpy(Lx).cuda()}
    out = gfbp.decode_batch(gfbp.DeviceCode(ext), dfr, schedule=schedule, max_iter=20)
    r = oracle.decode(ext, likelihoods=Lx.astype(np.float64), schedule=sched(schedule), max_iter=20)
    g = {k: v.cpu().numpy() for k, v in out.items()}
    assert (r["xhat"][:, -2] == 0).all() and (r["xhat"][:, -1] == 3).all()
    assert np.array_equal(g["xhat"], r["xhat"]) and np.array_equal(g["iters"], r["iters"])


# --------------------------------------------------------------- visiting order and source chain
@pytest.mark.parametrize("prior", ["uniform", "markov"])
def test_visit_order_and_source_chain(gfbp, prior):
    """A SUS visiting order other than 0..n-1 and a source chain over
    scattered columns (gfbp_code_desc visit_order, source_cols), against the
    reference with the same orders: messages after iterations 1-3, decisions,
    and the orders matter (the identity orders give other messages)."""
    q = 8
    base, enc = wl.regular_code(240, 3, 6, q, seed=61)
    rng = np.random.default_rng(62)
    perm = rng.permutation(base.n)  # column j of the new code is column perm[j] of the old
    inv = np.argsort(perm)
    code = wl.Code(q, base.n, base.m, base.row_ptr, inv[base.col].astype(np.int32), base.coef, poly=base.poly,
                   n_info=base.n_info)
    code.source_cols = inv[np.arange(base.n_info)].astype(np.int32)  # the chain in the old order
    code.visit_order = rng.permutation(base.n).astype(np.int32)
    M = wl.self_transition_matrix(q, 0.75)
    kw = dict(prior="markov", markov_M=M, markov_pi=wl.stationary(M)) if prior == "markov" else {}
    f0 = wl.make_frames(base, enc, 100, 63, "bsc", 0.1, source="markov" if kw else "iid",
                        markov=M if kw else None)
    fr = wl.Frames("bsc", f0.param, f0.codeword[:, perm], rx=f0.rx[:, perm])
    messages_close(gfbp, code, fr.subset(range(48)), "sus", iters=(1, 2, 3), label="orders", **kw)
    messages_close(gfbp, code, fr.subset(range(48)), "pus", iters=(1, 2), label="orders", **kw)
    for sch in ("pus", "sus"):
        _decide(gfbp, code, fr, sch, f"orders {prior} {sch}", max_iter=60, **kw)
    plain = wl.Code(q, code.n, code.m, code.row_ptr, code.col, code.coef, poly=code.poly, n_info=code.n_info)
    plain.source_cols = code.source_cols
    a = _gpu(gfbp, code, fr, "sus", max_iter=2, early_stop=False, snap_iter=2, **kw)
    b = _gpu(gfbp, plain, fr, "sus", max_iter=2, early_stop=False, snap_iter=2, **kw)
    assert np.abs(a["snap_q"] - b["snap_q"]).max() > 1e-3


# --------------------------------------------------------------- per-frame channels
@pytest.mark.parametrize("schedule", ["pus", "sus"])
def test_per_frame_channel_kinds(gfbp, schedule):
    """One batch mixing BSC, BEC and BI-AWGN frames (gfbp_batch channel_of)
    equals each channel's frames decoded alone, bitwise."""
    import torch

    q = 16
    code, enc = wl.regular_code(200, 3, 6, q, seed=71)
    parts = [wl.make_frames(code, enc, 30, 72, "bsc", 0.06), wl.make_frames(code, enc, 25, 73, "bec", 0.35),
             wl.make_frames(code, enc, 35, 74, "biawgn", 0.8)]
    mix = gfbp.frames_for_session(parts)
    mix["channel_of"] = mix["channel"]  # per-frame kinds (device uint8)
    mix["channel"] = "bsc"
    assert torch.equal(mix["channel_of"].cpu(), torch.from_numpy(
        np.concatenate([np.full(p.F, gfbp.CHANNELS[p.channel], np.uint8) for p in parts])))
    g = gpu_decode(gfbp, code, mix, schedule, max_iter=40, posterior=True)
    o = 0
    for p in parts:
        a = _gpu(gfbp, code, p, schedule, max_iter=40, posterior=True)
        for k in ("xhat", "iters", "converged", "posterior"):
            assert np.array_equal(g[k][o:o + p.F], a[k]), f"{p.channel} {k}"
        o += p.F


# --------------------------------------------------------------- batching properties
@pytest.mark.parametrize("schedule", ["pus", "sus"])
def test_frame_alone_equals_frame_in_batch_and_runs_repeat(gfbp, schedule):
    code, enc = wl.regular_code(200, 3, 6, 16, seed=17)
    fr = wl.make_frames(code, enc, 37, 18, "bsc", 0.07)
    a = _gpu(gfbp, code, fr, schedule, max_iter=40, posterior=True)
    b = _gpu(gfbp, code, fr, schedule, max_iter=40, posterior=True)
    for k in ("xhat", "iters", "converged", "posterior"):
        assert np.array_equal(a[k], b[k]), f"run-to-run difference in {k}"
    for f in (0, 5, 36):
        one = _gpu(gfbp, code, fr.subset([f]), schedule, max_iter=40, posterior=True)
        assert np.array_equal(one["posterior"][0], a["posterior"][f])
        assert one["iters"][0] == a["iters"][f]


@pytest.mark.parametrize("schedule", ["pus", "sus"])
def test_markov_posteriors_alone_equal_in_batch(gfbp, schedule):
    """With a Markov source, frames that stop at different iterations: each
    frame's posterior, decisions and iteration count in the batch equal those
    of the frame decoded alone (the posterior read back is the frame's own
    last one)."""
    q = 16
    code, enc = wl.regular_code(200, 3, 6, q, seed=27)
    M = wl.self_transition_matrix(q, 0.7)
    kw = dict(prior="markov", markov_M=M, markov_pi=wl.stationary(M), max_iter=40, posterior=True)
    fr = wl.make_frames(code, enc, 60, 28, "bsc", np.linspace(0.03, 0.12, 60), source="markov", markov=M)
    a = _gpu(gfbp, code, fr, schedule, **kw)
    assert len(set(a["iters"].tolist())) > 3  # frames stop at different iterations
    for f in (0, 7, 30, 59):
        one = _gpu(gfbp, code, fr.subset([f]), schedule, **kw)
        assert one["iters"][0] == a["iters"][f] and np.array_equal(one["xhat"][0], a["xhat"][f])
        assert np.array_equal(one["posterior"][0], a["posterior"][f]), f"frame {f}"


@pytest.mark.parametrize("schedule,q", [("pus", 8), ("sus", 8), ("sus-in-sweep", 8), ("pus", 2), ("sus", 2)])
def test_frame_compaction_changes_nothing(gfbp, schedule, q):
    """Moving running frames into finished slots (on by default) gives bitwise
    the outputs of decoding with every frame in place, with a Markov prior and
    a syndrome (and, for priors assigned during the sweep, the source symbols'
    pseudo-posteriors the next sweep reads); the batch mixes fast and slow
    frames so that compaction runs several times."""
    code, enc = wl.regular_code(240, 3, 6, q, seed=37)
    M = wl.self_transition_matrix(q, 0.7)
    pi = wl.stationary(M)
    fr = wl.make_frames(code, enc, 700, 38, "bsc", np.linspace(0.02, 0.14, 700), source="markov", markov=M)
    z = np.random.default_rng(39).integers(0, q, size=(fr.F, code.m)).astype(np.uint8)
    z[::3] = 0
    fr.syndrome = z
    dfr = gfbp.frames_to_device(fr)
    outs = [gpu_decode(gfbp, code, dfr, schedule[:3], max_iter=60, prior="markov", markov_M=M, markov_pi=pi,
                       compact=compact, prior_in_sweep=schedule.endswith("in-sweep"), onchip=False)
            for compact in (False, True)]
    it = outs[0]["iters"]
    assert it.min() < 10 and (it == 60).sum() > 20  # fast and slow frames
    for k in ("xhat", "iters", "converged", "guards"):
        assert np.array_equal(outs[0][k], outs[1][k]), k


def test_edge_cases(gfbp):
    import torch

    code, enc = _small_code(4, 48, seed=19)
    fr = wl.make_frames(code, enc, 1, 20, "bsc", 0.05)
    for sch in ("pus", "sus"):
        g = _gpu(gfbp, code, fr, sch, max_iter=1)
        r = _ref(code, fr, sch, max_iter=1)
        assert np.array_equal(g["xhat"], r["xhat"]) and np.array_equal(g["iters"], r["iters"])
    # zero frames is a no-op
    dcode = gfbp.DeviceCode(code)
    empty = {"channel": "bsc", "F": 0, "param": torch.zeros(0, device="cuda"),
             "rx": torch.zeros((0, code.n), dtype=torch.uint8, device="cuda")}
    out = gfbp.decode_batch(dcode, empty, schedule="pus")
    assert out["xhat"].shape == (0, code.n)
    # workspace too small is refused
    with pytest.raises(gfbp.GfbpError) as ei:
        gfbp.decode_batch(dcode, gfbp.frames_to_device(fr), workspace=torch.empty(16, dtype=torch.uint8, device="cuda"))
    assert ei.value.status == -5
    # a channel whose input is missing is refused before any launch
    with pytest.raises(gfbp.GfbpError) as ei:
        gfbp.decode_batch(dcode, {"channel": "biawgn", "F": 1, "param": torch.ones(1, device="cuda")})
    assert ei.value.status == -1
    # LIKELIHOOD with the MN evidence mode is refused
    with pytest.raises(gfbp.GfbpError):
        gfbp.decode_batch(dcode, {"channel": "likelihood", "F": 1, "evidence": "mn",
                                  "likelihood": torch.ones((1, code.n, 4), device="cuda")})


@pytest.mark.parametrize("schedule", ["pus", "sus"])
def test_largest_shape_gf64_n8000_sampled(gfbp, schedule):
    """The largest shape the workloads use: GF(64), N = 8000, (3,6) (E =
    24000, so q-message offsets pass 2^32 at 4096 frames), syndrome-form
    BI-AWGN frames, in the bench's batch size; pseudo-posteriors and
    decisions after 3 iterations of the first, a middle and the last frame
    against the reference."""
    import torch

    code = wl.make_code(8000, 4000, 3, 64, seed=0xC0DE8000)
    fr = wl.make_coset_frames(code, 4096, 0xDA7A8000, "biawgn", 0.75)
    assert code.E * 64 * 4096 > 2 ** 32
    dcode = gfbp.DeviceCode(code)
    out = gfbp.decode_batch(dcode, gfbp.frames_to_device(fr), schedule=schedule, max_iter=3, early_stop=False,
                            posterior=True)
    torch.cuda.synchronize()
    idx = [0, 2047, 4095]
    post = out["posterior"][idx].cpu().numpy()
    xh = out["xhat"][idx].cpu().numpy()
    it = out["iters"][idx].cpu().numpy()
    del out
    torch.cuda.empty_cache()
    r = oracle.decode(code, fr.subset(idx), schedule=sched(schedule), max_iter=3, early_stop=False, posterior=True,
                      gap_trace=True)
    assert np.abs(post - r["posterior"]).max() <= MSG_TOL
    # decisions differ only where the reference's two largest entries are within the message tolerance
    P = np.sort(r["posterior"], axis=2)
    off = xh != r["xhat"]
    assert (P[:, :, -1] - P[:, :, -2])[off].max(initial=0.0) < 2 * MSG_TOL
    assert np.array_equal(it, r["iters"])


def _random_irregular_code(rng, q, n, m):
    """Column degrees 1..5, rows of 2..16 entries, random nonzero coefficients."""
    while True:
        cols_of_row = [set() for _ in range(m)]
        for j in range(n):
            for i in rng.choice(m, size=int(rng.integers(1, 6)), replace=False):
                cols_of_row[i].add(j)
        sizes = [len(r) for r in cols_of_row]
        if min(sizes) >= 2 and max(sizes) <= 16:
            break
    row_ptr = np.zeros(m + 1, dtype=np.int32)
    row_ptr[1:] = np.cumsum(sizes)
    col = np.array([c for r in cols_of_row for c in sorted(r)], dtype=np.int32)
    coef = rng.integers(1, q, size=len(col)).astype(np.uint8)
    code = wl.Code(q=q, n=n, m=m, row_ptr=row_ptr, col=col, coef=coef)
    code.n_info = n // 2
    return code


@pytest.mark.parametrize("seed", range(8))
def test_random_irregular_codes(gfbp, seed):
    """Seeded random irregular codes (every field, column degrees 1-5, rows up
    to 16, syndromes z != 0, a random channel, Markov prior or not): messages
    after 2 iterations and decisions after up to 40, both schedules."""
    rng = np.random.default_rng([0x12E6, seed])
    q = int(2 ** (1 + seed % 6))
    n = int(rng.integers(40, 160))
    code = _random_irregular_code(rng, q, n, int(n * rng.uniform(0.4, 0.7)))
    channel, param = [("bsc", 0.04), ("bec", 0.3), ("biawgn", 0.7)][seed % 3]
    markov = seed % 2 == 1
    M = wl.self_transition_matrix(q, 0.75) if markov else None
    if markov and seed % 4 == 3:
        M = 0.5 * M + 0.5 * rng.dirichlet(np.ones(q), size=q)
    fr = wl.make_coset_frames(code, 70, 500 + seed, channel, param, source="markov" if markov else "iid", markov=M)
    kw = dict(prior="markov", markov_M=M, markov_pi=wl.stationary(M)) if markov else {}
    for sch in ("pus", "sus"):
        messages_close(gfbp, code, fr, sch, iters=(2,), label=f"random {seed}", **kw)
        _decide(gfbp, code, fr, sch, f"random seed {seed} q={q} n={n} {channel} markov={markov} {sch}",
                max_iter=40, **kw)


def test_column_without_edges(gfbp):
    """A column in no check: its pseudo-posterior is its channel likelihood
    alone, under every schedule (the sequential step still decides it)."""
    code, enc = _small_code(8, 48, seed=23)
    fr = wl.make_frames(code, enc, 20, 24, "bsc", 0.05)
    ext = wl.Code(code.q, code.n + 1, code.m, code.row_ptr, code.col, code.coef, poly=code.poly, n_info=code.n_info)
    extra = np.random.default_rng(25).integers(0, code.q, size=(fr.F, 1)).astype(np.uint8)
    fr2 = wl.Frames("bsc", fr.param, np.hstack([fr.codeword, extra]), rx=np.hstack([fr.rx, extra]))
    for sch, strict in (("pus", False), ("sus", False), ("sus", True)):
        g = _gpu(gfbp, ext, fr2, sch, max_iter=30, sus_strict=strict)
        r = _ref(ext, fr2, sch, max_iter=30)
        assert np.array_equal(g["xhat"], r["xhat"]) and np.array_equal(g["iters"], r["iters"]), f"{sch} strict={strict}"
        assert np.array_equal(g["xhat"][:, -1], extra[:, 0])


def test_degree_limits(gfbp):
    """Row degree 16 and column degree 8 (the kernels' limits)."""
    q = 4
    code = wl.make_code(64, 32, 8, q, seed=21, reject_4cycles=False)
    assert code.row_degrees().max() == 16 and code.col_degrees().max() == 8
    code, enc = wl.systematic(code)
    fr = wl.make_frames(code, enc, 9, 22, "bsc", 0.02)
    for sch in ("pus", "sus"):
        g = _gpu(gfbp, code, fr, sch, max_iter=2, early_stop=False, snap_iter=2)
        r = _ref(code, fr, sch, max_iter=2, early_stop=False, snap_iter=2)
        assert np.abs(g["snap_q"] - r["snap_q"]).max() <= MSG_TOL


# --------------------------------------------------------------- MN syndrome form (Section 2)
# The syndrome-form stand-ins are decoded near their threshold, where a few
# frames run tens of iterations on the edge of failing: there about 0.1% of
# frames (SUS: 3 of 2100 over these cases) drift apart after 8-19 iterations
# and flip a decision whose reference margin is 1e-3..1e-2, after the GPU's
# float32-stored messages have moved away from the float64 ones (the gate logs
# each such frame's posterior drift by iteration).  These gates allow 0.5% of
# such frames; the workload-size gates (test_gpu_configs.py) keep 0.1%.
MN_BUDGET = 0.005

_MN_SOURCES = {
    "iid": (None, None),
    "4s": (wl.PAPER_MARKOV_4S, wl.stationary(wl.PAPER_MARKOV_4S)),
    "2s": wl.lift_binary_chain(wl.PAPER_MARKOV_2S, 3),
}


@pytest.mark.parametrize("q,source,channel,param", [(2, "iid", "bsc", 0.1), (4, "4s", "bec", 0.55),
                                                    (8, "2s", "biawgn", 1.1), (4, "4s", "bsc", 0.17),
                                                    (8, "2s", "bec", 0.6), (4, "iid", "biawgn", 0.9)])
@pytest.mark.parametrize("schedule", ["pus", "sus"])
def test_mn_syndrome_form(gfbp, q, source, channel, param, schedule):
    """H = [A B], x = (source, noise), z = B r: the decoder sees z and the
    channel outputs at the noise columns; the GPU computes the noise symbols'
    evidence itself (GFBP_EVIDENCE_MN), the reference independently."""
    code = wl.mn_code(60, 180, q, seed=400 + q)
    M, start = _MN_SOURCES[source]
    fr = wl.make_mn_frames(code, 300, 401 + q, channel, param, source="iid" if M is None else "markov",
                           markov=M, start=start)
    kw = {} if M is None else dict(prior="markov", markov_M=M, markov_pi=start)
    messages_close(gfbp, code, fr.subset(range(64)), schedule, iters=(1, 2), label=f"MN {channel}", **kw)
    _, g, r = _decide(gfbp, code, fr, schedule, f"MN q={q} {source} {channel} {schedule}", max_iter=80,
                      budget=MN_BUDGET, **kw)
    ok = g["converged"].astype(bool)
    assert r["converged"].mean() > 0.5  # a meaningful share of frames decodes
    assert np.array_equal(wl.syndromes(code, g["xhat"][ok]), fr.syndrome[ok])


@pytest.mark.parametrize("q,source,channel,param", [(4, "4s", "bsc", 0.17), (8, "2s", "biawgn", 1.1)])
@pytest.mark.parametrize("schedule", ["pus", "sus"])
def test_mn_pool_form(gfbp, q, source, channel, param, schedule):
    """The syndrome form on the pooled-B stand-in (few dependency levels: SUS
    runs by level launches, not by runs of thin levels): decisions under the
    gate, messages after iterations 1 and 2, and levelled SUS bitwise the
    strict column order."""
    code = wl.mn_code(60, 180, q, seed=430 + q, b_form="pool", pool=12)
    M, start = _MN_SOURCES[source]
    fr = wl.make_mn_frames(code, 300, 431 + q, channel, param, source="markov", markov=M, start=start)
    kw = dict(prior="markov", markov_M=M, markov_pi=start)
    assert gfbp.DeviceCode(code).info.sus_levels == _sus_levels(code) < 60
    messages_close(gfbp, code, fr.subset(range(64)), schedule, iters=(1, 2), label="MN pool", **kw)
    _, g, r = _decide(gfbp, code, fr, schedule, f"MN pool q={q} {source} {channel} {schedule}", max_iter=80,
                      budget=MN_BUDGET, **kw)
    assert r["converged"].mean() > 0.5
    if schedule == "sus":
        a = _gpu(gfbp, code, fr.subset(range(40)), "sus", max_iter=60, posterior=True, **kw)
        b = _gpu(gfbp, code, fr.subset(range(40)), "sus", sus_strict=True, max_iter=60, posterior=True, **kw)
        for k in a:
            assert np.array_equal(a[k], b[k]), f"levelled and strict SUS differ in {k}"


@pytest.mark.parametrize("q,source,channel,param", [(4, "4s", "bsc", 0.17), (8, "2s", "biawgn", 1.1)])
def test_mn_syndrome_form_prior_in_sweep(gfbp, q, source, channel, param):
    """The MN syndrome form with the source priors assigned during the SUS
    sweep (in-sweep timing): messages after iterations 2 and 3, then decisions."""
    code = wl.mn_code(60, 180, q, seed=410 + q)
    M, start = _MN_SOURCES[source]
    fr = wl.make_mn_frames(code, 300, 411 + q, channel, param, source="markov", markov=M, start=start)
    kw = dict(prior="markov", markov_M=M, markov_pi=start, prior_in_sweep=True)
    messages_close(gfbp, code, fr.subset(range(64)), "sus", iters=(2, 3), label="MN in-sweep", **kw)
    _, g, r = _decide(gfbp, code, fr, "sus", f"MN in-sweep q={q} {source} {channel}", max_iter=80,
                      budget=MN_BUDGET, **kw)
    assert r["converged"].mean() > 0.5


@pytest.mark.parametrize("schedule", ["pus", "sus"])
def test_trace_of_correct_source_bits(gfbp, schedule):
    """The per-iteration count of correct source bits (Fig. 1 diagnostic)
    equals the count from the reference's decisions after each iteration, on
    frames whose decisions match the reference's at every iteration."""
    import torch

    q, p = 4, 2
    code = wl.mn_code(60, 180, q, seed=420)
    M, start = _MN_SOURCES["4s"]
    fr = wl.make_mn_frames(code, 120, 421, "biawgn", 1.2, source="markov", markov=M, start=start)
    kw = dict(prior="markov", markov_M=M, markov_pi=start)
    dcode = gfbp.DeviceCode(code)
    out = gfbp.decode_batch(dcode, gfbp.frames_to_device(fr), schedule=schedule, max_iter=60,
                            truth=torch.from_numpy(fr.codeword).cuda(), **kw)
    torch.cuda.synchronize()
    g = {k: v.cpu().numpy() for k, v in out.items()}
    r = oracle.decode(code, fr, schedule=sched(schedule), max_iter=60, trace=True, **kw)
    K = code.n_info
    same = (g["xhat"] == r["xhat"]).all(axis=1) & (g["iters"] == r["iters"]) & (r["converged"] == 1)
    assert same.mean() > 0.9
    exact = 0
    for f in np.nonzero(same)[0]:
        t = int(r["iters"][f])
        wrong = np.unpackbits((r["trace"][f, :t, :K] ^ fr.codeword[f, None, :K])[..., None], axis=-1).sum(axis=(1, 2))
        exact += int(np.array_equal(g["trace"][f, :t], p * K - wrong))
        assert g["trace"][f, t - 1] == p * K - wrong[-1], f"frame {f}"  # the final decision is the same
        assert (g["trace"][f, t:] == 0).all()
    assert exact >= 0.95 * same.sum(), f"{exact} of {int(same.sum())} traces identical"


# --------------------------------------------------------------- SUS by dependency levels
def _sus_levels(code):
    rows = code.row_of_edge()
    top = -np.ones(code.m, dtype=np.int64)
    nlev = 0
    for j in range(code.n):
        r = rows[code.col == j]
        lv = int(top[r].max()) + 1 if len(r) else 0
        top[r] = lv
        nlev = max(nlev, lv + 1)
    return nlev


@pytest.mark.parametrize("q,channel,param,prior", [(4, "bsc", 0.07, "uniform"), (16, "biawgn", 0.85, "uniform"),
                                                   (8, "bsc", 0.1, "markov"), (64, "bec", 0.4, "uniform")])
def test_levelled_sus_is_bitwise_the_strict_sweep(gfbp, q, channel, param, prior):
    """Columns of one dependency level share no check, so running a level at
    once reproduces the strict column order exactly."""
    code, enc = wl.regular_code(300 if q < 64 else 120, 3, 6, q, seed=31 + q)
    kw = {}
    src = "iid"
    if prior == "markov":
        M = wl.self_transition_matrix(q, 0.7)
        kw = dict(prior="markov", markov_M=M, markov_pi=wl.stationary(M))
        src = "markov"
    fr = wl.make_frames(code, enc, 50, 32 + q, channel, param, source=src, markov=kw.get("markov_M"))
    dcode = gfbp.DeviceCode(code)
    assert dcode.info.sus_levels == _sus_levels(code)
    assert dcode.info.sus_levels < code.n // 3
    for extra in (dict(max_iter=40, posterior=True), dict(max_iter=3, early_stop=False, snap_iter=2)):
        a = _gpu(gfbp, code, fr, "sus", **extra, **kw)
        b = _gpu(gfbp, code, fr, "sus", sus_strict=True, **extra, **kw)
        for k in a:
            assert np.array_equal(a[k], b[k]), f"levelled and strict SUS differ in {k}"


@pytest.mark.parametrize("q,source", [(4, "4s"), (8, "2s")])
def test_thin_level_runs_are_bitwise_the_strict_sweep(gfbp, q, source):
    """An MN syndrome-form code (B's chain: most levels hold one or two
    columns, walked in runs of levels per tile): levelled SUS, also with the
    priors assigned during the sweep, equals the strict column order."""
    M, start = _MN_SOURCES[source]
    code = wl.mn_code(60, 180, q, seed=41 + q)
    fr = wl.make_mn_frames(code, 40, 42 + q, "bsc", 0.12, source="markov", markov=M, start=start)
    for in_sweep in (False, True):
        kw = dict(prior="markov", markov_M=M, markov_pi=start, prior_in_sweep=in_sweep)
        for extra in (dict(max_iter=60, posterior=True), dict(max_iter=3, early_stop=False, snap_iter=3)):
            a = _gpu(gfbp, code, fr, "sus", **extra, **kw)
            b = _gpu(gfbp, code, fr, "sus", sus_strict=True, **extra, **kw)
            for k in a:
                assert np.array_equal(a[k], b[k]), f"in_sweep={in_sweep}: levelled and strict SUS differ in {k}"


# --------------------------------------------------------------- kernel shapes and the tuner
@pytest.mark.parametrize("q", [2, 4, 8, 16, 32, 64])
def test_every_kernel_shape_matches_the_reference(gfbp, q):
    """Each allowed entries-per-lane choice (EL = 2, 4, 8) is a different
    register/lane split of the same arithmetic; all must match the oracle."""
    import torch

    code, enc = _small_code(q, 72, seed=300 + q)
    fr = wl.make_frames(code, enc, 13, 301 + q, "bsc", 0.08)
    dcode = gfbp.DeviceCode(code)
    dfr = gfbp.frames_to_device(fr)
    for sch in ("pus", "sus"):
        r = _ref(code, fr, sch, max_iter=2, early_stop=False, snap_iter=2)
        for el in (2, 4, 8, 16):
            if el > q or el == 16:
                with pytest.raises(gfbp.GfbpError):
                    dcode.set_shape(sch, el)
                continue
            dcode.set_shape(sch, el)
            assert dcode.shape(sch) == el
            out = gfbp.decode_batch(dcode, dfr, schedule=sch, max_iter=2, early_stop=False, snap_iter=2)
            torch.cuda.synchronize()
            for key in ("snap_q", "snap_r", "snap_Q"):
                err = np.abs(out[key].cpu().numpy() - r[key]).max()
                assert err <= MSG_TOL, f"q={q} {sch} EL={el} {key}: {err:.3g}"


def test_tuner_keeps_an_allowed_shape_and_decodes_correctly(gfbp):
    code, enc = wl.regular_code(240, 3, 6, 16, seed=41)
    fr = wl.make_frames(code, enc, 200, 42, "bsc", 0.07)
    dcode = gfbp.DeviceCode(code)
    dfr = gfbp.frames_to_device(fr)
    for sch in ("pus", "sus"):
        el = gfbp.tune(dcode, dfr, schedule=sch, trial_iters=2)
        assert el in (2, 4, 8) and dcode.shape(sch) == el
        out = gfbp.decode_batch(dcode, dfr, schedule=sch, max_iter=50)
        g = {k: v.cpu().numpy() for k, v in out.items()}
        r = _ref(code, fr, sch, max_iter=50)
        classify(gfbp, code, fr, g, r, sch, f"tuned EL={el} {sch}", max_iter=50)


def test_stream_copy_rate_copies_and_reports_a_rate(gfbp):
    import torch

    src = torch.randint(0, 256, (64 << 20,), dtype=torch.uint8, device="cuda")
    dst = torch.zeros_like(src)
    rate = gfbp.stream_copy_rate(dst, src, reps=2)
    assert torch.equal(dst, src)
    assert 1e11 < rate < 1e14  # bytes/s read + write (the buffers fit the last-level cache)
    tail = torch.randint(0, 256, (4096 + 48,), dtype=torch.uint8, device="cuda")  # not a whole block of vectors
    out = torch.zeros_like(tail)
    gfbp.stream_copy_rate(out, tail, reps=1)
    assert torch.equal(out, tail)
