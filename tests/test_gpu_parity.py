"""GPU decoder against the reference decoder, through the C ABI.

Same seeded inputs on both sides.  Bars:
  * messages (q, r, Q) after the first iterations within 1e-4 absolute;
  * BEC with an i.i.d. source: messages bit-identical (every value is dyadic);
  * decisions and iteration counts identical on >= 99.9% of frames, the
    exceptions (logged) being frames the reference itself did not converge
    on ("chaotic") and frames whose reference outcome changes when its own
    float64 inputs are rounded to float32 or moved by a relative 1e-6
    ("precision-sensitive");
  * FER and mean iterations within each other's 95% confidence intervals.
"""
import math

import numpy as np
import pytest

import oracle
from paper_cs_0605069_amd import workloads as wl

pytestmark = pytest.mark.gpu

MSG_TOL = 1e-4


@pytest.fixture(scope="module")
def gfbp():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_cs_0605069_amd as g

    g.lib()
    return g


def _gpu(gfbp, code, fr, schedule, **kw):
    import torch

    dcode = gfbp.DeviceCode(code)
    out = gfbp.decode_batch(dcode, gfbp.frames_to_device(fr), schedule=schedule, **kw)
    torch.cuda.synchronize()
    return {k: v.cpu().numpy() for k, v in out.items()}


def _ref(code, fr, schedule, **kw):
    return oracle.decode(code, fr, schedule=gfbp_sched(schedule), **kw)


def gfbp_sched(s):
    return {"pus": oracle.PUS, "sus": oracle.SUS}[s]


def _small_code(q, n, seed, d_v=3, d_c=6):
    m = n * d_v // d_c
    return wl.systematic(wl.make_code(n, m, d_v, q, seed, reject_4cycles=False))


def _precision_sensitive(code, fr, schedule, idx, **kw):
    """Frames (of idx) whose reference outcome is not determined at float32
    precision: it changes when the reference's own float64 inputs (channel
    likelihoods, Markov matrix and start distribution) are rounded to float32,
    as the GPU decoder stores them, or perturbed by a relative 1e-6 (a few
    float32 rounding steps) in either of two seeded random directions, or
    when the reference keeps its messages in float32 (as the GPU does), or
    also drops r entries below the resolution of a double-precision
    transform (4e-16 of the largest; the GPU evaluates Eq. (3) through a
    Walsh-Hadamard transform, whose small outputs are differences of
    order-one terms)."""
    if len(idx) == 0:
        return np.zeros(0, dtype=bool)
    sub = fr.subset(idx)
    L = sub.lik.astype(np.float64) if sub.lik is not None else oracle.frame_likelihoods(code, sub)
    kw = {k: v for k, v in kw.items() if k not in ("snap_iter", "posterior")}
    sch = gfbp_sched(schedule)
    a = oracle.decode(code, likelihoods=L, syndrome=sub.syndrome, schedule=sch, **kw)
    rnd = dict(kw)
    if "markov_M" in rnd:
        rnd["markov_M"] = np.asarray(rnd["markov_M"]).astype(np.float32).astype(np.float64)
        rnd["markov_pi"] = np.asarray(rnd["markov_pi"]).astype(np.float32).astype(np.float64)
    variants = [L.astype(np.float32).astype(np.float64)]
    rng = np.random.default_rng(0x5E45)
    for _ in range(2):
        variants.append(L * (1.0 + 1e-6 * rng.uniform(-1, 1, size=L.shape)))
    moved = np.zeros(len(idx), dtype=bool)
    for Lv in variants:
        b = oracle.decode(code, likelihoods=Lv, syndrome=sub.syndrome, schedule=sch, **rnd)
        moved |= (a["xhat"] != b["xhat"]).any(axis=1) | (a["iters"] != b["iters"])
    for model in (1, 2):
        b = oracle.decode(code, likelihoods=L, syndrome=sub.syndrome, schedule=sch, precision_model=model, **kw)
        moved |= (a["xhat"] != b["xhat"]).any(axis=1) | (a["iters"] != b["iters"])
    return moved


def _near_tie(code, fr, schedule, idx, upto, gap=1e-3, **kw):
    """Frames (of idx) with a near tie in the reference: at some iteration
    t <= upto[k], some symbol's two largest pseudo-posterior entries differ by
    less than `gap` (the decision there is not determined by the arithmetic's
    last bits; float32 messages may break the tie the other way)."""
    if len(idx) == 0:
        return np.zeros(0, dtype=bool)
    sub = fr.subset(idx)
    L = sub.lik.astype(np.float64) if sub.lik is not None else oracle.frame_likelihoods(code, sub)
    kw = {k: v for k, v in kw.items() if k not in ("snap_iter", "posterior", "max_iter", "early_stop")}
    sch = gfbp_sched(schedule)
    tie = np.zeros(len(idx), dtype=bool)
    for t in range(1, int(max(upto)) + 1):
        o = oracle.decode(code, likelihoods=L, syndrome=sub.syndrome, schedule=sch, max_iter=t, early_stop=False,
                          posterior=True, **kw)
        P = np.sort(o["posterior"], axis=2)
        tie |= ((P[:, :, -1] - P[:, :, -2]).min(axis=1) < gap) & (t <= np.asarray(upto))
    return tie


def _compare_decisions(g, r, label, min_frac=0.999, recheck=None, near_tie=None):
    """Identical decisions and iteration counts on >= min_frac of the frames;
    frames the reference did not converge on (chaotic), frames whose
    reference outcome is not determined at float32 input precision
    (recheck(idx) -> bool mask) and near-tie frames (near_tie(idx, upto) ->
    bool mask, upto = the first iteration at which either side stopped) are
    logged exceptions."""
    same = (g["xhat"] == r["xhat"]).all(axis=1) & (g["iters"] == r["iters"])
    chaotic = r["converged"] == 0
    bad = ~same & ~chaotic
    sensitive = np.zeros_like(bad)
    if recheck is not None and bad.any():
        bi = np.nonzero(bad)[0]
        sens = recheck(bi)
        sensitive[bi[sens]] = True
        bad &= ~sensitive
    ties = np.zeros_like(bad)
    if near_tie is not None and bad.any():
        bi = np.nonzero(bad)[0]
        nt = near_tie(bi, np.minimum(g["iters"][bi], r["iters"][bi]))
        ties[bi[nt]] = True
        bad &= ~ties
    F = len(same)
    print(f"[{label}] frames={F} identical={int(same.sum())} chaotic-differing={int((~same & chaotic).sum())} "
          f"precision-sensitive={int(sensitive.sum())} near-tie={int(ties.sum())} other-differing={int(bad.sum())} "
          f"mean_iters gpu={g['iters'].mean():.3f} ref={r['iters'].mean():.3f} "
          f"FER gpu={1 - g['converged'].mean():.4f} ref={1 - r['converged'].mean():.4f}")
    for name, mask in (("chaotic", ~same & chaotic), ("precision-sensitive", sensitive), ("near-tie", ties),
                       ("differing", bad)):
        if mask.any():
            idx = np.nonzero(mask)[0][:8]
            print(f"[{label}] {name} frames {idx.tolist()} iters gpu={g['iters'][idx].tolist()} "
                  f"ref={r['iters'][idx].tolist()}")
    assert bad.sum() <= math.floor((1 - min_frac) * F), f"{label}: {int(bad.sum())} frames differ"
    return same


def _wilson(k, n, z=1.96):
    """95% Wilson score interval of a binomial proportion k/n."""
    p = k / n
    c = (p + z * z / (2 * n)) / (1 + z * z / n)
    h = z * math.sqrt(p * (1 - p) / n + z * z / (4 * n * n)) / (1 + z * z / n)
    return c - h, c + h


def _fer_ci_overlap(conv_a, conv_b):
    """The frame error rates' 95% Wilson intervals overlap."""
    a = _wilson(int((conv_a == 0).sum()), len(conv_a))
    b = _wilson(int((conv_b == 0).sum()), len(conv_b))
    return a[0] <= b[1] and b[0] <= a[1]


def _ci_overlap(a, b):
    """95% CIs of two means (normal approximation) overlap."""
    ma, mb = a.mean(), b.mean()
    sa = 1.96 * a.std(ddof=1) / math.sqrt(len(a)) if len(a) > 1 else 0.0
    sb = 1.96 * b.std(ddof=1) / math.sqrt(len(b)) if len(b) > 1 else 0.0
    return abs(ma - mb) <= sa + sb + 1e-12


# --------------------------------------------------------------- messages
@pytest.mark.parametrize("q", [2, 4, 8, 16, 32, 64])
@pytest.mark.parametrize("schedule", ["pus", "sus"])
def test_messages_after_first_iterations(gfbp, q, schedule):
    code, enc = _small_code(q, 72, seed=100 + q)
    F = 13  # not a multiple of the frames per wavefront: ragged tail
    fr = wl.make_frames(code, enc, F, 200 + q, "bsc", 0.09)
    for it in (1, 2, 3):
        g = _gpu(gfbp, code, fr, schedule, max_iter=it, early_stop=False, snap_iter=it)
        r = _ref(code, fr, schedule, max_iter=it, early_stop=False, snap_iter=it)
        for key in ("snap_q", "snap_r", "snap_Q"):
            err = np.abs(g[key] - r[key]).max()
            assert err <= MSG_TOL, f"q={q} {schedule} iter {it} {key}: max abs error {err:.3g}"


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


# --------------------------------------------------------------- decisions
@pytest.mark.parametrize("schedule", ["pus", "sus"])
def test_config1_all_frames(gfbp, schedule):
    """GF(4), (3,6), N=504, BSC 0.06, 2000 frames, max 200 iterations."""
    code, enc = wl.regular_code(504, 3, 6, 4, seed=0xC0DE0001)
    fr = wl.make_frames(code, enc, 2000, 0xDA7A0001, "bsc", 0.06)
    g = _gpu(gfbp, code, fr, schedule, max_iter=200)
    r = _ref(code, fr, schedule, max_iter=200)
    _compare_decisions(g, r, f"C1 {schedule}",
                       recheck=lambda idx: _precision_sensitive(code, fr, schedule, idx, max_iter=200))
    assert _ci_overlap(g["iters"].astype(float), r["iters"].astype(float))
    assert _fer_ci_overlap(g["converged"], r["converged"])


@pytest.mark.parametrize("channel,param", [("bec", 0.42), ("biawgn", 0.85)])
@pytest.mark.parametrize("schedule", ["pus", "sus"])
def test_other_channels(gfbp, channel, param, schedule):
    code, enc = wl.regular_code(240, 3, 6, 8, seed=9)
    fr = wl.make_frames(code, enc, 150, 10, channel, param)
    g = _gpu(gfbp, code, fr, schedule, max_iter=60)
    r = _ref(code, fr, schedule, max_iter=60)
    _compare_decisions(g, r, f"{channel} {schedule}",
                       recheck=lambda idx: _precision_sensitive(code, fr, schedule, idx, max_iter=60))
    for it in (1, 3):
        g = _gpu(gfbp, code, fr, schedule, max_iter=it, early_stop=False, snap_iter=it)
        r = _ref(code, fr, schedule, max_iter=it, early_stop=False, snap_iter=it)
        assert np.abs(g["snap_q"] - r["snap_q"]).max() <= MSG_TOL


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
    for it in (1, 2, 4):
        g = _gpu(gfbp, code, fr, schedule, max_iter=it, early_stop=False, snap_iter=it, **kw)
        r = _ref(code, fr, schedule, max_iter=it, early_stop=False, snap_iter=it, **kw)
        for key in ("snap_q", "snap_r", "snap_Q"):
            err = np.abs(g[key] - r[key]).max()
            assert err <= MSG_TOL, f"{schedule} iter {it} {key}: {err:.3g}"
    g = _gpu(gfbp, code, fr, schedule, max_iter=100, **kw)
    r = _ref(code, fr, schedule, max_iter=100, **kw)
    _compare_decisions(g, r, f"markov {kind} q={q} {schedule}",
                       recheck=lambda idx: _precision_sensitive(code, fr, schedule, idx, max_iter=100, **kw))


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
    for it in (1, 2, 4):
        g = _gpu(gfbp, code, fr, "sus", max_iter=it, early_stop=False, snap_iter=it, sus_strict=strict, **kw)
        r = _ref(code, fr, "sus", max_iter=it, early_stop=False, snap_iter=it, **kw)
        for key in ("snap_q", "snap_r", "snap_Q"):
            err = np.abs(g[key] - r[key]).max()
            assert err <= MSG_TOL, f"iter {it} {key}: {err:.3g}"
        if it == 2:  # the timing matters from iteration 2 on
            d = _gpu(gfbp, code, fr, "sus", max_iter=2, early_stop=False, snap_iter=2, prior="markov",
                     markov_M=M, markov_pi=pi)
            assert np.abs(d["snap_Q"] - g["snap_Q"]).max() > 1e-3
    g = _gpu(gfbp, code, fr, "sus", max_iter=100, sus_strict=strict, **kw)
    r = _ref(code, fr, "sus", max_iter=100, **kw)
    _compare_decisions(g, r, f"in-sweep {kind} strict={strict}",
                       recheck=lambda idx: _precision_sensitive(code, fr, "sus", idx, max_iter=100, **kw))


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
    d = gfbp.SessionDesc(64, gfbp.SCHEDULES["sus"], 10, 0, None, None, gfbp.OPT_PRIOR_IN_SWEEP)
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
    H = code.dense()
    from tests import _gf

    T = _gf.mul_table(code.p)
    z = np.zeros((F, code.m), dtype=np.uint8)
    for i in range(code.m):
        for j in np.nonzero(H[i])[0]:
            z[:, i] ^= T[H[i, j], x[:, j]].astype(np.uint8)
    noisy = wl.bsc(x, code.p, 0.05, 15)
    L = np.stack([oracle.likelihood(code.p, "bsc", 0.05, rx=int(v)) for v in noisy.ravel()]).reshape(F, code.n, q)
    dcode = gfbp.DeviceCode(code)
    dfr = {"channel": "likelihood", "F": F, "likelihood": torch.from_numpy(L.astype(np.float32)).cuda(),
           "syndrome": torch.from_numpy(z).cuda()}
    out = gfbp.decode_batch(dcode, dfr, schedule=schedule, max_iter=50)
    g = {k: v.cpu().numpy() for k, v in out.items()}
    r = oracle.decode(code, likelihoods=L.astype(np.float32).astype(np.float64), syndrome=z,
                      schedule=gfbp_sched(schedule), max_iter=50)
    _compare_decisions(g, r, f"coset {schedule}")
    assert (g["xhat"][g["converged"] == 1] == x[g["converged"] == 1]).mean() > 0.99


# --------------------------------------------------------------- full sizes, sampled frames
@pytest.mark.parametrize("schedule", ["pus", "sus"])
def test_config2_full_batch_sampled(gfbp, schedule):
    """GF(16), (3,6), N=2000, BI-AWGN 1.0 dB, 4096 frames in one launch; the
    reference decodes every 256th frame."""
    code, enc = wl.regular_code(2000, 3, 6, 16, seed=0xC0DE0002)
    sigma = wl.sigma_from_ebn0(1.0, code.n_info / code.n)
    fr = wl.make_frames(code, enc, 4096, 0xDA7A0002, "biawgn", sigma)
    g = _gpu(gfbp, code, fr, schedule, max_iter=100)
    idx = np.arange(0, 4096, 256)
    r = _ref(code, fr.subset(idx), schedule, max_iter=100)
    gs = {k: v[idx] for k, v in g.items()}
    sub = fr.subset(idx)
    _compare_decisions(gs, r, f"C2 1.0dB {schedule}", min_frac=0.9,
                       recheck=lambda i: _precision_sensitive(code, sub, schedule, i, max_iter=100))


@pytest.mark.parametrize("channel,param", [("bsc", 0.08), ("bec", 0.45)])
def test_config3_full_batch_sampled(gfbp, channel, param):
    """GF(8), (3,6), N=3000, Markov source (self-transition 0.7), 4096 frames."""
    q = 8
    code, enc = wl.regular_code(3000, 3, 6, q, seed=0xC0DE0003)
    M = wl.self_transition_matrix(q, 0.7)
    pi = wl.stationary(M)
    fr = wl.make_frames(code, enc, 4096, 0xDA7A0003, channel, param, source="markov", markov=M)
    kw = dict(prior="markov", markov_M=M, markov_pi=pi, max_iter=100)
    idx = np.arange(0, 4096, 512)
    for schedule in ("pus", "sus"):
        g = _gpu(gfbp, code, fr, schedule, **kw)
        r = _ref(code, fr.subset(idx), schedule, **kw)
        gs = {k: v[idx] for k, v in g.items()}
        sub = fr.subset(idx)
        _compare_decisions(gs, r, f"C3 {channel} {schedule}", min_frac=0.875,
                           recheck=lambda i: _precision_sensitive(code, sub, schedule, i, **kw))


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


@pytest.mark.parametrize("schedule,q", [("pus", 8), ("sus", 8), ("sus-in-sweep", 8), ("pus", 2), ("sus", 2)])
def test_frame_compaction_changes_nothing(gfbp, schedule, q):
    """Moving running frames into finished slots (on by default) gives bitwise
    the outputs of decoding with every frame in place, with a Markov prior and
    a syndrome (and, for priors assigned during the sweep, the source symbols'
    pseudo-posteriors the next sweep reads); the batch mixes fast and slow
    frames so that compaction runs several times."""
    import torch

    code, enc = wl.regular_code(240, 3, 6, q, seed=37)
    M = wl.self_transition_matrix(q, 0.7)
    pi = wl.stationary(M)
    fr = wl.make_frames(code, enc, 700, 38, "bsc", np.linspace(0.02, 0.14, 700), source="markov", markov=M)
    z = np.random.default_rng(39).integers(0, q, size=(fr.F, code.m)).astype(np.uint8)
    z[::3] = 0
    fr.syndrome = z
    dcode = gfbp.DeviceCode(code)
    dfr = gfbp.frames_to_device(fr)
    outs = []
    for compact in (False, True):
        o = gfbp.decode_batch(dcode, dfr, schedule=schedule[:3], max_iter=60, prior="markov", markov_M=M,
                              markov_pi=pi, compact=compact, prior_in_sweep=schedule.endswith("in-sweep"))
        torch.cuda.synchronize()
        outs.append({k: v.cpu().numpy() for k, v in o.items()})
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
    r = oracle.decode(code, fr.subset(idx), schedule=gfbp_sched(schedule), max_iter=3, early_stop=False,
                      posterior=True)
    assert np.abs(post - r["posterior"]).max() <= MSG_TOL
    assert (xh == r["xhat"]).mean() > 0.999  # decisions off only where two entries nearly tie
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
        g = _gpu(gfbp, code, fr, sch, max_iter=2, early_stop=False, snap_iter=2, **kw)
        r = _ref(code, fr, sch, max_iter=2, early_stop=False, snap_iter=2, **kw)
        for key in ("snap_q", "snap_r", "snap_Q"):
            err = np.abs(g[key] - r[key]).max()
            assert err <= MSG_TOL, f"seed {seed} q={q} {sch} {key}: {err:.3g}"
        g = _gpu(gfbp, code, fr, sch, max_iter=40, **kw)
        r = _ref(code, fr, sch, max_iter=40, **kw)
        _compare_decisions(g, r, f"random seed {seed} q={q} n={n} {channel} markov={markov} {sch}",
                           recheck=lambda idx: _precision_sensitive(code, fr, sch, idx, max_iter=40, **kw),
                           near_tie=lambda idx, upto: _near_tie(code, fr, sch, idx, upto, **kw))


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
_MN_SOURCES = {
    "iid": (None, None),
    "4s": (wl.PAPER_MARKOV_4S, wl.stationary(wl.PAPER_MARKOV_4S)),
    "2s": wl.lift_binary_chain(wl.PAPER_MARKOV_2S, 3),
}


@pytest.mark.parametrize("q,source,channel,param", [(2, "iid", "bsc", 0.1), (4, "4s", "bec", 0.55),
                                                    (8, "2s", "biawgn", 1.1), (4, "4s", "bsc", 0.17),
                                                    (8, "2s", "bec", 0.6)])
@pytest.mark.parametrize("schedule", ["pus", "sus"])
def test_mn_syndrome_form(gfbp, q, source, channel, param, schedule):
    """H = [A B], x = (source, noise), z = B r: the decoder sees only z, the
    noise symbols' likelihoods and the source model (Section 2)."""
    code = wl.mn_code(60, 180, q, seed=400 + q)
    M, start = _MN_SOURCES[source]
    fr = wl.make_mn_frames(code, 300, 401 + q, channel, param, source="iid" if M is None else "markov",
                           markov=M, start=start)
    kw = {} if M is None else dict(prior="markov", markov_M=M, markov_pi=start)
    g = _gpu(gfbp, code, fr, schedule, max_iter=80, **kw)
    r = oracle.decode(code, likelihoods=fr.lik.astype(np.float64), syndrome=fr.syndrome,
                      schedule=gfbp_sched(schedule), max_iter=80, **kw)
    same = _compare_decisions(g, r, f"MN q={q} {source} {channel} {schedule}",
                              recheck=lambda idx: _precision_sensitive(code, fr, schedule, idx, max_iter=80, **kw),
                              near_tie=lambda idx, upto: _near_tie(code, fr, schedule, idx, upto, **kw))
    ok = g["converged"].astype(bool)
    assert r["converged"].mean() > 0.5  # a meaningful share of frames decodes
    assert np.array_equal(wl.syndromes(code, g["xhat"][ok]), fr.syndrome[ok])


@pytest.mark.parametrize("q,source,channel,param", [(4, "4s", "bsc", 0.17), (8, "2s", "biawgn", 1.1)])
def test_mn_syndrome_form_prior_in_sweep(gfbp, q, source, channel, param):
    """The MN syndrome form with the source priors assigned during the SUS
    sweep (R7(ii) timing): messages after iterations 2 and 3, then decisions."""
    code = wl.mn_code(60, 180, q, seed=410 + q)
    M, start = _MN_SOURCES[source]
    fr = wl.make_mn_frames(code, 300, 411 + q, channel, param, source="markov", markov=M, start=start)
    kw = dict(prior="markov", markov_M=M, markov_pi=start, prior_in_sweep=True)
    L = fr.lik.astype(np.float64)
    for it in (2, 3):
        g = _gpu(gfbp, code, fr, "sus", max_iter=it, early_stop=False, snap_iter=it, **kw)
        r = oracle.decode(code, likelihoods=L, syndrome=fr.syndrome, schedule=oracle.SUS, max_iter=it,
                          early_stop=False, snap_iter=it, **kw)
        for key in ("snap_q", "snap_r", "snap_Q"):
            err = np.abs(g[key] - r[key]).max()
            assert err <= MSG_TOL, f"iter {it} {key}: {err:.3g}"
    g = _gpu(gfbp, code, fr, "sus", max_iter=80, **kw)
    r = oracle.decode(code, likelihoods=L, syndrome=fr.syndrome, schedule=oracle.SUS, max_iter=80, **kw)
    _compare_decisions(g, r, f"MN in-sweep q={q} {source} {channel}",
                       recheck=lambda idx: _precision_sensitive(code, fr, "sus", idx, max_iter=80, **kw),
                       near_tie=lambda idx, upto: _near_tie(code, fr, "sus", idx, upto, **kw))
    assert r["converged"].mean() > 0.5


@pytest.mark.parametrize("schedule", ["pus", "sus"])
def test_trace_of_correct_source_bits(gfbp, schedule):
    """The per-iteration count of correct source bits (Fig. 1 diagnostic)
    equals the count from the reference's decisions after each iteration
    (frames whose decisions match the reference's at every iteration: a
    near-tie at some iteration may flip a bit there and be corrected later;
    the test needs such frames to be rare and their final counts equal)."""
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
    r = oracle.decode(code, likelihoods=fr.lik.astype(np.float64), syndrome=fr.syndrome,
                      schedule=gfbp_sched(schedule), max_iter=60, trace=True, **kw)
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
    M, start = (wl.PAPER_MARKOV_4S, wl.stationary(wl.PAPER_MARKOV_4S)) if source == "4s" else \
        wl.lift_binary_chain(wl.PAPER_MARKOV_2S, 3)
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
    register/lane split of the same arithmetic (a different mix of register
    butterflies, row-swap butterflies and lane exchanges); all must match the
    oracle."""
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
        _compare_decisions(g, r, f"tuned EL={el} {sch}",
                           recheck=lambda idx: _precision_sensitive(code, fr, sch, idx, max_iter=50))
