"""Sessions (continuous batching) through the C ABI.

A frame's arithmetic does not depend on the other frames, so a frame decoded
in a session -- admitted at any time, next to any other frames, in any slot --
must give bitwise the result of gfbp_decode_batch (which the parity tests tie
to the reference decoder).
"""
import numpy as np
import pytest

from paper_cs_0605069_amd import workloads as wl

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gfbp():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_cs_0605069_amd as g

    g.lib()
    return g


def _slice(d, lo, hi):
    return {k: (v[lo:hi] if hasattr(v, "shape") and v is not None else v) for k, v in d.items()}


def _drain(sess, dfr, F, step_iters=3, max_rounds=10000, stream=None):
    """Offer frames in order as slots free up; step; collect.  Returns
    {id: (iters, converged, xhat)}."""
    done = {}
    nxt = 0
    for _ in range(max_rounds):
        if nxt < F:
            k = sess.admit(np.arange(nxt, F), _slice(dfr, nxt, F), stream=stream)
            nxt += k
        sess.step(step_iters, stream=stream)
        ids, it, cv, xh = sess.poll(stream=stream)
        for r in range(len(ids)):
            done[int(ids[r])] = (int(it[r]), int(cv[r]), xh[r].copy())
        if len(done) == F:
            return done
    raise AssertionError("session did not finish")


def _batch(gfbp, dcode, fr, schedule, max_iter, **kw):
    import torch

    # sessions run the tiled kernels: the batch decode through them too
    out = gfbp.decode_batch(dcode, gfbp.frames_to_device(fr), schedule=schedule, max_iter=max_iter, onchip=False,
                            **kw)
    torch.cuda.synchronize()
    return {k: v.cpu().numpy() for k, v in out.items()}


@pytest.mark.parametrize("schedule", ["pus", "sus"])
def test_session_equals_batch_with_staggered_admission(gfbp, schedule):
    code, enc = wl.regular_code(240, 3, 6, 8, seed=51)
    fr = wl.make_frames(code, enc, 300, 52, "bsc", 0.085)
    dcode = gfbp.DeviceCode(code)
    ref = _batch(gfbp, dcode, fr, schedule, 60)
    sess = gfbp.Session(dcode, n_slots=128, schedule=schedule, max_iter=60)
    got = _drain(sess, gfbp.frames_for_session([fr]), fr.F)
    assert sess.running == 0 and sess.free_slots == 128
    for f in range(fr.F):
        it, cv, xh = got[f]
        assert it == ref["iters"][f] and cv == ref["converged"][f], f"frame {f}"
        assert np.array_equal(xh, ref["xhat"][f]), f"frame {f}"


@pytest.mark.parametrize("kind", ["self", "general"])
@pytest.mark.parametrize("schedule", ["pus", "sus"])
def test_session_step_graphs_equal_batch(gfbp, schedule, kind):
    """Replayed step graphs (one per launch bound, captured as the number of
    frames in flight rises and falls) give the eager results; with a
    self-transition and with a general Markov matrix."""
    import torch

    q = 16
    code, enc = wl.regular_code(200, 3, 6, q, seed=61)
    M = wl.self_transition_matrix(q, 0.8)
    if kind == "general":
        M = 0.5 * M + 0.5 * np.random.default_rng(0x3A8).dirichlet(np.ones(q), size=q)
    pi = wl.stationary(M)
    fr = wl.make_frames(code, enc, 700, 62, "bsc", 0.06, source="markov", markov=M)
    dcode = gfbp.DeviceCode(code)
    ref = _batch(gfbp, dcode, fr, schedule, 40, prior="markov", markov_M=M, markov_pi=pi)
    dfr = gfbp.frames_for_session([fr])
    dfr["markov"] = torch.ones(fr.F, dtype=torch.uint8, device="cuda")
    stream = torch.cuda.Stream()
    torch.cuda.synchronize()
    sess = gfbp.Session(dcode, n_slots=256, schedule=schedule, max_iter=40, markov_M=M, markov_pi=pi,
                        step_graphs=True)
    with torch.cuda.stream(stream):
        got = _drain(sess, dfr, fr.F, step_iters=2, stream=stream)
    assert sess.running == 0
    for f in range(fr.F):
        it, cv, xh = got[f]
        assert it == ref["iters"][f] and cv == ref["converged"][f] and np.array_equal(xh, ref["xhat"][f]), f"frame {f}"
    sess.close()


@pytest.mark.parametrize("schedule", ["pus", "sus"])
def test_session_mixes_channels_and_priors(gfbp, schedule):
    import torch

    q = 8
    code, enc = wl.regular_code(180, 3, 6, q, seed=53)
    M = wl.self_transition_matrix(q, 0.7)
    pi = wl.stationary(M)
    groups = [wl.make_frames(code, enc, 40, 54, "bsc", 0.08),
              wl.make_frames(code, enc, 40, 55, "bec", 0.4),
              wl.make_frames(code, enc, 40, 56, "biawgn", 0.8, source="markov", markov=M),
              wl.make_frames(code, enc, 40, 57, "bsc", 0.1, source="markov", markov=M)]
    markov = [False, False, True, True]
    dcode = gfbp.DeviceCode(code)
    dfr = gfbp.frames_for_session(groups)
    dfr["markov"] = torch.from_numpy(np.concatenate([np.full(g.F, int(m), np.uint8) for g, m in zip(groups, markov)])).cuda()
    sess = gfbp.Session(dcode, n_slots=64, schedule=schedule, max_iter=50, markov_M=M, markov_pi=pi)
    got = _drain(sess, dfr, dfr["F"], step_iters=2)
    base = 0
    for g, m in zip(groups, markov):
        kw = dict(prior="markov", markov_M=M, markov_pi=pi) if m else {}
        ref = _batch(gfbp, dcode, g, schedule, 50, **kw)
        for f in range(g.F):
            it, cv, xh = got[base + f]
            assert it == ref["iters"][f] and cv == ref["converged"][f] and np.array_equal(xh, ref["xhat"][f]), \
                f"{g.channel} markov={m} frame {f}"
        base += g.F


def test_session_admission_and_accounting(gfbp):
    code, enc = wl.regular_code(120, 3, 6, 4, seed=58)
    fr = wl.make_frames(code, enc, 100, 59, "bsc", 0.05)
    dcode = gfbp.DeviceCode(code)
    sess = gfbp.Session(dcode, n_slots=40, schedule="pus", max_iter=30)
    assert sess.free_slots == 64  # rounded up to a multiple of 64
    dfr = gfbp.frames_for_session([fr])
    k = sess.admit(np.arange(100), dfr)
    assert k == 64 and sess.free_slots == 0 and sess.running == 64
    assert sess.admit(np.arange(64, 100), _slice(dfr, 64, 100)) == 0
    ids, it, cv, xh = sess.poll()
    assert len(ids) == 0  # nothing stepped yet
    sess.step(30)
    ids, it, cv, xh = sess.poll()
    assert len(ids) == 64 and sorted(ids.tolist()) == list(range(64))
    assert sess.free_slots == 64 and sess.running == 0
    assert (it >= 1).all() and (it <= 30).all()


def test_session_bytes_match_the_memory_it_takes(gfbp):
    import torch

    code, enc = wl.regular_code(120, 3, 6, 16, seed=60)
    dcode = gfbp.DeviceCode(code)
    need = gfbp.Session.bytes_needed(dcode, 256, "sus")
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]
    sess = gfbp.Session(dcode, n_slots=256, schedule="sus")
    torch.cuda.synchronize()
    free1 = torch.cuda.mem_get_info()[0]
    assert need > 0
    assert free0 - free1 >= need * 0.9
    sess.close()


def test_session_sized_by_device_bytes_and_timestamps(gfbp):
    """n_slots = 0: the session takes as many 64-slot tiles as device_bytes
    holds; poll returns device-clock admission and retirement times."""
    import torch

    code, enc = wl.regular_code(240, 3, 6, 16, seed=64)
    dcode = gfbp.DeviceCode(code)
    per64 = gfbp.Session.bytes_needed(dcode, 64, "sus")
    budget = 5 * per64 + per64 // 2
    assert gfbp.Session.bytes_needed(dcode, 0, "sus", device_bytes=budget) == gfbp.Session.bytes_needed(dcode, 320, "sus")
    sess = gfbp.Session(dcode, n_slots=0, schedule="sus", max_iter=40, device_bytes=budget)
    assert sess.free_slots == 320
    with pytest.raises(gfbp.GfbpError):
        gfbp.Session(dcode, n_slots=0, schedule="sus", device_bytes=per64 // 2)
    fr = wl.make_frames(code, enc, 100, 65, "bsc", 0.07)
    assert sess.admit(np.arange(100), gfbp.frames_for_session([fr])) == 100
    hz = gfbp.device_clock_hz()
    assert hz > 0
    done = {}
    for _ in range(40):
        sess.step(1)
        ids, it, cv, xh, ts = sess.poll(timestamps=True)
        for k in range(len(ids)):
            done[int(ids[k])] = (int(it[k]), ts[k])
        if len(done) == 100:
            break
    assert len(done) == 100
    spans = np.array([(int(t[1]) - int(t[0])) / hz for _, t in done.values()])
    assert (spans > 0).all() and (spans < 10).all()
    # frames that ran more iterations retired later
    fast = [t[1] for i, t in done.values() if i <= 3]
    slow = [t[1] for i, t in done.values() if i >= 8]
    if fast and slow:
        assert min(slow) > min(fast)
    torch.cuda.synchronize()
