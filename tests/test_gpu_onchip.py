"""Whole decodes in LDS (codes over GF(2), GF(4), GF(8) whose frame state fits
in a workgroup's LDS).

  * bitwise the tiled decode at the same lanes per vector (PUS: one lane, q
    entries; SUS: two entries per lane; the same arithmetic), over both
    schedules, every channel, the three priors
    (a general Markov matrix too), syndromes z != 0, frame counts that leave
    a partly filled last workgroup, fixed iteration counts;
  * the launch is the in-LDS kernel (the profiler's kernel kinds), and a
    code too large for LDS falls back to the tiled kernels;
  * against the reference decoder: the GF(4) N = 504 workload of the
    benchmark's configurations runs here by default (tests/test_gpu_configs.py
    checks every frame of it), and an MN syndrome-form case below.
"""
import numpy as np
import pytest

import oracle
from paper_cs_0605069_amd import workloads as wl
from tests._parity import classify, sched

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gfbp():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_cs_0605069_amd as g

    g.lib()
    return g


def _host(o):
    return {k: v.cpu().numpy() for k, v in o.items()}


def _both(gfbp, code, dfr, schedule, **kw):
    """The in-LDS decode and the tiled decode at its lanes per vector (PUS:
    one lane, q entries; SUS: two entries per lane)."""
    import torch

    dcode = gfbp.DeviceCode(code)
    dcode.set_shape(schedule, code.q if schedule == "pus" else 2)
    gfbp.profile_reset()
    gfbp.profile_enable(True)
    a = _host(gfbp.decode_batch(dcode, dfr, schedule=schedule, **kw))
    torch.cuda.synchronize()
    gfbp.profile_enable(False)
    prof = gfbp.profile_read()
    b = _host(gfbp.decode_batch(dcode, dfr, schedule=schedule, onchip=False, **kw))
    return a, b, prof


_CASES = [
    # q, n, channel, prior, syndrome, schedule, frames
    (4, 300, "bsc", "uniform", False, "pus", 333), (4, 300, "bsc", "uniform", False, "sus", 333),
    (8, 240, "biawgn", "markov", True, "pus", 257), (8, 240, "biawgn", "markov", True, "sus", 257),
    (2, 600, "bec", "uniform", True, "sus", 130), (2, 600, "biawgn", "static", False, "pus", 130),
    (8, 180, "bec", "static", True, "sus", 97), (4, 504, "bsc", "markov", False, "pus", 65),
    (4, 240, "biawgn", "general", True, "sus", 70), (8, 200, "bsc", "general", False, "pus", 1),
]


@pytest.mark.parametrize("q,n,channel,prior,syn,schedule,frames", _CASES)
def test_onchip_equals_tiled(gfbp, q, n, channel, prior, syn, schedule, frames):
    code, enc = wl.regular_code(n, 3, 6, q, seed=700 + q + n)
    M = wl.self_transition_matrix(q, 0.7)
    if prior == "general":
        M = 0.5 * M + 0.5 * np.random.default_rng(701).dirichlet(np.ones(q), size=q)
    kw = {}
    if prior in ("markov", "general"):
        kw = dict(prior="markov", markov_M=M, markov_pi=wl.stationary(M))
    elif prior == "static":
        kw = dict(prior="static", static_prior=np.random.default_rng(702).dirichlet(np.ones(q), size=code.n_info))
    param = {"bsc": 0.08, "bec": 0.42, "biawgn": 0.8}[channel]
    if syn:
        fr = wl.make_coset_frames(code, frames, 703 + q, channel, param)
    else:
        fr = wl.make_frames(code, enc, frames, 704 + q, channel, param,
                            source="markov" if "prior" in kw and kw["prior"] == "markov" else "iid",
                            markov=M if kw.get("prior") == "markov" else None)
    dfr = gfbp.frames_to_device(fr)
    a, b, prof = _both(gfbp, code, dfr, schedule, max_iter=60, **kw)
    assert prof.get("onchip", {}).get("launches", 0) == 1, prof.keys()
    for k in ("xhat", "iters", "converged", "guards"):
        assert np.array_equal(a[k], b[k]), f"{k}: in-LDS and tiled decodes differ"
    # and a fixed number of iterations without early stopping
    a, b, _ = _both(gfbp, code, dfr, schedule, max_iter=4, early_stop=False, **kw)
    for k in ("xhat", "iters", "converged", "guards"):
        assert np.array_equal(a[k], b[k]), f"fixed iterations, {k}"


@pytest.mark.parametrize("q,seed", [(2, 0), (4, 1), (4, 2)])
def test_onchip_irregular_codes_equal_tiled(gfbp, q, seed):
    """Irregular codes beyond the small degree class (rows up to 16 entries,
    columns up to 5), with a column in no check, syndromes and a Markov
    prior: bitwise the tiled decode."""
    from tests.test_gpu_parity import _random_irregular_code

    rng = np.random.default_rng([0x0C41, seed])
    n = int(rng.integers(60, 200))
    base = _random_irregular_code(rng, q, n, int(n * rng.uniform(0.4, 0.7)))
    code = wl.Code(q, n + 1, base.m, base.row_ptr, base.col, base.coef, poly=base.poly,
                   n_info=base.n_info)  # column n: in no check
    M = 0.5 * wl.self_transition_matrix(q, 0.75) + 0.5 * rng.dirichlet(np.ones(q), size=q)
    fr = wl.make_coset_frames(code, 90, 720 + seed, "biawgn", 0.75, source="markov", markov=M)
    kw = dict(prior="markov", markov_M=M, markov_pi=wl.stationary(M))
    for sch in ("pus", "sus"):
        a, b, prof = _both(gfbp, code, gfbp.frames_to_device(fr), sch, max_iter=40, **kw)
        assert prof["onchip"]["launches"] == 1
        for k in ("xhat", "iters", "converged", "guards"):
            assert np.array_equal(a[k], b[k]), f"{sch} {k}"


def test_guard_events_equal_tiled(gfbp):
    """All-zero likelihood rows (normalisation guards) counted alike."""
    import torch

    q = 4
    code, enc = wl.regular_code(120, 3, 6, q, seed=710)
    F = 70
    lik = np.random.default_rng(711).random((F, code.n, q)).astype(np.float32)
    lik[::5, 7, :] = 0.0
    lik[::7, 11, :] = 0.0
    dfr = {"F": F, "channel": "likelihood", "likelihood": torch.from_numpy(lik).cuda()}
    for sch in ("pus", "sus"):
        a, b, prof = _both(gfbp, code, dfr, sch, max_iter=20)
        assert prof["onchip"]["launches"] == 1
        assert (a["guards"] > 0).any()
        for k in ("xhat", "iters", "converged", "guards"):
            assert np.array_equal(a[k], b[k]), f"{sch} {k}"


def test_large_code_takes_the_tiled_kernels(gfbp):
    import torch

    q = 8
    code, enc = wl.regular_code(3000, 3, 6, q, seed=712)  # 9000 edges x 8 x 4 B x 2: more than a workgroup's LDS
    fr = wl.make_frames(code, enc, 64, 713, "bsc", 0.06)
    dcode = gfbp.DeviceCode(code)
    gfbp.profile_reset()
    gfbp.profile_enable(True)
    gfbp.decode_batch(dcode, gfbp.frames_to_device(fr), schedule="pus", max_iter=20)
    torch.cuda.synchronize()
    gfbp.profile_enable(False)
    prof = gfbp.profile_read()
    assert "onchip" not in prof and prof["check"]["launches"] > 0


@pytest.mark.parametrize("schedule", ["pus", "sus"])
def test_onchip_mn_form_against_the_reference(gfbp, schedule):
    """The syndrome form (noise evidence from the channel outputs, a Markov
    source on the source symbols) decoded in LDS, against the reference."""
    q = 8
    code = wl.mn_code(60, 180, q, seed=714, b_form="pool", pool=12)
    M, start = wl.lift_binary_chain(wl.PAPER_MARKOV_2S, 3)
    fr = wl.make_mn_frames(code, 200, 715, "bsc", 0.12, source="markov", markov=M, start=start)
    kw = dict(prior="markov", markov_M=M, markov_pi=start)
    dcode = gfbp.DeviceCode(code)
    import torch

    gfbp.profile_reset()
    gfbp.profile_enable(True)
    g = _host(gfbp.decode_batch(dcode, gfbp.frames_to_device(fr), schedule=schedule, max_iter=80, **kw))
    torch.cuda.synchronize()
    gfbp.profile_enable(False)
    assert gfbp.profile_read()["onchip"]["launches"] == 1
    r = oracle.decode(code, fr, schedule=sched(schedule), max_iter=80, **kw)
    classify(gfbp, code, fr, g, r, schedule, f"in-LDS MN q={q} {schedule}", budget=0.005, max_iter=80, **kw)
    assert r["converged"].mean() > 0.5
