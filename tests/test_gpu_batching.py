"""Uneven batches: one call over several codes (code by code on the plain
kernels, or the persistent work-list kernel), against the plain kernels and
the reference decoder; and sessions as one HIP graph.

The persistent path (GFBP_OPT_PERSISTENT) must give, frame by frame, bitwise
the decisions, iteration counts, convergence flags and guard counts of the
plain kernels at the same lane split: same device functions, same
arithmetic order.  The code-by-code path runs the plain kernels themselves.
"""
import numpy as np
import pytest

import oracle
from paper_cs_0605069_amd import workloads as wl
from tests._parity import classify, gpu_decode, sched

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gfbp():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_cs_0605069_amd as g

    g.lib()
    return g


def _groups(code, F, seed):
    """F frames of one code, channels cycling BSC / BEC / BI-AWGN, Eb/N0 ~ U[1, 2] dB."""
    rng = np.random.default_rng([seed, 11])
    rate = code.n_info / code.n
    out = []
    for k, kind in enumerate(("bsc", "bec", "biawgn")):
        nf = F // 3 + (1 if k < F % 3 else 0)
        if nf == 0:
            continue
        eb = rng.uniform(1.0, 2.0, size=nf)
        prm = np.array([wl.channel_for(kind, e, rate) for e in eb])
        out.append(wl.make_coset_frames(code, nf, seed * 10 + k, kind, prm))
    return out


_CASES = [
    # q, n, channel, prior, syndrome, schedule
    (4, 300, "bsc", "uniform", False, "pus"), (4, 300, "bsc", "uniform", False, "sus"),
    (16, 400, "biawgn", "markov", True, "pus"), (16, 400, "biawgn", "markov", True, "sus"),
    (64, 240, "bec", "static", True, "sus"), (2, 600, "biawgn", "uniform", True, "sus"),
    (8, 360, "bsc", "markov", False, "sus"), (32, 200, "bsc", "uniform", True, "pus"),
]


@pytest.mark.parametrize("q,n,channel,prior,syn,schedule", _CASES)
@pytest.mark.parametrize("el,waves", [(4, 8), (8, 4)])
def test_persistent_equals_plain(gfbp, q, n, channel, prior, syn, schedule, el, waves):
    code, enc = wl.regular_code(n, 3, 6, q, seed=80 + q)
    M = wl.self_transition_matrix(q, 0.7)
    kw = {}
    if prior == "markov":
        kw = dict(prior="markov", markov_M=M, markov_pi=wl.stationary(M))
    elif prior == "static":
        kw = dict(prior="static", static_prior=np.random.default_rng(81).dirichlet(np.ones(q), size=code.n_info))
    param = {"bsc": 0.07, "bec": 0.4, "biawgn": 0.8}[channel]
    fr = wl.make_frames(code, enc, 333, 82 + q, channel, param, source="markov" if prior == "markov" else "iid",
                        markov=M if prior == "markov" else None)
    if syn:  # a random syndrome per frame (coset decoding)
        fr = wl.make_coset_frames(code, 333, 84 + q, channel, param)
    dfr = gfbp.frames_to_device(fr)
    dcode = gfbp.DeviceCode(code)
    dcode.set_shape(schedule, gfbp.persist_entries_per_lane(q, el))  # the same lane split (rounding order)
    out = gfbp.decode_batch(dcode, dfr, schedule=schedule, max_iter=50, onchip=False, **kw)
    a = {k: v.cpu().numpy() for k, v in out.items()}
    b = gpu_decode(gfbp, code, dfr, schedule, max_iter=50, persistent=True, persist_el=el, persist_waves=waves, **kw)
    for k in ("xhat", "iters", "converged", "guards"):
        assert np.array_equal(a[k], b[k]), f"{k}: persistent and plain differ"


def test_persistent_mn_form_per_frame_channels(gfbp):
    """The syndrome form (the decoder computes the noise evidence) with the
    frames' channel kinds given per frame, plain against persistent."""
    import torch

    q = 8
    code = wl.mn_code(60, 180, q, seed=90)
    M, start = wl.lift_binary_chain(wl.PAPER_MARKOV_2S, 3)
    parts = [wl.make_mn_frames(code, 40, 91 + k, ch, prm, source="markov", markov=M, start=start)
             for k, (ch, prm) in enumerate((("bsc", 0.15), ("bec", 0.5), ("biawgn", 1.0)))]
    dfr = gfbp.ragged_frames(parts, [code] * 3)
    kw = dict(prior="markov", markov_M=M, markov_pi=start, max_iter=60)
    dcode = gfbp.DeviceCode(code)
    for sch in ("pus", "sus"):
        dcode.set_shape(sch, gfbp.persist_entries_per_lane(q))  # the persistent path's lane split
        a = {k: v.cpu().numpy() for k, v in gfbp.decode_batch(dcode, dfr, schedule=sch, onchip=False, **kw).items()}
        b = gpu_decode(gfbp, code, dfr, sch, persistent=True, **kw)
        for k in ("xhat", "iters", "converged", "guards"):
            assert np.array_equal(a[k], b[k]), f"{sch} {k}"
        o = 0
        for p in parts:  # and each channel's frames alone (a batch-wide channel)
            c = {k: v.cpu().numpy() for k, v in gfbp.decode_batch(dcode, gfbp.frames_to_device(p), schedule=sch,
                                                                   onchip=False, **kw).items()}
            assert np.array_equal(c["xhat"], a["xhat"][o:o + p.F]) and np.array_equal(c["iters"], a["iters"][o:o + p.F])
            o += p.F
    assert torch.cuda.is_available()


def _pool_batch(gfbp, n_codes, frames, seed, nmax, with_big):
    """Frames over a pool of codes (q in {4, 16, 64}); returns the codes, the
    per-code frame groups and the batch's code index (frames of one code in
    a row, codes in pool order)."""
    pool = wl.mixed_pool(n_codes, seed=seed, n_range=(256, nmax))
    if with_big:  # a GF(64) code of n >= 4000
        big = wl.mixed_pool(1, seed=seed + 1, qs=(64,), n_range=(4000, 4600))
        pool = pool + big
    rng = np.random.default_rng([seed, 2])
    counts = np.bincount(rng.integers(0, len(pool), size=frames), minlength=len(pool))
    counts[counts == 0] = 1
    if with_big:
        counts[-1] = max(counts[-1], 12)
    groups = [_groups(code, int(F), seed * 100 + k) for k, (code, F) in enumerate(zip(pool, counts))]
    return pool, groups


@pytest.mark.parametrize("schedule", ["pus", "sus"])
def test_multi_code_batch(gfbp, schedule):
    """One gfbp_decode_batch call over frames of 9 codes (q in {4, 16, 64},
    one GF(64) code of n >= 4000), BSC / BEC / BI-AWGN frames mixed per frame,
    syndromes z != 0: every frame equals, bitwise, the plain decode of its
    code's frames; 48 frames (every code, the GF(64) n >= 4000 ones
    included) against the reference, from this call and from the same call
    through the persistent kernels."""
    pool, groups = _pool_batch(gfbp, 8, 600, 0xB47C, 1500, True)
    assert {c.q for c in pool} >= {4, 16, 64} and max(c.n for c in pool if c.q == 64) >= 4000
    dcodes = [gfbp.DeviceCode(c) for c in pool]
    flat, codes_of, index = [], [], []
    for k, gs in enumerate(groups):
        for g in gs:
            flat.append(g)
            codes_of.append(pool[k])
            index += [k] * g.F
    index = np.array(index, dtype=np.int32)
    dfr = gfbp.ragged_frames(flat, codes_of)
    out = gfbp.decode_multi(dcodes, index, dfr, schedule=schedule, max_iter=60)
    xh = out["xhat"].cpu().numpy()
    it = out["iters"].cpu().numpy()
    cv = out["converged"].cpu().numpy()
    po = gfbp.decode_multi(dcodes, index, dfr, schedule=schedule, max_iter=60, persistent=True)
    p_xh, p_it, p_cv = (po[k].cpu().numpy() for k in ("xhat", "iters", "converged"))
    offs = np.concatenate([[0], np.cumsum([pool[k].n for k in index])])
    f0 = 0
    picks = []
    for g, code in zip(flat, codes_of):
        k = pool.index(code)
        e = gpu_decode(gfbp, code, gfbp.frames_to_device(g), schedule, max_iter=60)
        for f in range(g.F):
            ff = f0 + f
            assert it[ff] == e["iters"][f] and cv[ff] == e["converged"][f], f"frame {ff}"
            assert np.array_equal(xh[offs[ff]:offs[ff + 1]], e["xhat"][f]), f"frame {ff}"
        picks.append((k, g, list(range(f0, f0 + min(g.F, 2 if code.q < 64 else 4)))))
        f0 += g.F
    # the reference on a deterministic sample: the first frames of every group
    n_ref = 0
    for k, g, rows in picks:
        code = pool[k]
        sub = g.subset(np.arange(len(rows)))
        r = oracle.decode(code, sub, schedule=sched(schedule), max_iter=60)
        gg = {"xhat": np.stack([xh[offs[ff]:offs[ff + 1]] for ff in rows]), "iters": it[rows], "converged": cv[rows]}
        classify(gfbp, code, sub, gg, r, schedule, f"multi-code q={code.q} n={code.n} {g.channel} {schedule}",
                 max_iter=60)
        pg = {"xhat": np.stack([p_xh[offs[ff]:offs[ff + 1]] for ff in rows]), "iters": p_it[rows],
              "converged": p_cv[rows]}
        classify(gfbp, code, sub, pg, r, schedule,
                 f"multi-code persistent q={code.q} n={code.n} {g.channel} {schedule}", max_iter=60)
        n_ref += len(rows)
    assert n_ref >= 48


def test_uneven_batch_graph_equals_plain_kernels(gfbp):
    """Sessions of several codes stepped as one HIP graph equal the plain decode."""
    import torch

    pool = wl.mixed_pool(6, seed=61, n_range=(256, 900))
    assert {c.q for c in pool} >= {4, 16}
    stream = torch.cuda.Stream()
    sessions, expect, dcodes = [], [], []
    for ci, code in enumerate(pool):
        schedule = "pus" if ci % 2 == 0 else "sus"
        groups = _groups(code, 40, 62 + ci)
        dcode = gfbp.DeviceCode(code)
        dcodes.append(dcode)
        dfr = gfbp.frames_for_session(groups)
        dfr["syndrome"] = torch.from_numpy(np.concatenate([g.syndrome for g in groups])).cuda()
        d0 = gfbp.frames_to_device(groups[0])
        gfbp.tune(dcode, d0, schedule=schedule, trial_iters=2)
        ref = {}
        base = 0
        for g in groups:
            out = gfbp.decode_batch(dcode, gfbp.frames_to_device(g), schedule=schedule, max_iter=40,
                                    onchip=False)  # sessions run the tiled kernels
            torch.cuda.synchronize()
            for f in range(g.F):
                ref[base + f] = (int(out["iters"][f]), int(out["converged"][f]), out["xhat"][f].cpu().numpy())
            base += g.F
        sess = gfbp.Session(dcode, n_slots=64, schedule=schedule, max_iter=40, has_syndrome=True)
        with torch.cuda.stream(stream):
            assert sess.admit(np.arange(base), dfr, stream=stream) == base
        sessions.append(sess)
        expect.append(ref)
    torch.cuda.synchronize()
    graph = gfbp.Graph(sessions, iters=4, stream=stream)
    got = [dict() for _ in pool]
    for replay in range(40):
        graph.launch(stream)
        stream.synchronize()
        for k, sess in enumerate(sessions):
            ids, it, cv, xh = sess.poll(stream=stream)
            for r in range(len(ids)):
                got[k][int(ids[r])] = (int(it[r]), int(cv[r]), xh[r].copy())
        if all(len(got[k]) == len(expect[k]) for k in range(len(pool))):
            break
    for k in range(len(pool)):
        assert len(got[k]) == len(expect[k]), f"code {k}: {len(got[k])} of {len(expect[k])} frames finished"
        for f, (it, cv, xh) in expect[k].items():
            g = got[k][f]
            assert g[0] == it and g[1] == cv and np.array_equal(g[2], xh), f"code {k} frame {f}"
    graph.close()
