"""Uneven batches as one HIP graph, against the plain per-code kernels.

Frames of several codes (q in {4, 16, 64}, column weight 2-3, rate 1/3-1/2,
different lengths) and channels (BSC, BEC, BI-AWGN at 1-2 dB, capacity
matched) go into one session per code; the kernel shape of each code is
autotuned on its frames; one HIP graph holds several iterations of every
session and is replayed, with eager polls between replays, until every frame
has finished.  Each frame must equal, bitwise, its gfbp_decode_batch result.
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


def _groups(code, F, seed):
    """F frames of one code, channels cycling BSC / BEC / BI-AWGN, Eb/N0 ~ U[1, 2] dB."""
    rng = np.random.default_rng([seed, 11])
    rate = code.n_info / code.n
    out = []
    for k, kind in enumerate(("bsc", "bec", "biawgn")):
        nf = F // 3 + (1 if k < F % 3 else 0)
        eb = rng.uniform(1.0, 2.0, size=nf)
        prm = np.array([wl.channel_for(kind, e, rate) for e in eb])
        out.append(wl.make_coset_frames(code, nf, seed * 10 + k, kind, prm))
    return out


def test_uneven_batch_graph_equals_plain_kernels(gfbp):
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
        # autotune the kernel shape on this code's frames (first group)
        d0 = gfbp.frames_to_device(groups[0])
        gfbp.tune(dcode, d0, schedule=schedule, trial_iters=2)
        # eager plain-kernel results per channel group
        ref = {}
        base = 0
        for g in groups:
            out = gfbp.decode_batch(dcode, gfbp.frames_to_device(g), schedule=schedule, max_iter=40)
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
