"""gfbp_decode_batch_noalloc (the entry point for callers that cannot
allocate) against gfbp_decode_batch, through the C ABI: two calls in a row,
the second with a smaller batch, each equal bitwise to the allocating entry
point; a batch beyond the static scratch is refused with a clear error."""
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


def _outputs(torch, F, n):
    return {"xhat": torch.empty((F, n), dtype=torch.uint8, device="cuda"),
            "iters": torch.empty(F, dtype=torch.int32, device="cuda"),
            "converged": torch.empty(F, dtype=torch.uint8, device="cuda"),
            "guards": torch.empty(F, dtype=torch.int32, device="cuda")}


def _host(o):
    return {k: v.cpu().numpy() for k, v in o.items()}


@pytest.mark.parametrize("schedule", ["pus", "sus"])
def test_noalloc_equals_decode_batch_twice(gfbp, schedule):
    import torch

    q = 16
    code, enc = wl.regular_code(400, 3, 6, q, seed=97)
    M = wl.self_transition_matrix(q, 0.7)
    pi = wl.stationary(M)
    dcode = gfbp.DeviceCode(code)
    Mt = torch.as_tensor(M.astype(np.float32), device="cuda")
    pt = torch.as_tensor(pi.astype(np.float32), device="cuda")
    for F, seed in ((700, 98), (130, 99)):  # the second call smaller, on the scratch the first one left
        fr = wl.make_frames(code, enc, F, seed, "bsc", 0.09, source="markov", markov=M)
        dfr = gfbp.frames_to_device(fr)
        ref = gfbp.decode_batch(dcode, dfr, schedule=schedule, max_iter=60, prior="markov", markov_M=M,
                                markov_pi=pi)
        torch.cuda.synchronize()
        out = gfbp.decode_batch_noalloc([dcode], dfr, _outputs(torch, F, code.n), schedule=schedule, max_iter=60,
                                        prior="markov", prior_tensors=(Mt, pt, None, 0))
        torch.cuda.synchronize()
        a, b = _host(ref), _host(out)
        for k in ("xhat", "iters", "converged", "guards"):
            assert np.array_equal(a[k], b[k]), f"F={F} {k}"
        assert (b["converged"] == 1).mean() > 0.5


@pytest.mark.parametrize("schedule", ["pus", "sus"])
def test_noalloc_small_code_in_lds_twice(gfbp, schedule):
    """A code small enough for the whole decode in LDS (GF(4) N = 504): the
    no-allocation entry, on the static scratch, equals the allocating one,
    twice, the second call smaller."""
    import torch

    code, enc = wl.regular_code(504, 3, 6, 4, seed=107)
    dcode = gfbp.DeviceCode(code)
    for F, seed in ((700, 108), (130, 109)):
        fr = wl.make_frames(code, enc, F, seed, "bsc", 0.07)
        dfr = gfbp.frames_to_device(fr)
        ref = _host(gfbp.decode_batch(dcode, dfr, schedule=schedule, max_iter=80))
        torch.cuda.synchronize()
        got = _host(gfbp.decode_batch_noalloc([dcode], dfr, _outputs(torch, F, code.n), schedule=schedule,
                                              max_iter=80))
        for k in ("xhat", "iters", "converged", "guards"):
            assert np.array_equal(ref[k], got[k]), f"F={F} {k}"
        assert (got["converged"] == 1).mean() > 0.5


def test_noalloc_multi_code_twice_and_refusal(gfbp):
    """A batch over two codes of different fields (the no-allocation entry
    takes the persistent kernels, run one after the other on the stream,
    against the persistent path of gfbp_decode_batch), twice, the second
    smaller."""
    import torch

    codes = [wl.regular_code(300, 3, 6, 4, seed=101)[0], wl.regular_code(200, 3, 6, 64, seed=102)[0]]
    dcodes = [gfbp.DeviceCode(c) for c in codes]
    for F0, F1, seed in ((200, 60, 103), (40, 12, 104)):
        frs = [wl.make_coset_frames(codes[0], F0, seed, "biawgn", 0.8),
               wl.make_coset_frames(codes[1], F1, seed + 1, "bsc", 0.05)]
        dfr = gfbp.ragged_frames(frs, codes)
        index = np.array([0] * F0 + [1] * F1, dtype=np.int32)
        ref = _host(gfbp.decode_multi(dcodes, index, dfr, schedule="sus", max_iter=50, persistent=True))
        n_tot = F0 * codes[0].n + F1 * codes[1].n
        outs = _outputs(torch, F0 + F1, 1)
        outs["xhat"] = torch.empty(n_tot, dtype=torch.uint8, device="cuda")
        got = _host(gfbp.decode_batch_noalloc(dcodes, dfr, outs, schedule="sus", max_iter=50, code_index=index))
        for k in ("xhat", "iters", "converged", "guards"):
            assert np.array_equal(ref[k], got[k]), f"{F0}+{F1} {k}"
    # beyond the scratch: refused, nothing run
    big, enc = wl.regular_code(2000, 3, 6, 64, seed=105)
    fr = wl.make_frames(big, enc, 400, 106, "bsc", 0.05)
    with pytest.raises(gfbp.GfbpError) as ei:
        gfbp.decode_batch_noalloc([gfbp.DeviceCode(big)], gfbp.frames_to_device(fr), _outputs(torch, 400, big.n),
                                  schedule="pus")
    assert ei.value.status == -5 and "scratch" in str(ei.value)
