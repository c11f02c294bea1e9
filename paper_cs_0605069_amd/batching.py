"""Uneven batches: many codes' frames decoded together in one call.

Frames of a pool of codes (q in {4, 16, 64}, column weight 2-3, rate 1/3-1/2,
n uniform in 256..8000) and channels (BSC, BEC, BI-AWGN at Eb/N0 ~ U[1, 2] dB,
capacity matched; the channel kind given per frame) are decoded four ways:

* one call, code by code: one ``gfbp_decode_batch`` call over every frame (a
  code index per frame); the library decodes each code's frames with the
  plain kernels, the codes concurrently on its worker threads;
* one call, persistent: the same call with ``GFBP_OPT_PERSISTENT``: one
  persistent work-list kernel per field, run concurrently as one HIP graph
  launch, with its tile shape (entries per lane, i.e. frames per tile, and
  wavefronts per workgroup) chosen by ``gfbp_tune_persistent``;
* plain: ``gfbp_decode_batch`` on each (code, channel) group in turn;
* sessions (``--sessions``): one session per code, all stepped as one HIP
  graph replayed until every frame is done.

Every code's kernel shape is autotuned first (the plain ways use it).  The
code-by-code results must equal the plain ones bitwise (checked here and in
tests/test_gpu_batching.py); the persistent ones differ only where a
different lane split rounds differently.  tests/uneven_batch_reference.py
decodes the same batch and checks a deterministic sample of its frames
against the float64 reference decoder.

``python -m paper_cs_0605069_amd.batching`` prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import sys
import time

import numpy as np

from . import (DeviceCode, Graph, Session, decode_batch, decode_multi, frames_for_session, frames_to_device,
               ragged_frames, tune)
from . import workloads as wl


def make_groups(code: wl.Code, F: int, seed: int):
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


def build(frames: int, codes: int, nmax: int):
    pool = wl.mixed_pool(codes, seed=0xC0DE0004, n_range=(256, nmax))
    rng = np.random.default_rng([0xDA7A0004, 1])
    counts = np.bincount(rng.integers(0, len(pool), size=frames), minlength=len(pool))
    items = []
    for ci, (code, F) in enumerate(zip(pool, counts)):
        if F:
            items.append((ci, code, make_groups(code, int(F), 0xDA7A0004 + ci)))
    return pool, items


def batch_inputs(frames: int, codes: int, nmax: int):
    """The uneven batch on the host: the code pool, the (code index, code,
    frame groups) items, the groups in batch order with their codes, and each
    frame's code index."""
    pool, items = build(frames, codes, nmax)
    flat, flat_codes, index = [], [], []
    for ci, code, groups in items:
        for g in groups:
            flat.append(g)
            flat_codes.append(code)
            index += [ci] * g.F
    return pool, items, flat, flat_codes, np.array(index, dtype=np.int32)


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--frames", type=int, default=10000)
    ap.add_argument("--codes", type=int, default=64)
    ap.add_argument("--nmax", type=int, default=8000)
    ap.add_argument("--schedule", default="sus")
    ap.add_argument("--max-iter", type=int, default=100)
    ap.add_argument("--repeats", type=int, default=2, help="timed runs of each way (the fastest is kept)")
    ap.add_argument("--no-tune", action="store_true")
    ap.add_argument("--sessions", action="store_true", help="also time one graph over one session per code")
    ap.add_argument("--iters", type=int, default=4, help="iterations per session-graph replay (even)")
    args = ap.parse_args()
    import torch

    torch.cuda.set_device(0)
    pool, items, flat, flat_codes, index = batch_inputs(args.frames, args.codes, args.nmax)
    F = len(index)
    dcodes = [DeviceCode(c) for c in pool]
    dfr = ragged_frames(flat, flat_codes)
    stream = torch.cuda.Stream()
    eq_frame = np.array([c.E * c.q for c in pool], dtype=np.float64)
    print(f"# {F} frames over {len(items)} codes built", file=sys.stderr, flush=True)

    # every code's plain kernel shape, tuned on its last group
    dev_groups = []
    for ci, code, groups in items:
        dcode = dcodes[ci]
        tune(dcode, frames_to_device(groups[-1]), schedule=args.schedule, trial_iters=2)
        dev_groups.append((ci, dcode, [frames_to_device(g) for g in groups]))
    offs = np.concatenate([[0], np.cumsum([pool[k].n for k in index])])

    def timed(run):
        best, out = None, None
        for _ in range(args.repeats):
            t0 = time.perf_counter()
            with torch.cuda.stream(stream):
                o = run()
            stream.synchronize()
            dt = time.perf_counter() - t0
            if best is None or dt < best:
                best, out = dt, o
        return best, out

    def host(out):
        return out["iters"].cpu().numpy(), out["converged"].cpu().numpy(), out["xhat"].cpu().numpy()

    def differing(a, b):
        mism = (a[0] != b[0]) | (a[1] != b[1])
        mism |= np.array([not np.array_equal(a[2][offs[f]:offs[f + 1]], b[2][offs[f]:offs[f + 1]]) for f in range(F)])
        return int(mism.sum())

    # one call, code by code
    decode_multi(dcodes, index, dfr, schedule=args.schedule, max_iter=2, stream=stream)
    torch.cuda.synchronize()
    one_s, one_out = timed(lambda: decode_multi(dcodes, index, dfr, schedule=args.schedule, max_iter=args.max_iter,
                                                stream=stream))
    one = host(one_out)
    print(f"# one call, code by code: {one_s:.3f} s", file=sys.stderr, flush=True)

    # one call, persistent kernels
    el = waves = 0
    with torch.cuda.stream(stream):
        if not args.no_tune:
            t = decode_multi(dcodes, index, dfr, schedule=args.schedule, max_iter=args.max_iter, stream=stream,
                             tune_iters=2)
            el, waves = t["persist_el"], t["persist_waves"]
        decode_multi(dcodes, index, dfr, schedule=args.schedule, max_iter=2, stream=stream, persistent=True,
                     persist_el=el, persist_waves=waves)
    torch.cuda.synchronize()
    best, p_out = timed(lambda: decode_multi(dcodes, index, dfr, schedule=args.schedule, max_iter=args.max_iter,
                                             stream=stream, persistent=True, persist_el=el, persist_waves=waves))
    pers = host(p_out)
    print(f"# one call, persistent: {best:.3f} s", file=sys.stderr, flush=True)

    # plain kernels, one (code, channel) group after another
    for _, dcode, dg in dev_groups[:2]:  # warm-up
        decode_batch(dcode, dg[0], schedule=args.schedule, max_iter=2)
    torch.cuda.synchronize()

    def plain_all():
        return [decode_batch(dcode, d, schedule=args.schedule, max_iter=args.max_iter, stream=stream)
                for _, dcode, dg in dev_groups for d in dg]

    best_plain, plain_out = timed(plain_all)
    plain = (np.concatenate([o["iters"].cpu().numpy() for o in plain_out]),
             np.concatenate([o["converged"].cpu().numpy() for o in plain_out]),
             np.concatenate([o["xhat"].cpu().numpy().ravel() for o in plain_out]))
    print(f"# plain: {best_plain:.3f} s", file=sys.stderr, flush=True)

    def eq_of(it):
        return float((it * eq_frame[index]).sum())

    res = {"frames": int(F), "codes": len(items), "schedule": args.schedule, "max_iter": args.max_iter,
           "q_counts": {str(q): int(sum(1 for k in index if pool[k].q == q)) for q in sorted({c.q for c in pool})},
           "n_max": int(max(c.n for c in pool)),
           "one_call_s": one_s, "one_call_edge_q_per_s": eq_of(one[0]) / one_s, "one_call_frames_per_s": F / one_s,
           "persistent_s": best, "persistent_edge_q_per_s": eq_of(pers[0]) / best,
           "persistent_frames_per_s": F / best, "persist_el": el, "persist_waves": waves,
           "plain_s": best_plain, "plain_edge_q_per_s": eq_of(plain[0]) / best_plain,
           "plain_frames_per_s": F / best_plain,
           "one_call_vs_plain_frames_differing": differing(one, plain),
           "persistent_vs_plain_frames_differing": differing(pers, plain),
           "mean_iters": float(one[0].mean()), "fer": float(1 - one[1].mean())}
    if res["one_call_vs_plain_frames_differing"]:
        print("# the one-call results differ from the plain decode", file=sys.stderr, flush=True)

    if args.sessions:
        sessions = []
        for ci, code, groups in items:
            Fc = sum(g.F for g in groups)
            d = frames_for_session(groups)
            d["syndrome"] = torch.from_numpy(np.concatenate([g.syndrome for g in groups])).cuda()
            sessions.append((ci, Session(dcodes[ci], n_slots=Fc, schedule=args.schedule, max_iter=args.max_iter,
                                         has_syndrome=True), Fc, d))
        torch.cuda.synchronize()
        graph = Graph([s for _, s, _, _ in sessions], iters=args.iters, stream=stream)
        t0 = time.perf_counter()
        for ci, sess, Fc, d in sessions:
            with torch.cuda.stream(stream):
                assert sess.admit(np.arange(Fc), d, stream=stream) == Fc
        done, g_eq, replays = 0, 0.0, 0
        while done < F:
            graph.launch(stream)
            replays += 1
            for ci, sess, Fc, _ in sessions:
                if sess.running:
                    ids, it, cv, xh = sess.poll(want_xhat=False, stream=stream)
                    done += len(ids)
                    g_eq += float(it.sum()) * eq_frame[ci]
        stream.synchronize()
        dt = time.perf_counter() - t0
        graph.close()
        res.update({"sessions_graph_s": dt, "sessions_graph_edge_q_per_s": g_eq / dt,
                    "sessions_graph_frames_per_s": F / dt, "sessions_graph_replays": replays})

    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    sys.exit(main())
