"""Uneven batches: many codes' frames decoded together through one HIP graph.

Frames of a pool of codes (q in {4, 16, 64}, column weight 2-3, rate 1/3-1/2,
n uniform in 256..8000) and channels (BSC, BEC, BI-AWGN at Eb/N0 ~ U[1, 2] dB,
capacity matched) are decoded two ways:

* graph: one session per code holds all of that code's frames; each code's
  kernel shape is autotuned on its frames; one HIP graph holds `iters`
  iterations of every session (one branch per session) and is replayed, with
  the finished frames collected between replays, until every frame is done;
* plain: ``gfbp_decode_batch`` on each (code, channel) group in turn.

Both give bitwise the same per-frame results (tests/test_gpu_batching.py);
this reports the wall time and edge-q update rate of each way.

``python -m paper_cs_0605069_amd.batching`` prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import sys
import time

import numpy as np

from . import DeviceCode, Graph, Session, decode_batch, frames_for_session, frames_to_device, tune
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


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--frames", type=int, default=10000)
    ap.add_argument("--codes", type=int, default=64)
    ap.add_argument("--nmax", type=int, default=8000)
    ap.add_argument("--schedule", default="sus")
    ap.add_argument("--max-iter", type=int, default=100)
    ap.add_argument("--iters", type=int, default=4, help="iterations per graph replay (even)")
    args = ap.parse_args()
    import torch

    torch.cuda.set_device(0)
    pool = wl.mixed_pool(args.codes, seed=0xC0DE0004, n_range=(256, args.nmax))
    rng = np.random.default_rng([0xDA7A0004, 1])
    counts = np.bincount(rng.integers(0, len(pool), size=args.frames), minlength=len(pool))
    stream = torch.cuda.Stream()
    items = []
    for ci, (code, F) in enumerate(zip(pool, counts)):
        if F == 0:
            continue
        groups = make_groups(code, int(F), 0xDA7A0004 + ci)
        dcode = DeviceCode(code)
        tune(dcode, frames_to_device(groups[-1]), schedule=args.schedule, trial_iters=2)
        items.append((code, dcode, groups))
    eq_frame = {id(c): c.E * c.q for c, _, _ in items}
    torch.cuda.synchronize()

    # plain kernels, one (code, channel) group after another
    dev_groups = [(code, dcode, [frames_to_device(g) for g in groups]) for code, dcode, groups in items]
    for _, dcode, dg in dev_groups[:2]:  # warm-up
        decode_batch(dcode, dg[0], schedule=args.schedule, max_iter=2)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    plain_eq = 0.0
    for code, dcode, dg in dev_groups:
        for d in dg:
            o = decode_batch(dcode, d, schedule=args.schedule, max_iter=args.max_iter, stream=stream)
            plain_eq += float(o["iters"].sum().item()) * eq_frame[id(code)]
    stream.synchronize()
    t_plain = time.perf_counter() - t0

    # one graph over one session per code
    sessions = []
    for code, dcode, groups in items:
        F = sum(g.F for g in groups)
        dfr = frames_for_session(groups)
        dfr["syndrome"] = torch.from_numpy(np.concatenate([g.syndrome for g in groups])).cuda()
        sess = Session(dcode, n_slots=F, schedule=args.schedule, max_iter=args.max_iter, has_syndrome=True)
        sessions.append((code, sess, F, dfr))
    torch.cuda.synchronize()
    graph = Graph([s for _, s, _, _ in sessions], iters=args.iters, stream=stream)
    t0 = time.perf_counter()
    for code, sess, F, dfr in sessions:
        with torch.cuda.stream(stream):
            assert sess.admit(np.arange(F), dfr, stream=stream) == F
    done, graph_eq, replays = 0, 0.0, 0
    while done < args.frames:
        graph.launch(stream)
        replays += 1
        for code, sess, F, _ in sessions:
            if sess.running:
                ids, it, cv, xh = sess.poll(want_xhat=False, stream=stream)
                done += len(ids)
                graph_eq += float(it.sum()) * eq_frame[id(code)]
    stream.synchronize()
    t_graph = time.perf_counter() - t0
    graph.close()
    print(json.dumps({
        "frames": int(args.frames), "codes": len(items), "schedule": args.schedule, "max_iter": args.max_iter,
        "plain_s": t_plain, "plain_edge_q_per_s": plain_eq / t_plain, "plain_frames_per_s": args.frames / t_plain,
        "graph_s": t_graph, "graph_edge_q_per_s": graph_eq / t_graph, "graph_frames_per_s": args.frames / t_graph,
        "graph_replays": replays, "iters_per_replay": args.iters}), flush=True)


if __name__ == "__main__":
    sys.exit(main())
