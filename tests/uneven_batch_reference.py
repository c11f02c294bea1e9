"""The uneven batch of ``paper_cs_0605069_amd.batching`` (10,000 frames over
64 codes of the mixed pool: q in {4, 16, 64}, n up to 8000, per-frame
channels) decoded in one ``gfbp_decode_batch`` call (code by code, or with
--persistent the persistent kernels at their tuned shape), and a
deterministic sample of its frames (every k-th frame)
decoded by the float64 reference decoder: how many frames agree in decisions
and iteration count, and both sides' FER and mean iterations on the sample.
Not collected by pytest (a long GPU run); run as

    python tests/uneven_batch_reference.py --schedule sus --frames-checked 512

and it prints one JSON line.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--frames", type=int, default=10000)
    ap.add_argument("--codes", type=int, default=64)
    ap.add_argument("--nmax", type=int, default=8000)
    ap.add_argument("--schedule", default="sus")
    ap.add_argument("--max-iter", type=int, default=100)
    ap.add_argument("--frames-checked", type=int, default=512)
    ap.add_argument("--persistent", action="store_true")
    args = ap.parse_args()
    import torch

    import oracle
    import paper_cs_0605069_amd as gfbp
    from paper_cs_0605069_amd.batching import batch_inputs

    torch.cuda.set_device(0)
    pool, items, flat, flat_codes, index = batch_inputs(args.frames, args.codes, args.nmax)
    F = len(index)
    dcodes = [gfbp.DeviceCode(c) for c in pool]
    dfr = gfbp.ragged_frames(flat, flat_codes)
    t = {"persist_el": 0, "persist_waves": 0}
    if args.persistent:
        t = gfbp.decode_multi(dcodes, index, dfr, schedule=args.schedule, max_iter=args.max_iter, tune_iters=2)
    out = gfbp.decode_multi(dcodes, index, dfr, schedule=args.schedule, max_iter=args.max_iter,
                            persistent=args.persistent, persist_el=t["persist_el"], persist_waves=t["persist_waves"])
    torch.cuda.synchronize()
    g_it = out["iters"].cpu().numpy()
    g_cv = out["converged"].cpu().numpy()
    g_xh = out["xhat"].cpu().numpy()
    offs = np.concatenate([[0], np.cumsum([pool[k].n for k in index])])
    step = max(1, F // args.frames_checked)
    pick = np.arange(0, F, step)[:args.frames_checked]
    sch = {"pus": oracle.PUS, "sus": oracle.SUS}[args.schedule]
    t0 = time.perf_counter()
    same, r_it, r_cv, base = 0, [], [], 0
    for g, code in zip(flat, flat_codes):
        rows = pick[(pick >= base) & (pick < base + g.F)]
        if len(rows):
            r = oracle.decode(code, g.subset(rows - base), schedule=sch, max_iter=args.max_iter)
            for k, f in enumerate(rows):
                same += int(g_it[f] == r["iters"][k] and np.array_equal(g_xh[offs[f]:offs[f + 1]], r["xhat"][k]))
            r_it.append(r["iters"])
            r_cv.append(r["converged"])
            print(f"# reference: {len(np.concatenate(r_it))} of {len(pick)} frames", file=sys.stderr, flush=True)
        base += g.F
    r_it, r_cv = np.concatenate(r_it), np.concatenate(r_cv)
    print(json.dumps({"frames": int(F), "schedule": args.schedule, "persistent": args.persistent,
                      "persist_el": t["persist_el"],
                      "persist_waves": t["persist_waves"], "frames_checked": int(len(pick)),
                      "identical": int(same), "reference_s": time.perf_counter() - t0,
                      "reference_threads": oracle.max_threads(),
                      "reference_mean_iters": float(r_it.mean()), "gpu_mean_iters_same_frames": float(g_it[pick].mean()),
                      "reference_fer": float(1 - r_cv.mean()), "gpu_fer_same_frames": float(1 - g_cv[pick].mean())}),
          flush=True)


if __name__ == "__main__":
    sys.exit(main())
