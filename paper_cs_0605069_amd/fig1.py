"""Stand-in for the paper's Fig. 1: per-iteration progress of PUS vs SUS.

Fig. 1 plots, against the current fraction P of correctly decoded bits, the
ratio of the mean progress per iteration of the two schedules,
<dP_PUS> / <dP_SUS> (about 1/2 through decoding), for a rate-1/3 MN code over
GF(8) with N = 3333 source symbols (9999 bits), a 2-state Markov source and
a BSC with f = 0.23, over 10,000 samples.  Here the MN stand-in code of
``workloads.mn_code`` is used (the paper's construction is not specified),
with f scaled to the stand-in's own threshold region (``--scale``).

P(t) is the fraction of source bits whose decision equals the truth after
iteration t (from ``gfbp_result.trace``), P(0) that of the decision taken
from the prior alone; dP(t) = P(t) - P(t-1) for every iteration a sample ran.
Progress steps are grouped by P(t-1) into bins, and each bin reports the mean
dP of each schedule and their ratio.

``python -m paper_cs_0605069_amd.fig1`` prints one JSON line per bin and a
summary line.
"""
from __future__ import annotations

import argparse
import json
import sys

import numpy as np

from . import DeviceCode, decode_batch, frames_to_device
from . import workloads as wl


def progress(trace: np.ndarray, iters: np.ndarray, p0: np.ndarray, nbits: int):
    """(P(t-1), dP(t)) pairs of every iteration each sample ran."""
    P = np.concatenate([p0[:, None], trace / float(nbits)], axis=1)  # [F][1 + max_iter]
    t = np.arange(1, trace.shape[1] + 1)[None, :]
    ran = t <= iters[:, None]
    return P[:, :-1][ran], (P[:, 1:] - P[:, :-1])[ran]


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--samples", type=int, default=10000)
    ap.add_argument("--batch", type=int, default=2000)
    ap.add_argument("--f", type=float, default=0.23)
    ap.add_argument("--scale", type=float, default=0.85)
    ap.add_argument("--max-iter", type=int, default=300)
    ap.add_argument("--bins", default="0.5,0.6,0.7,0.8,0.85,0.9,0.95,0.98,0.99,0.995,0.999,1.0")
    args = ap.parse_args()
    import torch

    torch.cuda.set_device(0)
    q, p, N = 8, 3, 3333
    code = wl.mn_code(N, 3 * N, q, seed=0xC0DE0F01)
    M, start = wl.lift_binary_chain(wl.PAPER_MARKOV_2S, p)
    kw = dict(prior="markov", markov_M=M, markov_pi=start)
    dcode = DeviceCode(code)
    f = args.f * args.scale
    prior_guess = int(np.argmax(start))  # decision from the source prior alone (uniform channel term)
    pairs = {"pus": ([], []), "sus": ([], [])}
    iters = {"pus": [], "sus": []}
    for b0 in range(0, args.samples, args.batch):
        F = min(args.batch, args.samples - b0)
        fr = wl.make_mn_frames(code, F, 0xDA7A0F01 * 1000 + b0, "bsc", f, source="markov", markov=M, start=start)
        d = frames_to_device(fr)
        truth = torch.from_numpy(fr.codeword).cuda()
        wrong0 = np.unpackbits((fr.codeword[:, :N] ^ prior_guess)[..., None], axis=-1).sum(axis=(1, 2))
        p0 = 1.0 - wrong0 / float(N * p)
        for s in ("pus", "sus"):
            out = decode_batch(dcode, d, schedule=s, max_iter=args.max_iter, truth=truth, **kw)
            torch.cuda.synchronize()
            it = out["iters"].cpu().numpy()
            Pp, dP = progress(out["trace"].cpu().numpy(), it, p0, N * p)
            pairs[s][0].append(Pp)
            pairs[s][1].append(dP)
            iters[s].append(it)
    edges = [float(x) for x in args.bins.split(",")]
    Pp = {s: np.concatenate(pairs[s][0]) for s in pairs}
    dP = {s: np.concatenate(pairs[s][1]) for s in pairs}
    for lo, hi in zip(edges[:-1], edges[1:]):
        row = {"P_from": lo, "P_to": hi}
        for s in ("pus", "sus"):
            sel = (Pp[s] >= lo) & ((Pp[s] < hi) if hi < 1.0 else (Pp[s] <= hi))
            row[f"steps_{s}"] = int(sel.sum())
            row[f"mean_dP_{s}"] = float(dP[s][sel].mean()) if sel.any() else None
        if row["mean_dP_pus"] is not None and row["mean_dP_sus"]:
            row["ratio_pus_over_sus"] = row["mean_dP_pus"] / row["mean_dP_sus"]
        print(json.dumps(row), flush=True)
    it = {s: np.concatenate(iters[s]) for s in iters}
    print(json.dumps({"summary": True, "q": q, "N": N, "f": f, "samples": args.samples,
                      "mean_iters_pus": float(it["pus"].mean()), "mean_iters_sus": float(it["sus"].mean()),
                      "ratio_of_means": float(it["sus"].mean() / it["pus"].mean())}), flush=True)


if __name__ == "__main__":
    sys.exit(main())
