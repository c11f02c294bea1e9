"""Stand-ins for the paper's Table 1: SUS vs PUS on MN syndrome-form codes.

The paper decodes rate-1/3 MacKay-Neal codes (H = [A B], Section 2) with
N = 10000 / log2(q) source symbols over the BSC, the BEC and the BI-AWGN
channel, for GF(2) with an i.i.d. source, GF(4) with its 4-state Markov
source and GF(8) with its 2-state Markov source, and reports the mean
iteration counts of both schedules, their ratio of means, the mean and
standard deviation of the per-sample ratio, and the bit error rate (Table 1).
Its codes come from the Kanter-Saad construction, which it does not specify;
``workloads.mn_code`` (A with column weight 3, lower-triangular B) stands in,
so the iteration counts and error rates are not the paper's: the comparison
is the schedules' ratio.  ``--b-form chain`` (the default) gives B a
dual-diagonal chain, whose noise columns a sequential sweep must visit one
after another; ``--b-form pool`` places each column's second entry in a
random later row, which leaves the sweep a few tens of dependency levels.

``python -m paper_cs_0605069_amd.table1`` decodes every setting with both
schedules on the same samples and prints one JSON line per setting;
``--schedules pus,sus,sus-in-sweep`` adds SUS with the Markov priors assigned
during the sweep (the same as SUS for the i.i.d. rows).
"""
from __future__ import annotations

import argparse
import json
import math
import sys
import time

import numpy as np

from . import DeviceCode, decode_batch, frames_to_device
from . import workloads as wl

# (channel, q, source, noise parameter) of the nine rows of Table 1
SETTINGS = [
    ("bsc", 2, "iid", 0.155), ("bsc", 4, "4s", 0.227), ("bsc", 8, "2s", 0.230),
    ("bec", 2, "iid", 0.58), ("bec", 4, "4s", 0.78), ("bec", 8, "2s", 0.76),
    ("biawgn", 2, "iid", 0.98), ("biawgn", 4, "4s", 1.64), ("biawgn", 8, "2s", 1.66),
]


def source_model(name: str, q: int):
    """(transition matrix, start distribution) of a source over GF(q)."""
    if name == "iid":
        return None, None
    if name == "4s":
        assert q == 4
        M = wl.PAPER_MARKOV_4S
        return M, wl.stationary(M)
    if name == "2s":
        return wl.lift_binary_chain(wl.PAPER_MARKOV_2S, int(round(math.log2(q))))
    raise ValueError(name)


def run_setting(channel: str, q: int, source: str, param: float, samples: int, batch: int, max_iter: int,
                seed: int, scale: float = 1.0, source_bits: int = 10000, schedules=("pus", "sus"),
                b_form: str = "chain", pool: int = 1000) -> dict:
    import torch

    p = int(round(math.log2(q)))
    N = source_bits // p
    code = wl.mn_code(N, 3 * N, q, seed=seed, b_form=b_form, pool=pool)
    M, start = source_model(source, q)
    kw = {} if M is None else dict(prior="markov", markov_M=M, markov_pi=start)
    dcode = DeviceCode(code)
    it = {s: [] for s in schedules}
    conv = {s: [] for s in schedules}
    berr = {s: 0 for s in schedules}
    gpu_s = {s: 0.0 for s in schedules}
    prm = param * scale
    for b0 in range(0, samples, batch):
        F = min(batch, samples - b0)
        fr = wl.make_mn_frames(code, F, seed * 1000 + b0, channel, prm, source="iid" if M is None else "markov",
                               markov=M, start=start)
        d = frames_to_device(fr)
        torch.cuda.synchronize()
        for s in schedules:
            t0 = time.perf_counter()
            out = decode_batch(dcode, d, schedule=s[:3], max_iter=max_iter,
                               prior_in_sweep=s.endswith("in-sweep") and M is not None, **kw)
            torch.cuda.synchronize()
            gpu_s[s] += time.perf_counter() - t0
            print(f"# {channel} q={q} {source} {s}: frames {b0}..{b0 + F} in {time.perf_counter() - t0:.1f} s",
                  file=sys.stderr, flush=True)
            xh = out["xhat"].cpu().numpy()
            it[s].append(out["iters"].cpu().numpy())
            conv[s].append(out["converged"].cpu().numpy().astype(bool))
            # bit errors over the source bits
            diff = xh[:, :N] ^ fr.codeword[:, :N]
            berr[s] += int(np.unpackbits(diff[..., None], axis=-1).sum())
    res = {"channel": channel, "q": q, "source": source, "noise": prm, "N": N, "M": 3 * N, "E": code.E,
           "samples": samples, "max_iter": max_iter, "b_form": b_form, "sus_levels": dcode.info.sus_levels}
    ti = {s: np.concatenate(it[s]).astype(np.float64) for s in schedules}
    cv = {s: np.concatenate(conv[s]) for s in schedules}
    for s in schedules:
        res[f"t_{s}"] = float(ti[s].mean())
        res[f"t_{s}_converged"] = float(ti[s][cv[s]].mean()) if cv[s].any() else None
        res[f"fer_{s}"] = float(1.0 - cv[s].mean())
        res[f"ber_{s}"] = berr[s] / float(samples * N * p)
        res[f"edge_q_per_s_{s}"] = float(ti[s].sum() * code.E * q / gpu_s[s])
        res[f"seconds_{s}"] = gpu_s[s]
    for s in schedules:
        if s == "pus" or "pus" not in schedules:
            continue
        tag = "" if s == "sus" else f"_{s.replace('-', '_')}"
        both = cv["pus"] & cv[s]
        res[f"ratio_of_means{tag}"] = res[f"t_{s}"] / res["t_pus"]
        if both.any():
            r = ti[s][both] / ti["pus"][both]
            res[f"mean_of_ratios{tag}"] = float(r.mean())
            res[f"stdev_of_ratios{tag}"] = float(r.std())
            res[f"both_converged{tag}"] = int(both.sum())
    return res


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--samples", type=int, default=6000)
    ap.add_argument("--batch", type=int, default=2000)
    ap.add_argument("--max-iter", type=int, default=300)
    ap.add_argument("--scale", type=float, default=1.0, help="multiply every noise parameter")
    ap.add_argument("--only", default="", help="comma-separated row numbers (1-9) to run")
    ap.add_argument("--schedules", default="pus,sus")
    ap.add_argument("--b-form", default="chain", choices=["chain", "pool"], help="form of the stand-in codes' B")
    ap.add_argument("--pool", type=int, default=1000, help="pool form: rows a column waits on average")
    args = ap.parse_args()
    import torch

    torch.cuda.set_device(0)
    rows = [int(x) for x in args.only.split(",") if x] or list(range(1, 10))
    for k in rows:
        channel, q, source, param = SETTINGS[k - 1]
        res = run_setting(channel, q, source, param, args.samples, args.batch, args.max_iter,
                          seed=0xC0DE0100 + k, scale=args.scale, schedules=tuple(args.schedules.split(",")),
                          b_form=args.b_form, pool=args.pool)
        res["row"] = k
        print(json.dumps(res), flush=True)


if __name__ == "__main__":
    sys.exit(main())
