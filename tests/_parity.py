"""Decision and statistics gates of the GPU parity tests.

A frame is identical when the GPU and the reference decoder give the same
decision vector and the same iteration count.  At least 99.9% of the frames
must be identical (at most floor(0.001 F) others); a differing frame is
excused, and logged, only as
  * near-tie: in the reference, the smallest gap between the two largest
    pseudo-posterior entries of a symbol (over the symbols) falls below 1e-3
    at some iteration up to the first iteration at which the GPU's decision
    vector differs from the reference's (reading R14: the decision there is
    not fixed by the arithmetic's last bits), or
  * chaotic: neither side converged (both ran max_iter iterations).
A frame that only one side decoded is never chaotic: it counts as differing
unless it is a near-tie, and it enters the frame error rate of its side.
FER (Wilson) and mean-iteration (Student-t normal approximation) 95%
intervals of the two sides must overlap.

Every gate appends its per-class counts as one JSON line to the file named by
the GFBP_PARITY_LOG environment variable, when set.
"""
from __future__ import annotations

import json
import math
import os

import numpy as np

import oracle

MSG_TOL = 1e-4
GAP = 1e-3


def sched(s):
    return {"pus": oracle.PUS, "sus": oracle.SUS}[s]


def gpu_decode(gfbp, code, dfr, schedule, **kw):
    import torch

    dcode = gfbp.DeviceCode(code)
    out = gfbp.decode_batch(dcode, dfr, schedule=schedule, **kw)
    torch.cuda.synchronize()
    return {k: v.cpu().numpy() for k, v in out.items()}


def _oracle_kw(kw):
    return {k: v for k, v in kw.items() if k in ("prior", "markov_M", "markov_pi", "static_prior", "prior_in_sweep")}


def first_divergence(gfbp, code, fr, schedule, idx, ref_trace, horizon, **kw):
    """For the frames idx: the first iteration t (1-based) after which the
    GPU's decision vector differs from the reference's decision vector
    ref_trace[k][t-1]; horizon[k] (the last iteration to look at) when none
    does."""
    import torch

    idx = np.asarray(idx)
    sub = fr.subset(idx)
    dfr = gfbp.frames_to_device(sub)
    dcode = gfbp.DeviceCode(code)
    first = np.asarray(horizon, dtype=np.int64).copy()
    open_ = np.ones(len(idx), dtype=bool)
    gkw = {k: v for k, v in kw.items() if k not in ("max_iter", "early_stop", "posterior", "snap_iter")}
    for t in range(1, int(max(horizon)) + 1):
        if not open_.any():
            break
        out = gfbp.decode_batch(dcode, dfr, schedule=schedule, max_iter=t, early_stop=False, **gkw)
        torch.cuda.synchronize()
        xh = out["xhat"].cpu().numpy()
        diff = (xh != ref_trace[:, t - 1, :]).any(axis=1) & open_ & (t <= np.asarray(horizon))
        first[diff] = t
        open_ &= ~diff
        open_ &= t < np.asarray(horizon)
    return first


def posterior_error_trace(gfbp, code, fr, schedule, idx, upto, **kw):
    """For frames idx: the largest absolute difference between the GPU's and
    the reference's pseudo-posteriors after each iteration 1..upto[k]
    (NaN past a frame's own limit): how the two computations drift apart."""
    import torch

    idx = np.asarray(idx)
    sub = fr.subset(idx)
    dfr = gfbp.frames_to_device(sub)
    dcode = gfbp.DeviceCode(code)
    okw = _oracle_kw(kw)
    gkw = {k: v for k, v in kw.items() if k not in ("max_iter", "early_stop", "posterior", "snap_iter")}
    T = int(max(upto))
    err = np.full((len(idx), T), np.nan)
    for t in range(1, T + 1):
        out = gfbp.decode_batch(dcode, dfr, schedule=schedule, max_iter=t, early_stop=False, posterior=True, **gkw)
        torch.cuda.synchronize()
        r = oracle.decode(code, sub, schedule=sched(schedule), max_iter=t, early_stop=False, posterior=True, **okw)
        e = np.abs(out["posterior"].cpu().numpy() - r["posterior"]).max(axis=(1, 2))
        err[:, t - 1] = np.where(t <= np.asarray(upto), e, np.nan)
    return err


def classify(gfbp, code, fr, g, r, schedule, label, budget=0.001, **kw):
    """Class of every frame (identical / near-tie / chaotic / differing) and
    the gates (at most floor(budget F) differing frames); returns the
    identical mask.  For each differing frame the per-iteration posterior
    drift up to its divergence is logged."""
    F = len(g["iters"])
    max_iter = int(kw.get("max_iter", 100))
    same = (g["xhat"] == r["xhat"]).all(axis=1) & (g["iters"] == r["iters"])
    both_failed = (g["converged"] == 0) & (r["converged"] == 0)
    chaotic = ~same & both_failed
    cand = np.nonzero(~same & ~both_failed)[0]
    ties = np.zeros(F, dtype=bool)
    first = {}
    if len(cand):
        okw = _oracle_kw(kw)
        sub = fr.subset(cand)
        horizon = np.minimum(np.maximum(g["iters"][cand], r["iters"][cand]), max_iter)
        tr = oracle.decode(code, sub, schedule=sched(schedule), max_iter=int(horizon.max()), early_stop=False,
                           trace=True, gap_trace=True, **okw)
        d = first_divergence(gfbp, code, fr, schedule, cand, tr["trace"], horizon, **kw)
        for k, f in enumerate(cand):
            gaps = tr["gap_trace"][k, : int(d[k])]
            first[int(f)] = (int(d[k]), float(np.nanmin(gaps)) if len(gaps) else float("nan"))
            ties[f] = bool(len(gaps) and np.nanmin(gaps) < GAP)
    bad = ~same & ~chaotic & ~ties
    drift = {}
    if bad.any():
        bi = np.nonzero(bad)[0]
        upto = np.array([first[int(f)][0] for f in bi])
        err = posterior_error_trace(gfbp, code, fr, schedule, bi, upto, **kw)
        for k, f in enumerate(bi):
            e = err[k, : upto[k]]
            above = np.nonzero(e > MSG_TOL)[0]
            drift[int(f)] = {"divergence": int(upto[k]), "smallest_gap": first[int(f)][1],
                             "first_iteration_above_1e-4": int(above[0]) + 1 if len(above) else None,
                             "posterior_error_by_iteration": [float(x) for x in e]}
    counts = {"label": label, "frames": int(F), "identical": int(same.sum()), "near_tie": int(ties.sum()),
              "chaotic": int(chaotic.sum()), "differing": int(bad.sum()),
              "allowed_differing": int(math.floor(budget * F)), "differing_drift": drift,
              "mean_iters_gpu": float(g["iters"].mean()), "mean_iters_ref": float(r["iters"].mean()),
              "fer_gpu": float(1 - g["converged"].mean()), "fer_ref": float(1 - r["converged"].mean())}
    print(json.dumps(counts))
    for name, mask in (("near-tie", ties), ("chaotic", chaotic), ("differing", bad)):
        if mask.any():
            fi = np.nonzero(mask)[0][:8]
            print(f"[{label}] {name} frames {fi.tolist()} iters gpu={g['iters'][fi].tolist()} "
                  f"ref={r['iters'][fi].tolist()} (first divergence, smallest gap before it) "
                  f"{[first.get(int(f)) for f in fi]}")
    log = os.environ.get("GFBP_PARITY_LOG")
    if log:
        with open(log, "a") as fh:
            fh.write(json.dumps(counts) + "\n")
    assert bad.sum() <= counts["allowed_differing"], f"{label}: {int(bad.sum())} frames differ (not near-ties)"
    assert fer_ci_overlap(g["converged"], r["converged"]), f"{label}: FER intervals do not overlap"
    assert mean_ci_overlap(g["iters"].astype(float), r["iters"].astype(float)), \
        f"{label}: mean-iteration intervals do not overlap"
    return same


def wilson(k, n, z=1.96):
    """95% Wilson score interval of a binomial proportion k/n."""
    p = k / n
    c = (p + z * z / (2 * n)) / (1 + z * z / n)
    h = z * math.sqrt(p * (1 - p) / n + z * z / (4 * n * n)) / (1 + z * z / n)
    return c - h, c + h


def fer_ci_overlap(conv_a, conv_b):
    a = wilson(int((conv_a == 0).sum()), len(conv_a))
    b = wilson(int((conv_b == 0).sum()), len(conv_b))
    return a[0] <= b[1] and b[0] <= a[1]


def mean_ci_overlap(a, b):
    """95% intervals of two means (normal approximation) overlap."""
    sa = 1.96 * a.std(ddof=1) / math.sqrt(len(a)) if len(a) > 1 else 0.0
    sb = 1.96 * b.std(ddof=1) / math.sqrt(len(b)) if len(b) > 1 else 0.0
    return abs(a.mean() - b.mean()) <= sa + sb + 1e-12


def messages_close(gfbp, code, fr, schedule, iters=(1, 2, 3, 4, 5), label="", **kw):
    """q, r and Q after each listed iteration within MSG_TOL of the reference."""
    okw = _oracle_kw(kw)
    gkw = {k: v for k, v in kw.items() if k not in ("max_iter", "early_stop")}
    dfr = gfbp.frames_to_device(fr)
    worst = 0.0
    for it in iters:
        g = gpu_decode(gfbp, code, dfr, schedule, max_iter=it, early_stop=False, snap_iter=it, **gkw)
        r = oracle.decode(code, fr, schedule=sched(schedule), max_iter=it, early_stop=False, snap_iter=it, **okw)
        for key in ("snap_q", "snap_r", "snap_Q"):
            err = float(np.abs(g[key] - r[key]).max())
            worst = max(worst, err)
            assert err <= MSG_TOL, f"{label} {schedule} iter {it} {key}: max abs error {err:.3g}"
    return worst


def summary(log_path: str) -> str:
    """Markdown table of the per-class counts a GPU run appended to
    GFBP_PARITY_LOG (``python -m tests._parity LOG``)."""
    rows = [json.loads(ln) for ln in open(log_path) if ln.strip()]
    out = ["| gate | frames | identical | near-tie | chaotic | differing (allowed) | FER GPU / ref | mean iters GPU / ref |",
           "|---|---:|---:|---:|---:|---:|---:|---:|"]
    tot = dict(frames=0, identical=0, near_tie=0, chaotic=0, differing=0)
    for d in rows:
        for k in tot:
            tot[k] += d[k]
        out.append(f"| {d['label']} | {d['frames']} | {d['identical']} | {d['near_tie']} | {d['chaotic']} | "
                   f"{d['differing']} ({d['allowed_differing']}) | {d['fer_gpu']:.4f} / {d['fer_ref']:.4f} | "
                   f"{d['mean_iters_gpu']:.3f} / {d['mean_iters_ref']:.3f} |")
    out.append(f"| **all gates** | {tot['frames']} | {tot['identical']} | {tot['near_tie']} | {tot['chaotic']} | "
               f"{tot['differing']} | | |")
    drift = [(d["label"], f, v) for d in rows for f, v in d.get("differing_drift", {}).items()]
    if drift:
        out += ["", "Differing frames: divergence iteration, the reference's smallest top-two gap before it, the "
                    "first iteration whose GPU-vs-reference posterior difference exceeds 1e-4, and that difference "
                    "at the divergence.", "",
                "| gate | frame | divergence | smallest gap | first > 1e-4 | posterior difference at divergence |",
                "|---|---:|---:|---:|---:|---:|"]
        for label, f, v in drift:
            e = v["posterior_error_by_iteration"]
            out.append(f"| {label} | {f} | {v['divergence']} | {v['smallest_gap']:.2e} | "
                       f"{v['first_iteration_above_1e-4']} | {e[-1]:.2e} |")
    return "\n".join(out) + "\n"


if __name__ == "__main__":
    import sys

    print(summary(sys.argv[1]), end="")
