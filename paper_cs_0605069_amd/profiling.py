"""Summaries of rocprofv3 output for the decoder's kernels.

Two summaries, each a short markdown file that states the command it came
from:

* ``stats``: the per-kernel table of a ``rocprofv3 --kernel-trace --stats
  --output-format csv`` run (calls, average and total duration, share);
* ``traffic``: HBM bytes per dispatch from two ``rocprofv3 --pmc`` runs of
  the same program, one with ``FETCH_SIZE`` and one with ``WRITE_SIZE``
  (KiB per dispatch).  Each counter is scaled by what it reads for a plain
  device-to-device copy of known size made in the same run (the largest
  ``copyBuffer`` dispatch), so the figure is in true bytes.  The file ends
  with a JSON block (kernel -> bytes per dispatch, the kernel shapes and a
  hash of the kernel sources) that ``bench.py`` reads back; the figures are
  only used while the hash still matches the sources.

Usage::

    python -m paper_cs_0605069_amd.profiling stats KERNEL_STATS.csv --command CMD --out FILE.md
    python -m paper_cs_0605069_amd.profiling traffic FETCH.csv WRITE.csv --copy-bytes B \\
        --shapes pus=8,sus=4 --command CMD --out FILE.md
"""
from __future__ import annotations

import argparse
import csv
import glob
import hashlib
import json
import os
import re
from collections import defaultdict

HERE = os.path.dirname(os.path.abspath(__file__))

# decoder kernels as the library's tracer names them
KINDS = {"k_init": "init", "k_check": "check", "k_variable": "variable", "k_sequential": "sequential",
         "k_sus_level": "sus_level", "k_sus_run": "sus_run", "k_syndrome": "syndrome", "k_retire": "retire", "k_markov": "markov",
         "k_out_xhat": "output", "k_out_vectors": "output", "k_tiles": "tiles", "k_state_init": "state_init",
         "k_move_frames": "compact", "k_onchip": "onchip"}


def source_hash() -> str:
    """sha256 over the HIP sources of the library (file names and contents)."""
    h = hashlib.sha256()
    for p in sorted(glob.glob(os.path.join(HERE, "csrc", "*"))):
        if p.endswith((".hip", ".h")):
            h.update(os.path.basename(p).encode())
            with open(p, "rb") as f:
                h.update(f.read())
    return h.hexdigest()


def short_name(name: str) -> str:
    m = re.search(r"(k_\w+)(<[^>(]*>)?", name)
    if m:
        return m.group(1) + (m.group(2) or "")
    return name[:48]


def kind_of(name: str) -> str | None:
    m = re.search(r"(k_\w+)", name)
    return KINDS.get(m.group(1)) if m else None


def stats(path: str) -> list[dict]:
    rows = list(csv.DictReader(open(path)))
    out = []
    for r in rows:
        out.append({"kernel": short_name(r["Name"]), "calls": int(r["Calls"]),
                    "total_ms": float(r["TotalDurationNs"]) / 1e6, "avg_us": float(r["AverageNs"]) / 1e3,
                    "pct": float(r["Percentage"])})
    out.sort(key=lambda x: -x["total_ms"])
    return out


def _roofline(line: dict, key: str) -> dict:
    """The roofline record `key` of a bench JSON line, in the main line's
    field names (the GF(64) leg's records use achieved_GBps and no peak)."""
    r = dict(line[key] if "." not in key else line[key.split(".")[0]][key.split(".")[1]])
    if "achieved" not in r:
        r["achieved"] = r["achieved_GBps"]
        r["peak"] = 8000.0
    return r


def stats_markdown(path: str, command: str, bench_line: str | None = None, plain_line: str | None = None,
                   key: str = "roofline") -> str:
    rows = stats(path)
    lines = ["# Kernel time: rocprofv3 --kernel-trace --stats", "", "Command:", "", "```", command, "```", "",
             "| kernel | calls | avg µs | total ms | % of GPU time |", "|---|---:|---:|---:|---:|"]
    for r in rows:
        lines.append(f"| `{r['kernel']}` | {r['calls']} | {r['avg_us']:.2f} | {r['total_ms']:.2f} | {r['pct']:.2f} |")
    if bench_line:
        # the same run's own HIP-event figures for the dominant kernel
        last = [ln for ln in open(bench_line).read().splitlines() if ln.startswith("{")][-1]
        roof = _roofline(json.loads(last), key)
        k = roof["kernel"]
        calls = sum(r["calls"] for r in rows if kind_of(r["kernel"]) == k)
        tot = sum(r["total_ms"] for r in rows if kind_of(r["kernel"]) == k)
        launches = f" over {roof['launches']} launches" if "launches" in roof else ""
        lines += ["", f"Dominant kernel `{k}`: the program's HIP events give {roof['avg_launch_ms'] * 1e3:.2f} µs "
                      f"average{launches}; this trace gives {tot / max(calls, 1) * 1e3:.2f} µs "
                      f"over {calls} dispatches.  Algorithmic bytes per launch {roof['algo_bytes_per_launch'] / 1e6:.3f} MB, "
                      f"achieved {roof['achieved']:.0f} GB/s ({roof['frac'] * 100:.1f}% of {roof['peak']:.0f} GB/s)."]
    if plain_line:
        # the same bench without the profiler attached
        last = [ln for ln in open(plain_line).read().splitlines() if ln.startswith("{")][-1]
        roof = _roofline(json.loads(last), key if key == "roofline" else "gf64." + key)
        launches = f" over {roof['launches']} launches" if "launches" in roof else ""
        lines += ["", f"The same bench without the profiler (its default steps): `{roof['kernel']}` "
                      f"{roof['avg_launch_ms'] * 1e3:.2f} µs average{launches}, "
                      f"{roof['achieved']:.0f} GB/s ({roof['frac'] * 100:.1f}% of {roof['peak']:.0f} GB/s)."]
    return "\n".join(lines) + "\n"


def counter_means(path: str, counter: str) -> tuple[dict, dict, float]:
    """Per-kernel mean of `counter` over dispatches (KiB), dispatch counts, and
    the counter value of the largest copyBuffer dispatch."""
    tot, cnt = defaultdict(float), defaultdict(int)
    copy = 0.0
    per_dispatch = defaultdict(float)
    names = {}
    for r in csv.DictReader(open(path)):
        if r["Counter_Name"] != counter:
            continue
        key = r["Dispatch_Id"]
        per_dispatch[key] += float(r["Counter_Value"])
        names[key] = r["Kernel_Name"]
    for key, v in per_dispatch.items():
        name = names[key]
        if "copyBuffer" in name:
            copy = max(copy, v)
            continue
        k = short_name(name)
        tot[k] += v
        cnt[k] += 1
    return {k: tot[k] / cnt[k] for k in tot}, dict(cnt), copy


def traffic_markdown(fetch_csv: str, write_csv: str, copy_bytes: int, shapes: str, command: str) -> str:
    f_mean, f_cnt, f_copy = counter_means(fetch_csv, "FETCH_SIZE")
    w_mean, w_cnt, w_copy = counter_means(write_csv, "WRITE_SIZE")
    if f_copy <= 0 or w_copy <= 0:
        raise SystemExit("no copyBuffer dispatch found: run the program with its copy probe")
    f_scale = copy_bytes / (f_copy * 1024.0)
    w_scale = copy_bytes / (w_copy * 1024.0)
    lines = ["# HBM traffic per dispatch: rocprofv3 --pmc FETCH_SIZE, then WRITE_SIZE", "", "Commands (two runs):", "",
             "```", command, "```", "",
             f"Calibration: a plain device-to-device copy of {copy_bytes} bytes read FETCH_SIZE = {f_copy:.1f} KiB "
             f"and WRITE_SIZE = {w_copy:.1f} KiB, so bytes = FETCH_SIZE x {f_scale * 1024:.1f} + "
             f"WRITE_SIZE x {w_scale * 1024:.1f} (factors {f_scale:.3f} and {w_scale:.3f} on KiB x 1024).", "",
             "| kernel | dispatches | FETCH_SIZE KiB | WRITE_SIZE KiB | HBM MB per dispatch (scaled) |",
             "|---|---:|---:|---:|---:|"]
    kernels = {}
    for k in sorted(set(f_mean) & set(w_mean), key=lambda k: -(f_mean[k] + w_mean[k])):
        b = f_mean[k] * 1024 * f_scale + w_mean[k] * 1024 * w_scale
        lines.append(f"| `{k}` | {f_cnt[k]} | {f_mean[k]:.1f} | {w_mean[k]:.1f} | {b / 1e6:.3f} |")
        kind = kind_of(k)
        if kind:
            e = kernels.setdefault(kind, {"bytes_per_dispatch": 0.0, "dispatches": 0})
            n0 = e["dispatches"]
            e["bytes_per_dispatch"] = (e["bytes_per_dispatch"] * n0 + b * f_cnt[k]) / (n0 + f_cnt[k])
            e["dispatches"] = n0 + f_cnt[k]
    block = {"source_sha256": source_hash(), "shapes": dict(kv.split("=") for kv in shapes.split(",") if kv),
             "fetch_scale": f_scale, "write_scale": w_scale, "kernels": kernels}
    lines += ["", "```json", json.dumps(block, indent=1), "```"]
    return "\n".join(lines) + "\n"


def read_traffic(path: str) -> dict | None:
    """The JSON block of a traffic summary, or None when missing or stale."""
    try:
        text = open(path).read()
    except OSError:
        return None
    m = re.search(r"```json\n(.*?)\n```", text, re.S)
    if not m:
        return None
    block = json.loads(m.group(1))
    if block.get("source_sha256") != source_hash():
        return None
    return block


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    sub = ap.add_subparsers(dest="cmd", required=True)
    a = sub.add_parser("stats")
    a.add_argument("csv")
    a.add_argument("--command", required=True)
    a.add_argument("--out", required=True)
    a.add_argument("--bench-line", help="the program's own output (its last JSON line) to compare against")
    a.add_argument("--plain-line", help="output of the same program run without the profiler")
    a.add_argument("--key", default="roofline", help="roofline record of the JSON line (e.g. sus_roofline)")
    b = sub.add_parser("traffic")
    b.add_argument("fetch_csv")
    b.add_argument("write_csv")
    b.add_argument("--copy-bytes", type=int, required=True)
    b.add_argument("--shapes", default="")
    b.add_argument("--command", required=True)
    b.add_argument("--out", required=True)
    args = ap.parse_args()
    if args.cmd == "stats":
        text = stats_markdown(args.csv, args.command, args.bench_line, args.plain_line, args.key)
    else:
        text = traffic_markdown(args.fetch_csv, args.write_csv, args.copy_bytes, args.shapes, args.command)
    with open(args.out, "w") as f:
        f.write(text)
    print(text)


if __name__ == "__main__":
    main()
