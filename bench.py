"""Benchmark: GF(q) LDPC belief-propagation decoding, PUS and SUS, one MI355X.

Workload (one "step"): GF(16), regular (3,6), rate 1/2, N = 2000 symbols
(8000 bits); BPSK over BI-AWGN at Eb/N0 = 0.8, 1.0, 1.2, 1.4, 1.6 dB, 4096
frames per point, each point decoded in one launch under the parallel (PUS)
and then the sequential (SUS) schedule, max 100 iterations, early stopping
on H x = 0.  Inputs (code, codewords, channel outputs) are seeded synthetic
data generated once and resident in device memory before timing starts.

Reported value: edge-q message updates per second over the whole step, where
a frame that ran t iterations counts t * E * q updates (E = edges, q = field
size).  Also per schedule: updates/s, frames/s, mean iterations, decode-call
latency; the roofline of the dominant kernel from HIP events recorded around
each launch during the timed steps, beside the bandwidth a plain streaming
copy reaches on the same device (measured after the timed steps); the
reference decoder timed on a bounded
sample of the same frames on the host cores; a GF(64) leg; a serving leg
(continuous batching of a Poisson stream of mixed-code frames: throughput and
p50/p99 frame latency per schedule); a Table-1 stand-in leg (both
schedules' iteration counts and GPU time on a syndrome-form MN code); and
an uneven-batch leg (10,000 frames of 64 codes in one call per schedule,
code by code, and the same call as one persistent launch).

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--cpu-frames S]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK = 8.0e12  # MI355X HBM3E, bytes/s
EBN0 = (0.8, 1.0, 1.2, 1.4, 1.6)
N_SYM, DV, DC, Q = 2000, 3, 6, 16
FRAMES = 4096
MAX_ITER = 100
CODE_SEED, DATA_SEED = 0xC0DE0002, 0xDA7A0002


def make_workload():
    from paper_cs_0605069_amd import workloads as wl

    code, enc = wl.regular_code(N_SYM, DV, DC, Q, seed=CODE_SEED)
    rate = code.n_info / code.n
    points = []
    for i, eb in enumerate(EBN0):
        sigma = wl.sigma_from_ebn0(eb, rate)
        points.append((eb, wl.make_frames(code, enc, FRAMES, DATA_SEED * 16 + i, "biawgn", sigma)))
    return code, points


def cpu_baseline(code, points, n_frames: int, rec=None):
    """Reference decoder on every k-th frame of the step (all points), both
    schedules; with the timed steps' records `rec`, also both sides' FER and
    mean iterations on those frames and how many ran the same iterations."""
    import oracle
    from paper_cs_0605069_amd import workloads as wl

    per_point = max(1, n_frames // len(points))
    stride = FRAMES // per_point
    idx = np.arange(0, FRAMES, stride)[:per_point]
    subs = [fr.subset(idx) for _, fr in points]
    fr = wl.Frames("biawgn", np.concatenate([s.param for s in subs]), np.concatenate([s.codeword for s in subs]),
                   y=np.concatenate([s.y for s in subs]))
    threads = oracle.max_threads()
    eq = 0.0
    t0 = time.perf_counter()
    iters = {}
    outs = {}
    for name, sch in (("pus", oracle.PUS), ("sus", oracle.SUS)):
        out = oracle.decode(code, fr, schedule=sch, max_iter=MAX_ITER)
        eq += float(out["iters"].sum()) * code.E * code.q
        iters[name] = float(out["iters"].mean())
        outs[name] = out
    dt = time.perf_counter() - t0
    res = {"value": eq / dt, "unit": "edge·q updates/s", "cores": threads, "kind": "oracle",
           "sample": f"{fr.F} frames (every {stride}th of each of the {len(points)} Eb/N0 points), "
                     f"PUS and SUS, max {MAX_ITER} iterations, float64, {dt:.1f} s wall",
           "frames_per_s": 2 * fr.F / dt, "mean_iters": iters}
    if rec:
        side = {}
        for name, out in outs.items():
            g_it = np.concatenate([next(r for r in rec if r["sched"] == name and r["ebn0"] == eb)["iters"][idx]
                                   for eb, _ in points])
            g_cv = np.concatenate([next(r for r in rec if r["sched"] == name and r["ebn0"] == eb)["conv"][idx]
                                   for eb, _ in points])
            side[name] = {"frames": int(fr.F), "same_iterations": int((g_it == out["iters"]).sum()),
                          "mean_iters_gpu": float(g_it.mean()), "mean_iters_reference": float(out["iters"].mean()),
                          "fer_gpu": float(1 - g_cv.mean()), "fer_reference": float(1 - out["converged"].mean())}
        res["gpu_on_the_same_frames"] = side
    return res


def gf64_leg(gfbp, torch, steps: int, traffic_path: str = "", shapes: dict | None = None) -> dict:
    """GF(64) (3,6) rate-1/2 N=2000, BI-AWGN at 1.6 dB, 4096 frames, max 100
    iterations, autotuned: per schedule edge-q/s, frames/s and the roofline of
    its dominant kernel, with the measured HBM traffic of that kernel when a
    current traffic summary exists (not part of `value`)."""
    from paper_cs_0605069_amd import workloads as wl

    code, enc = wl.systematic(wl.make_code(2000, 1000, 3, 64, seed=0xC0DE0040))
    fr = wl.make_frames(code, enc, 4096, 0xDA7A0040, "biawgn", wl.sigma_from_ebn0(1.6, code.n_info / code.n))
    dcode = gfbp.DeviceCode(code)
    d = gfbp.frames_to_device(fr)
    res = {"workload": "GF(64) regular (3,6) rate-1/2 LDPC, N=2000 symbols, BI-AWGN 1.6 dB, 4096 frames, "
                       "max 100 iterations", "edges": code.E, "q": 64}
    for s in ("pus", "sus"):
        if shapes and s in shapes:
            dcode.set_shape(s, shapes[s])
            res[f"{s}_entries_per_lane"] = dcode.shape(s)
        else:
            res[f"{s}_entries_per_lane"] = gfbp.tune(dcode, d, schedule=s, trial_iters=3)
        gfbp.decode_batch(dcode, d, schedule=s, max_iter=100)
        torch.cuda.synchronize()
        gfbp.profile_reset()
        gfbp.profile_enable(True)
        t0 = time.perf_counter()
        its = []
        for _ in range(steps):
            o = gfbp.decode_batch(dcode, d, schedule=s, max_iter=100)
            its.append(o["iters"].cpu().numpy())
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        gfbp.profile_enable(False)
        prof = gfbp.profile_read()
        it = np.concatenate(its)
        res[f"{s}_edge_q_per_s"] = float(it.sum()) * code.E * code.q / wall
        res[f"{s}_frames_per_s"] = len(it) / wall
        res[f"{s}_mean_iters"] = float(it.mean())
        ks = {k: v for k, v in prof.items() if k in ("check", "variable", "sus_level")}
        dom = max(ks, key=lambda k: ks[k]["total_ms"])
        ach = ks[dom]["algo_bytes"] / (ks[dom]["total_ms"] / 1e3)
        algo = ks[dom]["algo_bytes"] / ks[dom]["launches"]
        res[f"{s}_roofline"] = {"kernel": dom, "achieved_GBps": ach / 1e9, "frac": ach / HBM_PEAK,
                                "avg_launch_ms": ks[dom]["total_ms"] / ks[dom]["launches"],
                                "algo_bytes_per_launch": algo, "traffic": None}
        if traffic_path:
            from paper_cs_0605069_amd.profiling import read_traffic

            tr = read_traffic(traffic_path)
            el = res[f"{s}_entries_per_lane"]
            if tr and dom in tr["kernels"] and int(tr["shapes"].get(s, -1)) == el:
                res[f"{s}_roofline"]["traffic"] = tr["kernels"][dom]["bytes_per_dispatch"]
                res[f"{s}_roofline"]["traffic_over_algorithmic"] = tr["kernels"][dom]["bytes_per_dispatch"] / algo
        # the same kernel with every frame running (fixed iterations, no early stop): its
        # bandwidth at full occupancy, without the convergence tail's small launches
        gfbp.profile_reset()
        gfbp.profile_enable(True)
        gfbp.decode_batch(dcode, d, schedule=s, max_iter=4, early_stop=False)
        torch.cuda.synchronize()
        gfbp.profile_enable(False)
        full = gfbp.profile_read()[dom]
        fa = full["algo_bytes"] / (full["total_ms"] / 1e3)
        res[f"{s}_roofline"]["all_frames_active"] = {"iterations": 4, "achieved_GBps": fa / 1e9, "frac": fa / HBM_PEAK,
                                                     "avg_launch_ms": full["total_ms"] / full["launches"]}
    return res


def configs_workloads():
    """The two other fixed workloads: (label, code, frames, decode keywords)."""
    from paper_cs_0605069_amd import workloads as wl

    out = []
    code, enc = wl.regular_code(504, 3, 6, 4, seed=0xC0DE0001)
    out.append(("gf4_n504_bsc", code, wl.make_frames(code, enc, 2000, 0xDA7A0001, "bsc", 0.06), {"max_iter": 200}))
    code, enc = wl.regular_code(3000, 3, 6, 8, seed=0xC0DE0003)
    M = wl.self_transition_matrix(8, 0.7)
    kw = {"max_iter": 100, "prior": "markov", "markov_M": M, "markov_pi": wl.stationary(M)}
    for ch, par in (("bsc", 0.08), ("bec", 0.45)):
        fr = wl.make_frames(code, enc, 4096, 0xDA7A0003 + (ch == "bec"), ch, par, source="markov", markov=M)
        out.append((f"gf8_n3000_markov_{ch}", code, fr, kw))
    return out


LDS_PEAK = 256 * 128 * 2.4e9   # MI355X: 256 CUs x 128 bytes per clock x 2.4 GHz
FP64_PEAK = 78.6e12            # MI355X fp64 vector


def onchip_counts(code) -> tuple[float, float]:
    """Algorithmic LDS bytes and float64 operations of one frame-iteration of
    the in-LDS decode: each edge reads its row's other q-vectors and writes
    its r (check side); each column reads its r-vectors and prior and writes
    its q-vectors (variable side); transforms cost q log2 q additions, every
    product and normalisation q operations."""
    q, p = code.q, int(np.log2(code.q))
    dc = np.diff(code.row_ptr).astype(float)
    dv = np.bincount(code.col, minlength=code.n).astype(float)
    lds = 4.0 * q * (float((dc * (dc - 1)).sum()) + 3.0 * code.E + code.n)
    flops = float((dc * ((dc - 1) * (q * p + q) + q * p + q)).sum()) + \
        float((q * dv + 2 * q + dv * ((dv - 1) * q + 2 * q)).sum())
    return lds, flops


def configs_leg(gfbp, torch, calls: int = 2) -> tuple[dict, list]:
    """GF(4) (3,6) N=504 over BSC 0.06 (2000 frames, max 200 iterations) and
    GF(8) (3,6) N=3000 with a Markov source (self-transition 0.7) over BSC 0.08
    and BEC 0.45 (4096 frames each, max 100), every frame of a workload in one
    launch, the kernel shape tuned per schedule: edge-q/s, frames/s, mean
    iterations and FER per schedule over `calls` timed calls, each kernel's
    algorithmic GB/s (the Markov prior kernel among them) and the SUS/PUS
    iteration ratios (not part of `value`).  Also returns, per workload, the
    decoded iterations and convergence for the reference decoder's sample."""
    out, samples = {}, []
    for label, code, fr, kw in configs_workloads():
        dcode = gfbp.DeviceCode(code)
        d = gfbp.frames_to_device(fr)
        res = {"workload": f"GF({code.q}) (3,6) N={code.n}, {fr.channel.upper()} {float(fr.param[0])}"
                           + (", Markov source (self-transition 0.7)" if "prior" in kw else ", i.i.d. source")
                           + f", {fr.F} frames in one launch, max {kw['max_iter']} iterations",
               "edges": code.E, "q": code.q}
        got = {}
        for s in ("pus", "sus"):
            res[s] = {"entries_per_lane": gfbp.tune(dcode, d, schedule=s, trial_iters=3, **{k: v for k, v in kw.items()
                                                                                          if k != "max_iter"})}
            gfbp.decode_batch(dcode, d, schedule=s, **kw)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(calls):
                o = gfbp.decode_batch(dcode, d, schedule=s, **kw)
                it, cv = o["iters"].cpu().numpy(), o["converged"].cpu().numpy()
            torch.cuda.synchronize()
            wall = time.perf_counter() - t0
            # the kernels of one more call, timed one by one (events around
            # each launch: outside the timed calls above)
            gfbp.profile_reset()
            gfbp.profile_enable(True)
            gfbp.decode_batch(dcode, d, schedule=s, **kw)
            torch.cuda.synchronize()
            gfbp.profile_enable(False)
            prof = gfbp.profile_read()
            res[s].update({"edge_q_per_s": calls * float(it.sum()) * code.E * code.q / wall,
                           "frames_per_s": calls * fr.F / wall, "mean_iters": float(it.mean()),
                           "fer": float(1 - cv.mean()),
                           "kernels": {k: {"launches": v["launches"], "avg_us": v["total_ms"] / v["launches"] * 1e3,
                                           "GBps_algorithmic": v["algo_bytes"] / (v["total_ms"] / 1e3) / 1e9,
                                           "frac_of_hbm_peak": v["algo_bytes"] / (v["total_ms"] / 1e3) / HBM_PEAK}
                                       for k, v in prof.items() if v["launches"] and v["total_ms"]}})
            got[s] = (it, cv)
            if "onchip" in prof:
                # the whole decode in LDS: what bounds it is latency (the frames
                # that run to max_iter), not HBM; its LDS and fp64 rates, also
                # with every frame running a fixed 20 iterations
                lds_b, flops = onchip_counts(code)
                k = prof["onchip"]
                fi = float(it.sum())
                sec = k["total_ms"] / 1e3
                full = {}
                gfbp.profile_reset()
                gfbp.profile_enable(True)
                gfbp.decode_batch(dcode, d, schedule=s, **{**kw, "max_iter": 20, "early_stop": False})
                torch.cuda.synchronize()
                gfbp.profile_enable(False)
                k2 = gfbp.profile_read()["onchip"]
                sec2 = k2["total_ms"] / 1e3
                full = {"frame_iterations": 20 * fr.F, "kernel_ms": k2["total_ms"],
                        "lds_GBps": 20 * fr.F * lds_b / sec2 / 1e9, "lds_frac": 20 * fr.F * lds_b / sec2 / LDS_PEAK,
                        "fp64_TFLOPs": 20 * fr.F * flops / sec2 / 1e12,
                        "fp64_frac": 20 * fr.F * flops / sec2 / FP64_PEAK}
                res[s]["onchip"] = {"bound": "latency", "kernel_ms": k["total_ms"], "frame_iterations": fi,
                                    "lds_bytes_per_frame_iteration": lds_b, "fp64_ops_per_frame_iteration": flops,
                                    "lds_GBps": fi * lds_b / sec / 1e9, "lds_frac": fi * lds_b / sec / LDS_PEAK,
                                    "fp64_TFLOPs": fi * flops / sec / 1e12, "fp64_frac": fi * flops / sec / FP64_PEAK,
                                    "lds_peak_GBps": LDS_PEAK / 1e9, "fp64_peak_TFLOPs": FP64_PEAK / 1e12,
                                    "every_frame_running": full}
        pi, si = got["pus"][0].astype(float), got["sus"][0].astype(float)
        res["sus_over_pus"] = {"ratio_of_means": si.mean() / pi.mean(), "mean_of_ratios": float(np.mean(si / pi)),
                               "stdev_of_ratios": float(np.std(si / pi))}
        out[label] = res
        samples.append((label, code, fr, kw, got))
        del dcode, d
        print(f"# configs leg {label} done", file=sys.stderr, flush=True)
    return out, samples


def cpu_baseline_configs(samples, frames: int = 256) -> dict:
    """Reference decoder on every k-th frame (`frames` of each workload of the
    configs leg), both schedules: its edge-q/s and frames/s, and both sides'
    mean iterations and FER on those frames."""
    import oracle

    out = {}
    for label, code, fr, kw, got in samples:
        stride = max(1, fr.F // frames)
        idx = np.arange(0, fr.F, stride)[:frames]
        sub = fr.subset(idx)
        okw = {k: v for k, v in kw.items() if k in ("prior", "markov_M", "markov_pi", "max_iter")}
        r = {"frames": int(len(idx)), "stride": int(stride), "cores": oracle.max_threads()}
        eq, t0 = 0.0, time.perf_counter()
        for name, sch in (("pus", oracle.PUS), ("sus", oracle.SUS)):
            o = oracle.decode(code, sub, schedule=sch, **okw)
            eq += float(o["iters"].sum()) * code.E * code.q
            g_it, g_cv = got[name][0][idx], got[name][1][idx]
            r[name] = {"mean_iters_reference": float(o["iters"].mean()), "mean_iters_gpu": float(g_it.mean()),
                       "fer_reference": float(1 - o["converged"].mean()), "fer_gpu": float(1 - g_cv.mean()),
                       "same_iterations": int((g_it == o["iters"]).sum())}
        dt = time.perf_counter() - t0
        r.update({"edge_q_per_s": eq / dt, "frames_per_s": 2 * len(idx) / dt, "seconds": dt})
        out[label] = r
    return out


def uneven_leg(gfbp, torch) -> dict:
    """The uneven batch: 10,000 frames over 64 codes of the mixed pool (q in
    {4, 16, 64}, n 256-8000, BSC / BEC / BI-AWGN per frame at Eb/N0 ~ U[1, 2]
    dB), each code's kernel shape tuned on its frames, then the whole batch in
    one gfbp_decode_batch call per schedule (code by code, the codes
    concurrent), max 100 iterations; best of two timed calls, and each
    kernel's algorithmic rate from one more, profiled call; then the same call
    on the persistent work-list kernels in one launch, their tile shape tuned
    first (none of it part of `value`)."""
    from paper_cs_0605069_amd.batching import batch_inputs

    pool, items, flat, flat_codes, index = batch_inputs(10000, 64, 8000)
    dcodes = [gfbp.DeviceCode(c) for c in pool]
    dfr = gfbp.ragged_frames(flat, flat_codes)
    eq_frame = np.array([c.E * c.q for c in pool], dtype=np.float64)
    out = {"workload": "10,000 frames over 64 codes (q in {4, 16, 64}, n 256-8000, rate 1/3-1/2, column weight "
                       "2-3), BSC/BEC/BI-AWGN per frame at Eb/N0 ~ U[1, 2] dB, syndromes z != 0, max 100 "
                       "iterations, one call per schedule",
           "frames": int(len(index)), "codes": len(items)}
    for s in ("sus", "pus"):
        for ci, code, groups in items:
            gfbp.tune(dcodes[ci], gfbp.frames_to_device(groups[-1]), schedule=s, trial_iters=2)
        gfbp.decode_multi(dcodes, index, dfr, schedule=s, max_iter=2)
        torch.cuda.synchronize()
        best, its = None, None
        for _ in range(2):
            t0 = time.perf_counter()
            o = gfbp.decode_multi(dcodes, index, dfr, schedule=s, max_iter=100)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            if best is None or dt < best:
                best, its = dt, o["iters"].cpu().numpy()
        out[s] = {"seconds": best, "frames_per_s": len(index) / best,
                  "edge_q_per_s": float((its * eq_frame[index]).sum()) / best, "mean_iters": float(its.mean())}
        # the same call on the persistent work-list kernels (one HIP graph
        # launch, one kernel per field), their tile shape tuned first
        t = gfbp.decode_multi(dcodes, index, dfr, schedule=s, max_iter=100, tune_iters=2)
        el, waves = t["persist_el"], t["persist_waves"]
        gfbp.decode_multi(dcodes, index, dfr, schedule=s, max_iter=2, persistent=True, persist_el=el,
                          persist_waves=waves)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        o = gfbp.decode_multi(dcodes, index, dfr, schedule=s, max_iter=100, persistent=True, persist_el=el,
                              persist_waves=waves)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        pits = o["iters"].cpu().numpy()
        out[s]["persistent_one_launch"] = {
            "seconds": dt, "frames_per_s": len(index) / dt,
            "edge_q_per_s": float((pits * eq_frame[index]).sum()) / dt, "mean_iters": float(pits.mean()),
            "entries_per_lane": el, "wavefronts_per_workgroup": waves,
            "frames_with_other_iteration_count": int((pits != its).sum())}
        # the kernels of one more call, each launch timed by the library (HIP
        # events on the decode streams; the codes' kernels overlap, so these
        # are per-kernel rates, not shares of the wall time above)
        gfbp.profile_reset()
        gfbp.profile_enable(True)
        gfbp.decode_multi(dcodes, index, dfr, schedule=s, max_iter=100)
        torch.cuda.synchronize()
        gfbp.profile_enable(False)
        prof = gfbp.profile_read()
        out[s]["kernels"] = {k: {"launches": v["launches"], "avg_us": v["total_ms"] / v["launches"] * 1e3,
                                 "GBps_algorithmic": v["algo_bytes"] / (v["total_ms"] / 1e3) / 1e9}
                             for k, v in prof.items() if v["launches"] and v["total_ms"]}
        print(f"# uneven batch {s}: {best:.3f} s", file=sys.stderr, flush=True)
    return out


def mn_leg(samples: int = 3000) -> dict:
    """The paper's setting on a stand-in code whose sweep is not serial: Table
    1's row 9 (BI-AWGN, GF(8), the 2-state Markov source lifted to symbols,
    rate-1/3 syndrome-form code with 10^4 source bits and a pooled B) at 0.85
    of the paper's sigma, `samples` frames in one launch per schedule, max 300
    iterations: mean iterations of both schedules, their ratios (the Table 1
    quantities) and the GPU time of each schedule (not part of `value`)."""
    from paper_cs_0605069_amd import table1

    channel, q, source, param = table1.SETTINGS[8]
    r = table1.run_setting(channel, q, source, param, samples, samples, 300, seed=0xC0DE0100 + 9, scale=0.85,
                           b_form="pool")
    keep = ("noise", "N", "M", "E", "samples", "sus_levels", "t_pus", "t_sus", "ratio_of_means", "mean_of_ratios",
            "stdev_of_ratios", "fer_pus", "fer_sus", "ber_pus", "ber_sus", "seconds_pus", "seconds_sus",
            "edge_q_per_s_pus", "edge_q_per_s_sus")
    out = {"workload": "Table 1 row 9 stand-in: BI-AWGN, GF(8), 2-state Markov source, rate-1/3 MN code with "
                       "10^4 source bits and a pooled B, sigma = 0.85 x 1.66, max 300 iterations"}
    out.update({k: r[k] for k in keep if k in r})
    out["sus_over_pus_gpu_time"] = r["seconds_sus"] / r["seconds_pus"]
    return out


def serving_leg(gfbp, torch, seconds: float, rate: float, schedules=("sus", "pus")) -> tuple[dict, dict]:
    """Continuous batching of the mixed-code stream: Poisson arrivals at `rate`
    frames/s for `seconds`, frames from 16 codes of the uneven pool (q in
    {4, 16, 64} with GF(64) weighted 30%, n up to 8000, BSC / BEC / BI-AWGN at
    Eb/N0 ~ U[1, 2] dB, half with the Markov source), admitted into resident
    slots as they arrive, converged frames retired at once; per schedule the
    sustained throughput and p50/p99 frame latency (arrival to result on the
    host, and admission to retirement on the device clock; throughput both over
    the whole run and over the arrival window after its first second).  Also
    returns, per schedule, the served sample that the CPU baseline leg checks
    with the reference decoder (the first frame of each request group of the
    codes of n <= 2500)."""
    from paper_cs_0605069_amd import serving
    from paper_cs_0605069_amd import workloads as wl

    pool = wl.mixed_pool(16, seed=0xC0DE0005, n_range=(256, 8000), q_weights=[0.35, 0.35, 0.3])
    samples = {}
    out = {"workload": f"Poisson arrivals at {rate:.0f} frames/s for {seconds:.0f} s over 16 codes "
                       "(q in {4, 16, 64}, GF(64) 30%, n 256-8000, BSC/BEC/BI-AWGN at 1-2 dB, half Markov), "
                       "max 100 iterations"}
    for sch in schedules:
        n = int(rate * seconds)
        queues, markov = serving.make_requests(pool, n, rate, seed=0xDA7A0005, pool_max=512)
        # the reference sample: the first frame of every group of the codes of n <= 2500 (bounded run time)
        small = [cq for cq in queues if cq.code.n <= 2500]
        keep = [int(cq.ids[pos[0]]) for cq in small for g, m, pos in cq.groups]
        srv = serving.Server(queues, 1024, sch, 100, 200 << 30, step_iters=2, markov=markov, keep_ids=keep)
        st = srv.run(deadline=seconds + 15.0)
        lat = np.array(st.latency) * 1e3
        dlat = np.array(st.device_latency) * 1e3
        at = np.array(st.answer_time)
        res = {"offered_per_s": rate, "offered": st.offered, "answered": st.done, "wall_s": st.wall,
               "throughput_frames_per_s": st.done / st.wall,
               "steady_throughput_frames_per_s": float(((at >= 1.0) & (at <= seconds)).sum() / (seconds - 1.0)),
               "arrival_window_s": seconds,
               "frame_latency_ms_p50": float(np.percentile(lat, 50)), "frame_latency_ms_p99": float(np.percentile(lat, 99)),
               "device_latency_ms_p50": float(np.percentile(dlat, 50)),
               "device_latency_ms_p99": float(np.percentile(dlat, 99)),
               "mean_iters": float(np.mean(st.iters)), "fer": 1 - st.converged / max(1, st.done),
               "edge_q_per_s": st.edge_q / st.wall}
        # the served frames the CPU baseline leg decodes with the reference decoder
        samples[sch] = [(cq.code, markov[cq.code.q], g, m, st.results.get(int(cq.ids[pos[0]])))
                        for cq in small for g, m, pos in cq.groups]
        out[sch] = res
        print(f"# serving {sch}: {res['throughput_frames_per_s']:.0f} frames/s, p99 {res['frame_latency_ms_p99']:.0f} ms",
              file=sys.stderr, flush=True)
        del queues, srv
        torch.cuda.empty_cache()
    return out, samples


def cpu_baseline_serving(samples: dict) -> dict:
    """Part of the CPU baseline leg: the reference decoder on the served sample
    (the first frame of every request group of the serving leg's codes of
    n <= 2500): agreement with the served answers and the reference's rate."""
    import oracle

    res = {}
    for sch, items in samples.items():
        same = tot = 0
        t0 = time.perf_counter()
        sch_o = {"pus": oracle.PUS, "sus": oracle.SUS}[sch]
        for code, (M, pi), g, m, got in items:
            if got is None:
                continue
            kw = dict(prior="markov", markov_M=M, markov_pi=pi) if m else {}
            r = oracle.decode(code, g.subset([0]), schedule=sch_o, max_iter=100, **kw)
            it, cv, xh = got
            same += int(it == r["iters"][0] and np.array_equal(xh, r["xhat"][0]))
            tot += 1
        dt = time.perf_counter() - t0
        res[sch] = {"frames": tot, "identical": same, "seconds": dt, "frames_per_s": tot / dt if dt else None,
                    "threads": oracle.max_threads()}
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--cpu-frames", type=int, default=500)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--schedules", default="pus,sus")
    ap.add_argument("--no-tune", action="store_true", help="keep the default kernel shape instead of autotuning")
    ap.add_argument("--shapes", default="", help="fix entries per lane instead of autotuning, e.g. pus=8,sus=4")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MiB",
                    help="after the timed steps, copy this many MiB device-to-device (counter calibration)")
    ap.add_argument("--no-gf64", action="store_true", help="skip the GF(64) leg")
    ap.add_argument("--traffic", default=os.path.join(ROOT, "profiles", "traffic_gf16_n2000_bi-awgn.txt"),
                    help="measured HBM traffic summary to report beside the roofline")
    ap.add_argument("--traffic-gf64", default=os.path.join(ROOT, "profiles", "traffic_gf64_n2000_bi-awgn.txt"),
                    help="the same for the GF(64) leg")
    ap.add_argument("--leg", default="", choices=["", "gf64", "serving", "mn", "uneven", "configs"],
                    help="run only this leg and print its JSON (profiling)")
    ap.add_argument("--serving-seconds", type=float, default=6.0)
    ap.add_argument("--serving-rate", type=float, default=20000.0)
    ap.add_argument("--no-serving", action="store_true")
    ap.add_argument("--no-mn", action="store_true", help="skip the Table-1 stand-in leg (SUS and PUS on an MN code)")
    ap.add_argument("--no-uneven", action="store_true", help="skip the uneven-batch leg (64 codes in one call)")
    ap.add_argument("--no-configs", action="store_true",
                    help="skip the GF(4) N=504 and GF(8) N=3000 Markov workloads")
    ap.add_argument("--no-copy-rate", action="store_true", help="skip measuring the achievable streaming-copy bandwidth")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: frames are independent and this decoder has no multi-GPU path "
              "(run it with --gpus 1).", file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_cs_0605069_amd as gfbp

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    fixed = {}
    if args.shapes:
        for kv in args.shapes.split(","):
            k, v = kv.split("=")
            fixed[k] = int(v)
    if args.leg == "gf64":
        res = gf64_leg(gfbp, torch, max(1, args.steps), args.traffic_gf64, fixed)
        if args.copy_probe:
            a = torch.empty(args.copy_probe << 20, dtype=torch.uint8, device="cuda")
            torch.empty_like(a).copy_(a)
            torch.cuda.synchronize()
        print(json.dumps(res), flush=True)
        return
    if args.leg == "serving":
        print(json.dumps(serving_leg(gfbp, torch, args.serving_seconds, args.serving_rate)[0]), flush=True)
        return
    if args.leg == "mn":
        print(json.dumps(mn_leg()), flush=True)
        return
    if args.leg == "uneven":
        print(json.dumps(uneven_leg(gfbp, torch)), flush=True)
        return
    if args.leg == "configs":
        print(json.dumps(configs_leg(gfbp, torch)[0]), flush=True)
        return
    code, points = make_workload()
    dcode = gfbp.DeviceCode(code)
    scheds = [s for s in args.schedules.split(",") if s]
    dev_points = [(eb, gfbp.frames_to_device(fr)) for eb, fr in points]
    ws = {s: torch.empty(dcode.workspace_size(FRAMES, s), dtype=torch.uint8, device="cuda") for s in scheds}
    outs = {s: {"xhat": torch.empty((FRAMES, code.n), dtype=torch.uint8, device="cuda"),
                "iters": torch.empty(FRAMES, dtype=torch.int32, device="cuda"),
                "converged": torch.empty(FRAMES, dtype=torch.uint8, device="cuda"),
                "guards": torch.empty(FRAMES, dtype=torch.int32, device="cuda")} for s in scheds}
    shapes = {}
    if args.shapes:
        for kv in args.shapes.split(","):
            k, v = kv.split("=")
            dcode.set_shape(k, int(v))
        shapes = {s: dcode.shape(s) for s in scheds}
    elif not args.no_tune:
        eb, d = dev_points[len(dev_points) // 2]
        for s in scheds:
            shapes[s] = gfbp.tune(dcode, d, schedule=s, trial_iters=3, workspace=ws[s], outputs=outs[s])
    else:
        shapes = {s: dcode.shape(s) for s in scheds}
    torch.cuda.synchronize()

    def step(record):
        for eb, d in dev_points:
            for s in scheds:
                t0 = time.perf_counter()
                o = gfbp.decode_batch(dcode, d, schedule=s, max_iter=MAX_ITER, workspace=ws[s], outputs=outs[s])
                torch.cuda.synchronize()
                dt = time.perf_counter() - t0
                if record is not None:
                    it = o["iters"].cpu().numpy()
                    cv = o["converged"].cpu().numpy()
                    record.append({"sched": s, "ebn0": eb, "ms": dt * 1e3, "iters": it, "conv": cv,
                                   "fer": 1.0 - float(cv.mean())})

    for _ in range(args.warmup):
        step(None)
    gfbp.profile_reset()
    gfbp.profile_enable(True)
    rec = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        step(rec)
        print(f"# step {k + 1}/{args.steps} done", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    gfbp.profile_enable(False)
    prof = gfbp.profile_read()
    if args.copy_probe:
        a = torch.empty(args.copy_probe << 20, dtype=torch.uint8, device="cuda")
        torch.empty_like(a).copy_(a)
        torch.cuda.synchronize()

    EQ = code.E * code.q
    total_eq = sum(float(r["iters"].sum()) * EQ for r in rec)
    per = {}
    for s in scheds:
        rs = [r for r in rec if r["sched"] == s]
        ms = np.array([r["ms"] for r in rs])
        eq = sum(float(r["iters"].sum()) * EQ for r in rs)
        per[s] = {"edge_q_per_s": eq / (ms.sum() / 1e3), "frames_per_s": len(rs) * FRAMES / (ms.sum() / 1e3),
                  "mean_iters": float(np.mean([r["iters"].mean() for r in rs])),
                  "decode_call_ms_p50": float(np.percentile(ms, 50)), "decode_call_ms_p99": float(np.percentile(ms, 99)),
                  "fer_by_ebn0": {str(r["ebn0"]): round(r["fer"], 4) for r in rs[:len(EBN0)]},
                  "mean_iters_by_ebn0": {str(r["ebn0"]): round(float(r["iters"].mean()), 3) for r in rs[:len(EBN0)]},
                  "decode_call_ms_by_ebn0": {str(eb): round(float(np.mean([r["ms"] for r in rs if r["ebn0"] == eb])), 3)
                                             for eb in EBN0}}
    if "pus" in per and "sus" in per:
        pi = np.concatenate([r["iters"] for r in rec if r["sched"] == "pus"]).astype(float)
        si = np.concatenate([r["iters"] for r in rec if r["sched"] == "sus"]).astype(float)
        per["sus_over_pus"] = {"ratio_of_means": si.mean() / pi.mean(), "mean_of_ratios": float(np.mean(si / pi)),
                               "stdev_of_ratios": float(np.std(si / pi))}

    iter_kernels = {k: v for k, v in prof.items() if k in ("check", "variable", "sequential", "sus_level")}
    dom = max(iter_kernels, key=lambda k: iter_kernels[k]["total_ms"]) if iter_kernels else None
    roof = None
    if dom:
        d = prof[dom]
        ach = d["algo_bytes"] / (d["total_ms"] / 1e3)
        algo = d["algo_bytes"] / d["launches"]
        roof = {"bound": "hbm", "kernel": dom, "achieved": ach / 1e9, "peak": HBM_PEAK / 1e9, "unit": "GB/s",
                "frac": ach / HBM_PEAK, "traffic": None,
                "avg_launch_ms": d["total_ms"] / d["launches"], "launches": d["launches"],
                "algo_bytes_per_launch": algo}
        from paper_cs_0605069_amd.profiling import read_traffic

        tr = read_traffic(args.traffic)
        dsch = "pus" if dom in ("check", "variable") else "sus"  # the schedule whose kernel shape it is
        if tr and dom in tr["kernels"] and dsch in shapes and int(tr["shapes"].get(dsch, -1)) == shapes[dsch]:
            roof["traffic"] = tr["kernels"][dom]["bytes_per_dispatch"]
            roof["traffic_unit"] = "HBM bytes per launch (FETCH_SIZE + WRITE_SIZE, copy-calibrated)"
            roof["traffic_over_algorithmic"] = roof["traffic"] / algo
        if not args.no_copy_rate:
            # what a plain streaming kernel reaches on this device (2 GiB copy,
            # after the timed steps), beside the nominal peak
            src = torch.empty(1 << 31, dtype=torch.uint8, device="cuda")
            dst = torch.empty_like(src)
            cr = gfbp.stream_copy_rate(dst, src, reps=5)
            del src, dst
            roof["achievable_copy"] = cr / 1e9
            roof["frac_of_achievable_copy"] = ach / cr
    kernels = {k: {"launches": v["launches"], "avg_ms": v["total_ms"] / v["launches"],
                   "share_of_gpu_time": v["total_ms"] / max(1e-9, sum(x["total_ms"] for x in prof.values())),
                   "GBps_algorithmic": (v["algo_bytes"] / (v["total_ms"] / 1e3) / 1e9) if v["total_ms"] else 0.0,
                   "frac_of_hbm_peak": (v["algo_bytes"] / (v["total_ms"] / 1e3) / HBM_PEAK) if v["total_ms"] else 0.0}
               for k, v in prof.items()}

    gf64 = None if args.no_gf64 else gf64_leg(gfbp, torch, max(1, args.steps), args.traffic_gf64)
    srv, srv_samples = (None, None) if args.no_serving else serving_leg(gfbp, torch, args.serving_seconds,
                                                                         args.serving_rate)
    mn = None if args.no_mn else mn_leg()
    uneven = None if args.no_uneven else uneven_leg(gfbp, torch)
    cfgs, cfg_samples = (None, None) if args.no_configs else configs_leg(gfbp, torch)
    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(code, points, args.cpu_frames, rec)
        if cfg_samples:
            cpu["configs_sample"] = cpu_baseline_configs(cfg_samples)
        if srv_samples:
            cpu["serving_sample"] = cpu_baseline_serving(srv_samples)
            for sch, r in cpu["serving_sample"].items():
                srv[sch]["reference_sample"] = r

    line = {
        "metric": "edge·q message updates/s (PUS and SUS)",
        "value": total_eq / wall,
        "unit": "edge·q updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": wall / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "message_storage": "f32",
        "data": "synthetic",
        "config": {"workload": f"GF({Q}) regular ({DV},{DC}) rate-1/2 LDPC, N={N_SYM} symbols, BI-AWGN "
                               f"Eb/N0 {EBN0[0]}-{EBN0[-1]} dB step 0.2, {FRAMES} frames per point, max {MAX_ITER} "
                               f"iterations, {'+'.join(s.upper() for s in scheds)}",
                   "edges": code.E, "q": code.q, "frames_per_step": FRAMES * len(EBN0) * len(scheds),
                   "entries_per_lane": shapes},
        "frames_per_s": len(rec) * FRAMES / wall,
        "schedules": per,
        "roofline": roof,
        "kernels": kernels,
        "cpu_baseline": cpu,
        "gf64": gf64,
        "serving": srv,
        "mn_table1_row9": mn,
        "uneven_batch": uneven,
        "configs": cfgs,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
