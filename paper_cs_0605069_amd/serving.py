"""Serving: continuous batching of decode requests over several codes.

A :class:`Server` keeps one session (resident frame slots, see
``gfbp_session_*``) per code, created on first use if the device-memory budget
allows.  Requests (frames with their arrival times) are admitted into free
slots as they arrive; each round of the serving loop advances every session
by a few iterations on its own stream (so sessions' kernels overlap on the
device), then collects finished frames and records their latency (arrival to
collection).  Converged frames leave early; slots are reused at once.

``python -m paper_cs_0605069_amd.serving`` runs a Poisson arrival stream over
a mixed pool of codes and prints throughput and p50/p99 latency per rate.
"""
from __future__ import annotations

import argparse
import json
import sys
import time
from dataclasses import dataclass, field

import numpy as np

from . import DeviceCode, Session, frames_for_session, frames_to_device, tune
from . import workloads as wl


@dataclass
class CodeQueue:
    """Frames of one code, resident on the device, offered in arrival order."""

    code: wl.Code
    frames: dict  # device tensors from frames_for_session (+ markov, syndrome)
    arrival: np.ndarray  # seconds, nondecreasing
    ids: np.ndarray  # global request ids
    next_arrived: int = 0
    next_admitted: int = 0
    dcode: DeviceCode | None = None
    session: Session | None = None
    stream: object = None


@dataclass
class Stats:
    latency: list = field(default_factory=list)
    iters: list = field(default_factory=list)
    converged: int = 0
    done: int = 0
    results: dict = field(default_factory=dict)


class Server:
    def __init__(self, queues: list[CodeQueue], slots: int, schedule: str, max_iter: int, budget_bytes: int,
                 step_iters: int = 2, markov: dict | None = None, keep_results: bool = False, autotune: bool = True):
        self.queues = queues
        self.slots = slots
        self.schedule = schedule
        self.max_iter = max_iter
        self.budget = budget_bytes
        self.used = 0
        self.step_iters = step_iters
        self.markov = markov or {}
        self.keep = keep_results
        self.autotune = autotune
        self.refused = 0
        self.opened = 0

    def prepare(self):
        """Upload every code and (if asked) autotune its kernel shape on a few
        of its own frames, before the clock starts."""
        for cq in self.queues:
            if cq.dcode is None:
                cq.dcode = DeviceCode(cq.code)
            if self.autotune and getattr(cq, "groups", None):
                g = max(cq.groups, key=lambda x: x[0].F)[0]
                tune(cq.dcode, frames_to_device(g.subset(np.arange(min(g.F, 64)))), schedule=self.schedule,
                     trial_iters=2)

    def _open(self, cq: CodeQueue) -> bool:
        import torch

        if cq.session is not None:
            return True
        if cq.dcode is None:
            cq.dcode = DeviceCode(cq.code)
        M, pi = self.markov.get(cq.code.q, (None, None))
        need = Session.bytes_needed(cq.dcode, self.slots, self.schedule, markov=M is not None, has_syndrome=True)
        if self.used + need > self.budget:
            self.refused += 1
            return False
        cq.session = Session(cq.dcode, self.slots, self.schedule, self.max_iter, has_syndrome=True,
                             markov_M=M, markov_pi=pi)
        cq.stream = torch.cuda.Stream()
        cq.need = need
        self.used += need
        self.opened += 1
        return True

    def _close(self, cq: CodeQueue):
        cq.stream.synchronize()
        cq.session.close()
        cq.session = None
        self.used -= cq.need

    def run(self, duration: float | None = None, stats: Stats | None = None) -> Stats:
        """Serve every request (or until `duration` seconds); returns statistics."""
        import torch

        self.prepare()
        torch.cuda.synchronize()
        st = stats or Stats()
        total = sum(len(cq.arrival) for cq in self.queues)
        t0 = time.perf_counter()
        while st.done < total:
            now = time.perf_counter() - t0
            if duration is not None and now > duration:
                break
            for cq in self.queues:
                cq.next_arrived = int(np.searchsorted(cq.arrival, now, side="right"))
                if cq.next_admitted < cq.next_arrived and self._open(cq):
                    lo, hi = cq.next_admitted, cq.next_arrived
                    sl = {k: (v[lo:hi] if hasattr(v, "shape") and v is not None else v) for k, v in cq.frames.items()}
                    with torch.cuda.stream(cq.stream):
                        cq.next_admitted += cq.session.admit(cq.ids[lo:hi], sl, stream=cq.stream)
            busy = [cq for cq in self.queues if cq.session is not None and cq.session.running > 0]
            for cq in busy:
                cq.session.step(self.step_iters, stream=cq.stream)
            for cq in busy:
                ids, it, cv, xh = cq.session.poll(want_xhat=self.keep, stream=cq.stream)
                t = time.perf_counter() - t0
                for r in range(len(ids)):
                    gid = int(ids[r])
                    k = int(np.searchsorted(cq.ids, gid))
                    st.latency.append(t - cq.arrival[k])
                    st.iters.append(int(it[r]))
                    st.converged += int(cv[r])
                    if self.keep:
                        st.results[gid] = (int(it[r]), int(cv[r]), xh[r].copy())
                st.done += len(ids)
            for cq in self.queues:
                # a session whose requests have all been answered gives its memory back
                if cq.session is not None and cq.session.running == 0 and cq.next_admitted == len(cq.arrival):
                    self._close(cq)
            if not busy:
                if not any(cq.session is not None for cq in self.queues) and any(
                        cq.next_admitted < cq.next_arrived for cq in self.queues):
                    raise RuntimeError("device-memory budget too small for any session")
                time.sleep(0.0002)
        st.wall = time.perf_counter() - t0
        return st


def poisson_times(n: int, rate: float, seed: int) -> np.ndarray:
    rng = np.random.default_rng([seed, 9])
    return np.cumsum(rng.exponential(1.0 / rate, size=n))


def make_requests(pool: list[wl.Code], n_frames: int, rate: float, seed: int, markov_share: float = 0.5,
                  stay: float = 0.7):
    """Poisson stream over the pool: each request picks a code uniformly, a
    channel (BSC, BEC, BI-AWGN) uniformly, Eb/N0 ~ U[1, 2] dB (channel
    parameter matched to that Eb/N0 at the code's rate) and, with probability
    `markov_share`, a Markov source (self-transition `stay`) on its
    information symbols.  Returns (queues, markov) where markov maps q to
    (M, pi); each queue also keeps its host frame groups as
    ``groups = [(Frames, is_markov, global ids)]``."""
    import torch

    rng = np.random.default_rng([seed, 10])
    t = poisson_times(n_frames, rate, seed)
    which = rng.integers(0, len(pool), size=n_frames)
    queues, markov = [], {}
    for ci, code in enumerate(pool):
        idx = np.nonzero(which == ci)[0]
        if len(idx) == 0:
            continue
        M = wl.self_transition_matrix(code.q, stay)
        markov[code.q] = (M, wl.stationary(M))
        rate_c = code.n_info / code.n
        kinds = rng.integers(0, 3, size=len(idx))
        mk = rng.random(len(idx)) < markov_share
        groups = []
        for k, kind in enumerate(("bsc", "bec", "biawgn")):
            for m in (False, True):
                sel = np.nonzero((kinds == k) & (mk == m))[0]
                if len(sel) == 0:
                    continue
                eb = rng.uniform(1.0, 2.0, size=len(sel))
                prm = np.array([wl.channel_for(kind, e, rate_c) for e in eb])
                g = wl.make_coset_frames(code, len(sel), seed * 100 + ci * 6 + k * 2 + int(m), kind, prm,
                                         source="markov" if m else "iid", markov=M if m else None)
                groups.append((g, m, idx[sel]))
        gids = np.concatenate([ids for _, _, ids in groups])
        dfr = frames_for_session([g for g, _, _ in groups])
        dfr["markov"] = torch.from_numpy(np.concatenate([np.full(g.F, int(m), np.uint8) for g, m, _ in groups])).cuda()
        dfr["syndrome"] = torch.from_numpy(np.concatenate([g.syndrome for g, _, _ in groups])).cuda()
        order = np.argsort(gids, kind="stable")  # this code's frames in arrival order
        perm = torch.from_numpy(order).cuda()
        dfr = {k: (v[perm].contiguous() if hasattr(v, "shape") and v is not None else v) for k, v in dfr.items()}
        cq = CodeQueue(code=code, frames=dfr, arrival=t[gids[order]], ids=gids[order].astype(np.int64))
        cq.groups = groups
        queues.append(cq)
    return queues, markov


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--rates", default="2000,5000,10000,20000")
    ap.add_argument("--frames", type=int, default=6000, help="requests per rate")
    ap.add_argument("--codes", type=int, default=6)
    ap.add_argument("--nmax", type=int, default=4000)
    ap.add_argument("--slots", type=int, default=512)
    ap.add_argument("--schedule", default="sus")
    ap.add_argument("--max-iter", type=int, default=100)
    ap.add_argument("--budget-gb", type=float, default=64.0)
    ap.add_argument("--step-iters", type=int, default=2)
    args = ap.parse_args()
    import torch

    torch.cuda.set_device(0)
    pool = wl.mixed_pool(args.codes, seed=0xC0DE0005, n_range=(256, args.nmax), q_weights=[0.35, 0.35, 0.3])
    for rate in [float(r) for r in args.rates.split(",")]:
        queues, markov = make_requests(pool, args.frames, rate, seed=0xDA7A0005)
        srv = Server(queues, args.slots, args.schedule, args.max_iter, int(args.budget_gb * 2 ** 30),
                     step_iters=args.step_iters, markov=markov)
        st = srv.run()
        lat = np.array(st.latency) * 1e3
        print(json.dumps({"rate": rate, "frames": st.done, "wall_s": st.wall, "throughput": st.done / st.wall,
                          "p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
                          "mean_iters": float(np.mean(st.iters)), "fer": 1 - st.converged / max(1, st.done),
                          "sessions": srv.opened, "schedule": args.schedule}),
              flush=True)


if __name__ == "__main__":
    sys.exit(main())
