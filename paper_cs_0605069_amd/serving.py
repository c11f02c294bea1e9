"""Serving: continuous batching of decode requests over several codes.

A :class:`Server` keeps one session (resident frame slots, see
``gfbp_session_*``) per code, created on first use if the device-memory budget
allows (and closed again, giving its memory back, once all its requests are
answered).  Requests (frames with their arrival times) are admitted into free
slots as they arrive; each round of the serving loop advances every session
with running frames by a few iterations on its own stream (so sessions'
kernels overlap on the device), then collects finished frames and records
their latency (arrival to collection on the host).  Converged frames leave
early; their slots are reused at once.

Request inputs come from a per-code pool of frames resident in device memory;
the k-th request of a code uses pool frame k mod P, so long arrival streams
need no more input memory than the pool.

``python -m paper_cs_0605069_amd.serving`` runs Poisson arrival streams over a
mixed pool of codes and prints, per rate, the sustained throughput and the
p50/p99 latency.
"""
from __future__ import annotations

import argparse
import json
import sys
import time
from dataclasses import dataclass, field

import numpy as np

from . import DeviceCode, Graph, Session, frames_for_session, frames_to_device, tune
from . import workloads as wl


@dataclass
class CodeQueue:
    """Requests for one code, offered in arrival order; their inputs are the
    device-resident pool `frames` (P frames; request k uses frame k mod P)."""

    code: wl.Code
    frames: dict  # device tensors from frames_for_session (+ markov, syndrome)
    arrival: np.ndarray  # seconds, nondecreasing
    ids: np.ndarray  # global request ids, increasing
    P: int = 0
    groups: list = field(default_factory=list)  # host frames: (Frames, is_markov, pool positions)
    next_arrived: int = 0
    next_admitted: int = 0
    dcode: DeviceCode | None = None
    session: Session | None = None
    stream: object = None
    need: int = 0


@dataclass
class Stats:
    latency: list = field(default_factory=list)  # arrival to collection on the host, seconds
    device_latency: list = field(default_factory=list)  # admission to retirement on the device clock, seconds
    answer_time: list = field(default_factory=list)  # collection time of each answer since the start, seconds
    iters: list = field(default_factory=list)
    edge_q: float = 0.0  # edge-q updates of the answered frames (iterations x E x q)
    converged: int = 0
    done: int = 0
    offered: int = 0
    wall: float = 0.0
    results: dict = field(default_factory=dict)


class Server:
    def __init__(self, queues: list[CodeQueue], slots: int, schedule: str, max_iter: int, budget_bytes: int,
                 step_iters: int = 2, markov: dict | None = None, keep_results: bool = False, autotune: bool = True,
                 graph: bool = False, step_graphs: bool = False, keep_ids=None, independent: bool = False):
        """keep_results: keep every answered frame's (iterations, converged,
        decisions) in Stats.results; keep_ids: keep only those requests'."""
        self.queues = queues
        self.slots = slots
        self.schedule = schedule
        self.max_iter = max_iter
        self.budget = budget_bytes
        self.used = 0
        self.step_iters = step_iters
        self.markov = markov or {}
        self.keep_ids = None if keep_ids is None else set(int(i) for i in keep_ids)
        self.keep = keep_results or self.keep_ids is not None
        self.autotune = autotune
        self.refused = 0
        self.opened = 0
        # optionally one HIP graph stepping every session at once, when all of
        # them are open from the start (sessions are then kept open until the
        # end); its grids cover every slot, which costs more than it saves
        # while few frames are in flight
        self.use_graph = graph
        # optionally each session replays its own captured step (one per
        # power-of-two bound on the tiles in flight): half the host's launch
        # cost of a SUS step, but no gain in latency, which the device's time
        # per launch bounds
        self.step_graphs = step_graphs
        # optionally each session on its own clock: a session is stepped
        # again as soon as its previous step has finished (an event on its
        # stream says so), instead of every busy session once per round
        self.independent = independent and not graph
        self.graph = None
        self.gstream = None
        from . import device_clock_hz

        self.clock_hz = float(device_clock_hz())

    def prepare(self, prewarm: bool = True):
        """Before the clock starts: upload every code, (if asked) autotune its
        kernel shape on a few of its own frames, and open as many sessions as
        the budget holds, in arrival order of their first request (the others
        open later as memory frees up)."""
        for cq in self.queues:
            if cq.dcode is None:
                cq.dcode = DeviceCode(cq.code)
            if self.autotune and cq.groups:
                g = max(cq.groups, key=lambda x: x[0].F)[0]
                tune(cq.dcode, frames_to_device(g.subset(np.arange(min(g.F, 64)))), schedule=self.schedule,
                     trial_iters=2)
        if prewarm:
            for cq in sorted(self.queues, key=lambda c: c.arrival[0] if len(c.arrival) else np.inf):
                self._open(cq)
        if self.use_graph and prewarm and all(cq.session is not None for cq in self.queues) \
                and self.step_iters % 2 == 0:
            import torch

            self.gstream = torch.cuda.Stream()
            for cq in self.queues:
                cq.stream = self.gstream  # admissions and polls in order with the graph
            torch.cuda.synchronize()
            self.graph = Graph([cq.session for cq in self.queues], iters=self.step_iters, stream=self.gstream)

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
                             markov_M=M, markov_pi=pi, step_graphs=self.step_graphs)
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

    def _admit(self, cq: CodeQueue):
        import torch

        lo, hi = cq.next_admitted, cq.next_arrived
        while lo < hi:
            p0 = lo % cq.P
            cnt = min(hi - lo, cq.P - p0)  # contiguous pool frames
            sl = {k: (v[p0:p0 + cnt] if hasattr(v, "shape") and v is not None else v) for k, v in cq.frames.items()}
            with torch.cuda.stream(cq.stream):
                k = cq.session.admit(cq.ids[lo:lo + cnt], sl, stream=cq.stream)
            lo += k
            cq.next_admitted = lo
            if k < cnt:
                break  # no free slot left

    def run(self, deadline: float | None = None, stats: Stats | None = None, prewarm: bool = True) -> Stats:
        """Serve every request, or until `deadline` seconds after the start;
        returns statistics (requests not answered by then are not counted)."""
        import torch

        self.prepare(prewarm)
        torch.cuda.synchronize()
        st = stats or Stats()
        total = sum(len(cq.arrival) for cq in self.queues)
        st.offered = total
        inflight = {}  # independent sessions: the event after each one's step in flight
        t0 = time.perf_counter()
        while st.done < total:
            now = time.perf_counter() - t0
            if deadline is not None and now > deadline:
                break
            for cq in self.queues:
                cq.next_arrived = int(np.searchsorted(cq.arrival, now, side="right"))
                # (admission waits on the session's stream: not while its step runs)
                if cq.next_admitted < cq.next_arrived and id(cq) not in inflight and self._open(cq):
                    self._admit(cq)
            busy = [cq for cq in self.queues if cq.session is not None and cq.session.running > 0]
            if self.independent:
                ready = []
                for cq in busy:
                    ev = inflight.get(id(cq))
                    if ev is None:  # idle: start its next step
                        cq.session.step(self.step_iters, stream=cq.stream)
                        ev = torch.cuda.Event()
                        ev.record(cq.stream)
                        inflight[id(cq)] = ev
                    elif ev.query():  # its step has finished: collect, then step again
                        del inflight[id(cq)]
                        ready.append(cq)
                polled = ready
            elif self.graph is not None:
                if busy:
                    self.graph.launch(self.gstream)
                polled = busy
            else:
                for cq in busy:
                    cq.session.step(self.step_iters, stream=cq.stream)
                polled = busy
            for cq in polled:
                ids, it, cv, xh, ts = cq.session.poll(want_xhat=self.keep, stream=cq.stream, timestamps=True)
                t = time.perf_counter() - t0
                if len(ids):
                    k = np.searchsorted(cq.ids, ids)
                    st.latency.extend((t - cq.arrival[k]).tolist())
                    st.answer_time.extend([t] * len(ids))
                    st.device_latency.extend(((ts[:, 1].astype(np.int64) - ts[:, 0].astype(np.int64)) / self.clock_hz)
                                             .tolist())
                    st.iters.extend(it.tolist())
                    st.edge_q += float(it.sum()) * cq.code.E * cq.code.q
                    st.converged += int(cv.sum())
                    if self.keep:
                        for r in range(len(ids)):
                            if self.keep_ids is None or int(ids[r]) in self.keep_ids:
                                st.results[int(ids[r])] = (int(it[r]), int(cv[r]), xh[r].copy())
                    st.done += len(ids)
            for cq in self.queues:
                # a session whose requests have all been answered gives its memory back
                if self.graph is None and cq.session is not None and cq.session.running == 0 \
                        and cq.next_admitted == len(cq.arrival) and id(cq) not in inflight:
                    self._close(cq)
            if self.independent and busy and not polled:
                time.sleep(0.00005)  # every busy session's step still running
            if not busy:
                if not any(cq.session is not None for cq in self.queues) and any(
                        cq.next_admitted < cq.next_arrived for cq in self.queues):
                    raise RuntimeError("device-memory budget too small for any session")
                time.sleep(0.0002)
        st.wall = time.perf_counter() - t0
        if self.graph is not None:
            self.gstream.synchronize()
            self.graph.close()
            self.graph = None
            for cq in self.queues:
                if cq.session is not None:
                    self._close(cq)
        return st


def poisson_times(n: int, rate: float, seed: int) -> np.ndarray:
    rng = np.random.default_rng([seed, 9])
    return np.cumsum(rng.exponential(1.0 / rate, size=n))


def make_requests(pool: list[wl.Code], n_frames: int, rate: float, seed: int, markov_share: float = 0.5,
                  stay: float = 0.7, pool_max: int | None = None):
    """Poisson stream of n_frames requests over the pool: each request picks a
    code uniformly, a channel (BSC, BEC, BI-AWGN) uniformly, Eb/N0 ~ U[1, 2] dB
    (channel parameter matched to that Eb/N0 at the code's rate) and, with
    probability `markov_share`, a Markov source (self-transition `stay`) on its
    information symbols.  At most pool_max distinct frames are generated per
    code (request k of a code uses frame k mod P).  Returns (queues, markov)
    where markov maps q to (M, pi)."""
    import torch

    rng = np.random.default_rng([seed, 10])
    t = poisson_times(n_frames, rate, seed)
    which = rng.integers(0, len(pool), size=n_frames)
    queues, markov = [], {}
    for ci, code in enumerate(pool):
        idx = np.nonzero(which == ci)[0]
        if len(idx) == 0:
            continue
        P = len(idx) if pool_max is None else min(len(idx), pool_max)
        M = wl.self_transition_matrix(code.q, stay)
        markov[code.q] = (M, wl.stationary(M))
        rate_c = code.n_info / code.n
        kinds = rng.integers(0, 3, size=P)
        mk = rng.random(P) < markov_share
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
                groups.append((g, m, sel))
        pos = np.concatenate([sel for _, _, sel in groups])
        dfr = frames_for_session([g for g, _, _ in groups])
        dfr["markov"] = torch.from_numpy(np.concatenate([np.full(g.F, int(m), np.uint8) for g, m, _ in groups])).cuda()
        dfr["syndrome"] = torch.from_numpy(np.concatenate([g.syndrome for g, _, _ in groups])).cuda()
        order = torch.from_numpy(np.argsort(pos, kind="stable")).cuda()  # pool order
        dfr = {k: (v[order].contiguous() if hasattr(v, "shape") and v is not None else v) for k, v in dfr.items()}
        queues.append(CodeQueue(code=code, frames=dfr, arrival=t[idx], ids=idx.astype(np.int64), P=P, groups=groups))
    return queues, markov


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--rates", default="5000,10000,20000,30000,50000,100000,200000", help="arrival rates, frames/s")
    ap.add_argument("--seconds", type=float, default=10.0, help="arrival window per rate")
    ap.add_argument("--drain", type=float, default=10.0, help="extra seconds allowed to answer the window's requests")
    ap.add_argument("--codes", type=int, default=16)
    ap.add_argument("--nmax", type=int, default=8000)
    ap.add_argument("--pool", type=int, default=2048, help="distinct frames per code")
    ap.add_argument("--slots", type=int, default=1024)
    ap.add_argument("--schedules", default="sus,pus")
    ap.add_argument("--max-iter", type=int, default=100)
    ap.add_argument("--budget-gb", type=float, default=200.0)
    ap.add_argument("--step-iters", type=int, default=2)
    ap.add_argument("--graph", action="store_true", help="step all sessions as one HIP graph")
    ap.add_argument("--step-graphs", action="store_true", help="replay a captured graph per session step")
    ap.add_argument("--independent", action="store_true",
                    help="step each session again as soon as its previous step has finished")
    args = ap.parse_args()
    import torch

    torch.cuda.set_device(0)
    pool = wl.mixed_pool(args.codes, seed=0xC0DE0005, n_range=(256, args.nmax), q_weights=[0.35, 0.35, 0.3])
    for schedule in args.schedules.split(","):
        for rate in [float(r) for r in args.rates.split(",")]:
            n = int(rate * args.seconds)
            queues, markov = make_requests(pool, n, rate, seed=0xDA7A0005, pool_max=args.pool)
            srv = Server(queues, args.slots, schedule, args.max_iter, int(args.budget_gb * 2 ** 30),
                         step_iters=args.step_iters, markov=markov, graph=args.graph,
                         step_graphs=args.step_graphs, independent=args.independent)
            st = srv.run(deadline=args.seconds + args.drain)
            lat = np.array(st.latency) * 1e3
            print(json.dumps({
                "schedule": schedule, "rate": rate, "offered": st.offered, "answered": st.done,
                "wall_s": round(st.wall, 3), "throughput_frames_per_s": st.done / st.wall,
                "p50_ms": float(np.percentile(lat, 50)) if len(lat) else None,
                "p99_ms": float(np.percentile(lat, 99)) if len(lat) else None,
                "mean_iters": float(np.mean(st.iters)) if st.iters else None,
                "edge_q_per_s": st.edge_q / st.wall if st.wall else None,
                "fer": 1 - st.converged / max(1, st.done), "sessions_opened": srv.opened,
                "codes": args.codes, "slots": args.slots, "step_iters": args.step_iters,
                "graph": args.graph, "step_graphs": args.step_graphs, "independent": args.independent}),
                flush=True)
            del queues, srv
            torch.cuda.empty_cache()


if __name__ == "__main__":
    sys.exit(main())
