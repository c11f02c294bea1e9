"""Reference decoder (plain C, double precision) and its ctypes binding.

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the benchmark's
CPU-baseline leg may load this package; the decoding product never does.  It
shares no code with the GPU decoder: see ``gfbp_oracle.c`` for the paper
passages each function follows.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "liboracle.so")
_lib = None

PUS, SUS = 0, 1
CHANNELS = {"bsc": 0, "bec": 1, "biawgn": 2, "likelihood": 3}


SANITIZED_DIR_ENV = "GFBP_SANITIZED_DIR"  # directory of a sanitizer build (see the sanitizer test)
SANITIZE_FLAGS = ["-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined", "-fno-sanitize-recover=all"]


def build(verbose: bool = False, out_dir: str | None = None, sanitize: bool = False) -> str:
    """Compile the reference decoder with gcc next to this file (or into
    out_dir; sanitize: with the address and undefined-behaviour sanitizers)."""
    src = os.path.join(_HERE, "gfbp_oracle.c")
    so = os.path.join(out_dir, "liboracle.so") if out_dir else _SO
    tmp = so + ".tmp"
    cmd = ["gcc", *(SANITIZE_FLAGS if sanitize else ["-O2"]), "-fopenmp", "-fPIC", "-shared", "-o", tmp, src, "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.check_call(cmd)
    os.replace(tmp, so)
    return so


class _Code(ctypes.Structure):
    _fields_ = [("p", ctypes.c_int), ("poly", ctypes.c_uint), ("n", ctypes.c_int), ("m", ctypes.c_int),
                ("n_info", ctypes.c_int), ("row_ptr", ctypes.c_void_p), ("col", ctypes.c_void_p),
                ("coef", ctypes.c_void_p), ("visit", ctypes.c_void_p), ("source", ctypes.c_void_p)]


class _Batch(ctypes.Structure):
    _fields_ = [("n_frames", ctypes.c_int), ("schedule", ctypes.c_int), ("max_iter", ctypes.c_int),
                ("early_stop", ctypes.c_int), ("channel", ctypes.c_int), ("evidence", ctypes.c_int),
                ("param", ctypes.c_void_p), ("rx", ctypes.c_void_p), ("erasure", ctypes.c_void_p),
                ("y", ctypes.c_void_p), ("likelihood", ctypes.c_void_p), ("syndrome", ctypes.c_void_p),
                ("prior", ctypes.c_int), ("markov_M", ctypes.c_void_p), ("markov_pi", ctypes.c_void_p),
                ("static_P", ctypes.c_void_p), ("static_per_symbol", ctypes.c_int), ("snap_iter", ctypes.c_int),
                ("n_threads", ctypes.c_int), ("prior_in_sweep", ctypes.c_int)]


class _Result(ctypes.Structure):
    _fields_ = [("xhat", ctypes.c_void_p), ("iters", ctypes.c_void_p), ("converged", ctypes.c_void_p),
                ("posterior", ctypes.c_void_p), ("snap_q", ctypes.c_void_p), ("snap_r", ctypes.c_void_p),
                ("snap_Q", ctypes.c_void_p), ("xhat_trace", ctypes.c_void_p), ("gap_trace", ctypes.c_void_p),
                ("guards", ctypes.c_void_p)]


def _load():
    global _lib
    if _lib is None:
        san = os.environ.get(SANITIZED_DIR_ENV)
        so = os.path.join(san, "liboracle.so") if san else _SO
        if not os.path.exists(so):
            build(out_dir=san)
        lib = ctypes.CDLL(so)
        lib.ref_gf_mul.argtypes = [ctypes.c_int, ctypes.c_uint, ctypes.c_int, ctypes.c_int]
        lib.ref_gf_inv.argtypes = [ctypes.c_int, ctypes.c_uint, ctypes.c_int]
        lib.ref_likelihood.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_int, ctypes.c_int,
                                       ctypes.c_void_p, ctypes.c_void_p]
        lib.ref_check_update.argtypes = [ctypes.c_int, ctypes.c_uint, ctypes.c_int, ctypes.c_void_p, ctypes.c_int,
                                         ctypes.c_void_p, ctypes.c_void_p]
        lib.ref_markov_prior.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p,
                                         ctypes.c_void_p, ctypes.c_void_p]
        lib.ref_markov_prior.restype = ctypes.c_int
        lib.ref_noise_evidence.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_int,
                                           ctypes.c_void_p, ctypes.c_void_p]
        lib.ref_frame_likelihoods.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_void_p,
                                              ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
        lib.ref_decode.argtypes = [ctypes.POINTER(_Code), ctypes.POINTER(_Batch), ctypes.POINTER(_Result)]
        lib.ref_decode.restype = ctypes.c_int
        lib.ref_max_threads.restype = ctypes.c_int
        _lib = lib
    return _lib


def _ptr(a):
    return None if a is None else a.ctypes.data


def gf_mul(p: int, poly: int, a: int, b: int) -> int:
    return _load().ref_gf_mul(p, poly, a, b)


def gf_inv(p: int, poly: int, a: int) -> int:
    return _load().ref_gf_inv(p, poly, a)


def likelihood(p: int, channel: str, param: float, rx: int = 0, er: int = 0, y=None) -> np.ndarray:
    out = np.zeros(1 << p, dtype=np.float64)
    yy = None if y is None else np.ascontiguousarray(y, dtype=np.float32)
    _load().ref_likelihood(p, CHANNELS[channel], float(param), int(rx), int(er), _ptr(yy), out.ctypes.data)
    return out


def noise_evidence(p: int, channel: str, param: float, er: int = 0, y=None) -> np.ndarray:
    """P(noise symbol = a | channel output) of one noise symbol of the
    MacKay-Neal syndrome form (Section 2)."""
    out = np.zeros(1 << p, dtype=np.float64)
    yy = None if y is None else np.ascontiguousarray(y, dtype=np.float32)
    _load().ref_noise_evidence(p, CHANNELS[channel], float(param), int(er), _ptr(yy), out.ctypes.data)
    return out


def frame_likelihoods(code, frames) -> np.ndarray:
    """Channel likelihoods L[f][j][a] of every symbol of every frame."""
    F, n, p = frames.F, code.n, code.p
    out = np.zeros((F, n, 1 << p))
    param = np.ascontiguousarray(frames.param, dtype=np.float64)
    rx = None if frames.rx is None else np.ascontiguousarray(frames.rx, dtype=np.uint8)
    er = None if frames.erasure is None else np.ascontiguousarray(frames.erasure, dtype=np.uint8)
    y = None if frames.y is None else np.ascontiguousarray(frames.y, dtype=np.float32)
    _load().ref_frame_likelihoods(p, CHANNELS[frames.channel], F, n, param.ctypes.data, _ptr(rx), _ptr(er), _ptr(y),
                                  out.ctypes.data)
    return out


def check_update(p: int, poly: int, h, z: int, qin: np.ndarray) -> np.ndarray:
    """All r-messages of one check (Eq. (3)) from its q-messages qin[dc][q]."""
    h = np.ascontiguousarray(h, dtype=np.uint8)
    qin = np.ascontiguousarray(qin, dtype=np.float64)
    out = np.zeros_like(qin)
    _load().ref_check_update(p, poly, len(h), h.ctypes.data, int(z), qin.ctypes.data, out.ctypes.data)
    return out


def markov_prior(Q: np.ndarray, M: np.ndarray, pi: np.ndarray) -> np.ndarray:
    Q = np.ascontiguousarray(Q, dtype=np.float64)
    M = np.ascontiguousarray(M, dtype=np.float64)
    pi = np.ascontiguousarray(pi, dtype=np.float64)
    K, q = Q.shape
    out = np.zeros_like(Q)
    _load().ref_markov_prior(q, K, Q.ctypes.data, M.ctypes.data, pi.ctypes.data, out.ctypes.data)
    return out


def max_threads() -> int:
    return _load().ref_max_threads()


def decode(code, frames=None, schedule: int = PUS, max_iter: int = 100, early_stop: bool = True,
           prior: str = "uniform", markov_M=None, markov_pi=None, static_prior=None, snap_iter: int = 0,
           posterior: bool = False, trace: bool = False, gap_trace: bool = False, n_threads: int = 0,
           likelihoods=None, syndrome=None, prior_in_sweep: bool = False) -> dict:
    """Decode every frame of ``frames`` (a ``workloads.Frames``) on ``code``.

    ``likelihoods`` [F][n][q] replaces the channel when given.  Frames whose
    ``evidence`` attribute is "mn" are in the MacKay-Neal syndrome form: the
    source columns carry no channel evidence and every other column is a
    noise symbol whose evidence comes from the channel output at that column.
    ``prior``: "uniform", "markov" (``markov_M``, ``markov_pi``) or "static"
    (``static_prior`` [q], or [n_info][q] in chain order).  The code's
    optional ``visit_order`` [n] and ``source_cols`` [n_info] attributes set
    the SUS visiting order and the source chain.  ``prior_in_sweep`` (SUS
    with the Markov prior): each source symbol's prior is assigned when its
    column is visited, from the newest pseudo-posteriors of its chain
    neighbours, instead of after each iteration.  Returns a dict of numpy
    arrays: xhat, iters, converged, guards and, when asked, posterior,
    snap_q / snap_r / snap_Q (messages after iteration ``snap_iter``), trace
    (decisions after each iteration) and gap_trace (after each iteration,
    the smallest gap over the columns between the two largest
    pseudo-posterior entries).
    """
    lib = _load()
    q, n, m, E = code.q, code.n, code.m, code.E
    evidence = 0
    if likelihoods is not None:
        lk = np.ascontiguousarray(likelihoods, dtype=np.float64)
        F = lk.shape[0]
        ch, param, rx, er, y = 3, np.zeros(F), None, None, None
        syn = syndrome
    else:
        F = frames.F
        ch = CHANNELS[frames.channel]
        evidence = 1 if getattr(frames, "evidence", "symbol") == "mn" else 0
        lk = None
        param = np.ascontiguousarray(frames.param, dtype=np.float64)
        rx = None if frames.rx is None else np.ascontiguousarray(frames.rx, dtype=np.uint8)
        er = None if frames.erasure is None else np.ascontiguousarray(frames.erasure, dtype=np.uint8)
        y = None if frames.y is None else np.ascontiguousarray(frames.y, dtype=np.float32)
        syn = frames.syndrome if syndrome is None else syndrome
    syn = None if syn is None else np.ascontiguousarray(syn, dtype=np.uint8)
    rp = np.ascontiguousarray(code.row_ptr, dtype=np.int32)
    cl = np.ascontiguousarray(code.col, dtype=np.int32)
    cf = np.ascontiguousarray(code.coef, dtype=np.uint8)
    vo = getattr(code, "visit_order", None)
    sc = getattr(code, "source_cols", None)
    vo = None if vo is None else np.ascontiguousarray(vo, dtype=np.int32)
    sc = None if sc is None else np.ascontiguousarray(sc, dtype=np.int32)
    Mk = pk = sp = None
    prior_kind = {"uniform": 0, "markov": 1, "static": 2}[prior]
    per_symbol = 0
    if prior == "markov":
        Mk = np.ascontiguousarray(markov_M, dtype=np.float64)
        pk = np.ascontiguousarray(markov_pi, dtype=np.float64)
    elif prior == "static":
        sp = np.ascontiguousarray(static_prior, dtype=np.float64)
        per_symbol = int(sp.ndim == 2)
    out = {
        "xhat": np.zeros((F, n), dtype=np.uint8),
        "iters": np.zeros(F, dtype=np.int32),
        "converged": np.zeros(F, dtype=np.uint8),
        "guards": np.zeros(F, dtype=np.int32),
    }
    if posterior:
        out["posterior"] = np.zeros((F, n, q))
    if snap_iter:
        out["snap_q"] = np.zeros((F, E, q))
        out["snap_r"] = np.zeros((F, E, q))
        out["snap_Q"] = np.zeros((F, n, q))
    if trace:
        out["trace"] = np.zeros((F, max_iter, n), dtype=np.uint8)
    if gap_trace:
        out["gap_trace"] = np.full((F, max_iter), np.nan)
    c = _Code(code.p, code.poly, n, m, code.n_info, rp.ctypes.data, cl.ctypes.data, cf.ctypes.data, _ptr(vo),
              _ptr(sc))
    b = _Batch(F, schedule, max_iter, int(early_stop), ch, evidence, param.ctypes.data, _ptr(rx), _ptr(er), _ptr(y),
               _ptr(lk), _ptr(syn), prior_kind, _ptr(Mk), _ptr(pk), _ptr(sp), per_symbol, snap_iter, n_threads,
               int(bool(prior_in_sweep)))
    r = _Result(out["xhat"].ctypes.data, out["iters"].ctypes.data, out["converged"].ctypes.data,
                _ptr(out.get("posterior")), _ptr(out.get("snap_q")), _ptr(out.get("snap_r")),
                _ptr(out.get("snap_Q")), _ptr(out.get("trace")), _ptr(out.get("gap_trace")), out["guards"].ctypes.data)
    rc = lib.ref_decode(ctypes.byref(c), ctypes.byref(b), ctypes.byref(r))
    if rc != 0:
        raise RuntimeError(f"ref_decode failed ({rc})")
    return out
