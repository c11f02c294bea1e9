"""gfbp — GF(2^p) LDPC belief-propagation decoding on AMD Instinct MI355X.

Thin ctypes binding of the C ABI in ``include/gfbp.h`` (library
``libgfbp.so`` next to this file).  The binding only marshals arguments: it
allocates device buffers with PyTorch (memory and streams are PyTorch's) and
passes raw pointers; every step of decoding runs in the HIP kernels of the
library.  If the library is missing the binding raises: there is no fallback.

Method: Yacov et al., "Parallel vs. Sequential Belief Propagation Decoding of
LDPC Codes over GF(q) and Markov Sources", Section 2 (schedules PUS and SUS,
Eqs. (3), (4), (5), dynamical Markov block priors Eq. (7)).
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libgfbp.so")

PUS, SUS = 0, 1
CH_BSC, CH_BEC, CH_BIAWGN, CH_LIKELIHOOD = 0, 1, 2, 3
PRIOR_UNIFORM, PRIOR_MARKOV, PRIOR_STATIC = 0, 1, 2
PRIORS = {"uniform": PRIOR_UNIFORM, "markov": PRIOR_MARKOV, "static": PRIOR_STATIC}
EVIDENCE_SYMBOL, EVIDENCE_MN = 0, 1
OPT_SUS_STRICT = 1
OPT_NO_COMPACT = 2
OPT_STEP_GRAPHS = 4
OPT_PRIOR_IN_SWEEP = 8
OPT_PERSISTENT = 16
OPT_NO_ONCHIP = 32
CHANNELS = {"bsc": CH_BSC, "bec": CH_BEC, "biawgn": CH_BIAWGN, "likelihood": CH_LIKELIHOOD}
SCHEDULES = {"pus": PUS, "sus": SUS, PUS: PUS, SUS: SUS}

EXPORTS = ("gfbp_code_build", "gfbp_code_free", "gfbp_code_info_get", "gfbp_workspace_size",
           "gfbp_batch_workspace_size", "gfbp_decode_batch", "gfbp_decode_batch_noalloc", "gfbp_tune_persistent",
           "gfbp_device_clock_hz", "gfbp_stream_copy_rate",
           "gfbp_profile_enable", "gfbp_profile_reset", "gfbp_profile_read", "gfbp_code_set_shape",
           "gfbp_code_get_shape", "gfbp_tune", "gfbp_session_bytes", "gfbp_session_create", "gfbp_session_destroy",
           "gfbp_session_admit", "gfbp_session_step", "gfbp_session_poll", "gfbp_session_free_slots",
           "gfbp_session_running", "gfbp_graph_capture", "gfbp_graph_launch", "gfbp_graph_destroy",
           "gfbp_last_error", "gfbp_version")


class CodeDesc(ctypes.Structure):
    _fields_ = [("q", ctypes.c_int32), ("poly", ctypes.c_int32), ("n", ctypes.c_int32), ("m", ctypes.c_int32),
                ("n_info", ctypes.c_int32), ("row_ptr", ctypes.c_void_p), ("col", ctypes.c_void_p),
                ("coef", ctypes.c_void_p), ("visit_order", ctypes.c_void_p), ("source_cols", ctypes.c_void_p)]


class CodeInfo(ctypes.Structure):
    _fields_ = [("q", ctypes.c_int32), ("p", ctypes.c_int32), ("n", ctypes.c_int32), ("m", ctypes.c_int32),
                ("n_info", ctypes.c_int32), ("n_edges", ctypes.c_int32), ("max_row_degree", ctypes.c_int32),
                ("max_col_degree", ctypes.c_int32), ("poly", ctypes.c_int32), ("sus_levels", ctypes.c_int32),
                ("sus_levels_in_sweep", ctypes.c_int32)]


class Batch(ctypes.Structure):
    _fields_ = [("n_frames", ctypes.c_int32), ("schedule", ctypes.c_int32), ("max_iter", ctypes.c_int32),
                ("early_stop", ctypes.c_int32), ("channel", ctypes.c_int32), ("param", ctypes.c_void_p),
                ("rx", ctypes.c_void_p), ("erasure", ctypes.c_void_p), ("y", ctypes.c_void_p),
                ("likelihood", ctypes.c_void_p), ("syndrome", ctypes.c_void_p), ("prior", ctypes.c_int32),
                ("markov_M", ctypes.c_void_p), ("markov_pi", ctypes.c_void_p), ("options", ctypes.c_int32),
                ("truth", ctypes.c_void_p), ("evidence", ctypes.c_int32), ("channel_of", ctypes.c_void_p),
                ("static_prior", ctypes.c_void_p), ("static_per_symbol", ctypes.c_int32), ("n_codes", ctypes.c_int32),
                ("code_index", ctypes.c_void_p), ("persist_el", ctypes.c_int32), ("persist_waves", ctypes.c_int32)]


class Result(ctypes.Structure):
    _fields_ = [("xhat", ctypes.c_void_p), ("iters", ctypes.c_void_p), ("converged", ctypes.c_void_p),
                ("posterior", ctypes.c_void_p), ("guards", ctypes.c_void_p), ("snap_iter", ctypes.c_int32),
                ("snap_q", ctypes.c_void_p), ("snap_r", ctypes.c_void_p), ("snap_Q", ctypes.c_void_p),
                ("trace", ctypes.c_void_p)]


class KernelStats(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char * 32), ("launches", ctypes.c_int64), ("total_ms", ctypes.c_double),
                ("algo_bytes", ctypes.c_double), ("edge_q", ctypes.c_double)]


class SessionDesc(ctypes.Structure):
    _fields_ = [("n_slots", ctypes.c_int32), ("schedule", ctypes.c_int32), ("max_iter", ctypes.c_int32),
                ("has_syndrome", ctypes.c_int32), ("markov_M", ctypes.c_void_p), ("markov_pi", ctypes.c_void_p),
                ("options", ctypes.c_int32), ("device_bytes", ctypes.c_int64)]


class FramesIn(ctypes.Structure):
    _fields_ = [("channel", ctypes.c_void_p), ("markov", ctypes.c_void_p), ("param", ctypes.c_void_p),
                ("rx", ctypes.c_void_p), ("erasure", ctypes.c_void_p), ("y", ctypes.c_void_p),
                ("syndrome", ctypes.c_void_p)]


class Retired(ctypes.Structure):
    _fields_ = [("id", ctypes.c_int64), ("iters", ctypes.c_int32), ("converged", ctypes.c_int32),
                ("t_admit", ctypes.c_uint64), ("t_retire", ctypes.c_uint64)]


_lib = None


def lib():
    """The loaded C library (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} not found: build the HIP library first (__graft_entry__.build())")
    L = ctypes.CDLL(LIB_PATH)
    L.gfbp_code_build.argtypes = [ctypes.POINTER(CodeDesc), ctypes.POINTER(ctypes.c_void_p)]
    L.gfbp_code_build.restype = ctypes.c_int32
    L.gfbp_code_free.argtypes = [ctypes.c_void_p]
    L.gfbp_code_free.restype = ctypes.c_int32
    L.gfbp_code_info_get.argtypes = [ctypes.c_void_p, ctypes.POINTER(CodeInfo)]
    L.gfbp_code_info_get.restype = ctypes.c_int32
    L.gfbp_workspace_size.argtypes = [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32]
    L.gfbp_workspace_size.restype = ctypes.c_size_t
    L.gfbp_batch_workspace_size.argtypes = [ctypes.c_void_p, ctypes.POINTER(Batch)]
    L.gfbp_batch_workspace_size.restype = ctypes.c_size_t
    L.gfbp_decode_batch.argtypes = [ctypes.c_void_p, ctypes.POINTER(Batch), ctypes.POINTER(Result), ctypes.c_void_p,
                                    ctypes.c_size_t, ctypes.c_void_p]
    L.gfbp_decode_batch.restype = ctypes.c_int32
    L.gfbp_decode_batch_noalloc.argtypes = [ctypes.c_void_p, ctypes.POINTER(Batch), ctypes.POINTER(Result),
                                            ctypes.c_void_p]
    L.gfbp_decode_batch_noalloc.restype = ctypes.c_int32
    L.gfbp_tune_persistent.argtypes = [ctypes.c_void_p, ctypes.POINTER(Batch), ctypes.POINTER(Result), ctypes.c_void_p,
                                       ctypes.c_size_t, ctypes.c_void_p, ctypes.c_int32,
                                       ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32)]
    L.gfbp_tune_persistent.restype = ctypes.c_int32
    L.gfbp_device_clock_hz.restype = ctypes.c_uint64
    L.gfbp_stream_copy_rate.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int32,
                                        ctypes.c_void_p, ctypes.POINTER(ctypes.c_double)]
    L.gfbp_stream_copy_rate.restype = ctypes.c_int32
    L.gfbp_profile_enable.argtypes = [ctypes.c_int32]
    L.gfbp_profile_enable.restype = ctypes.c_int32
    L.gfbp_profile_reset.restype = ctypes.c_int32
    L.gfbp_profile_read.argtypes = [ctypes.POINTER(KernelStats), ctypes.c_int32]
    L.gfbp_profile_read.restype = ctypes.c_int32
    L.gfbp_code_set_shape.argtypes = [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32]
    L.gfbp_code_set_shape.restype = ctypes.c_int32
    L.gfbp_code_get_shape.argtypes = [ctypes.c_void_p, ctypes.c_int32]
    L.gfbp_code_get_shape.restype = ctypes.c_int32
    L.gfbp_tune.argtypes = [ctypes.c_void_p, ctypes.POINTER(Batch), ctypes.POINTER(Result), ctypes.c_void_p,
                            ctypes.c_size_t, ctypes.c_void_p, ctypes.c_int32, ctypes.POINTER(ctypes.c_int32)]
    L.gfbp_tune.restype = ctypes.c_int32
    L.gfbp_session_bytes.argtypes = [ctypes.c_void_p, ctypes.POINTER(SessionDesc)]
    L.gfbp_session_bytes.restype = ctypes.c_size_t
    L.gfbp_session_create.argtypes = [ctypes.c_void_p, ctypes.POINTER(SessionDesc), ctypes.POINTER(ctypes.c_void_p)]
    L.gfbp_session_create.restype = ctypes.c_int32
    L.gfbp_session_destroy.argtypes = [ctypes.c_void_p]
    L.gfbp_session_destroy.restype = ctypes.c_int32
    L.gfbp_session_admit.argtypes = [ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p, ctypes.POINTER(FramesIn),
                                     ctypes.POINTER(ctypes.c_int32), ctypes.c_void_p]
    L.gfbp_session_admit.restype = ctypes.c_int32
    L.gfbp_session_step.argtypes = [ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p]
    L.gfbp_session_step.restype = ctypes.c_int32
    L.gfbp_session_poll.argtypes = [ctypes.c_void_p, ctypes.POINTER(Retired), ctypes.c_void_p, ctypes.c_int32,
                                    ctypes.POINTER(ctypes.c_int32), ctypes.c_void_p]
    L.gfbp_session_poll.restype = ctypes.c_int32
    L.gfbp_session_free_slots.argtypes = [ctypes.c_void_p]
    L.gfbp_session_free_slots.restype = ctypes.c_int32
    L.gfbp_session_running.argtypes = [ctypes.c_void_p]
    L.gfbp_session_running.restype = ctypes.c_int32
    L.gfbp_graph_capture.argtypes = [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32, ctypes.c_void_p,
                                     ctypes.POINTER(ctypes.c_void_p)]
    L.gfbp_graph_capture.restype = ctypes.c_int32
    L.gfbp_graph_launch.argtypes = [ctypes.c_void_p, ctypes.c_void_p]
    L.gfbp_graph_launch.restype = ctypes.c_int32
    L.gfbp_graph_destroy.argtypes = [ctypes.c_void_p]
    L.gfbp_graph_destroy.restype = ctypes.c_int32
    L.gfbp_last_error.restype = ctypes.c_char_p
    L.gfbp_version.restype = ctypes.c_char_p
    _lib = L
    return L


class GfbpError(RuntimeError):
    def __init__(self, status: int, where: str):
        msg = lib().gfbp_last_error().decode()
        super().__init__(f"{where} failed with status {status}: {msg}")
        self.status = status


def _check(status: int, where: str):
    if status != 0:
        raise GfbpError(status, where)


def version() -> str:
    return lib().gfbp_version().decode()


def profile_enable(on: bool = True):
    _check(lib().gfbp_profile_enable(int(bool(on))), "gfbp_profile_enable")


def profile_reset():
    _check(lib().gfbp_profile_reset(), "gfbp_profile_reset")


def profile_read() -> dict:
    """Per-kernel totals since the last reset: {name: {launches, total_ms, algo_bytes, edge_q}}."""
    buf = (KernelStats * 16)()
    n = lib().gfbp_profile_read(buf, 16)
    return {buf[i].name.decode(): {"launches": int(buf[i].launches), "total_ms": float(buf[i].total_ms),
                                   "algo_bytes": float(buf[i].algo_bytes), "edge_q": float(buf[i].edge_q)}
            for i in range(min(n, 16))}


def last_error() -> str:
    return lib().gfbp_last_error().decode()


class DeviceCode:
    """A code built on the current HIP device (``gfbp_code_build``).

    ``code`` is any object with q, n, m, n_info, row_ptr, col, coef and
    (optionally) poly attributes, such as ``workloads.Code``.
    """

    def __init__(self, code):
        L = lib()
        self._rp = np.ascontiguousarray(code.row_ptr, dtype=np.int32)
        self._col = np.ascontiguousarray(code.col, dtype=np.int32)
        self._coef = np.ascontiguousarray(code.coef, dtype=np.uint8)
        vo, sc = getattr(code, "visit_order", None), getattr(code, "source_cols", None)
        self._vo = None if vo is None else np.ascontiguousarray(vo, dtype=np.int32)
        self._sc = None if sc is None else np.ascontiguousarray(sc, dtype=np.int32)
        d = CodeDesc(int(code.q), int(getattr(code, "poly", 0)), int(code.n), int(code.m), int(code.n_info),
                     self._rp.ctypes.data, self._col.ctypes.data, self._coef.ctypes.data,
                     None if self._vo is None else self._vo.ctypes.data,
                     None if self._sc is None else self._sc.ctypes.data)
        h = ctypes.c_void_p()
        _check(L.gfbp_code_build(ctypes.byref(d), ctypes.byref(h)), "gfbp_code_build")
        self.handle = h
        info = CodeInfo()
        _check(L.gfbp_code_info_get(h, ctypes.byref(info)), "gfbp_code_info_get")
        self.info = info

    def close(self):
        if getattr(self, "handle", None):
            lib().gfbp_code_free(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def q(self):
        return self.info.q

    @property
    def n(self):
        return self.info.n

    @property
    def m(self):
        return self.info.m

    @property
    def E(self):
        return self.info.n_edges

    def set_shape(self, schedule, entries_per_lane: int):
        _check(lib().gfbp_code_set_shape(self.handle, SCHEDULES[schedule], int(entries_per_lane)), "gfbp_code_set_shape")

    def shape(self, schedule) -> int:
        return int(lib().gfbp_code_get_shape(self.handle, SCHEDULES[schedule]))

    def workspace_size(self, n_frames: int, schedule, prior: int = PRIOR_UNIFORM) -> int:
        return int(lib().gfbp_workspace_size(self.handle, int(n_frames), SCHEDULES[schedule], int(prior)))


def _dptr(t):
    return None if t is None else t.data_ptr()


def frames_to_device(frames, device="cuda"):
    """Copy a ``workloads.Frames`` batch to device tensors (marshalling only)."""
    import torch

    def dev(a, dt):
        return None if a is None else torch.from_numpy(np.ascontiguousarray(a)).to(device=device, dtype=dt)

    return {
        "channel": frames.channel,
        "F": frames.F,
        "evidence": getattr(frames, "evidence", "symbol"),
        "param": dev(frames.param.astype(np.float32), torch.float32),
        "rx": dev(frames.rx, torch.uint8),
        "erasure": dev(frames.erasure, torch.uint8),
        "y": dev(frames.y, torch.float32),
        "syndrome": dev(frames.syndrome, torch.uint8),
        "likelihood": dev(getattr(frames, "lik", None), torch.float32),
    }


def _codes_array(dcodes):
    arr = (ctypes.c_void_p * len(dcodes))(*[d.handle.value for d in dcodes])
    return arr


def _batch(F, sch, max_iter, early_stop, dframes, prior, Mt, pt, Pt, per_symbol, options, truth, n_codes, code_index,
           persist_el=0, persist_waves=0):
    ev = dframes.get("evidence", "symbol")
    return Batch(F, sch, int(max_iter), int(bool(early_stop)), CHANNELS[dframes.get("channel", "bsc")],
                 _dptr(dframes.get("param")), _dptr(dframes.get("rx")), _dptr(dframes.get("erasure")),
                 _dptr(dframes.get("y")), _dptr(dframes.get("likelihood")), _dptr(dframes.get("syndrome")),
                 PRIORS[prior], _dptr(Mt), _dptr(pt), int(options), _dptr(truth),
                 EVIDENCE_MN if ev == "mn" else EVIDENCE_SYMBOL, _dptr(dframes.get("channel_of")), _dptr(Pt),
                 int(per_symbol), int(n_codes), None if code_index is None else code_index.ctypes.data,
                 int(persist_el), int(persist_waves))


def _prior_tensors(prior, markov_M, markov_pi, static_prior, dev):
    import torch

    Mt = pt = Pt = None
    per_symbol = 0
    if prior == "markov":
        Mt = torch.as_tensor(np.asarray(markov_M, dtype=np.float32), device=dev).contiguous()
        pt = torch.as_tensor(np.asarray(markov_pi, dtype=np.float32), device=dev).contiguous()
    elif prior == "static":
        sp = np.asarray(static_prior, dtype=np.float32)
        per_symbol = int(sp.ndim == 2)
        Pt = torch.as_tensor(sp, device=dev).contiguous()
    return Mt, pt, Pt, per_symbol


def decode_batch(dcode: DeviceCode, dframes: dict, schedule="pus", max_iter: int = 100, early_stop: bool = True,
                 prior: str = "uniform", markov_M=None, markov_pi=None, posterior: bool = False, guards: bool = True,
                 snap_iter: int = 0, workspace=None, stream=None, outputs: dict | None = None,
                 sus_strict: bool = False, tune_iters: int = 0, compact: bool = True, truth=None,
                 prior_in_sweep: bool = False, static_prior=None, persistent: bool = False, persist_el: int = 0,
                 persist_waves: int = 0, onchip: bool = True) -> dict:
    """``gfbp_decode_batch`` on device tensors of one code; returns device tensors.

    dframes: dict from :func:`frames_to_device` (or with the same keys; an
    optional ``channel_of`` uint8 [F] gives each frame's channel kind, and
    ``evidence`` "mn" selects the MacKay-Neal syndrome form).
    prior: "uniform", "markov" (markov_M, markov_pi) or "static"
    (static_prior [q] or [n_info][q] in chain order).
    workspace: optional preallocated uint8 device tensor of at least
    ``gfbp_batch_workspace_size`` bytes, 256-byte aligned.
    outputs: optional preallocated output tensors (xhat, iters, converged).
    truth: optional device uint8 [F][n] true symbols; then out["trace"] [F][max_iter]
    counts the correct source bits after each iteration (the Fig. 1 diagnostic).
    prior_in_sweep: SUS with the Markov prior assigns each source symbol's
    prior at its column's vertical pass (``GFBP_OPT_PRIOR_IN_SWEEP``).
    persistent: decode through the persistent work-list kernel
    (``GFBP_OPT_PERSISTENT``) with tile shape persist_el / persist_waves.
    onchip=False: the tiled kernels even where the frames' state fits in LDS
    (``GFBP_OPT_NO_ONCHIP``).
    """
    import torch

    F = int(dframes["F"])
    n, q, E = dcode.n, dcode.q, dcode.E
    dev = torch.device("cuda", torch.cuda.current_device())
    sch = SCHEDULES[schedule]
    out = dict(outputs) if outputs else {}
    out.setdefault("xhat", torch.empty((F, n), dtype=torch.uint8, device=dev))
    out.setdefault("iters", torch.empty((F,), dtype=torch.int32, device=dev))
    out.setdefault("converged", torch.empty((F,), dtype=torch.uint8, device=dev))
    if posterior:
        out.setdefault("posterior", torch.empty((F, n, q), dtype=torch.float32, device=dev))
    if guards:
        out.setdefault("guards", torch.empty((F,), dtype=torch.int32, device=dev))
    if truth is not None:
        out.setdefault("trace", torch.empty((F, int(max_iter)), dtype=torch.int32, device=dev))
    if snap_iter:
        out["snap_q"] = torch.zeros((F, E, q), dtype=torch.float32, device=dev)
        out["snap_r"] = torch.zeros((F, E, q), dtype=torch.float32, device=dev)
        out["snap_Q"] = torch.zeros((F, n, q), dtype=torch.float32, device=dev)
    Mt, pt, Pt, per_symbol = _prior_tensors(prior, markov_M, markov_pi, static_prior, dev)
    opts = ((OPT_SUS_STRICT if sus_strict else 0) | (0 if compact else OPT_NO_COMPACT) |
            (OPT_PRIOR_IN_SWEEP if prior_in_sweep else 0) | (OPT_PERSISTENT if persistent else 0) |
            (0 if onchip else OPT_NO_ONCHIP))
    b = _batch(F, sch, max_iter, early_stop, dframes, prior, Mt, pt, Pt, per_symbol, opts, truth, 1, None,
               persist_el, persist_waves)
    codes = _codes_array([dcode])
    ws_bytes = int(lib().gfbp_batch_workspace_size(codes, ctypes.byref(b)))
    if workspace is None:
        workspace = torch.empty((max(ws_bytes, 1),), dtype=torch.uint8, device=dev)
    r = Result(_dptr(out["xhat"]), _dptr(out["iters"]), _dptr(out["converged"]), _dptr(out.get("posterior")),
               _dptr(out.get("guards")), int(snap_iter), _dptr(out.get("snap_q")), _dptr(out.get("snap_r")),
               _dptr(out.get("snap_Q")), _dptr(out.get("trace")))
    st = torch.cuda.current_stream() if stream is None else stream
    if tune_iters:
        chosen = ctypes.c_int32(0)
        _check(lib().gfbp_tune(dcode.handle, ctypes.byref(b), ctypes.byref(r), workspace.data_ptr(), workspace.numel(),
                               ctypes.c_void_p(st.cuda_stream), int(tune_iters), ctypes.byref(chosen)), "gfbp_tune")
        out["entries_per_lane"] = int(chosen.value)
        return out
    _check(lib().gfbp_decode_batch(codes, ctypes.byref(b), ctypes.byref(r), workspace.data_ptr(),
                                   workspace.numel(), ctypes.c_void_p(st.cuda_stream)), "gfbp_decode_batch")
    return out


def ragged_frames(frames_list, codes_list, device="cuda"):
    """Concatenate ``workloads.Frames`` batches (frames_list[k] on codes_list[k],
    in order) into the ragged device inputs of a multi-code
    ``gfbp_decode_batch``: per-symbol arrays one frame after the other with each
    frame's own n (and p or q), syndromes with each frame's m, a per-frame
    channel kind and parameters."""
    import torch

    def cat(parts, dtype):
        parts = [np.ascontiguousarray(x, dtype=dtype).ravel() for x in parts]
        return torch.from_numpy(np.concatenate(parts) if parts else np.zeros(0, dtype)).to(device)

    ev = {getattr(f, "evidence", "symbol") for f in frames_list}
    if len(ev) > 1:
        raise ValueError("one evidence mode per batch")
    rx, er, y, lik, syn, ch, prm = [], [], [], [], [], [], []
    for fr in frames_list:
        F, n = fr.codeword.shape
        rx.append(fr.rx if fr.rx is not None else np.zeros((F, n), np.uint8))
        er.append(fr.erasure if fr.erasure is not None else np.zeros((F, n), np.uint8))
        if fr.y is not None:
            y.append(fr.y)
        if getattr(fr, "lik", None) is not None:
            lik.append(fr.lik)
        if fr.syndrome is not None:
            syn.append(fr.syndrome)
        ch.append(np.full(F, CHANNELS[fr.channel], np.uint8))
        prm.append(fr.param.astype(np.float32))
    any_y = any(fr.y is not None for fr in frames_list)
    if any_y:  # frames of other channels hold zeros in y (unread)
        y = []
        for fr, code in zip(frames_list, codes_list):
            F, n = fr.codeword.shape
            y.append(fr.y if fr.y is not None else np.zeros((F, n, code.p), np.float32))
    out = {"F": sum(fr.F for fr in frames_list), "channel": frames_list[0].channel, "evidence": ev.pop(),
           "channel_of": cat(ch, np.uint8), "param": cat(prm, np.float32), "rx": cat(rx, np.uint8),
           "erasure": cat(er, np.uint8)}
    if any_y:
        out["y"] = cat(y, np.float32)
    if lik:
        out["likelihood"] = cat(lik, np.float32)
    if syn:
        if len(syn) != len(frames_list):
            raise ValueError("syndromes for every entry or none")
        out["syndrome"] = cat(syn, np.uint8)
    return out


def persist_entries_per_lane(q: int, el: int = 0, narrow: bool = True) -> int:
    """Entries per lane the persistent path gives field q's tiles for the batch
    shape persist_el = el (0 = 4), as gfbp_batch.persist_el states: at most
    max(2, q/4) (at most 16 frames per tile), at most 4 outside the narrow
    degree class, at most q."""
    e = min(el or 4, 4 if not narrow else 8)
    return min(e, max(2, q // 4), q)


def decode_multi(dcodes, code_index, dframes: dict, schedule="pus", max_iter: int = 100, early_stop: bool = True,
                 prior: str = "uniform", markov_M=None, markov_pi=None, static_prior=None, workspace=None,
                 stream=None, persist_el: int = 0, persist_waves: int = 0, tune_iters: int = 0,
                 persistent: bool = False, prior_in_sweep: bool = False) -> dict:
    """``gfbp_decode_batch`` over several codes: frame f is on
    dcodes[code_index[f]]; dframes holds ragged inputs (see
    :func:`ragged_frames`).  By default the library decodes code by code with
    the plain kernels, the codes concurrently; persistent=True takes the
    persistent work-list kernels (``GFBP_OPT_PERSISTENT``, tile shape
    persist_el / persist_waves).  Returns device tensors xhat (ragged, sum of
    n), iters, converged and guards; with tune_iters, runs
    ``gfbp_tune_persistent`` instead and returns the chosen shape."""
    import torch

    ci = np.ascontiguousarray(code_index, dtype=np.int32)
    F = len(ci)
    if int(dframes["F"]) != F:
        raise ValueError("code_index and dframes disagree on the number of frames")
    dev = torch.device("cuda", torch.cuda.current_device())
    ns = np.array([d.n for d in dcodes], dtype=np.int64)
    out = {"xhat": torch.empty((int(ns[ci].sum()),), dtype=torch.uint8, device=dev),
           "iters": torch.empty((F,), dtype=torch.int32, device=dev),
           "converged": torch.empty((F,), dtype=torch.uint8, device=dev),
           "guards": torch.empty((F,), dtype=torch.int32, device=dev)}
    Mt, pt, Pt, per_symbol = _prior_tensors(prior, markov_M, markov_pi, static_prior, dev)
    opts = (OPT_PERSISTENT if persistent or tune_iters else 0) | (OPT_PRIOR_IN_SWEEP if prior_in_sweep else 0)
    b = _batch(F, SCHEDULES[schedule], max_iter, early_stop, dframes, prior, Mt, pt, Pt, per_symbol, opts, None,
               len(dcodes), ci, persist_el, persist_waves)
    codes = _codes_array(dcodes)
    ws_bytes = int(lib().gfbp_batch_workspace_size(codes, ctypes.byref(b)))
    if tune_iters:  # room for every candidate shape
        ws_bytes = max(ws_bytes, max(int(lib().gfbp_batch_workspace_size(codes, ctypes.byref(
            _batch(F, SCHEDULES[schedule], max_iter, early_stop, dframes, prior, Mt, pt, Pt, per_symbol, opts, None,
                   len(dcodes), ci, el, wv)))) for el in (4, 8) for wv in (4, 8)))
    if workspace is None:
        workspace = torch.empty((max(ws_bytes, 1),), dtype=torch.uint8, device=dev)
    r = Result(_dptr(out["xhat"]), _dptr(out["iters"]), _dptr(out["converged"]), None, _dptr(out["guards"]), 0,
               None, None, None, None)
    st = torch.cuda.current_stream() if stream is None else stream
    if tune_iters:
        el, wv = ctypes.c_int32(0), ctypes.c_int32(0)
        _check(lib().gfbp_tune_persistent(codes, ctypes.byref(b), ctypes.byref(r), workspace.data_ptr(),
                                          workspace.numel(), ctypes.c_void_p(st.cuda_stream), int(tune_iters),
                                          ctypes.byref(el), ctypes.byref(wv)), "gfbp_tune_persistent")
        out["persist_el"], out["persist_waves"] = int(el.value), int(wv.value)
        return out
    _check(lib().gfbp_decode_batch(codes, ctypes.byref(b), ctypes.byref(r), workspace.data_ptr(), workspace.numel(),
                                   ctypes.c_void_p(st.cuda_stream)), "gfbp_decode_batch")
    return out


def decode_batch_noalloc(dcodes, dframes: dict, outputs: dict, schedule="pus", max_iter: int = 100,
                         early_stop: bool = True, prior: str = "uniform", prior_tensors=(None, None, None, 0),
                         code_index=None, options: int = 0, stream=None):
    """``gfbp_decode_batch_noalloc``: decode with the library's static device
    scratch; the caller passes every device buffer (inputs in dframes, outputs
    xhat / iters / converged / guards in ``outputs``, prior tensors as
    (markov_M, markov_pi, static_prior, per_symbol)); nothing is allocated."""
    F = int(dframes["F"])
    Mt, pt, Pt, per_symbol = prior_tensors
    ci = None if code_index is None else np.ascontiguousarray(code_index, dtype=np.int32)
    b = _batch(F, SCHEDULES[schedule], max_iter, early_stop, dframes, prior, Mt, pt, Pt, per_symbol, options, None,
               len(dcodes), ci)
    r = Result(_dptr(outputs["xhat"]), _dptr(outputs["iters"]), _dptr(outputs["converged"]), None,
               _dptr(outputs.get("guards")), 0, None, None, None, None)
    _check(lib().gfbp_decode_batch_noalloc(_codes_array(dcodes), ctypes.byref(b), ctypes.byref(r),
                                           _stream_ptr(stream)), "gfbp_decode_batch_noalloc")
    return outputs


def device_clock_hz() -> int:
    return int(lib().gfbp_device_clock_hz())


def stream_copy_rate(dst, src, reps: int = 5, stream=None) -> float:
    """``gfbp_stream_copy_rate``: best read + write bytes/s of a streaming copy
    of src (a contiguous device tensor) into dst (same size)."""
    import torch

    assert dst.is_cuda and src.is_cuda and dst.is_contiguous() and src.is_contiguous()
    nbytes = src.numel() * src.element_size()
    assert dst.numel() * dst.element_size() == nbytes
    st = stream if stream is not None else torch.cuda.current_stream()
    rate = ctypes.c_double(0.0)
    _check(lib().gfbp_stream_copy_rate(dst.data_ptr(), src.data_ptr(), nbytes, int(reps), st.cuda_stream,
                                       ctypes.byref(rate)), "gfbp_stream_copy_rate")
    return float(rate.value)


def tune(dcode: DeviceCode, dframes: dict, schedule="pus", trial_iters: int = 3, **kw) -> int:
    """``gfbp_tune``: time every allowed kernel shape on this batch and keep the
    fastest for the schedule; returns the chosen entries per lane."""
    return decode_batch(dcode, dframes, schedule=schedule, tune_iters=trial_iters, **kw)["entries_per_lane"]


def _stream_ptr(stream):
    import torch

    st = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(st.cuda_stream)


class Session:
    """``gfbp_session_*``: continuous batching on one code (resident frame slots).

    Frames are admitted from device tensors (a dict with per-frame ``channel``
    codes, optional ``markov`` flags, ``param``, ``rx``, ``erasure``, ``y``,
    ``syndrome``), stepped, and collected by :meth:`poll`.
    """

    def __init__(self, dcode: DeviceCode, n_slots: int, schedule="pus", max_iter: int = 100,
                 has_syndrome: bool = False, markov_M=None, markov_pi=None, sus_strict: bool = False,
                 step_graphs: bool = False, device_bytes: int = 0):
        """step_graphs: replay a captured HIP graph for each even-iteration
        :meth:`step` on a created stream (the same work; fewer host launches).
        n_slots = 0: as many slots as ``device_bytes`` of device memory hold."""
        self.dcode = dcode
        self._M = None if markov_M is None else np.ascontiguousarray(markov_M, dtype=np.float32)
        self._pi = None if markov_pi is None else np.ascontiguousarray(markov_pi, dtype=np.float32)
        self.desc = SessionDesc(int(n_slots), SCHEDULES[schedule], int(max_iter), int(bool(has_syndrome)),
                                None if self._M is None else self._M.ctypes.data,
                                None if self._pi is None else self._pi.ctypes.data,
                                (OPT_SUS_STRICT if sus_strict else 0) | (OPT_STEP_GRAPHS if step_graphs else 0),
                                int(device_bytes))
        h = ctypes.c_void_p()
        _check(lib().gfbp_session_create(dcode.handle, ctypes.byref(self.desc), ctypes.byref(h)), "gfbp_session_create")
        self.handle = h
        self.n = dcode.n

    @staticmethod
    def bytes_needed(dcode: DeviceCode, n_slots: int, schedule="pus", markov: bool = False,
                     has_syndrome: bool = False, device_bytes: int = 0) -> int:
        q = dcode.q
        M = np.zeros((q, q), np.float32)
        d = SessionDesc(int(n_slots), SCHEDULES[schedule], 1, int(bool(has_syndrome)),
                        M.ctypes.data if markov else None, M.ctypes.data if markov else None, 0, int(device_bytes))
        return int(lib().gfbp_session_bytes(dcode.handle, ctypes.byref(d)))

    def close(self):
        if getattr(self, "handle", None):
            lib().gfbp_session_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def free_slots(self) -> int:
        return int(lib().gfbp_session_free_slots(self.handle))

    @property
    def running(self) -> int:
        return int(lib().gfbp_session_running(self.handle))

    def admit(self, ids, frames: dict, stream=None) -> int:
        ids = np.ascontiguousarray(ids, dtype=np.int64)
        fr = FramesIn(_dptr(frames["channel"]), _dptr(frames.get("markov")), _dptr(frames.get("param")),
                      _dptr(frames.get("rx")), _dptr(frames.get("erasure")), _dptr(frames.get("y")),
                      _dptr(frames.get("syndrome")))
        k = ctypes.c_int32(0)
        _check(lib().gfbp_session_admit(self.handle, len(ids), ids.ctypes.data, ctypes.byref(fr), ctypes.byref(k),
                                        _stream_ptr(stream)), "gfbp_session_admit")
        return int(k.value)

    def step(self, iters: int = 1, stream=None):
        _check(lib().gfbp_session_step(self.handle, int(iters), _stream_ptr(stream)), "gfbp_session_step")

    @property
    def n_slots(self) -> int:
        return self.free_slots + self.running

    def poll(self, cap: int | None = None, want_xhat: bool = True, stream=None, timestamps: bool = False):
        """Finished frames: (ids int64[k], iters int32[k], converged uint8[k], xhat uint8[k][n] or None)
        and, with timestamps, a fifth item: device clock ticks [k][2] at admission and retirement
        (:func:`device_clock_hz` per second)."""
        cap = int(cap or max(1, self.running))
        out = (Retired * cap)()
        xh = np.zeros((cap, self.n), dtype=np.uint8) if want_xhat else None
        k = ctypes.c_int32(0)
        _check(lib().gfbp_session_poll(self.handle, out, None if xh is None else xh.ctypes.data, cap, ctypes.byref(k),
                                       _stream_ptr(stream)), "gfbp_session_poll")
        k = int(k.value)
        ids = np.array([out[i].id for i in range(k)], dtype=np.int64)
        it = np.array([out[i].iters for i in range(k)], dtype=np.int32)
        cv = np.array([out[i].converged for i in range(k)], dtype=np.uint8)
        if timestamps:
            ts = np.array([(out[i].t_admit, out[i].t_retire) for i in range(k)], dtype=np.uint64).reshape(k, 2)
            return ids, it, cv, (None if xh is None else xh[:k]), ts
        return ids, it, cv, (None if xh is None else xh[:k])


def frames_for_session(frames_list, device="cuda"):
    """Concatenate ``workloads.Frames`` batches (any channels) into the device
    dict that :meth:`Session.admit` takes; frame order is preserved."""
    import torch

    kinds = {"bsc": CH_BSC, "bec": CH_BEC, "biawgn": CH_BIAWGN}
    F = sum(f.F for f in frames_list)
    n = frames_list[0].codeword.shape[1]
    ch = np.concatenate([np.full(f.F, kinds[f.channel], np.uint8) for f in frames_list])
    param = np.concatenate([f.param.astype(np.float32) for f in frames_list])
    need_rx = any(f.rx is not None for f in frames_list)
    need_er = any(f.erasure is not None for f in frames_list)
    need_y = any(f.y is not None for f in frames_list)
    p = None
    for f in frames_list:
        if f.y is not None:
            p = f.y.shape[2]
    rx = np.concatenate([f.rx if f.rx is not None else np.zeros((f.F, n), np.uint8) for f in frames_list]) if need_rx else None
    er = np.concatenate([f.erasure if f.erasure is not None else np.zeros((f.F, n), np.uint8) for f in frames_list]) if need_er else None
    y = np.concatenate([f.y if f.y is not None else np.zeros((f.F, n, p), np.float32) for f in frames_list]) if need_y else None
    dev = lambda a: None if a is None else torch.from_numpy(np.ascontiguousarray(a)).to(device)
    return {"F": F, "channel": dev(ch), "param": dev(param), "rx": dev(rx), "erasure": dev(er), "y": dev(y)}


class Graph:
    """``gfbp_graph_*``: `iters` iterations of several sessions as one HIP graph."""

    def __init__(self, sessions, iters: int, stream):
        arr = (ctypes.c_void_p * len(sessions))(*[x.handle.value for x in sessions])
        h = ctypes.c_void_p()
        _check(lib().gfbp_graph_capture(ctypes.cast(arr, ctypes.c_void_p), len(sessions), int(iters),
                                        ctypes.c_void_p(stream.cuda_stream), ctypes.byref(h)), "gfbp_graph_capture")
        self.handle = h
        self.sessions = list(sessions)
        self.iters = iters

    def launch(self, stream):
        _check(lib().gfbp_graph_launch(self.handle, ctypes.c_void_p(stream.cuda_stream)), "gfbp_graph_launch")

    def close(self):
        if getattr(self, "handle", None):
            lib().gfbp_graph_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
