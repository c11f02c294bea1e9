"""Seeded synthetic workloads for LDPC decoding over GF(2^p).

This module only *generates inputs*: random sparse parity-check matrices,
codewords whose information symbols follow an i.i.d. or first-order Markov
source, and their images through the binary symmetric, binary erasure and
binary-input AWGN channels.  It holds none of the decoder's arithmetic and is
shared, as the single source of inputs, by the decoder library's tests and
benchmarks and by the reference decoder's tests.

Conventions (Section 2 of the paper: symbols of GF(q) are sent as their binary
representation, and channel noise is added bitwise):

* GF(2^p) is taken in the polynomial basis of a fixed primitive polynomial
  (``DEFAULT_POLY``); bit b of a symbol is the coefficient of x^b and is
  transmitted b-th (least significant bit first).
* BPSK maps bit 0 to +1 and bit 1 to -1; sigma is the noise standard deviation.
* After :func:`systematic` the columns are ordered [information | parity] so
  that the information symbols are columns 0..K-1 in source order.

All randomness comes from ``numpy.random.default_rng([seed, stream])`` with a
distinct stream number per purpose, drawn with the frame index as the leading
array axis, so frame f of a workload does not depend on how many frames are
generated after it.
"""
from __future__ import annotations

import ctypes
import math
import os
from dataclasses import dataclass, field

import numpy as np

DEFAULT_POLY = {1: 0b11, 2: 0b111, 3: 0b1011, 4: 0b10011, 5: 0b100101, 6: 0b1000011}

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIBNAME = "libgfsynth.so"

# Markov transition matrices printed in the paper's results section (footnote
# to Table 1): the 2-state matrix, and the 4-state matrix whose rows sum to 1
# only to about 5e-7 (they are renormalised in double precision).
PAPER_MARKOV_2S = np.array([[0.89, 0.11], [0.11, 0.89]], dtype=np.float64)
PAPER_MARKOV_4S_RAW = np.array(
    [
        [0.808022, 0.0883281, 0.0130689, 0.0905813],
        [0.128676, 0.0514706, 0.0772059, 0.742647],
        [0.755814, 0.108527, 0.0116279, 0.124031],
        [0.866667, 0.0151111, 0.091556, 0.0266659],
    ],
    dtype=np.float64,
)
PAPER_MARKOV_4S = PAPER_MARKOV_4S_RAW / PAPER_MARKOV_4S_RAW.sum(axis=1, keepdims=True)


# --------------------------------------------------------------------------
# native encoder
# --------------------------------------------------------------------------
_lib = None


# Directory of a sanitizer-instrumented build of the host libraries (set by
# the sanitizer test for the process it starts); unset: the in-tree build.
SANITIZED_DIR_ENV = "GFBP_SANITIZED_DIR"
SANITIZE_FLAGS = ["-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
                  "-fno-sanitize-recover=all"]


def _load():
    global _lib
    if _lib is not None:
        return _lib
    path = os.path.join(os.environ.get(SANITIZED_DIR_ENV) or _HERE, _LIBNAME)
    if not os.path.exists(path):
        raise RuntimeError(
            f"{path} is missing: build it first (python -c 'import __graft_entry__ as g; g.build()')"
        )
    lib = ctypes.CDLL(path)
    lib.synth_encoder_build.restype = ctypes.c_void_p
    lib.synth_encoder_build.argtypes = [
        ctypes.c_int, ctypes.c_uint, ctypes.c_int, ctypes.c_int,
        ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
    ]
    lib.synth_encoder_info.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
    lib.synth_encoder_encode.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p]
    lib.synth_encoder_free.argtypes = [ctypes.c_void_p]
    _lib = lib
    return lib


def build_native(verbose: bool = False, out_dir: str | None = None, sanitize: bool = False) -> str:
    """Compile the encoder helper with gcc into this directory (or out_dir;
    sanitize: with the address and undefined-behaviour sanitizers)."""
    import subprocess

    src = os.path.join(_HERE, "_encoder.c")
    out = os.path.join(out_dir or _HERE, _LIBNAME)
    tmp = out + ".tmp"
    cmd = ["gcc", *(SANITIZE_FLAGS if sanitize else ["-O2"]), "-fPIC", "-shared", "-o", tmp, src]
    if verbose:
        print(" ".join(cmd))
    subprocess.check_call(cmd)
    os.replace(tmp, out)
    return out


# --------------------------------------------------------------------------
# codes
# --------------------------------------------------------------------------
@dataclass
class Code:
    """A parity-check matrix H over GF(q) in compressed-row form.

    Edges (nonzeros of H) are numbered row by row; within a row by increasing
    column.  ``n_info`` columns 0..n_info-1 are information symbols when the
    code came from :func:`systematic`.
    """

    q: int
    n: int
    m: int
    row_ptr: np.ndarray  # int32 [m+1]
    col: np.ndarray  # int32 [E]
    coef: np.ndarray  # uint8 [E]
    poly: int = 0
    n_info: int = 0
    seed: int = 0
    meta: dict = field(default_factory=dict)
    visit_order: np.ndarray | None = None  # int32 [n]: SUS visiting order (None: 0..n-1)
    source_cols: np.ndarray | None = None  # int32 [n_info]: source chain's columns (None: 0..n_info-1)

    def __post_init__(self):
        if self.poly == 0:
            self.poly = DEFAULT_POLY[self.p]

    @property
    def p(self) -> int:
        return int(round(math.log2(self.q)))

    @property
    def E(self) -> int:
        return int(self.row_ptr[-1])

    def row_of_edge(self) -> np.ndarray:
        return np.repeat(np.arange(self.m, dtype=np.int32), np.diff(self.row_ptr))

    def dense(self) -> np.ndarray:
        H = np.zeros((self.m, self.n), dtype=np.uint8)
        H[self.row_of_edge(), self.col] = self.coef
        return H

    def col_degrees(self) -> np.ndarray:
        return np.bincount(self.col, minlength=self.n)

    def row_degrees(self) -> np.ndarray:
        return np.diff(self.row_ptr)


def _four_cycle_edges(var: np.ndarray, chk: np.ndarray, n: int, m: int) -> np.ndarray:
    """Indices of edges to move so that no two checks share two variables and
    no (check, variable) pair repeats.  ``var``/``chk`` list the edges."""
    order = np.lexsort((chk, var))
    v_s, c_s = var[order], chk[order]
    starts = np.searchsorted(v_s, np.arange(n))
    ends = np.searchsorted(v_s, np.arange(n), side="right")
    deg = ends - starts
    bad = []
    # multi-edges: consecutive equal (var, chk)
    dup = np.nonzero((v_s[1:] == v_s[:-1]) & (c_s[1:] == c_s[:-1]))[0]
    bad.extend(order[dup + 1].tolist())
    # 4-cycles: pairs of checks of a variable repeated across variables
    keys, owner = [], []
    dmax = int(deg.max()) if n else 0
    for a in range(dmax):
        for b in range(a + 1, dmax):
            ok = deg > b
            vi = np.nonzero(ok)[0]
            ca = c_s[starts[vi] + a]
            cb = c_s[starts[vi] + b]
            keys.append(ca.astype(np.int64) * m + cb)
            owner.append(order[starts[vi] + b])
    if keys:
        keys = np.concatenate(keys)
        owner = np.concatenate(owner)
        srt = np.argsort(keys, kind="stable")
        k_s = keys[srt]
        rep = np.nonzero(k_s[1:] == k_s[:-1])[0]
        bad.extend(owner[srt[rep + 1]].tolist())
    return np.unique(np.asarray(bad, dtype=np.int64))


def make_code(n: int, m: int, d_v: int, q: int, seed: int, reject_4cycles: bool = True,
              max_rounds: int = 20000) -> Code:
    """Random column-regular code: every column has weight ``d_v``; row weights
    are as equal as possible (floor/ceil of n*d_v/m).  Configuration model,
    then random edge swaps until there are no repeated edges (and, if asked, no
    4-cycles).  Nonzero coefficients are uniform on GF(q) minus {0}."""
    rng = np.random.default_rng([seed, 0xC0DE])
    E = n * d_v
    base, extra = divmod(E, m)
    rdeg = np.full(m, base, dtype=np.int64)
    rdeg[rng.permutation(m)[:extra]] += 1
    var = np.repeat(np.arange(n, dtype=np.int64), d_v)
    chk = np.repeat(np.arange(m, dtype=np.int64), rdeg)[rng.permutation(E)]
    for _ in range(max_rounds):
        if reject_4cycles:
            bad = _four_cycle_edges(var, chk, n, m)
        else:
            order = np.lexsort((chk, var))
            dup = np.nonzero((var[order][1:] == var[order][:-1]) & (chk[order][1:] == chk[order][:-1]))[0]
            bad = order[dup + 1]
        if len(bad) == 0:
            break
        partners = rng.integers(0, E, size=len(bad))
        for e1, e2 in zip(bad.tolist(), partners.tolist()):
            chk[e1], chk[e2] = chk[e2], chk[e1]
    else:
        raise RuntimeError("code construction did not converge; relax the constraints")
    order = np.lexsort((var, chk))
    chk, var = chk[order], var[order]
    row_ptr = np.zeros(m + 1, dtype=np.int32)
    row_ptr[1:] = np.cumsum(np.bincount(chk, minlength=m))
    coef = rng.integers(1, q, size=E).astype(np.uint8)
    return Code(q=q, n=n, m=m, row_ptr=row_ptr, col=var.astype(np.int32), coef=coef, seed=seed,
                meta={"d_v": d_v, "reject_4cycles": reject_4cycles})


class Encoder:
    """Systematic encoder of a code whose columns are [information | parity]."""

    def __init__(self, handle, n_info: int, rank: int, p: int):
        self._h = handle
        self.n_info = n_info
        self.rank = rank
        self.p = p

    def __del__(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.synth_encoder_free(self._h)
            self._h = None

    def encode(self, s: np.ndarray) -> np.ndarray:
        """Codewords [F][n] (information symbols first) for sources s [F][K]."""
        s = np.ascontiguousarray(s, dtype=np.uint8)
        F = s.shape[0]
        assert s.shape[1] == self.n_info
        par = np.zeros((F, self.rank), dtype=np.uint8)
        _load().synth_encoder_encode(self._h, F, s.ctypes.data, par.ctypes.data)
        return np.concatenate([s, par], axis=1)


def systematic(code: Code) -> tuple[Code, Encoder]:
    """Permute the columns of ``code`` to [information | parity] (keeping the
    relative order inside each part) and return it with its encoder."""
    lib = _load()
    order = np.zeros(code.n, dtype=np.int32)
    rp = np.ascontiguousarray(code.row_ptr, dtype=np.int32)
    cl = np.ascontiguousarray(code.col, dtype=np.int32)
    cf = np.ascontiguousarray(code.coef, dtype=np.uint8)
    h = lib.synth_encoder_build(code.p, code.poly, code.m, code.n, rp.ctypes.data, cl.ctypes.data,
                                cf.ctypes.data, order.ctypes.data)
    if not h:
        raise RuntimeError("encoder construction failed")
    k = ctypes.c_int32()
    r = ctypes.c_int32()
    lib.synth_encoder_info(h, ctypes.byref(k), ctypes.byref(r))
    newpos = np.empty(code.n, dtype=np.int32)
    newpos[order] = np.arange(code.n, dtype=np.int32)
    col = newpos[code.col]
    # re-sort edges inside each row by the new column index
    row = code.row_of_edge()
    srt = np.lexsort((col, row))
    out = Code(q=code.q, n=code.n, m=code.m, row_ptr=code.row_ptr.copy(), col=col[srt].astype(np.int32),
               coef=code.coef[srt].copy(), poly=code.poly, n_info=int(k.value), seed=code.seed,
               meta=dict(code.meta, rank=int(r.value)))
    return out, Encoder(h, int(k.value), int(r.value), code.p)


def regular_code(n: int, d_v: int, d_c: int, q: int, seed: int) -> tuple[Code, Encoder]:
    """Systematic (d_v, d_c)-regular code with no 4-cycles."""
    assert (n * d_v) % d_c == 0
    return systematic(make_code(n, n * d_v // d_c, d_v, q, seed))


# --------------------------------------------------------------------------
# sources and channels
# --------------------------------------------------------------------------
def self_transition_matrix(q: int, stay: float) -> np.ndarray:
    M = np.full((q, q), (1.0 - stay) / (q - 1), dtype=np.float64)
    np.fill_diagonal(M, stay)
    return M


def stationary(M: np.ndarray) -> np.ndarray:
    w, v = np.linalg.eig(M.T)
    i = int(np.argmin(np.abs(w - 1.0)))
    pi = np.real(v[:, i])
    pi = np.abs(pi) / np.abs(pi).sum()
    return pi


def iid_source(F: int, K: int, q: int, seed: int) -> np.ndarray:
    rng = np.random.default_rng([seed, 1])
    return rng.integers(0, q, size=(F, K)).astype(np.uint8)


def markov_source(F: int, K: int, M: np.ndarray, pi: np.ndarray, seed: int) -> np.ndarray:
    """First-order Markov chain: s_0 ~ pi, s_k | s_{k-1}=a ~ M[a, :]."""
    rng = np.random.default_rng([seed, 1])
    u = rng.random((F, K))
    cumM = np.cumsum(M, axis=1)
    cumM[:, -1] = 1.0
    cumpi = np.cumsum(pi)
    cumpi[-1] = 1.0
    s = np.zeros((F, K), dtype=np.int64)
    if K == 0:
        return s.astype(np.uint8)
    s[:, 0] = np.searchsorted(cumpi, u[:, 0], side="right")
    for k in range(1, K):
        rows = cumM[s[:, k - 1]]
        s[:, k] = (u[:, k:k + 1] >= rows).sum(axis=1)
    return np.minimum(s, M.shape[0] - 1).astype(np.uint8)


def symbol_bits(c: np.ndarray, p: int) -> np.ndarray:
    """[..., n] symbols -> [..., n, p] bits (bit b = coefficient of x^b)."""
    return ((c[..., None].astype(np.int64) >> np.arange(p)) & 1).astype(np.uint8)


def pack_bits(bits: np.ndarray) -> np.ndarray:
    p = bits.shape[-1]
    return (bits.astype(np.int64) << np.arange(p)).sum(axis=-1).astype(np.uint8)


def bsc(c: np.ndarray, p: int, f, seed: int) -> np.ndarray:
    """Received symbols: each bit flipped independently with probability f."""
    rng = np.random.default_rng([seed, 2])
    f = np.broadcast_to(np.asarray(f, dtype=np.float64).reshape(-1, 1, 1), (c.shape[0], 1, 1))
    flips = rng.random(c.shape + (p,)) < f
    return (c ^ pack_bits(flips)).astype(np.uint8)


def bec(c: np.ndarray, p: int, eps, seed: int) -> tuple[np.ndarray, np.ndarray]:
    """(received symbols with erased bits set to 0, erased-bit masks)."""
    rng = np.random.default_rng([seed, 2])
    eps = np.broadcast_to(np.asarray(eps, dtype=np.float64).reshape(-1, 1, 1), (c.shape[0], 1, 1))
    er = pack_bits(rng.random(c.shape + (p,)) < eps)
    return (c & ~er).astype(np.uint8), er.astype(np.uint8)


def biawgn(c: np.ndarray, p: int, sigma, seed: int) -> np.ndarray:
    """y = (1 - 2 bit) + sigma * n, float32 [F][n][p]."""
    rng = np.random.default_rng([seed, 2])
    sigma = np.broadcast_to(np.asarray(sigma, dtype=np.float64).reshape(-1, 1, 1), (c.shape[0], 1, 1))
    x = 1.0 - 2.0 * symbol_bits(c, p).astype(np.float64)
    return (x + sigma * rng.standard_normal(x.shape)).astype(np.float32)


def sigma_from_ebn0(ebn0_db: float, rate: float) -> float:
    """Noise std for unit-energy BPSK at Eb/N0 (dB) and code rate R:
    sigma^2 = 1 / (2 R 10^(Eb/N0 / 10))."""
    return math.sqrt(1.0 / (2.0 * rate * 10.0 ** (ebn0_db / 10.0)))


def biawgn_capacity(sigma: float, npts: int = 4001) -> float:
    """Capacity (bits/use) of the BPSK-input AWGN channel, by quadrature."""
    y = np.linspace(-1.0 - 12 * sigma, 1.0 + 12 * sigma, npts)
    dy = y[1] - y[0]
    g = lambda m: np.exp(-((y - m) ** 2) / (2 * sigma * sigma)) / math.sqrt(2 * math.pi * sigma * sigma)
    p0, p1 = g(1.0), g(-1.0)
    py = 0.5 * (p0 + p1)
    with np.errstate(divide="ignore", invalid="ignore"):
        t0 = np.where(p0 > 0, p0 * np.log2(p0 / py), 0.0)
    return float(np.sum(t0) * dy)


def h2(x: float) -> float:
    if x <= 0 or x >= 1:
        return 0.0
    return -x * math.log2(x) - (1 - x) * math.log2(1 - x)


def bsc_matching(cap: float) -> float:
    """Crossover f with 1 - h2(f) = cap (0 <= f <= 1/2)."""
    lo, hi = 0.0, 0.5
    for _ in range(80):
        mid = 0.5 * (lo + hi)
        if 1 - h2(mid) > cap:
            lo = mid
        else:
            hi = mid
    return 0.5 * (lo + hi)


@dataclass
class Frames:
    """One batch of received frames for one code and one channel kind."""

    channel: str  # "bsc" | "bec" | "biawgn"
    param: np.ndarray  # float64 [F]: f, eps or sigma
    codeword: np.ndarray  # uint8 [F][n]
    rx: np.ndarray | None = None  # uint8 [F][n]
    erasure: np.ndarray | None = None  # uint8 [F][n]
    y: np.ndarray | None = None  # float32 [F][n][p]
    syndrome: np.ndarray | None = None  # uint8 [F][m] (None means z = 0)
    lik: np.ndarray | None = None  # float32 [F][n][q] per-symbol likelihoods (channel "likelihood")
    # "symbol": the channel output at column j is about symbol x_j; "mn": the
    # MacKay-Neal syndrome form, where the output at a noise column j is the
    # received bit pattern of a transmitted symbol whose noise is x_j, and
    # source columns carry no channel output (their entries are 0)
    evidence: str = "symbol"

    @property
    def F(self) -> int:
        return int(self.codeword.shape[0])

    def subset(self, idx) -> "Frames":
        g = lambda a: None if a is None else np.ascontiguousarray(a[idx])
        return Frames(self.channel, self.param[idx].copy(), g(self.codeword), g(self.rx), g(self.erasure),
                      g(self.y), g(self.syndrome), g(self.lik), self.evidence)


def make_frames(code: Code, enc: Encoder, F: int, seed: int, channel: str, param,
                source: str = "iid", markov: np.ndarray | None = None,
                pi: np.ndarray | None = None) -> Frames:
    """Encode F source blocks and pass them through the channel."""
    K = code.n_info
    if source == "iid":
        s = iid_source(F, K, code.q, seed)
    elif source == "markov":
        assert markov is not None
        s = markov_source(F, K, markov, stationary(markov) if pi is None else pi, seed)
    elif source == "zero":
        s = np.zeros((F, K), dtype=np.uint8)
    else:
        raise ValueError(source)
    c = enc.encode(s)
    prm = np.broadcast_to(np.asarray(param, dtype=np.float64), (F,)).copy()
    p = code.p
    if channel == "bsc":
        return Frames("bsc", prm, c, rx=bsc(c, p, prm, seed))
    if channel == "bec":
        rx, er = bec(c, p, prm, seed)
        return Frames("bec", prm, c, rx=rx, erasure=er)
    if channel == "biawgn":
        return Frames("biawgn", prm, c, y=biawgn(c, p, prm, seed))
    raise ValueError(channel)


# --------------------------------------------------------------------------
# syndrome-form frames and the mixed-shape pool
# --------------------------------------------------------------------------
def gf_mul_table(p: int, poly: int | None = None) -> np.ndarray:
    """[q][q] products in GF(2^p) (carry-less multiplication, reduced)."""
    poly = DEFAULT_POLY[p] if poly is None else poly
    q = 1 << p
    a = np.arange(q, dtype=np.int64)[:, None]
    b = np.arange(q, dtype=np.int64)[None, :]
    r = np.zeros((q, q), dtype=np.int64)
    for i in range(p):
        r ^= np.where((b >> i) & 1, a << i, 0)
    for d in range(2 * p - 2, p - 1, -1):
        r = np.where((r >> d) & 1, r ^ (poly << (d - p)), r)
    return r.astype(np.uint8)


def syndromes(code: Code, x: np.ndarray) -> np.ndarray:
    """z = H x for every row of x [F][n]."""
    T = gf_mul_table(code.p, code.poly)
    z = np.zeros((x.shape[0], code.m), dtype=np.uint8)
    deg = np.diff(code.row_ptr)
    rows = np.nonzero(deg > 0)[0]
    if len(rows) == 0:
        return z
    for f0 in range(0, x.shape[0], 256):
        prod = T[code.coef[None, :], x[f0:f0 + 256][:, code.col]]  # [F][E], edges grouped by row
        z[f0:f0 + 256, rows] = np.bitwise_xor.reduceat(prod, code.row_ptr[rows], axis=1)
    return z


def make_coset_frames(code: Code, F: int, seed: int, channel: str, param, source: str = "iid",
                      markov: np.ndarray | None = None) -> Frames:
    """Syndrome-form frames (the paper's Eq. (2) setting): x has source
    symbols in columns 0..n_info-1 (i.i.d. or Markov) and uniform symbols
    elsewhere; the decoder is given z = H x and the channel output of x."""
    K = code.n_info
    rng = np.random.default_rng([seed, 3])
    x = rng.integers(0, code.q, size=(F, code.n)).astype(np.uint8)
    if source == "markov":
        x[:, :K] = markov_source(F, K, markov, stationary(markov), seed)
    prm = np.broadcast_to(np.asarray(param, dtype=np.float64), (F,)).copy()
    p = code.p
    if channel == "bsc":
        fr = Frames("bsc", prm, x, rx=bsc(x, p, prm, seed))
    elif channel == "bec":
        rx, er = bec(x, p, prm, seed)
        fr = Frames("bec", prm, x, rx=rx, erasure=er)
    elif channel == "biawgn":
        fr = Frames("biawgn", prm, x, y=biawgn(x, p, prm, seed))
    else:
        raise ValueError(channel)
    fr.syndrome = syndromes(code, x)
    return fr


def channel_for(kind: str, ebn0_db: float, rate: float) -> float:
    """Channel parameter for a frame drawn at Eb/N0 (dB): sigma for BI-AWGN;
    for BSC and BEC the parameter whose capacity equals the BI-AWGN capacity
    at that sigma (1 - h2(f) = C, eps = 1 - C)."""
    sigma = sigma_from_ebn0(ebn0_db, rate)
    if kind == "biawgn":
        return sigma
    cap = biawgn_capacity(sigma)
    return bsc_matching(cap) if kind == "bsc" else 1.0 - cap


def mixed_pool(n_codes: int, seed: int, qs=(4, 16, 64), n_range=(256, 8000), q_weights=None) -> list[Code]:
    """Codes for uneven batches: q from qs (optionally weighted), column weight
    2 or 3, rate 1/3 or 1/2, n uniform in n_range (even), m = round((1-R) n),
    row degrees balanced; n_info = n - m (source columns first)."""
    rng = np.random.default_rng([seed, 7])
    out = []
    for k in range(n_codes):
        q = int(rng.choice(qs, p=q_weights))
        dv = int(rng.choice([2, 3]))
        R = float(rng.choice([1 / 3, 1 / 2]))
        n = int(rng.integers(n_range[0] // 2, n_range[1] // 2 + 1)) * 2
        m = int(round((1 - R) * n))
        c = make_code(n, m, dv, q, seed=seed * 1000 + k)
        c.n_info = n - m
        c.meta.update(rate=R, d_v=dv)
        out.append(c)
    return out


# --------------------------------------------------------------------------
# MacKay-Neal syndrome form (Section 2): H = [A | B], x = (source, noise)
# --------------------------------------------------------------------------
def mn_code(N: int, M: int, q: int, seed: int, d_a: int = 3, extra: float = 0.5, b_form: str = "chain",
            pool: int = 1000) -> Code:
    """H = [A | B] over GF(q): A (M x N) with column weight d_a (rows balanced,
    no repeated edge, no 4-cycle inside A), B (M x M) lower triangular with a
    nonzero diagonal, hence invertible.  Columns 0..N-1 of H are the source
    symbols (n_info = N), columns N..N+M-1 the noise symbols.  Nonzero
    coefficients are uniform on GF(q) minus {0}.  B's form:

    * "chain": row i holds columns i and i-1 and, with probability `extra`,
      one random earlier column that has no such extra entry yet (a column
      of B has at most 3 entries).  Every noise column then shares a check
      with the previous one, so a sequential sweep's dependency levels
      number about M.
    * "pool": each column's second entry sits in a random later row: from
      row `pool` on, every row takes one random column from the columns
      still waiting (two per row once fewer rows than waiting columns
      remain), so each column of B has 2 entries (a few at the end 1) and
      each row at most 3.  Columns then wait about `pool` rows, and a
      sequential sweep's dependency levels number about M / pool plus a few.

    Both stand in for the paper's Kanter-Saad construction, which it does not
    specify."""
    if b_form not in ("chain", "pool"):
        raise ValueError(f"b_form {b_form!r}")
    A = make_code(N, M, d_a, q, seed)
    rng = np.random.default_rng([seed, 0xB])
    br, bc = [], []
    avail = []  # chain: columns < i-1 without an extra entry; pool: columns waiting for their second entry
    for i in range(M):
        br.append(i)
        bc.append(N + i)
        if b_form == "pool":
            if i >= 1:
                avail.append(i - 1)
            take = 2 if len(avail) > M - i else (1 if i >= pool else 0)
            for _ in range(min(take, len(avail))):
                k = int(rng.integers(0, len(avail)))
                avail[k], avail[-1] = avail[-1], avail[k]
                br.append(i)
                bc.append(N + avail.pop())
            continue
        if i >= 2:
            avail.append(i - 2)
        if i >= 1:
            br.append(i)
            bc.append(N + i - 1)
        if avail and rng.random() < extra:
            k = int(rng.integers(0, len(avail)))
            avail[k], avail[-1] = avail[-1], avail[k]
            br.append(i)
            bc.append(N + avail.pop())
    r = np.concatenate([A.row_of_edge(), np.array(br, dtype=np.int64)])
    c = np.concatenate([A.col.astype(np.int64), np.array(bc, dtype=np.int64)])
    h = np.concatenate([A.coef, rng.integers(1, q, size=len(br)).astype(np.uint8)])
    order = np.lexsort((c, r))
    row_ptr = np.zeros(M + 1, dtype=np.int32)
    row_ptr[1:] = np.cumsum(np.bincount(r, minlength=M))
    return Code(q=q, n=N + M, m=M, row_ptr=row_ptr, col=c[order].astype(np.int32), coef=h[order], n_info=N,
                seed=seed, meta={"mn": True, "N": N, "M": M, "d_a": d_a, "extra": extra, "b_form": b_form,
                                 "pool": pool})


def mn_encode(code: Code, s: np.ndarray) -> np.ndarray:
    """t = B^-1 A s for sources s [F][N] (Eq. (1)), by forward substitution
    (B is lower triangular with a nonzero diagonal)."""
    N, M, q = code.meta["N"], code.meta["M"], code.q
    T = gf_mul_table(code.p, code.poly)
    inv = np.zeros(q, dtype=np.uint8)
    for a in range(1, q):
        inv[a] = int(np.nonzero(T[a] == 1)[0][0])
    F = s.shape[0]
    t = np.zeros((F, M), dtype=np.uint8)
    for i in range(M):
        acc = np.zeros(F, dtype=np.uint8)
        diag = 0
        for e in range(code.row_ptr[i], code.row_ptr[i + 1]):
            j, h = int(code.col[e]), int(code.coef[e])
            if j < N:
                acc ^= T[h, s[:, j]]
            elif j - N < i:
                acc ^= T[h, t[:, j - N]]
            else:
                diag = h
        t[:, i] = T[inv[diag], acc]
    return t


def lift_binary_chain(M2: np.ndarray, p: int) -> tuple[np.ndarray, np.ndarray]:
    """Symbol-level chain (q x q transition matrix, start distribution) of a
    2-state chain over bits grouped into p-bit symbols, bit b of a symbol
    being the b-th bit sent: P(b | a) = M2[a_{p-1}, b_0] prod_k M2[b_{k-1}, b_k]."""
    q = 1 << p
    pi2 = stationary(M2)
    Mq = np.zeros((q, q))
    start = np.zeros(q)
    for b in range(q):
        inner = 1.0
        for k in range(1, p):
            inner *= M2[(b >> (k - 1)) & 1, (b >> k) & 1]
        start[b] = pi2[b & 1] * inner
        for a in range(q):
            Mq[a, b] = M2[(a >> (p - 1)) & 1, b & 1] * inner
    return Mq, start


def make_mn_frames(code: Code, F: int, seed: int, channel: str, param, source: str = "iid",
                   markov: np.ndarray | None = None, start: np.ndarray | None = None) -> Frames:
    """Frames of the MN syndrome form (Section 2, Eqs. (1)-(2)): sources s
    [F][N] (i.i.d. uniform or a Markov chain with transition matrix `markov`
    from `start`), t = B^-1 A s sent over the channel, r the received word
    (hard decisions for BI-AWGN, erased bits read as 0 for the BEC), and
    z = B r = A s + B n with n = r - t.  The frames hold only what the
    receiver has: z and the channel outputs, placed at the noise columns
    N..N+M-1 (rx = r, erasure masks, y); source columns have no channel output
    and hold zeros.  Turning the outputs into evidence about the noise symbols
    is the decoder's work (``evidence = "mn"``).  `codeword` holds the true
    x = (s, n)."""
    N, M, q, p = code.meta["N"], code.meta["M"], code.q, code.p
    if source == "iid":
        s = iid_source(F, N, q, seed)
    else:
        s = markov_source(F, N, markov, stationary(markov) if start is None else start, seed)
    t = mn_encode(code, s)
    prm = np.broadcast_to(np.asarray(param, dtype=np.float64), (F,)).copy()
    rx = np.zeros((F, N + M), dtype=np.uint8)
    er = y = None
    if channel == "bsc":
        r = bsc(t, p, prm, seed)
    elif channel == "bec":
        r, e = bec(t, p, prm, seed)
        er = np.zeros((F, N + M), dtype=np.uint8)
        er[:, N:] = e
    elif channel == "biawgn":
        yt = biawgn(t, p, prm, seed)
        r = pack_bits(yt < 0)
        y = np.zeros((F, N + M, p), dtype=np.float32)
        y[:, N:] = yt
    else:
        raise ValueError(channel)
    r = r.astype(np.uint8)
    rx[:, N:] = r
    n = (r ^ t).astype(np.uint8)
    x = np.concatenate([s, n], axis=1)
    z = syndromes(code, np.concatenate([np.zeros_like(s), r], axis=1))
    fr = Frames(channel, prm, x, rx=rx, erasure=er, y=y, evidence="mn")
    fr.syndrome = z
    return fr
