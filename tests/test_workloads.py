"""The seeded input generators (CPU): codes, encoders, syndrome-form frames,
the mixed pool and the MacKay-Neal (MN) syndrome form of Section 2."""
import numpy as np
import pytest

import oracle
from paper_cs_0605069_amd import workloads as wl


def _dense(code):
    H = np.zeros((code.m, code.n), dtype=np.int64)
    H[code.row_of_edge(), code.col] = code.coef
    return H


def test_regular_code_shape_and_no_four_cycles():
    code = wl.make_code(120, 60, 3, 8, seed=1)
    assert (code.col_degrees() == 3).all() and set(code.row_degrees().tolist()) == {6}
    B = (_dense(code) != 0).astype(np.int64)
    overlap = B @ B.T
    np.fill_diagonal(overlap, 0)
    assert overlap.max() <= 1  # two rows share at most one column


def test_systematic_codewords_satisfy_h():
    code, enc = wl.regular_code(96, 3, 6, 16, seed=2)
    fr = wl.make_frames(code, enc, 20, 3, "bsc", 0.0)
    assert (wl.syndromes(code, fr.codeword) == 0).all()


def test_coset_frames_carry_their_syndrome():
    code, _ = wl.regular_code(96, 3, 6, 4, seed=4)
    fr = wl.make_coset_frames(code, 10, 5, "bec", 0.3)
    assert np.array_equal(wl.syndromes(code, fr.codeword), fr.syndrome)


def test_mixed_pool_shapes():
    pool = wl.mixed_pool(12, seed=6, n_range=(256, 1000), q_weights=[0.35, 0.35, 0.3])
    for c in pool:
        assert c.q in (4, 16, 64) and 256 <= c.n <= 1000
        assert set(np.unique(c.col_degrees()).tolist()) <= {2, 3}
        assert c.meta["rate"] in (1 / 3, 1 / 2) and c.m == round((1 - c.meta["rate"]) * c.n)


@pytest.mark.parametrize("b_form", ["chain", "pool"])
@pytest.mark.parametrize("q", [2, 4, 8])
def test_mn_code_is_a_then_invertible_b(q, b_form):
    N, M = 30, 90
    code = wl.mn_code(N, M, q, seed=7, b_form=b_form, pool=10)
    H = _dense(code)
    A, B = H[:, :N], H[:, N:]
    assert code.n_info == N and (np.count_nonzero(A, axis=0) == 3).all()
    assert (np.triu(B, 1) == 0).all() and (np.diag(B) != 0).all()  # lower triangular, nonzero diagonal
    s = wl.iid_source(5, N, q, seed=8)
    t = wl.mn_encode(code, s)
    # B t = A s, i.e. H (s, t) = 0 ... checked through the syndrome map
    assert (wl.syndromes(code, np.concatenate([s, t], axis=1)) == 0).all()


def _sus_levels(code):
    """Number of dependency levels of a sequential sweep in column order
    (1 + the deepest earlier column sharing a check), by a plain loop."""
    rows_of = [[] for _ in range(code.n)]
    for e, (i, j) in enumerate(zip(code.row_of_edge(), code.col)):
        rows_of[int(j)].append(int(i))
    deepest = np.zeros(code.m, dtype=np.int64)
    top = 0
    for j in range(code.n):
        lv = 1 + max((int(deepest[i]) for i in rows_of[j]), default=0)
        for i in rows_of[j]:
            deepest[i] = max(deepest[i], lv)
        top = max(top, lv)
    return top


def test_mn_pool_form_shape_and_levels():
    """The pooled B: lower triangular with a nonzero diagonal, every noise
    column in two rows of B but the last, rows of B of at most 3 entries, and
    a sequential sweep of far fewer dependency levels than the chain form's
    (whose every noise column depends on the one before)."""
    N, M, q = 300, 900, 4
    chain = wl.mn_code(N, M, q, seed=31)
    pool = wl.mn_code(N, M, q, seed=31, b_form="pool", pool=60)
    B = _dense(pool)[:, N:]
    assert (np.triu(B, 1) == 0).all() and (np.diag(B) != 0).all()
    col_w = np.count_nonzero(B, axis=0)
    assert (col_w[:-1] == 2).all() and col_w[-1] == 1
    assert np.count_nonzero(B, axis=1).max() <= 3
    assert _sus_levels(chain) > M
    assert _sus_levels(pool) < M // 10
    with pytest.raises(ValueError):
        wl.mn_code(N, M, q, seed=31, b_form="other")


@pytest.mark.parametrize("channel,param", [("bsc", 0.1), ("bec", 0.3), ("biawgn", 0.8)])
def test_mn_frames_hold_only_what_the_receiver_has(channel, param):
    """z = H (s, n) = B r, and the channel outputs of the transmitted symbols
    t = B^-1 A s at the noise columns (source columns have none); the noise
    is what separates r from t."""
    q, p = 8, 3
    code = wl.mn_code(20, 60, q, seed=9)
    fr = wl.make_mn_frames(code, 6, 10, channel, param)
    N = 20
    assert fr.evidence == "mn" and fr.lik is None
    assert np.array_equal(wl.syndromes(code, fr.codeword), fr.syndrome)  # z = H (s, n)
    s, noise = fr.codeword[:, :N], fr.codeword[:, N:]
    t = wl.mn_encode(code, s)
    r = fr.rx[:, N:]
    assert (fr.rx[:, :N] == 0).all()
    assert np.array_equal(r ^ t, noise)
    zr = np.concatenate([np.zeros_like(s), r], axis=1)
    assert np.array_equal(wl.syndromes(code, zr), fr.syndrome)  # z = B r
    if channel == "bec":
        er = fr.erasure[:, N:]
        assert (fr.erasure[:, :N] == 0).all()
        assert ((noise & ~er) == 0).all() and ((r & er) == 0).all()  # unerased bits arrive as sent
    if channel == "biawgn":
        assert (fr.y[:, :N] == 0).all()
        assert np.array_equal(r, wl.pack_bits(fr.y[:, N:] < 0))  # hard decisions


def test_mn_bsc_noise_follows_the_papers_noise_prior():
    """The generator's BSC noise symbols have the distribution
    f^L (1-f)^(p-L) of Section 2 (L = ones in the symbol): empirical
    frequencies within five binomial standard deviations."""
    q, p, f = 8, 3, 0.17
    code = wl.mn_code(30, 90, q, seed=19)
    fr = wl.make_mn_frames(code, 400, 20, "bsc", f)
    noise = fr.codeword[:, 30:].ravel()
    emp = np.bincount(noise, minlength=q) / noise.size
    L = np.array([bin(a).count("1") for a in range(q)])
    want = f ** L * (1 - f) ** (p - L)
    assert (np.abs(emp - want) <= 5 * np.sqrt(want * (1 - want) / noise.size)).all()


def test_lifted_binary_chain():
    Mq, start = wl.lift_binary_chain(wl.PAPER_MARKOV_2S, 3)
    assert np.allclose(Mq.sum(axis=1), 1.0) and np.isclose(start.sum(), 1.0)
    assert np.allclose(start @ Mq, start)  # the start distribution is stationary
    # symbols of a long 2-state bit chain, grouped 3 bits at a time (bit b sent b-th)
    rng = np.random.default_rng(11)
    T = 3 * 60000
    bits = np.zeros(T, dtype=np.int64)
    u = rng.random(T)
    for k in range(1, T):
        bits[k] = bits[k - 1] ^ int(u[k] < wl.PAPER_MARKOV_2S[bits[k - 1], 1 - bits[k - 1]])
    sym = bits[0::3] | (bits[1::3] << 1) | (bits[2::3] << 2)
    emp = np.zeros((8, 8))
    np.add.at(emp, (sym[:-1], sym[1:]), 1.0)
    nrow = emp.sum(axis=1, keepdims=True)
    emp /= nrow
    tol = 5.0 * np.sqrt(Mq * (1 - Mq) / nrow) + 1e-3  # five binomial standard deviations
    assert (np.abs(emp - Mq) <= tol).all()


def test_mn_frames_decode_at_low_noise():
    q = 4
    code = wl.mn_code(40, 120, q, seed=12)
    M = wl.PAPER_MARKOV_4S
    fr = wl.make_mn_frames(code, 8, 13, "bsc", 0.02, source="markov", markov=M)
    for sch in (oracle.PUS, oracle.SUS):
        out = oracle.decode(code, fr, schedule=sch, max_iter=50, prior="markov", markov_M=M,
                            markov_pi=wl.stationary(M))
        assert out["converged"].all() and (out["xhat"] == fr.codeword).all()


def test_sigma_from_ebn0_closed_form():
    """sigma^2 = 1 / (2 R 10^(Eb/N0 / 10)): the benchmark's five points at R = 1/2."""
    got = [round(wl.sigma_from_ebn0(e, 0.5), 3) for e in (0.8, 1.0, 1.2, 1.4, 1.6)]
    assert got == [0.912, 0.891, 0.871, 0.851, 0.832]
    assert wl.sigma_from_ebn0(0.0, 0.5) == 1.0


@pytest.mark.parametrize("rate,limit_db", [(1 / 2, 0.187), (1 / 3, -0.495)])
def test_biawgn_capacity_at_the_bpsk_shannon_limits(rate, limit_db):
    """The BPSK-input AWGN channel's capacity equals the code rate at the
    textbook Shannon limits (Eb/N0 = 0.187 dB for R = 1/2, -0.495 dB for
    R = 1/3), and tends to 1 and 0 at the extremes."""
    assert abs(wl.biawgn_capacity(wl.sigma_from_ebn0(limit_db, rate)) - rate) < 2e-3
    assert wl.biawgn_capacity(0.2) > 0.9999 and wl.biawgn_capacity(20.0) < 0.01


def test_capacity_matched_channel_parameters():
    """R20: BSC and BEC parameters with the BI-AWGN capacity at the frame's sigma."""
    for e in (1.0, 1.5, 2.0):
        for R in (1 / 3, 1 / 2):
            C = wl.biawgn_capacity(wl.sigma_from_ebn0(e, R))
            f = wl.channel_for("bsc", e, R)
            assert 0 < f < 0.5 and abs(1 - wl.h2(f) - C) < 1e-9
            assert abs(wl.channel_for("bec", e, R) - (1 - C)) < 1e-12
            assert wl.channel_for("biawgn", e, R) == wl.sigma_from_ebn0(e, R)
