"""Values the paper prints (fixtures under tests/golden/, each citing its
place in the paper) against the workload generator and the Table-1 runner."""
import math
import os

import numpy as np

from paper_cs_0605069_amd import workloads as wl

HERE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _rows(name):
    with open(os.path.join(HERE, name)) as f:
        return [line.split() for line in f if line.strip() and not line.startswith("#")]


def _markov(tag):
    return np.array([[float(x) for x in r[1:]] for r in _rows("paper_markov_sources.txt") if r[0] == tag])


def _entropy_rate(M):
    """Bits per step of a stationary Markov chain: sum_a pi(a) H(M(a, .))."""
    pi = wl.stationary(M)
    logs = np.log2(np.where(M > 0, M, 1.0))
    return float(-(pi[:, None] * M * logs).sum())


def test_markov_sources_are_the_printed_matrices():
    assert np.array_equal(wl.PAPER_MARKOV_2S, _markov("2S"))
    assert np.array_equal(wl.PAPER_MARKOV_4S_RAW, _markov("4S"))
    # the printed 4S rows sum to 1 only to within ~5e-7; the generator renormalises them
    assert np.abs(_markov("4S").sum(axis=1) - 1).max() <= 6e-7
    assert np.allclose(wl.PAPER_MARKOV_4S.sum(axis=1), 1.0, atol=1e-15)


def test_markov_sources_have_the_stated_entropy():
    """The paper gives both sources entropy 1/2 per transmitted bit: the 2S
    chain (h2(0.11)) exactly to print precision, the 4S chain approximately."""
    h2 = lambda p: -p * math.log2(p) - (1 - p) * math.log2(1 - p)
    assert abs(_entropy_rate(_markov("2S")) - h2(0.11)) < 1e-12
    assert abs(_entropy_rate(_markov("2S")) - 0.5) < 1e-3
    assert 0.45 < _entropy_rate(wl.PAPER_MARKOV_4S) / 2 < 0.5


def test_lifted_2s_chain_keeps_the_bit_entropy():
    """Grouping p consecutive bits of the 2S chain into a GF(2^p) symbol
    changes nothing about the bit process: the symbol chain's entropy rate is
    p times the bit chain's."""
    for p in (1, 2, 3):
        Mq, start = wl.lift_binary_chain(_markov("2S"), p)
        assert abs(_entropy_rate(Mq) - p * _entropy_rate(_markov("2S"))) < 1e-12


def test_table1_settings_are_the_printed_rows():
    from paper_cs_0605069_amd import table1

    rows = _rows("paper_table1.txt")
    assert len(rows) == 9 == len(table1.SETTINGS)
    for r, (channel, q, source, noise) in zip(rows, table1.SETTINGS):
        assert (r[0], int(r[1]), r[2], float(r[3])) == (channel, q, source, noise)
        t_sus, t_pus, ratio = float(r[4]), float(r[5]), float(r[6])
        assert abs(t_sus / t_pus - ratio) < 2e-3  # the fixture's ratio column matches its means
