"""Pins of the oracle's counter-based generator and stream layout."""
import os

import numpy as np
import pytest

import oracle

GOLD = os.path.join(os.path.dirname(__file__), "golden", "philox4x32_10_kat.txt")


def _kat():
    rows = []
    for line in open(GOLD):
        if line.startswith("#") or not line.strip():
            continue
        v = [int(x, 16) for x in line.split()]
        rows.append((v[0:4], v[4:6], v[6:10]))
    return rows


@pytest.mark.parametrize("ctr,key,out", _kat())
def test_philox_known_answers(ctr, key, out):
    assert oracle.philox(ctr, key) == out


def test_stream_block_layout():
    # key = (lo32(seed), hi32(seed)); counter = (block, tag, lo32(id), hi32(id))
    seed = 0x0123456789ABCDEF
    eid = 0xFEDCBA9876543210
    got = oracle.stream_block(seed, eid, 3, 77)
    want = oracle.philox([77, 3, eid & 0xffffffff, eid >> 32], [seed & 0xffffffff, seed >> 32])
    assert got == want


def test_uniform53_bits():
    assert oracle.uniform53(0, 0) == 0.0
    top = oracle.uniform53(0xffffffff, 0xffffffff)
    assert top == (2 ** 53 - 1) / 2 ** 53 and top < 1.0
    rng = np.random.default_rng(1)
    for hi, lo in rng.integers(0, 2 ** 32, size=(200, 2)):
        u = oracle.uniform53(int(hi), int(lo))
        # the top 24 bits are the single-precision uniform (hi >> 8) * 2^-24
        assert int(u * 2 ** 24) == int(hi) >> 8
        assert u * 2 ** 53 == (int(hi) << 21) | (int(lo) >> 11)


def test_stream_uniformity():
    # trial uniforms of one electron are uniform on [0,1): Kolmogorov-Smirnov at 1e-3
    from scipy import stats
    us = []
    for b in range(4000):
        hi = oracle.stream_block(7, 3, oracle.TRIAL_HI, b)
        lo = oracle.stream_block(7, 3, oracle.TRIAL_LO, b)
        us += [oracle.uniform53(hi[i], lo[i]) for i in range(4)]
    assert stats.kstest(us, "uniform").pvalue > 1e-3
