"""Pins of the oracle's counter-based random stream (Philox4x32-10) and of the
sampling rules of Algorithm 3 (Section 3.1)."""
import os

import numpy as np
import pytest

from synth import rmat_csr

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _kat_rows():
    rows = []
    for line in open(os.path.join(GOLD, "philox4x32_10_kat.txt")):
        if line.startswith("#") or not line.strip():
            continue
        w = [int(x, 16) for x in line.split()]
        rows.append((w[0:4], w[4:6], w[6:10]))
    return rows


@pytest.mark.parametrize("ctr,key,want", _kat_rows())
def test_philox_known_answers(orc, ctr, key, want):
    assert list(orc.philox4x32_10(ctr, key)) == want


def test_stream_counter_layout(orc):
    # block = philox((src, epoch, level | tag << 8, kind<<24 | slot<<16 | block), seed)
    seed = 0x0123456789ABCDEF
    got = orc.stream_block(seed, 3, 7, 11, 12345, 1, 2, 5)
    want = orc.philox4x32_10([12345, 11, 3 | (7 << 8), (1 << 24) | (2 << 16) | 5],
                             [seed & 0xFFFFFFFF, seed >> 32])
    assert list(got) == list(want)


def test_sample_rules(orc):
    off, idx = rmat_csr(8, 8, seed=11)
    n = len(off) - 1
    k = 5
    deg = np.diff(off)
    for src in range(n):
        s = orc.draw_samples(off, idx, 4, 0, 0, 3, src, k)
        if deg[src] == 0:
            assert s[0] == -1
        else:
            assert s[0] in idx[off[src]:off[src + 1]]
        assert np.all((s[1:] >= 0) & (s[1:] < n))


def test_sample_words_map(orc):
    # positive uses word 0 of block 0 scaled to the degree; negative t uses word t.
    off, idx = rmat_csr(8, 8, seed=11)
    n = len(off) - 1
    src = int(np.argmax(np.diff(off)))
    words = np.concatenate([orc.stream_block(9, 2, 1, 4, src, 0, 0, b) for b in range(2)])
    s = orc.draw_samples(off, idx, 9, 2, 1, 4, src, 6)
    deg = off[src + 1] - off[src]
    assert s[0] == idx[off[src] + (int(words[0]) * int(deg) >> 32)]
    for t in range(1, 7):
        assert s[t] == (int(words[t]) * n) >> 32


def test_negative_uniformity_chi2(orc):
    # chi^2 goodness of fit of negative draws over 64 buckets (n = 64 vertices).
    from scipy.stats import chisquare
    off = np.zeros(65, np.int64)
    idx = np.zeros(0, np.int32)
    counts = np.zeros(64)
    for src in range(64):
        for ep in range(40):
            s = orc.draw_samples(off, idx, 77, 0, 0, ep, src, 15)
            np.add.at(counts, s[1:], 1)
    p = chisquare(counts).pvalue
    assert p > 1e-4


def test_positive_uniform_over_neighbours(orc):
    from scipy.stats import chisquare
    # star centre 0 with 16 leaves: positive draws of the centre over 4000 epochs
    n = 17
    off = np.zeros(n + 1, np.int64)
    off[1:] = 16
    off[1] = 16
    off = np.concatenate([[0], [16], 16 + np.arange(1, 17)]).astype(np.int64)
    idx = np.concatenate([np.arange(1, 17), np.zeros(16)]).astype(np.int32)
    counts = np.zeros(16)
    for ep in range(4000):
        s = orc.draw_samples(off, idx, 5, 0, 0, ep, 0, 0)
        counts[s[0] - 1] += 1
    assert chisquare(counts).pvalue > 1e-4


def test_sr_bits_layout(orc):
    # element e sits in 32-bit word w = e // 2; with L = d // 8 the word draws
    # from block w % L and takes half 2 * (w // L) + e % 2 (low half first)
    for d in (8, 32, 128, 256):
        L = d // 8
        for e in range(d):
            w = e // 2
            blk = orc.stream_block(5, 1, 0, 2, 9, 1, 3, w % L)
            h = 2 * (w // L) + e % 2
            word = int(blk[h // 2])
            want = (word >> 16) if h & 1 else (word & 0xFFFF)
            assert orc.sr_bits(5, 1, 0, 2, 9, 3, e, d) == want
    # every (block, half) pair of the d/8 blocks is used exactly once per row
    d = 64
    seen = {(((e // 2) % 8), 2 * ((e // 2) // 8) + e % 2) for e in range(d)}
    assert len(seen) == d
