"""Pins of the random-walk sampling reference (Section 3.2): walks are walks
of the graph with uniform transitions (chi-square), the pair offsets against
their closed-form count and a brute-force enumeration, the visiting order is
a permutation sorted by its Philox keys (the generator is pinned to the
published known-answer vectors), the pairs of an epoch are exactly the
within-window pairs of its walks, the training reduces to explicit UpdateEmbed
batches in visiting order (FP64, bit for bit), the zero learning rate and the
isolated-vertex cases, and walk-sampled training separates held-out edges."""
import numpy as np
import pytest
from scipy import stats

from synth import csr_from_pairs, evaluate_auc, init_rows, rmat_csr, split_edges

SEED = 11


def _graph(scale=8, ef=5, seed=3):
    sp = split_edges(*rmat_csr(scale, ef, seed), seed=2)
    return sp.offsets, sp.indices


def _with_isolated(off, idx, extra=3):
    """The graph with `extra` isolated vertices appended."""
    return np.concatenate([off, np.full(extra, off[-1], off.dtype)]), idx


@pytest.mark.parametrize("length", [0, 1, 5, 17])
def test_walks_follow_edges(orc, length):
    off, idx = _with_isolated(*_graph())
    n = len(off) - 1
    for v in range(0, n, 7):
        w = orc.walk(off, idx, v, length, SEED, epoch=3)
        assert w[0] == v
        if off[v + 1] == off[v]:
            assert len(w) == 1          # an isolated start has no step
            continue
        assert len(w) == length + 1     # symmetric graph: every step finds a neighbour
        for a, b in zip(w[:-1], w[1:]):
            assert b in idx[off[a]:off[a + 1]]


def test_walk_transitions_are_uniform(orc):
    # a hub with 7 neighbours that each link back only to the hub: every
    # second step leaves the hub to a uniform neighbour
    pairs = np.array([(0, i) for i in range(1, 8)])
    off, idx = csr_from_pairs(8, pairs[:, 0], pairs[:, 1])
    counts = np.zeros(8, np.int64)
    for ep in range(400):
        w = orc.walk(off, idx, 0, 20, SEED, epoch=ep)
        assert np.all(w[0::2] == 0)
        counts += np.bincount(w[1::2], minlength=8)
    assert counts[0] == 0
    assert stats.chisquare(counts[1:]).pvalue > 1e-3


def test_walks_differ_by_epoch_and_level(orc):
    off, idx = _graph()
    a = orc.walk(off, idx, 5, 30, SEED, epoch=0)
    assert not np.array_equal(a, orc.walk(off, idx, 5, 30, SEED, epoch=1))
    assert not np.array_equal(a, orc.walk(off, idx, 5, 30, SEED, level=1))
    assert np.array_equal(a, orc.walk(off, idx, 5, 30, SEED, epoch=0))


@pytest.mark.parametrize("length,window", [(10, 3), (5, 5), (5, 9), (1, 1), (0, 3), (80, 10), (4, 0)])
def test_pair_offsets(orc, length, window):
    a, b = orc.walk_offsets(length, window)
    want = [(i, j) for i in range(length) for j in range(i + 1, length + 1) if j - i <= window]
    assert list(zip(a.tolist(), b.tolist())) == want
    g = min(window, length)
    assert len(a) == g * length - g * (g - 1) // 2      # closed form


@pytest.mark.parametrize("n,P,epoch", [(1, 1, 0), (37, 5, 2), (200, 27, 0), (0, 4, 1)])
def test_order_is_a_key_sorted_permutation(orc, n, P, epoch):
    order = orc.walk_order(n, P, SEED, level=2, tag=5, epoch=epoch)
    assert np.array_equal(np.sort(order), np.arange(n * P))
    keys = np.array([orc.stream_block(SEED, 2, 5, epoch, int(q), 5, 0, 0)[0] for q in order], np.uint64)
    assert np.all(np.diff(keys.astype(np.int64)) >= 0)
    tie = np.diff(keys.astype(np.int64)) == 0
    assert np.all(np.diff(order)[tie] > 0)


@pytest.mark.parametrize("length,window,extra", [(6, 2, 0), (4, 4, 3), (1, 1, 2)])
def test_pairs_are_the_window_pairs_of_the_walks(orc, length, window, extra):
    off, idx = _with_isolated(*_graph(), extra)
    n = len(off) - 1
    src, pos = orc.walk_pairs(off, idx, length, window, SEED, epoch=4)
    a, b = orc.walk_offsets(length, window)
    P = len(a)
    order = orc.walk_order(n, P, SEED, epoch=4)
    assert len(src) == n * P
    want_void = 0
    for r, q in enumerate(order):
        v, l = divmod(int(q), P)
        w = orc.walk(off, idx, v, length, SEED, epoch=4)
        if b[l] >= len(w):
            want_void += 1
            assert src[r] == -1 and pos[r] == -1
        else:
            assert (src[r], pos[r]) == (w[a[l]], w[b[l]])
    assert want_void == extra * P
    assert np.count_nonzero(src < 0) == want_void


def _negatives(orc, r, epoch, k, n):
    words = np.concatenate([orc.stream_block(SEED, 0, 0, epoch, r, 6, 0, blk) for blk in range((k + 4) // 4)])
    return [int((int(words[t]) * n) >> 32) for t in range(1, k + 1)]


@pytest.mark.parametrize("k,length,window,epochs", [(0, 3, 1, 1), (2, 5, 2, 2), (5, 2, 2, 3)])
def test_training_is_explicit_batches_in_visiting_order(orc, k, length, window, epochs):
    off, idx = _with_isolated(*_graph(7, 4, 5), 2)
    n = len(off) - 1
    d = 16
    f = init_rows(n, d, 3) * 4
    M = f.astype(np.float64)
    done = orc.train_walks(off, idx, M, epochs, 0.05, k, length, window, SEED)
    R = f.astype(np.float64)
    want = 0
    for j in range(epochs):
        lr = orc.lr_at(0.05, j, epochs)
        src, pos = orc.walk_pairs(off, idx, length, window, SEED, epoch=j)
        for r in range(len(src)):
            if src[r] < 0:
                continue
            samp = np.array([[pos[r]] + _negatives(orc, r, j, k, n)], np.int32)
            want += orc.update_batch(R, np.array([src[r]], np.int32), samp, lr, SEED, epoch=j)
    assert done == want
    assert np.array_equal(M, R)


@pytest.mark.parametrize("bf16", [False, True])
def test_zero_lr_is_identity(orc, bf16):
    off, idx = _graph()
    n = len(off) - 1
    f = init_rows(n, 32, 3)
    M = orc.f32_to_bf16_rne(f).reshape(n, 32) if bf16 else f.astype(np.float64)
    M0 = M.copy()
    done = orc.train_walks(off, idx, M, 2, 0.0, 3, 4, 2, SEED)
    assert done > 0 and np.array_equal(M, M0)


def test_degenerate_sizes(orc):
    off, idx = _graph()
    n = len(off) - 1
    M = init_rows(n, 8, 3).astype(np.float64)
    M0 = M.copy()
    assert orc.train_walks(off, idx, M, 3, 0.05, 2, 0, 3, SEED) == 0       # no step, no pair
    assert orc.train_walks(off, idx, M, 3, 0.05, 2, 5, 0, SEED) == 0       # empty window
    assert orc.train_walks(off, idx, M, 0, 0.05, 2, 5, 2, SEED) == 0       # no epoch
    assert np.array_equal(M, M0)
    iso_off = np.zeros(5, np.int64)
    E = init_rows(4, 8, 3).astype(np.float64)
    assert orc.train_walks(iso_off, np.zeros(0, np.int32), E, 2, 0.05, 2, 4, 2, SEED) == 0


def test_walk_training_learns(orc):
    from scipy.spatial import cKDTree
    pts = np.random.default_rng(0).random((3000, 2))
    pairs = np.array(sorted(cKDTree(pts).query_pairs(0.03)))
    sp = split_edges(*csr_from_pairs(3000, pairs[:, 0], pairs[:, 1]), seed=2)
    M = (init_rows(sp.n, 32, 3) * 20).astype(np.float64)
    orc.train_walks(sp.offsets, sp.indices, M, 10, 0.045, 3, 6, 2, SEED)
    assert evaluate_auc(M, sp, seed=5) > 0.9


def test_bf16_training_tracks_fp64(orc):
    # stochastic rounding is unbiased: one BF16 epoch (each row rounded about
    # 35 times, each rounding off by up to one BF16 ulp, 2^-8 relative) drifts
    # from the FP64 epoch on the same samples like a random walk of those errors
    off, idx = _graph()
    n = len(off) - 1
    f = init_rows(n, 32, 3) * 4
    bits = orc.f32_to_bf16_rne(f).reshape(n, 32)
    R = orc.bf16_to_f64(bits)
    orc.train_walks(off, idx, bits, 1, 0.05, 3, 4, 2, SEED)
    orc.train_walks(off, idx, R, 1, 0.05, 3, 4, 2, SEED)
    got = orc.bf16_to_f64(bits)
    rel = np.abs(got - R).sum(1) / np.abs(R).sum(1)
    assert rel.mean() < 2e-2 and rel.max() < 6e-2
    assert abs(float(np.mean(got - R))) < 1e-4
