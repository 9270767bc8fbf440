"""Pins of the partitioned-embedding reference (Section 5): the inside-out
pair order against hand traces and its defining properties, the parts,
sample pools against a brute-force neighbour scan and a chi-square test, the
one-part one-sample case against sequential Algorithm 3 (bit for bit, FP64
and BF16), the zero learning rate, and the cap on positive samples."""
import numpy as np
import pytest

from synth import init_rows, rmat_csr, split_edges


def test_inside_out_hand_traces(orc):
    assert orc.inside_out(1) == [(0, 0)]
    assert orc.inside_out(2) == [(0, 0), (1, 0), (1, 1)]
    assert orc.inside_out(4) == [(0, 0), (1, 0), (1, 1), (2, 0), (2, 1), (2, 2),
                                 (3, 0), (3, 1), (3, 2), (3, 3)]


@pytest.mark.parametrize("K", [1, 2, 3, 5, 8, 13])
def test_inside_out_properties(orc, K):
    pairs = orc.inside_out(K)
    assert len(pairs) == K * (K + 1) // 2
    assert sorted(pairs) == sorted((a, b) for a in range(K) for b in range(a + 1))
    # consecutive kernels share a part except when a new part enters
    for (a0, b0), (a1, b1) in zip(pairs, pairs[1:]):
        assert a1 == a0 or (a1 == a0 + 1 and b1 == 0 and a0 == b0)


@pytest.mark.parametrize("n,K", [(10, 3), (7, 7), (1000, 6), (5, 1)])
def test_part_starts(orc, n, K):
    s = orc.part_starts(n, K)
    assert s[0] == 0 and s[-1] == n and np.all(np.diff(s) >= 0)
    assert np.diff(s).max() - np.diff(s).min() <= 1


def _graph(scale=9, ef=6, seed=3):
    sp = split_edges(*rmat_csr(scale, ef, seed), seed=2)
    return sp.offsets, sp.indices


@pytest.mark.parametrize("K,i,j", [(3, 0, 0), (3, 2, 0), (4, 3, 1), (1, 0, 0)])
def test_pool_brute_force(orc, K, i, j):
    off, idx = _graph()
    n = len(off) - 1
    st = orc.part_starts(n, K)
    B = 5
    src, pos, bb = orc.pool(off, idx, K, i, j, B, seed=11, round=2)
    want = []
    sides = [(i, j)] + ([(j, i)] if i != j else [])
    for s, o in sides:
        for u in range(st[s], st[s + 1]):
            nb = idx[off[u]:off[u + 1]]
            inpart = nb[(nb >= st[o]) & (nb < st[o + 1])]
            if len(inpart):
                want += [(u, b, set(inpart.tolist())) for b in range(B)]
    assert len(src) == len(want)
    for e, (u, b, allowed) in enumerate(want):
        assert src[e] == u and bb[e] == b
        assert int(pos[e]) in allowed


def test_pool_positives_uniform(orc):
    # a vertex with many neighbours in the opposite part: counts over rounds
    off, idx = _graph(10, 8)
    n = len(off) - 1
    K, B = 2, 5
    st = orc.part_starts(n, K)
    deg1 = [(len([x for x in idx[off[u]:off[u + 1]] if x >= st[1]]), u) for u in range(st[0], st[1])]
    c, u = max(deg1)
    assert c >= 20
    counts = {}
    for r in range(400):
        src, pos, _ = orc.pool(off, idx, K, 1, 0, B, seed=7, round=r)
        sel = pos[src == u]
        for p in sel.tolist():
            counts[p] = counts.get(p, 0) + 1
    obs = np.array(list(counts.values()), float)
    assert len(obs) == c
    exp = obs.sum() / c
    chi2 = ((obs - exp) ** 2 / exp).sum()
    # chi-square with c-1 degrees of freedom: mean c-1, sd sqrt(2(c-1)); 5 sd margin
    assert chi2 < (c - 1) + 5 * np.sqrt(2 * (c - 1))


@pytest.mark.parametrize("bf16", [False, True])
def test_one_part_one_sample_is_algorithm3(orc, bf16):
    off, idx = _graph(9, 6)
    n = len(off) - 1
    assert np.all(np.diff(off) > 0)          # no isolated vertex (split train graph)
    f = init_rows(n, 16, 3)
    if bf16:
        A = orc.f32_to_bf16_rne(f).reshape(n, 16)
        Bm = A.copy()
    else:
        A = f.astype(np.float64)
        Bm = A.copy()
    u1 = orc.train(off, idx, A, 6, 0.05, 3, seed=9, level=2, tag=5)
    u2, p2 = orc.train_partitioned(off, idx, Bm, 1, 1, 6, 0.05, 3, seed=9, level=2, tag=5)
    assert u1 == u2 and p2 == 6 * n
    assert np.array_equal(A, Bm)


def test_zero_learning_rate_is_identity(orc):
    off, idx = _graph()
    n = len(off) - 1
    M = init_rows(n, 8, 3).astype(np.float64)
    M0 = M.copy()
    orc.train_partitioned(off, idx, M, 3, 5, 10, 0.0, 3, seed=1)
    assert np.array_equal(M, M0)


def test_positive_cap(orc):
    off, idx = _graph()
    n = len(off) - 1
    K, B, e, k = 3, 5, 7, 2
    total = sum(len(orc.pool(off, idx, K, a, b, B, seed=1, round=r)[0])
                for r in range(2) for a, b in orc.inside_out(K))
    assert total > e * n                       # the cap binds in the second round
    M = init_rows(n, 8, 3).astype(np.float64)
    upd, pos = orc.train_partitioned(off, idx, M, K, B, e, 0.03, k, seed=1)
    assert pos == e * n
    assert pos * (1 + k) - upd >= 0 and pos * (1 + k) - upd < 0.05 * pos * k   # self-negatives only


def test_partitioned_training_learns(orc):
    # random geometric graph (4000 points, radius 0.03): strong locality, so
    # link prediction separates well once the rows are trained
    from scipy.spatial import cKDTree
    from synth import csr_from_pairs, evaluate_auc
    pts = np.random.default_rng(0).random((4000, 2))
    pairs = np.array(sorted(cKDTree(pts).query_pairs(0.03)))
    sp = split_edges(*csr_from_pairs(4000, pairs[:, 0], pairs[:, 1]), seed=2)
    M = init_rows(sp.n, 32, 3).astype(np.float64) * 20
    orc.train_partitioned(sp.offsets, sp.indices, M, 4, 5, 100, 0.045, 3, seed=4)
    assert evaluate_auc(M, sp, seed=5) > 0.85
