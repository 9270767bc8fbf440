"""Inputs and evaluator: R-MAT shape, CSR validity, the link-prediction split
of Section 6.1 and the AUCROC score against a brute-force pairwise count."""
import numpy as np
import pytest

from synth import check_csr, evaluate_auc, init_rows, rmat_csr, split_edges
from synth.rmat import rmat_pairs


def test_rmat_deterministic_and_simple():
    a = rmat_csr(10, 8, seed=5)
    b = rmat_csr(10, 8, seed=5)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
    check_csr(*a)
    c = rmat_csr(10, 8, seed=6)
    assert not np.array_equal(a[1][:100], c[1][:100])


def test_rmat_quadrant_frequencies():
    r, c = rmat_pairs(1, 0, 200000, seed=3)
    freq = np.bincount(r * 2 + c, minlength=4) / len(r)
    assert np.allclose(freq, [0.57, 0.19, 0.19, 0.05], atol=0.005)


def test_rmat_scale12_shape():
    off, idx = rmat_csr(12, 16, seed=1)
    assert len(off) == 4097
    m = len(idx) // 2
    assert 45000 < m < 52000           # ~74% of 65,536 draws survive dedup
    nonisolated = int((np.diff(off) > 0).sum())
    assert 3200 < nonisolated < 3500


def test_non_power_of_two_n():
    off, idx = rmat_csr(11, 4, seed=8, n=1500)
    assert len(off) == 1501
    check_csr(off, idx)


def test_split_invariants():
    off, idx = rmat_csr(10, 8, seed=1)
    sp = split_edges(off, idx, seed=2)
    m = len(idx) // 2
    assert len(sp.train_pos) == int(np.floor(0.8 * m))
    check_csr(sp.offsets, sp.indices)
    assert np.all(np.diff(sp.offsets) > 0)              # no isolated train vertex
    assert sp.test_pos.max() < sp.n
    assert np.all(np.diff(sp.old_id) > 0)               # relabelled in ascending old id
    # train CSR holds exactly the train edges
    nn = sp.n
    src = np.repeat(np.arange(nn), np.diff(sp.offsets))
    keys = np.sort((src * nn + sp.indices)[src < sp.indices])
    want = np.sort(sp.train_pos[:, 0] * nn + sp.train_pos[:, 1])
    assert np.array_equal(keys, want)
    # test edges map back to original edges
    oe = set(zip(*np.nonzero(np.zeros(0))))
    orig_src = np.repeat(np.arange(len(off) - 1), np.diff(off))
    okeys = set((orig_src * (len(off) - 1) + idx).tolist())
    for u, v in sp.test_pos[:200]:
        assert int(sp.old_id[u]) * (len(off) - 1) + int(sp.old_id[v]) in okeys


def _auc_bruteforce(y, s):
    pos, neg = s[y == 1], s[y == 0]
    tot = 0.0
    for p in pos:
        tot += np.sum(p > neg) + 0.5 * np.sum(p == neg)
    return tot / (len(pos) * len(neg))


def test_auc_matches_pairwise_count():
    from sklearn.metrics import roc_auc_score
    rng = np.random.default_rng(3)
    for _ in range(5):
        y = rng.integers(0, 2, size=60)
        y[0], y[1] = 0, 1
        s = np.round(rng.normal(size=60), 1)          # ties included
        assert roc_auc_score(y, s) == pytest.approx(_auc_bruteforce(y, s), abs=1e-12)


def test_random_embedding_auc_near_half():
    off, idx = rmat_csr(11, 8, seed=1)
    sp = split_edges(off, idx, seed=2)
    M = init_rows(sp.n, 16, seed=3)
    auc = evaluate_auc(M, sp, seed=5)
    assert 0.35 < auc < 0.65


def test_init_rows_range():
    M = init_rows(1000, 32, seed=3)
    assert M.dtype == np.float32 and M.shape == (1000, 32)
    assert np.abs(M).max() <= 0.5 / 32


def test_torch_rmat_matches_numpy():
    import torch
    r0, c0 = rmat_pairs(13, 12345, 5000, seed=9)
    r1, c1 = __import__("synth.rmat", fromlist=["rmat_pairs_torch"]).rmat_pairs_torch(13, 12345, 5000, 9, "cpu")
    assert np.array_equal(r0, r1.numpy()) and np.array_equal(c0, c1.numpy())
    from synth.rmat import rmat_csr_torch
    for args in ((10, 8, 3, None), (11, 5.5, 4, 1500)):
        off, idx = rmat_csr(args[0], args[1], seed=args[2], n=args[3])
        to, ti = rmat_csr_torch(args[0], args[1], args[2], "cpu", n=args[3], chunk=3000)
        assert np.array_equal(off, to.numpy()) and np.array_equal(idx, ti.numpy())


def test_drop_isolated_torch():
    import torch
    from synth.rmat import drop_isolated_torch
    off, idx = rmat_csr(10, 2, seed=4)
    o, x, old = drop_isolated_torch(torch.from_numpy(off), torch.from_numpy(idx))
    o, x, old = o.numpy(), x.numpy(), old.numpy()
    check_csr(o, x)
    assert np.all(np.diff(o) > 0)
    # same edge set after mapping back to old ids
    src = np.repeat(np.arange(len(o) - 1), np.diff(o))
    n0 = len(off) - 1
    a = np.sort(old[src] * n0 + old[x])
    s0 = np.repeat(np.arange(n0), np.diff(off))
    assert np.array_equal(a, np.sort(s0 * n0 + idx))


def test_device_split_protocol():
    # the torch split on the CPU device: train and test partition the edges,
    # the train CSR is valid, relabelling keeps old-id order, negatives avoid edges
    import torch
    from synth.linkpred import make_eval_pairs_torch, split_rmat_torch
    sp = split_rmat_torch(11, 8, 1, 2, "cpu", chunk=5000)
    off, idx = sp.offsets.numpy(), sp.indices.numpy()
    check_csr(off, idx)
    assert np.all(np.diff(off) > 0) and len(off) == sp.n + 1
    assert np.all(np.diff(sp.old_id.numpy()) > 0)
    full_off, full_idx = rmat_csr(11, 8, seed=1)
    N = len(full_off) - 1
    src = np.repeat(np.arange(N), np.diff(full_off))
    allk = np.sort((src * N + full_idx)[src < full_idx])
    old = sp.old_id.numpy()
    tr = sp.train_keys.numpy()
    tu, tv = tr // sp.n, tr % sp.n
    back = np.sort(old[tu] * N + old[tv])
    assert np.all(np.isin(back, allk))
    frac = len(tr) / len(allk)
    assert 0.78 < frac < 0.82
    te = sp.test_keys.numpy()
    assert not np.intersect1d(te, tr).size
    P = make_eval_pairs_torch(sp, 5, n_train=2000, n_test=2000)
    trs, tes = set(tr.tolist()), set(te.tolist())
    for (u, v), y in zip(P.xtr, P.ytr):
        k = min(u, v) * sp.n + max(u, v)
        assert (k in trs) == (y == 1) and u != v
    for (u, v), y in zip(P.xte, P.yte):
        k = min(u, v) * sp.n + max(u, v)
        assert (k in tes) == (y == 1) and (k not in trs)
