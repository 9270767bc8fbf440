"""Link-prediction protocol of Section 6.1 (data preparation for ML tasks).

* The undirected edges are shuffled (seeded) and split 80% / 20%.
* Vertices isolated in G_train are removed and the rest relabelled compactly
  in ascending old id; test edges with an endpoint outside V_train are
  dropped.
* The classifier is trained on all |E_train| train edges plus as many
  negatives drawn uniformly from (V_train x V_train) \\ E_train (u != v).
* Test set: E_test plus as many negatives outside E_train and E_test.
* A pair's feature is the element-wise product M[u] * M[v]; the classifier is
  scikit-learn's LogisticRegression with its defaults except
  max_iter=1000, so that it converges (the paper gives no
  hyperparameters); the score is AUCROC on the test set.

For large graphs the paper switches to SGDClassifier; here the training set
is subsampled (seeded) to ``max_train`` pairs instead, which keeps the
classifier identical across graph sizes.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from .rmat import csr_from_pairs


@dataclass
class LinkSplit:
    n: int                      # |V_train|
    offsets: np.ndarray         # train CSR (int64), relabelled ids
    indices: np.ndarray         # int32
    train_pos: np.ndarray       # [E_train, 2] int64, u < v (relabelled)
    test_pos: np.ndarray        # [E_test', 2] int64 (relabelled, both ends in V_train)
    old_id: np.ndarray          # old id of each train vertex
    seed: int


def _undirected_edges(offsets, indices):
    n = len(offsets) - 1
    src = np.repeat(np.arange(n, dtype=np.int64), np.diff(offsets))
    dst = indices.astype(np.int64)
    m = src < dst
    return src[m], dst[m]


def split_edges(offsets, indices, seed: int, train_frac: float = 0.8) -> LinkSplit:
    n0 = len(offsets) - 1
    eu, ev = _undirected_edges(offsets, indices)
    rng = np.random.default_rng(seed)
    perm = rng.permutation(len(eu))
    ntr = int(np.floor(train_frac * len(eu)))
    tr, te = perm[:ntr], perm[ntr:]
    used = np.zeros(n0, dtype=bool)
    used[eu[tr]] = True
    used[ev[tr]] = True
    newid = np.full(n0, -1, dtype=np.int64)
    n = int(used.sum())
    newid[used] = np.arange(n, dtype=np.int64)
    tu, tv = newid[eu[tr]], newid[ev[tr]]
    off, idx = csr_from_pairs(n, tu, tv)
    su, sv = newid[eu[te]], newid[ev[te]]
    keep = (su >= 0) & (sv >= 0)
    train_pos = np.stack([np.minimum(tu, tv), np.maximum(tu, tv)], axis=1)
    test_pos = np.stack([np.minimum(su[keep], sv[keep]),
                         np.maximum(su[keep], sv[keep])], axis=1)
    return LinkSplit(n=n, offsets=off, indices=idx, train_pos=train_pos,
                     test_pos=test_pos, old_id=np.nonzero(used)[0], seed=seed)


def _draw_negatives(n, count, forbidden_keys, rng):
    """``count`` pairs (u != v) uniform over V x V whose undirected key
    min*n+max is not in the sorted ``forbidden_keys``."""
    out = np.zeros((0, 2), dtype=np.int64)
    while len(out) < count:
        need = count - len(out)
        u = rng.integers(0, n, size=2 * need + 16)
        v = rng.integers(0, n, size=2 * need + 16)
        ok = u != v
        u, v = u[ok], v[ok]
        key = np.minimum(u, v) * n + np.maximum(u, v)
        pos = np.searchsorted(forbidden_keys, key)
        pos = np.minimum(pos, max(len(forbidden_keys) - 1, 0))
        hit = (len(forbidden_keys) > 0) & (forbidden_keys[pos] == key) if len(forbidden_keys) else np.zeros(len(key), bool)
        u, v = u[~hit], v[~hit]
        out = np.concatenate([out, np.stack([u, v], axis=1)[:need]])
    return out


@dataclass
class EvalPairs:
    xtr: np.ndarray     # [N, 2] classifier training pairs
    ytr: np.ndarray
    xte: np.ndarray     # [M, 2] test pairs
    yte: np.ndarray


def make_eval_pairs(split: LinkSplit, seed: int, max_train: int = 2_000_000,
                    max_test: int | None = None) -> EvalPairs:
    """The labelled pairs evaluate_auc scores (same draws for the same seed),
    built once so that several embeddings of one split can share them."""
    n = split.n
    rng = np.random.default_rng(seed)
    tr_keys = np.sort(split.train_pos[:, 0] * n + split.train_pos[:, 1])
    all_keys = np.sort(np.concatenate([tr_keys, split.test_pos[:, 0] * n + split.test_pos[:, 1]]))
    pos_tr = split.train_pos
    neg_tr = _draw_negatives(n, len(pos_tr), tr_keys, rng)
    pos_te = split.test_pos
    neg_te = _draw_negatives(n, len(pos_te), all_keys, rng)
    xtr = np.concatenate([pos_tr, neg_tr])
    ytr = np.concatenate([np.ones(len(pos_tr)), np.zeros(len(neg_tr))])
    if len(xtr) > max_train:
        sel = rng.choice(len(xtr), size=max_train, replace=False)
        xtr, ytr = xtr[sel], ytr[sel]
    xte = np.concatenate([pos_te, neg_te])
    yte = np.concatenate([np.ones(len(pos_te)), np.zeros(len(neg_te))])
    if max_test is not None and len(xte) > max_test:
        sel = rng.choice(len(xte), size=max_test, replace=False)
        xte, yte = xte[sel], yte[sel]
    return EvalPairs(xtr, ytr, xte, yte)


def auc_on_pairs(emb: np.ndarray, P: EvalPairs) -> float:
    """AUCROC of a logistic-regression link predictor on Hadamard features."""
    from sklearn.linear_model import LogisticRegression
    from sklearn.metrics import roc_auc_score

    emb = np.asarray(emb, dtype=np.float64)
    ftr = emb[P.xtr[:, 0]] * emb[P.xtr[:, 1]]
    fte = emb[P.xte[:, 0]] * emb[P.xte[:, 1]]
    clf = LogisticRegression(max_iter=1000)
    clf.fit(ftr, P.ytr)
    return float(roc_auc_score(P.yte, clf.decision_function(fte)))


def evaluate_auc(emb: np.ndarray, split: LinkSplit, seed: int,
                 max_train: int = 2_000_000, max_test: int | None = None) -> float:
    """AUCROC of a logistic-regression link predictor on Hadamard features."""
    return auc_on_pairs(emb, make_eval_pairs(split, seed, max_train, max_test))
