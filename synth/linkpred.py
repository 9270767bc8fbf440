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


# --------------------------------------------------------------------------- device (torch) versions
# For graphs too large for the host-side split above (billions of edges) the
# same protocol runs on torch tensors, with one change: an edge goes to the
# test set when a seeded hash of its key falls below 0.2 (an independent
# Bernoulli(0.2) draw per edge) instead of by a shuffled 80/20 cut.

def _s64(x: int) -> int:
    """uint64 value as the int64 with the same bits."""
    x &= (1 << 64) - 1
    return x - (1 << 64) if x >= (1 << 63) else x


_GOLD, _M1, _M2 = _s64(0x9E3779B97F4A7C15), _s64(0xBF58476D1CE4E5B9), _s64(0x94D049BB133111EB)   # SplitMix64


def _lsr(z, k: int):
    return (z >> k) & ((1 << (64 - k)) - 1)


def _mix64(z):
    """SplitMix64 output function on int64 tensors holding uint64 bits."""
    z = z + _GOLD
    z = (z ^ _lsr(z, 30)) * _M1
    z = (z ^ _lsr(z, 27)) * _M2
    return z ^ _lsr(z, 31)


@dataclass
class DeviceSplit:
    n: int                  # |V_train|
    offsets: object         # int64 [n+1] (device)
    indices: object         # int32 [nnz] (device)
    train_keys: object      # int64 sorted u*n+v (u < v, relabelled): the train edges
    test_keys: object       # int64 sorted u*n+v (u < v, relabelled): test edges inside V_train
    old_id: object          # int64 old id of each train vertex


def split_rmat_torch(scale: int, edge_factor: float, seed: int, split_seed: int, device,
                     test_frac: float = 0.2, chunk: int = 1 << 26, progress=None) -> DeviceSplit:
    """R-MAT graph (as rmat_csr) split for link prediction on `device`;
    progress(msg) is called after each stage when given."""
    say = progress or (lambda msg: None)
    import torch
    from .rmat import rmat_pairs_torch
    N = 1 << scale
    m = int(round(edge_factor * N))
    parts = []
    first = 0
    while first < m:
        cnt = min(chunk, m - first)
        r, c = rmat_pairs_torch(scale, first, cnt, seed, device)
        first += cnt
        keep = r != c
        lo, hi = torch.minimum(r[keep], c[keep]), torch.maximum(r[keep], c[keep])
        del r, c, keep
        parts.append(torch.unique(lo * N + hi))
        del lo, hi
        if len(parts) % 8 == 0:
            say(f"drew {first} of {m} pairs")
    keys = torch.unique(torch.cat(parts))
    del parts
    say(f"{keys.numel()} distinct undirected edges")
    # test iff the hash, read as an unsigned number, is below test_frac * 2^64;
    # xor with the sign bit makes signed order equal unsigned order
    salt = _s64(split_seed * 0x9E3779B97F4A7C15)
    h = _mix64(keys ^ salt)
    thr = _s64(int(test_frac * 2.0 ** 64) ^ (1 << 63))
    is_test = (h ^ _s64(1 << 63)) < thr
    del h
    test = keys[is_test]
    train = keys[~is_test]
    del keys, is_test
    tu, tv = torch.div(train, N, rounding_mode="floor"), None
    tv = train - tu * N
    used = torch.zeros(N, dtype=torch.bool, device=device)
    used[tu] = True
    used[tv] = True
    newid = torch.cumsum(used.to(torch.int64), 0) - 1
    n = int(used.sum().item())
    old_id = torch.nonzero(used).flatten()
    tu, tv = newid[tu], newid[tv]
    train_keys = tu * n + tv                      # relabelling is monotone: still sorted, u < v
    del train
    # CSR without sorting both directions at once: row x holds its smaller
    # neighbours (the reversed keys v*n+u, sorted) followed by its larger
    # ones (train_keys, already sorted); both blocks ascend and every smaller
    # neighbour precedes every larger one
    say(f"building the CSR of {2 * train_keys.numel()} train entries")
    rev, _ = torch.sort(tv * n + tu)
    del tu, tv
    rows_hi = torch.div(train_keys, n, rounding_mode="floor")
    rows_lo = torch.div(rev, n, rounding_mode="floor")
    deg_hi = torch.bincount(rows_hi, minlength=n)
    deg_lo = torch.bincount(rows_lo, minlength=n)
    offsets = torch.zeros(n + 1, dtype=torch.int64, device=device)
    offsets[1:] = torch.cumsum(deg_lo + deg_hi, 0)
    start_lo = torch.cumsum(deg_lo, 0) - deg_lo
    start_hi = torch.cumsum(deg_hi, 0) - deg_hi
    indices = torch.empty(int(offsets[-1].item()), dtype=torch.int32, device=device)
    i = torch.arange(rev.numel(), device=device, dtype=torch.int64)
    indices[offsets[rows_lo] + (i - start_lo[rows_lo])] = (rev - rows_lo * n).to(torch.int32)
    del i, rev, rows_lo
    j = torch.arange(train_keys.numel(), device=device, dtype=torch.int64)
    indices[offsets[rows_hi] + deg_lo[rows_hi] + (j - start_hi[rows_hi])] = (train_keys - rows_hi * n).to(torch.int32)
    del j, rows_hi, deg_lo, deg_hi, start_lo, start_hi
    su = torch.div(test, N, rounding_mode="floor")
    sv = test - su * N
    ok = used[su] & used[sv]
    test_keys = newid[su[ok]] * n + newid[sv[ok]]
    del su, sv, ok, test, used, newid
    return DeviceSplit(n, offsets, indices, train_keys, test_keys, old_id)


def _contains(sorted_keys, q):
    import torch
    if sorted_keys.numel() == 0:
        return torch.zeros_like(q, dtype=torch.bool)
    pos = torch.searchsorted(sorted_keys, q).clamp_(max=sorted_keys.numel() - 1)
    return sorted_keys[pos] == q


def _negatives(n, count, forbidden, gen, device):
    import torch
    out = []
    have = 0
    while have < count:
        need = count - have
        u = torch.randint(0, n, (2 * need + 16,), generator=gen, device=device)
        v = torch.randint(0, n, (2 * need + 16,), generator=gen, device=device)
        ok = u != v
        u, v = u[ok], v[ok]
        key = torch.minimum(u, v) * n + torch.maximum(u, v)
        bad = torch.zeros_like(key, dtype=torch.bool)
        for f in forbidden:
            bad |= _contains(f, key)
        pairs = torch.stack([u[~bad], v[~bad]], 1)[:need]
        out.append(pairs)
        have += len(pairs)
    return torch.cat(out)


def make_eval_pairs_torch(split: DeviceSplit, seed: int, n_train: int = 500_000, n_test: int = 1_000_000):
    """Classifier and test pairs of the link-prediction protocol on the
    device split: n_train/2 train edges and as many non-edges of G_train;
    n_test/2 test edges and as many pairs outside train and test edges."""
    import torch
    dev = split.train_keys.device
    gen = torch.Generator(device=dev)
    gen.manual_seed(seed)
    n = split.n

    def pick(keys, count):
        sel = torch.randint(0, keys.numel(), (count,), generator=gen, device=dev)
        k = keys[sel]
        u = torch.div(k, n, rounding_mode="floor")
        return torch.stack([u, k - u * n], 1)

    ptr = pick(split.train_keys, n_train // 2)
    ntr = _negatives(n, n_train // 2, [split.train_keys], gen, dev)
    pte = pick(split.test_keys, n_test // 2)
    nte = _negatives(n, n_test // 2, [split.train_keys, split.test_keys], gen, dev)
    xtr = torch.cat([ptr, ntr]).cpu().numpy()
    ytr = np.concatenate([np.ones(len(ptr)), np.zeros(len(ntr))])
    xte = torch.cat([pte, nte]).cpu().numpy()
    yte = np.concatenate([np.ones(len(pte)), np.zeros(len(nte))])
    return EvalPairs(xtr, ytr, xte, yte)


def auc_on_pairs_device(emb, P: EvalPairs) -> float:
    """auc_on_pairs with the Hadamard features gathered on the embedding's
    device (only the pairs' rows leave it)."""
    import torch
    from sklearn.linear_model import LogisticRegression
    from sklearn.metrics import roc_auc_score

    def feats(x):
        idx = torch.from_numpy(x).to(emb.device)
        return (emb[idx[:, 0]].float() * emb[idx[:, 1]].float()).cpu().numpy().astype(np.float64)

    clf = LogisticRegression(max_iter=1000)
    clf.fit(feats(P.xtr), P.ytr)
    return float(roc_auc_score(P.yte, clf.decision_function(feats(P.xte))))
