"""Learned prolongation -- FP64 reference (test infrastructure only).

Not part of the paper: the build replaces ExpandEmbedding's plain copy
(Algorithm 2) by an optional small network that predicts a fine row from
the coarse row it would have copied.  For fine vertex v of level i with
super vertex c = map_i[v]:

    x  = [ M_{i+1}[c] (d values), log1p(deg_i(v)), log(clsz(c)) ]   (d + 2)
    h  = GELU(W1 x + b1)                     W1: H x (d+2), exact erf GELU
    y  = M_{i+1}[c] + W2 h + b2              W2: d x H

so W2 = 0, b2 = 0 is exactly copy prolongation.  Training minimises the
mean squared error between y and the row the level's training finally
produced, with Adam (beta1 0.9, beta2 0.999, eps 1e-8).  GELU follows
Hendrycks and Gimpel (2016): x * Phi(x), Phi the standard normal CDF.
Matrix products use numpy; everything is float64.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

_SQRT2 = math.sqrt(2.0)
_SQRT2PI = math.sqrt(2.0 * math.pi)
_erf = np.vectorize(math.erf, otypes=[np.float64])


def gelu(z):
    z = np.asarray(z, np.float64)
    return z * 0.5 * (1.0 + _erf(z / _SQRT2))


def gelu_grad(z):
    """d/dz [z Phi(z)] = Phi(z) + z phi(z)."""
    z = np.asarray(z, np.float64)
    return 0.5 * (1.0 + _erf(z / _SQRT2)) + z * np.exp(-0.5 * z * z) / _SQRT2PI


def features(coarse_rows, deg, clsz):
    """[B, d+2]: coarse row, log1p(fine degree), log(cluster size)."""
    c = np.asarray(coarse_rows, np.float64)
    return np.concatenate([c, np.log1p(np.asarray(deg, np.float64))[:, None],
                           np.log(np.asarray(clsz, np.float64))[:, None]], axis=1)


@dataclass
class Params:
    W1: np.ndarray   # [H, d+2]
    b1: np.ndarray   # [H]
    W2: np.ndarray   # [d, H]
    b2: np.ndarray   # [d]

    def copy(self):
        return Params(self.W1.copy(), self.b1.copy(), self.W2.copy(), self.b2.copy())


def forward(P: Params, X, C):
    """Returns (y, cache).  X: [B, d+2] features, C: [B, d] coarse rows."""
    Z1 = X @ P.W1.T + P.b1
    A1 = gelu(Z1)
    Y = C + A1 @ P.W2.T + P.b2
    return Y, (X, Z1, A1)


def mse(Y, T):
    return float(np.mean((Y - T) ** 2))


def backward(P: Params, Y, T, cache):
    """Gradients of mse(Y, T) (mean over all B*d entries)."""
    X, Z1, A1 = cache
    B, d = Y.shape
    dY = 2.0 * (Y - T) / (B * d)
    dW2 = dY.T @ A1
    db2 = dY.sum(0)
    dA1 = dY @ P.W2
    dZ1 = dA1 * gelu_grad(Z1)
    dW1 = dZ1.T @ X
    db1 = dZ1.sum(0)
    return Params(dW1, db1, dW2, db2)


@dataclass
class AdamState:
    m: Params
    v: Params
    t: int = 0


def adam_init(P: Params) -> AdamState:
    z = Params(np.zeros_like(P.W1), np.zeros_like(P.b1), np.zeros_like(P.W2), np.zeros_like(P.b2))
    return AdamState(z, z.copy(), 0)


def adam_step(P: Params, g: Params, S: AdamState, lr, b1=0.9, b2=0.999, eps=1e-8):
    """Kingma and Ba (2015), bias-corrected."""
    S.t += 1
    for name in ("W1", "b1", "W2", "b2"):
        m = getattr(S.m, name)
        v = getattr(S.v, name)
        gr = getattr(g, name)
        m[...] = b1 * m + (1 - b1) * gr
        v[...] = b2 * v + (1 - b2) * gr * gr
        mh = m / (1 - b1 ** S.t)
        vh = v / (1 - b2 ** S.t)
        getattr(P, name)[...] -= lr * mh / (np.sqrt(vh) + eps)


def init_params(d, H, seed, w2_zero=True):
    """W1 ~ U(-1/sqrt(d+2), 1/sqrt(d+2)); W2 = 0 (starts as copy prolongation)."""
    rng = np.random.default_rng(seed)
    lim = 1.0 / math.sqrt(d + 2)
    W1 = rng.uniform(-lim, lim, size=(H, d + 2))
    b1 = np.zeros(H)
    W2 = np.zeros((d, H)) if w2_zero else rng.uniform(-1 / math.sqrt(H), 1 / math.sqrt(H), size=(d, H))
    return Params(W1, b1, W2, np.zeros(d))


# --------------------------------------------------------------------------- training on level pairs
def init_params_stream(d, H, seed):
    """The network's starting point as drawn from the counter-based stream
    (Philox4x32-10, Salmon et al. 2011) keyed by the 64-bit seed: element p
    of W1 (row-major, H x (d+2)) takes word 0 of the block with counter
    (p mod 2^32, p div 2^32, 0, kind 3 << 24), u = (word >> 8) / 2^24, and
    W1[p] = lim (2 u - 1), lim = 1/sqrt(d+2), evaluated in float32; b1, W2
    and b2 are zero (copy prolongation)."""
    from . import philox_many
    F = d + 2
    n = H * F
    p = np.arange(n, dtype=np.uint64)
    ctr = np.zeros((n, 4), np.uint32)
    ctr[:, 0] = (p & 0xFFFFFFFF).astype(np.uint32)
    ctr[:, 1] = (p >> np.uint64(32)).astype(np.uint32)
    ctr[:, 3] = np.uint32(3 << 24)
    r = philox_many(ctr, (seed & 0xFFFFFFFF, (seed >> 32) & 0xFFFFFFFF))
    lim = np.float32(1.0 / math.sqrt(F))
    u = (r[:, 0] >> np.uint32(8)).astype(np.float32) * np.float32(1.0 / 16777216.0)
    w = lim * (np.float32(2.0) * u - np.float32(1.0))
    return Params(w.astype(np.float64).reshape(H, F), np.zeros(H), np.zeros((d, H)), np.zeros(d))


def minibatch(step, batch, total, seed, tag):
    """Pair indices of one minibatch, drawn uniformly with replacement from
    the stream: row b takes the block with counter (b, step, tag << 8,
    kind 2 << 24) and index ((word0 << 32 | word1) >> 16) mod total."""
    from . import philox_many
    ctr = np.zeros((batch, 4), np.uint32)
    ctr[:, 0] = np.arange(batch, dtype=np.uint32)
    ctr[:, 1] = np.uint32(step)
    ctr[:, 2] = np.uint32((tag << 8) & 0xFFFFFFFF)
    ctr[:, 3] = np.uint32(2 << 24)
    r = philox_many(ctr, (seed & 0xFFFFFFFF, (seed >> 32) & 0xFFFFFFFF)).astype(np.uint64)
    return (((r[:, 0] << np.uint64(32)) | r[:, 1]) >> np.uint64(16)) % np.uint64(total)


def level_pairs(coarse, fine, mp, deg):
    """Training pairs of one fine level: for every fine vertex v the coarse
    row of its super vertex c = mp[v], the trained fine row, deg(v) and the
    size of cluster c."""
    mp = np.asarray(mp, np.int64)
    clsz = np.bincount(mp, minlength=len(coarse))
    return (np.asarray(coarse, np.float64)[mp], np.asarray(fine, np.float64), np.asarray(deg, np.int64), clsz[mp])


def train_pairs(P: Params, sources, steps, batch, lr, seed, tag, S: AdamState | None = None):
    """Adam on the MSE of minibatches drawn over the concatenated pairs of
    `sources` (level_pairs tuples, in order).  Returns the loss of every
    step before its update."""
    C = np.concatenate([s[0] for s in sources])
    T = np.concatenate([s[1] for s in sources])
    deg = np.concatenate([s[2] for s in sources])
    cl = np.concatenate([s[3] for s in sources])
    S = S or adam_init(P)
    losses = []
    for step in range(steps):
        u = minibatch(step, batch, len(C), seed, tag).astype(np.int64)
        Y, cache = forward(P, features(C[u], deg[u], cl[u]), C[u])
        losses.append(mse(Y, T[u]))
        adam_step(P, backward(P, Y, T[u], cache), S, lr)
    return np.array(losses)


def prolong_learned(P: Params, coarse, mp, deg):
    """Learned ExpandEmbedding: the fine row of every vertex v of the finer
    level from its super vertex's coarse row."""
    C, _, dg, cl = level_pairs(coarse, np.zeros((len(mp), np.asarray(coarse).shape[1])), mp, deg)
    return forward(P, features(C, dg, cl), C)[0]
