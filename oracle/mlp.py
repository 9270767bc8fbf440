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
