"""Pins of the learned-prolongation reference: GELU against its closed form
and known values, backward against central finite differences of the MSE,
the zero-output-layer case against copy prolongation, Adam's first step."""
import math

import numpy as np
import pytest

from oracle import mlp


def test_gelu_known_values():
    # x Phi(x): Phi(0) = 1/2, Phi(1) = 0.8413447460685429, Phi(-1) = 1 - Phi(1)
    assert mlp.gelu(0.0) == 0.0
    assert mlp.gelu(1.0) == pytest.approx(0.8413447460685429, rel=1e-15)
    assert mlp.gelu(-1.0) == pytest.approx(-0.15865525393145707, rel=1e-14)
    assert mlp.gelu(40.0) == pytest.approx(40.0)
    assert abs(mlp.gelu(-40.0)) < 1e-300
    assert mlp.gelu_grad(0.0) == pytest.approx(0.5)


def test_gelu_grad_finite_differences():
    z = np.linspace(-4, 4, 41)
    h = 1e-6
    fd = (mlp.gelu(z + h) - mlp.gelu(z - h)) / (2 * h)
    assert np.allclose(mlp.gelu_grad(z), fd, rtol=1e-8, atol=1e-10)


def _problem(seed, B=7, d=6, H=5):
    rng = np.random.default_rng(seed)
    C = rng.normal(size=(B, d)) * 0.3
    X = mlp.features(C, rng.integers(0, 50, B), rng.integers(1, 20, B))
    T = C + rng.normal(size=(B, d)) * 0.1
    P = mlp.init_params(d, H, seed, w2_zero=False)
    P.b1 = rng.normal(size=H) * 0.1
    P.b2 = rng.normal(size=d) * 0.1
    return P, X, C, T


def test_backward_matches_finite_differences():
    P, X, C, T = _problem(1)
    Y, cache = mlp.forward(P, X, C)
    g = mlp.backward(P, Y, T, cache)
    h = 1e-6
    for name in ("W1", "b1", "W2", "b2"):
        W = getattr(P, name)
        G = getattr(g, name)
        it = np.nditer(W, flags=["multi_index"])
        for _ in it:
            i = it.multi_index
            old = W[i]
            W[i] = old + h
            lp = mlp.mse(mlp.forward(P, X, C)[0], T)
            W[i] = old - h
            lm = mlp.mse(mlp.forward(P, X, C)[0], T)
            W[i] = old
            assert G[i] == pytest.approx((lp - lm) / (2 * h), rel=1e-6, abs=1e-10), (name, i)


def test_zero_output_layer_is_copy_prolongation():
    P, X, C, T = _problem(2)
    P.W2[...] = 0.0
    P.b2[...] = 0.0
    Y, _ = mlp.forward(P, X, C)
    assert np.array_equal(Y, C)


def test_features_layout():
    C = np.arange(6.0).reshape(2, 3)
    X = mlp.features(C, [0, 3], [1, 4])
    assert np.array_equal(X[:, :3], C)
    assert X[0, 3] == 0.0 and X[1, 3] == pytest.approx(math.log(4.0))
    assert X[0, 4] == 0.0 and X[1, 4] == pytest.approx(math.log(4.0))


def test_adam_first_step_is_signed_lr():
    # with bias correction the first Adam step moves every weight by
    # lr * g / (|g| + eps) -> lr * sign(g)
    P, X, C, T = _problem(3)
    Y, cache = mlp.forward(P, X, C)
    g = mlp.backward(P, Y, T, cache)
    Q = P.copy()
    S = mlp.adam_init(Q)
    mlp.adam_step(Q, g, S, 1e-3)
    for name in ("W1", "W2"):
        step = getattr(P, name) - getattr(Q, name)
        G = getattr(g, name)
        big = np.abs(G) > 1e-6
        assert np.allclose(step[big], 1e-3 * np.sign(G[big]), rtol=1e-3)


def test_adam_constant_gradient_steps_are_signed_lr():
    # under a constant gradient g the bias-corrected moments are exactly g and
    # g^2 at every step t (m_t = (1 - b1^t) g, v_t = (1 - b2^t) g^2), so each
    # of the first five steps moves a weight by lr * g / (|g| + eps); a wrong
    # bias-correction exponent changes every step from the second on
    P = mlp.Params(np.zeros((2, 3)), np.zeros(2), np.zeros((3, 2)), np.zeros(3))
    g = mlp.Params(np.array([[0.3, -2.0, 1e-3], [5.0, -0.25, 0.7]]), np.array([1.0, -1.0]),
                   np.full((3, 2), -0.125), np.array([0.5, 3.0, -7.0]))
    S = mlp.adam_init(P)
    lr, eps = 1e-2, 1e-8
    for t in range(1, 6):
        before = P.copy()
        mlp.adam_step(P, g, S, lr)
        for name in ("W1", "b1", "W2", "b2"):
            G = getattr(g, name)
            step = getattr(before, name) - getattr(P, name)
            assert np.allclose(step, lr * G / (np.abs(G) + eps), rtol=1e-9, atol=0), (t, name)


def test_adam_two_gradients_by_hand():
    # one weight, gradients 1 then -0.5, lr 0.1, beta 0.9 / 0.999, eps 1e-8:
    #   t=1: m = 0.1, v = 0.001, m^ = 1, v^ = 1       -> step 0.1 / (1 + 1e-8)
    #   t=2: m = 0.09 - 0.05 = 0.04, v = 0.000999 + 0.00025 = 0.001249,
    #        m^ = 0.04 / 0.19, v^ = 0.001249 / 0.001999
    P = mlp.Params(np.zeros((1, 1)), np.zeros(1), np.zeros((1, 1)), np.zeros(1))
    S = mlp.adam_init(P)
    one = lambda x: mlp.Params(np.full((1, 1), x), np.zeros(1), np.zeros((1, 1)), np.zeros(1))
    mlp.adam_step(P, one(1.0), S, 0.1)
    w1 = -0.1 / (1.0 + 1e-8)
    assert P.W1[0, 0] == pytest.approx(w1, rel=1e-14)
    mlp.adam_step(P, one(-0.5), S, 0.1)
    step2 = 0.1 * (0.04 / 0.19) / (math.sqrt(0.001249 / 0.001999) + 1e-8)
    assert P.W1[0, 0] == pytest.approx(w1 - step2, rel=1e-12)
    assert P.W1[0, 0] == pytest.approx(-0.1 - 0.02663370, abs=1e-7)   # 0.2105263 / 0.7904508 * 0.1


def test_training_reduces_mse():
    rng = np.random.default_rng(4)
    B, d, H = 256, 8, 16
    C = rng.normal(size=(B, d)) * 0.3
    deg = rng.integers(1, 30, B)
    X = mlp.features(C, deg, rng.integers(1, 10, B))
    T = C * 0.5 + 0.05 * np.log1p(deg)[:, None]     # learnable shift from the features
    P = mlp.init_params(d, H, 4)
    S = mlp.adam_init(P)
    first = mlp.mse(mlp.forward(P, X, C)[0], T)
    for _ in range(300):
        Y, cache = mlp.forward(P, X, C)
        mlp.adam_step(P, mlp.backward(P, Y, T, cache), S, 1e-2)
    assert mlp.mse(mlp.forward(P, X, C)[0], T) < 0.1 * first


def test_stream_init_is_uniform_copy_start():
    # W1 uniform on [-1/sqrt(d+2), 1/sqrt(d+2)] (mean 0, variance lim^2 / 3),
    # everything else zero, so the network starts as copy prolongation
    d, H = 64, 128
    P = mlp.init_params_stream(d, H, 4)
    lim = 1.0 / np.sqrt(d + 2)
    w = P.W1.ravel()
    assert np.all(np.abs(w) <= lim) and w.min() < -0.99 * lim and w.max() > 0.99 * lim
    assert abs(w.mean()) < 4 * lim / np.sqrt(3 * w.size)
    assert abs(w.var() / (lim * lim / 3) - 1) < 0.05
    assert not P.W2.any() and not P.b1.any() and not P.b2.any()
    assert np.array_equal(mlp.init_params_stream(d, H, 4).W1, P.W1)
    assert not np.array_equal(mlp.init_params_stream(d, H, 5).W1, P.W1)


def test_minibatch_uniform_over_pairs():
    total, batch = 97, 4096
    counts = np.zeros(total)
    for step in range(10):
        u = mlp.minibatch(step, batch, total, 4, 3)
        assert u.min() >= 0 and u.max() < total
        counts += np.bincount(u.astype(np.int64), minlength=total)
    exp = 10 * batch / total
    chi2 = float(((counts - exp) ** 2 / exp).sum())
    assert chi2 < 160            # 96 degrees of freedom; p < 1e-5 above
    assert not np.array_equal(mlp.minibatch(0, 64, total, 4, 3), mlp.minibatch(1, 64, total, 4, 3))
    assert not np.array_equal(mlp.minibatch(0, 64, total, 4, 3), mlp.minibatch(0, 64, total, 4, 4))


def test_train_pairs_learns_and_lr_zero_keeps():
    rng = np.random.default_rng(2)
    d, H, nc, nf = 32, 64, 50, 400
    coarse = rng.normal(size=(nc, d)) * 0.3
    mp = rng.integers(0, nc, size=nf)
    deg = rng.integers(1, 60, size=nf)
    fine = coarse[mp] + 0.05 * np.log1p(deg)[:, None]
    src = [mlp.level_pairs(coarse, fine, mp, deg)]
    P0 = mlp.init_params_stream(d, H, 4)
    P = P0.copy()
    mlp.train_pairs(P, src, 5, 64, 0.0, 4, 1)
    assert np.array_equal(P.W1, P0.W1) and not P.W2.any()
    losses = mlp.train_pairs(P, src, 300, 128, 3e-3, 4, 1)
    assert losses[-10:].mean() < 0.1 * losses[:10].mean()
    # W2 = 0: learned prolongation is the copy
    assert np.array_equal(mlp.prolong_learned(P0, coarse, mp, deg), coarse[mp])
    # the trained network moves every fine row toward its target
    err_l = np.mean((mlp.prolong_learned(P, coarse, mp, deg) - fine) ** 2)
    err_c = np.mean((coarse[mp] - fine) ** 2)
    assert err_l < 0.2 * err_c
