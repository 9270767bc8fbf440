"""Pins of the oracle's UpdateEmbed (Algorithm 1) and training loop
(Algorithm 3): closed forms, finite differences of the logistic loss of
Section 2, invariants of the update order, and BF16 stochastic rounding."""
import math

import numpy as np
import pytest

from synth import rmat_csr


def test_closed_form_d1(orc):
    # d = 1, one positive: score = (1 - sigma(vu)) lr; v' = v + score u;
    # u' = u + score v'.
    v, u, lr = 0.5, -0.25, 0.1
    M = np.array([[v], [u]], dtype=np.float64)
    orc.visit(M, 0, [1], lr)
    x = v * u
    g = (1.0 - 1.0 / (1.0 + math.exp(-x))) * lr
    v1 = v + g * u
    u1 = u + g * v1
    assert M[0, 0] == pytest.approx(v1, rel=1e-15)
    assert M[1, 0] == pytest.approx(u1, rel=1e-15)


def test_lr_zero_is_identity(orc):
    rng = np.random.default_rng(0)
    M = rng.normal(size=(6, 16))
    M0 = M.copy()
    orc.visit(M, 2, [3, 4, 5, 1], 0.0)
    assert np.array_equal(M, M0)


@pytest.mark.parametrize("b", [0, 1])
def test_gradient_matches_finite_differences(orc, b):
    # (s' - s) / lr = (b - sigma(s.u)) u must equal -dL/ds of
    # L = -[b log sigma(x) + (1-b) log(1-sigma(x))], x = s.u.
    rng = np.random.default_rng(1 + b)
    d = 8
    s = rng.normal(size=d) * 0.7
    u = rng.normal(size=d) * 0.7
    lr = 1e-3
    M = np.stack([s, u]).copy()
    samples = [1] if b == 1 else [-1, 1]
    orc.visit(M, 0, samples, lr)
    step = (M[0] - s) / lr
    h = 1e-6
    fd = np.zeros(d)
    for e in range(d):
        sp, sm = s.copy(), s.copy()
        sp[e] += h
        sm[e] -= h
        fd[e] = (orc.loss(float(sp @ u), b) - orc.loss(float(sm @ u), b)) / (2 * h)
    assert np.allclose(step, -fd, rtol=1e-7, atol=1e-9)
    # the sample-side gradient is symmetric: -dL/du = (b - sigma) s
    gu = np.zeros(d)
    for e in range(d):
        up, um = u.copy(), u.copy()
        up[e] += h
        um[e] -= h
        gu[e] = (orc.loss(float(s @ up), b) - orc.loss(float(s @ um), b)) / (2 * h)
    sig = 1 / (1 + math.exp(-float(s @ u)))
    assert np.allclose((b - sig) * s, -gu, rtol=1e-7, atol=1e-9)


def test_loss_stable_tails(orc):
    assert orc.loss(800.0, 1) == pytest.approx(0.0, abs=1e-300)
    assert orc.loss(-800.0, 1) == pytest.approx(800.0)
    assert orc.loss(800.0, 0) == pytest.approx(800.0)
    assert orc.loss(0.0, 1) == pytest.approx(math.log(2.0))


def test_edge_points_pull_together(orc):
    # With the sample row updated from the already-updated source row,
    # v'.u' - v.u = g (|u|^2 + |v|^2 + 2 g v.u + g^2 |u|^2): a positive update
    # (g > 0) raises the dot product, a negative one lowers it.
    rng = np.random.default_rng(7)
    for trial in range(20):
        d = 16
        v = rng.normal(size=d) * 0.3
        u = rng.normal(size=d) * 0.3
        lr = 0.05
        for b in (1, 0):
            M = np.stack([v, u]).copy()
            orc.visit(M, 0, [1] if b else [-1, 1], lr)
            x = v @ u
            g = (b - 1 / (1 + math.exp(-x))) * lr
            pred = g * (u @ u + v @ v + 2 * g * x + g * g * (u @ u))
            assert M[0] @ M[1] - x == pytest.approx(pred, rel=1e-9, abs=1e-15)
            assert (M[0] @ M[1] > x) == (b == 1)


def test_k2_converges(orc):
    # K_2, positives only: the dot product rises every epoch and sigma -> 1.
    off = np.array([0, 1, 2], np.int64)
    idx = np.array([1, 0], np.int32)
    M = np.array([[0.01, -0.02, 0.03], [0.02, 0.01, -0.01]], dtype=np.float64)
    last = M[0] @ M[1]
    for ep in range(200):
        orc.train(off, idx, M, 1, 0.5, 0, seed=1, level=0)
        cur = M[0] @ M[1]
        assert cur > last
        last = cur
    assert 1 / (1 + math.exp(-last)) > 0.95


def test_repeated_sample_sees_earlier_update(orc):
    # Sequential semantics within one source: samples [u, u] equal two
    # visits with [u] (FP64 storage makes the write-back/re-read exact).
    rng = np.random.default_rng(3)
    M = rng.normal(size=(5, 8)) * 0.2
    A = M.copy()
    orc.visit(A, 0, [-1, 3, 3], 0.03)
    B = M.copy()
    orc.visit(B, 0, [-1, 3], 0.03)
    orc.visit(B, 0, [-1, 3], 0.03)
    assert np.array_equal(A, B)


def test_skip_rules(orc):
    rng = np.random.default_rng(4)
    M = rng.normal(size=(4, 8))
    M0 = M.copy()
    assert orc.visit(M, 2, [-1, 2, 2], 0.1) == 0      # no positive, negatives == src
    assert np.array_equal(M, M0)
    assert orc.visit(M, 2, [1, 2, 3], 0.1) == 2
    assert np.array_equal(M[0], M0[0])


def test_update_batch_is_sequential_visits(orc):
    rng = np.random.default_rng(5)
    M = rng.normal(size=(10, 4))
    src = np.array([0, 4, 1])
    samp = np.array([[2, 3], [5, 6], [7, -1]], np.int32)
    A = M.copy()
    assert orc.update_batch(A, src, samp, 0.02) == 5
    B = M.copy()
    for s, sm in zip(src, samp):
        orc.visit(B, int(s), sm, 0.02)
    assert np.array_equal(A, B)


# ---------------------------------------------------------------- BF16 + SR
def _bf16_neighbours(x):
    u = np.float32(x).view(np.uint32)
    lo = np.uint16(u >> 16)
    return {int(lo), int(lo) + 1}


def test_sr_result_is_a_neighbour(orc):
    rng = np.random.default_rng(8)
    for x in rng.normal(size=300).astype(np.float32):
        for r in (0, 1, 0x7FFF, 0x8000, 0xFFFF, int(rng.integers(0, 65536))):
            h = orc.bf16_sr(float(x), r)
            assert h in _bf16_neighbours(x)
    assert orc.bf16_sr(1.0, 0xFFFF) == 0x3F80          # exact values never move
    assert orc.bf16_sr(float("inf"), 0xFFFF) == 0x7F80


def test_sr_unbiased(orc):
    # mean of 1e5 stochastic roundings of x equals x within 4 standard errors
    rng = np.random.default_rng(9)
    for x in (0.123456789, -3.3e-3, 7.77e4):
        lo = orc.bf16_to_f64(np.array([np.float32(x).view(np.uint32) >> 16], np.uint16))[0]
        r = rng.integers(0, 65536, size=100000)
        hs = np.array([orc.bf16_sr(x, int(v)) for v in r], np.uint16)
        vals = orc.bf16_to_f64(hs)
        spacing = abs(orc.bf16_to_f64(np.array([(np.float32(x).view(np.uint32) >> 16) + 1], np.uint16))[0] - lo)
        se = spacing * 0.5 / math.sqrt(len(r))
        assert abs(vals.mean() - float(np.float32(x))) < 4 * se


def test_rne_matches_numpy_cast(orc):
    import torch
    rng = np.random.default_rng(10)
    x = rng.normal(size=4096).astype(np.float32) * 10
    ours = orc.f32_to_bf16_rne(x)
    ref = torch.from_numpy(x).to(torch.bfloat16).view(torch.int16).numpy().view(np.uint16)
    assert np.array_equal(ours, ref)
    for v in x[:64]:
        assert orc.bf16_rne(float(v)) == int(orc.f32_to_bf16_rne(np.array([v]))[0])


def test_bf16_visit_uses_sr_bits(orc):
    # Sample-row element e of slot t is SR-rounded with the bits of (kind 1,
    # slot t, element e); the source row with slot 0xFF at write-back.
    rng = np.random.default_rng(11)
    d = 16
    f = rng.normal(size=(3, d)).astype(np.float32) * 0.3
    M = orc.f32_to_bf16_rne(f).reshape(3, d)
    s = orc.bf16_to_f64(M[0])
    m = orc.bf16_to_f64(M[1])
    lr, seed, level, tag, ep = 0.05, 99, 2, 3, 4
    x = s @ m
    g = (1.0 - 1.0 / (1.0 + math.exp(-x))) * lr
    s1 = s + g * m
    m1 = m + g * s1
    orc.visit(M, 0, [1], lr, seed, level, tag, ep)
    for e in range(d):
        assert M[1, e] == orc.bf16_sr(float(np.float32(m1[e])), orc.sr_bits(seed, level, tag, ep, 0, 0, e, d))
        assert M[0, e] == orc.bf16_sr(float(np.float32(s1[e])), orc.sr_bits(seed, level, tag, ep, 0, 0xFF, e, d))


def test_train_lr_schedule_and_determinism(orc):
    off, idx = rmat_csr(7, 6, seed=2)
    n = len(off) - 1
    rng = np.random.default_rng(12)
    M = rng.uniform(-0.5 / 16, 0.5 / 16, size=(n, 16))
    A, B = M.copy(), M.copy()
    ua = orc.train(off, idx, A, 3, 0.045, 2, seed=4, level=1)
    ub = orc.train(off, idx, B, 3, 0.045, 2, seed=4, level=1)
    assert ua == ub and np.array_equal(A, B)
    # equals explicit epochs: lr' = lr max(1 - j/e, 1e-4), samples of epoch j
    C = M.copy()
    for j in range(3):
        lrj = orc.lr_at(0.045, j, 3)
        samp = orc.draw_all(off, idx, 4, 1, 0, j, 2)
        orc.update_batch(C, np.arange(n), samp, lrj, seed=4, level=1, epoch=j)
    assert np.array_equal(A, C)
    deg0 = int((np.diff(off) == 0).sum())
    assert ua <= 3 * n * 3 and ua >= 3 * (n - deg0)


def test_hogwild_trainer_one_thread_is_sequential(orc):
    # the all-core timing variant with one thread is orc.train exactly; with
    # several threads it executes the same number of updates
    from synth import init_rows, rmat_csr
    off, idx = rmat_csr(10, 8, seed=5)
    n = len(off) - 1
    A = init_rows(n, 16, 3).astype(np.float64)
    B = A.copy()
    C = A.copy()
    u1 = orc.train(off, idx, A, 3, 0.05, 2, 4, level=1, tag=3)
    u2 = orc.train_hogwild(off, idx, B, 3, 0.05, 2, 4, 1, level=1, tag=3)
    u3 = orc.train_hogwild(off, idx, C, 3, 0.05, 2, 4, 4, level=1, tag=3)
    assert u1 == u2 == u3
    assert np.array_equal(A, B)
    assert np.all(np.isfinite(C)) and np.abs(C - A).max() < 0.05


@pytest.mark.parametrize("a", [0.0, 0.7, 2.5])
def test_running_loss_closed_form(orc, a):
    # lr = 0 and every row a * e_1: every update reads the dot a^2, so an
    # epoch's running loss (Section 2's objective over its executed updates)
    # is P log(1 + e^-a^2) + N log(1 + e^a^2), P and N its executed positive
    # and negative updates; the rows never change
    off, idx = rmat_csr(8, 4, seed=9)          # some vertices without neighbours
    n, d, k, epochs = len(off) - 1, 8, 3, 3
    M = np.zeros((n, d))
    M[:, 0] = a
    M0 = M.copy()
    u, loss = orc.train_loss(off, idx, M, epochs, 0.0, k, 4, level=2, tag=1)
    assert np.array_equal(M, M0)
    x = a * a
    total = 0
    for ep in range(epochs):
        dr = orc.draw_all(off, idx, 4, 2, 1, ep, k)
        src = np.arange(n)[:, None]
        P = int((dr[:, 0] >= 0).sum())
        N = int(((dr[:, 1:] >= 0) & (dr[:, 1:] != src)).sum())
        want = P * math.log1p(math.exp(-x)) + N * math.log1p(math.exp(x))
        assert loss[ep] == pytest.approx(want, rel=1e-12)
        total += P + N
    assert u == total
