"""Learned prolongation on the GPU against the FP64 reference (oracle/mlp.py):
the forward on real level hierarchies (ragged row counts, both row dtypes,
several widths), the zero output layer against copy prolongation,
gradients on explicit batches, Adam steps, and minibatch training that
lowers the loss.  The reference multiplies the same BF16-rounded weights and
inputs the GPU multiplies; the tolerances below bound what remains: the
GPU's BF16 rounding of hidden activations and output gradients, FP32
accumulation, and (rarely) a one-ulp difference in a rounded log feature."""
import numpy as np
import pytest
import torch

from oracle import mlp as OM
from tests.conftest import train_split

pytestmark = pytest.mark.gpu


def _bf(orc, a):
    """float32 values rounded to BF16 (nearest even), as float64."""
    return orc.bf16_to_f64(orc.f32_to_bf16_rne(np.asarray(a, np.float32)))


def _ulp_bf16(x):
    x = np.maximum(np.abs(x), 1e-30)
    return np.exp2(np.floor(np.log2(x)) - 7)


def _random_weights(d, H, seed, w2_zero=False):
    rng = np.random.default_rng(seed)
    F = d + 2
    W1 = rng.uniform(-1, 1, (H, F)) / np.sqrt(F)
    b1 = rng.normal(0, 0.1, H)
    W2 = np.zeros((d, H)) if w2_zero else rng.uniform(-1, 1, (d, H)) / np.sqrt(H)
    b2 = np.zeros(d) if w2_zero else rng.normal(0, 0.01, d)
    return np.concatenate([W1.ravel(), b1, W2.ravel(), b2]).astype(np.float32)


def _params(orc, flat, d, H, bf16_weights=True):
    F = d + 2
    a = H * F
    W1 = flat[:a].reshape(H, F)
    W2 = flat[a + H:a + H + d * H].reshape(d, H)
    r = (lambda w: _bf(orc, w)) if bf16_weights else (lambda w: w.astype(np.float64))
    return OM.Params(r(W1), flat[a:a + H].astype(np.float64), r(W2), flat[a + H + d * H:].astype(np.float64))


def _rows(t):
    return t.float().cpu().numpy().astype(np.float64)


def _reference(orc, flat, d, H, C, deg, clsz, C_input):
    """FP64 forward on BF16 weights and BF16 inputs; returns (Y, error bound
    scale per element without the output rounding)."""
    P = _params(orc, flat, d, H)
    X = OM.features(C_input, deg, clsz)
    X = _bf(orc, X.astype(np.float32))
    Y, (_, Z1, A1) = OM.forward(P, X, C)
    absW2 = np.abs(P.W2)
    scale = np.abs(A1) @ absW2.T                                  # sum_h |W2[m,h] A1[h]|
    # one BF16 ulp on either log feature, through |gelu'| <= 1.13
    fe = np.stack([_ulp_bf16(X[:, d]), _ulp_bf16(X[:, d + 1])], 1)   # [B, 2]
    zerr = fe @ np.abs(P.W1[:, d:d + 2]).T * 1.13                      # [B, H]
    return Y, scale, zerr @ absW2.T


def _check_close(Yg, Y, scale, ferr, bf16_out):
    tol = 2.0 ** -7 * scale + ferr + 1e-6 * np.abs(Y) + 1e-7
    if bf16_out:
        tol = tol + 2.0 ** -8 * np.abs(Y)
    bad = np.abs(Yg - Y) > tol
    assert not bad.any(), (int(bad.sum()), float(np.max(np.abs(Yg - Y) - tol)))


@pytest.mark.parametrize("dtype", [torch.float32, torch.bfloat16])
@pytest.mark.parametrize("d,H", [(32, 64), (128, 256), (256, 128), (64, 128), (256, 256)])
def test_prolong_matches_reference(gctx, orc, dtype, d, H):
    from paper_2110_10049_amd import gosh as G
    sp = train_split(12, 16)
    g = G.CSR.from_numpy(sp.offsets, sp.indices)
    lv = G.gosh_coarsen(gctx, g, 64)
    net = G.Mlp(gctx, d, H)
    flat = _random_weights(d, H, 7)
    net.set_weights(flat)
    gen = torch.Generator(device="cpu").manual_seed(11)
    print(f"[mlp prolong] d={d} H={H} dtype={dtype}", flush=True)
    for i in range(lv.count() - 1):
        nf, _ = lv.shape(i)
        nc, _ = lv.shape(i + 1)
        coarse = (torch.randn((nc, d), generator=gen) * 0.3).to(dtype).cuda()
        fine = torch.empty((nf, d), device="cuda", dtype=dtype)
        G.gosh_prolong(gctx, lv, i, coarse, fine, mlp=net)
        torch.cuda.synchronize()
        off, _, mp = lv.copy_out(i)
        cs = lv.cluster_sizes(i)
        C = _rows(coarse)[mp]
        Y, scale, ferr = _reference(orc, flat, d, H, C, np.diff(off), cs[mp], C)
        _check_close(_rows(fine), Y, scale, ferr, dtype == torch.bfloat16)


@pytest.mark.parametrize("dtype", [torch.float32, torch.bfloat16])
def test_zero_output_layer_is_copy(gctx, dtype):
    from paper_2110_10049_amd import gosh as G
    sp = train_split(12, 16)
    g = G.CSR.from_numpy(sp.offsets, sp.indices)
    lv = G.gosh_coarsen(gctx, g, 64)
    d, H = 128, 256
    net = G.Mlp(gctx, d, H)
    net.set_weights(_random_weights(d, H, 3, w2_zero=True))
    for i in range(lv.count() - 1):
        nf, _ = lv.shape(i)
        nc, _ = lv.shape(i + 1)
        coarse = torch.randn((nc, d), device="cuda").to(dtype)
        a = torch.empty((nf, d), device="cuda", dtype=dtype)
        b = torch.empty((nf, d), device="cuda", dtype=dtype)
        G.gosh_prolong(gctx, lv, i, coarse, a, mlp=net)
        G.gosh_prolong(gctx, lv, i, coarse, b)
        assert torch.equal(a, b)


def test_new_network_is_copy(gctx):
    # W2 = 0 and b2 = 0 at creation
    from paper_2110_10049_amd import gosh as G
    net = G.Mlp(gctx, 64, 128)
    W1, b1, W2, b2 = net.split(net.get_weights())
    assert np.all(W2 == 0) and np.all(b2 == 0) and np.all(b1 == 0)
    assert np.abs(W1).max() <= 1 / np.sqrt(66) and np.abs(W1).std() > 0.01


def test_weights_roundtrip(gctx):
    from paper_2110_10049_amd import gosh as G
    net = G.Mlp(gctx, 32, 64)
    w = _random_weights(32, 64, 5)
    net.set_weights(w)
    assert np.array_equal(net.get_weights(), w)


def _batch(rng, B, d, dtype):
    C = (rng.normal(size=(B, d)) * 0.3).astype(np.float32)
    T = (C + rng.normal(size=(B, d)) * 0.1).astype(np.float32)
    deg = rng.integers(0, 1000, B).astype(np.int32)
    cs = rng.integers(1, 50, B).astype(np.int32)
    tC = torch.from_numpy(C).to(dtype).cuda()
    tT = torch.from_numpy(T).to(dtype).cuda()
    return tC, tT, torch.from_numpy(deg).cuda(), torch.from_numpy(cs).cuda()


@pytest.mark.parametrize("dtype", [torch.float32, torch.bfloat16])
@pytest.mark.parametrize("d,H,B", [(128, 256, 1000), (128, 256, 1), (32, 64, 100), (256, 256, 333)])
def test_gradients_match_reference(gctx, orc, dtype, d, H, B):
    from paper_2110_10049_amd import gosh as G
    print(f"[mlp grad] d={d} H={H} B={B} dtype={dtype}", flush=True)
    rng = np.random.default_rng(B + d)
    net = G.Mlp(gctx, d, H)
    flat = _random_weights(d, H, 9)
    net.set_weights(flat)
    tC, tT, tdeg, tcs = _batch(rng, B, d, dtype)
    g, loss = net.grad(tC, tdeg, tcs, tT)
    g = g.cpu().numpy().astype(np.float64)
    P = _params(orc, flat, d, H)
    C = _rows(tC)
    X = _bf(orc, OM.features(C, tdeg.cpu().numpy(), tcs.cpu().numpy()).astype(np.float32))
    Y, cache = OM.forward(P, X, C)
    T = _rows(tT)
    ref = OM.backward(P, Y, T, cache)
    assert loss == pytest.approx(OM.mse(Y, T), rel=1e-2)
    got = net.split(g)
    tol = _grad_bounds(P, Y, T, cache)
    for name, gg in zip(("W1", "b1", "W2", "b2"), got):
        rr = getattr(ref, name)
        rel = np.linalg.norm(gg - rr) / max(np.linalg.norm(rr), 1e-30)
        ratio = np.abs(gg - rr) / tol[name]
        print(f"  {name} rel err {rel:.2e}, max |err| / bound {ratio.max():.3f}", flush=True)
        assert rel < 2e-2, (name, rel)
        # element by element, within the bound of the kernel's rounding points
        assert np.all(ratio <= 1.0), (name, float(ratio.max()))
    # the padding of the first layer's input never leaks into W1's gradient columns
    assert np.all(np.isfinite(g))


def _grad_bounds(P, Y, T, cache):
    """Per-element bound on |GPU gradient - FP64 gradient| when both multiply
    the same BF16 weights and BF16 inputs X, and the GPU (as documented for
    gosh_mlp_grad) also rounds the hidden activations A1, the output gradient
    dY and the hidden gradient dZ1 to BF16 (relative error <= u = 2^-9 each,
    round to nearest) and accumulates in FP32:
      |dY err|  <= u |dY| + (2 / (B d)) eY,  eY = u |A1| |W2|^T (the output's
                   error from A1's rounding)
      |dW2 err| <= |dY err|^T |A1| + u |dY|^T |A1|
      |dZ1 err| <= ((|dY err|) |W2|) * |gelu'(Z1)| + u |dZ1| (+ the kernel's
                   GELU', whose error is far below u)
      |dW1 err| <= |dZ1 err|^T |X|,  |db1 err| <= sum_b |dZ1 err|,
      |db2 err| <= sum_b |dY err|
    each doubled (second-order terms and FP32 accumulation), plus 1e-6 of the
    largest |gradient| of the tensor (FP32 sums that cancel)."""
    X, Z1, A1 = cache
    B, d = Y.shape
    u = 2.0 ** -9
    dY = 2.0 * (Y - T) / (B * d)
    eY = u * (np.abs(A1) @ np.abs(P.W2).T)
    edY = u * np.abs(dY) + (2.0 / (B * d)) * eY
    dZ1 = (dY @ P.W2) * OM.gelu_grad(Z1)
    edZ1 = (edY @ np.abs(P.W2)) * np.abs(OM.gelu_grad(Z1)) + u * np.abs(dZ1)
    raw = {"W2": edY.T @ np.abs(A1) + u * (np.abs(dY).T @ np.abs(A1)),
           "b2": edY.sum(0),
           "W1": edZ1.T @ np.abs(X),
           "b1": edZ1.sum(0)}
    ref = {"W2": dY.T @ A1, "b2": dY.sum(0), "W1": dZ1.T @ X, "b1": dZ1.sum(0)}
    return {k: 2.0 * v + 1e-6 * np.abs(ref[k]).max() for k, v in raw.items()}


def test_adam_steps_match_reference(gctx):
    from paper_2110_10049_amd import gosh as G
    d, H = 64, 128
    net = G.Mlp(gctx, d, H)
    flat = _random_weights(d, H, 13)
    net.set_weights(flat)
    rng = np.random.default_rng(2)
    P = OM.Params(*[x.astype(np.float64).copy() for x in net.split(flat)])
    S = OM.adam_init(P)
    for lr in (1e-3, 3e-3, 1e-3):
        g = rng.normal(size=net.nparams) * rng.choice([1e-6, 1e-3, 1.0], size=net.nparams)
        net.adam_step(torch.from_numpy(g.astype(np.float32)).cuda(), lr)
        g32 = g.astype(np.float32).astype(np.float64)
        OM.adam_step(P, OM.Params(*net.split(g32)), S, lr)
    want = np.concatenate([P.W1.ravel(), P.b1, P.W2.ravel(), P.b2])
    got = net.get_weights().astype(np.float64)
    assert np.allclose(got, want, rtol=0, atol=1e-6)


def test_training_lowers_loss_and_beats_copy(gctx):
    # fine rows are a fixed function of the coarse row and the fine degree
    from paper_2110_10049_amd import gosh as G
    sp = train_split(12, 16)
    g = G.CSR.from_numpy(sp.offsets, sp.indices)
    lv = G.gosh_coarsen(gctx, g, 64)
    d, H = 32, 64
    rng = np.random.default_rng(4)
    srcs, keep = [], []
    for i in range(lv.count() - 1):
        nf, _ = lv.shape(i)
        nc, _ = lv.shape(i + 1)
        off, _, mp = lv.copy_out(i)
        Cc = (rng.normal(size=(nc, d)) * 0.3).astype(np.float32)
        T = 0.5 * Cc[mp] + 0.05 * np.log1p(np.diff(off))[:, None].astype(np.float32)
        coarse = torch.from_numpy(Cc).cuda()
        fine = torch.from_numpy(T.astype(np.float32)).cuda()
        srcs.append((lv, i, coarse, fine))
        keep.append((T, mp))
    net = G.Mlp(gctx, d, H)
    losses = net.train(srcs, steps=400, batch=256, lr=1e-2, tag=1).cpu().numpy()
    assert np.all(np.isfinite(losses))
    first, last = losses[:10].mean(), losses[-10:].mean()
    print(f"[mlp train] loss {first:.4g} -> {last:.4g}", flush=True)
    assert last < 0.1 * first
    lv0, i0, coarse0, fine0 = srcs[0]
    out = torch.empty_like(fine0)
    G.gosh_prolong(gctx, lv0, 0, coarse0, out, mlp=net)
    cp = torch.empty_like(fine0)
    G.gosh_prolong(gctx, lv0, 0, coarse0, cp)
    e_mlp = torch.mean((out - fine0) ** 2).item()
    e_copy = torch.mean((cp - fine0) ** 2).item()
    assert e_mlp < 0.2 * e_copy


def test_training_is_deterministic(gctx):
    from paper_2110_10049_amd import gosh as G
    sp = train_split(12, 16)
    g = G.CSR.from_numpy(sp.offsets, sp.indices)
    lv = G.gosh_coarsen(gctx, g, 64)
    nf, _ = lv.shape(0)
    nc, _ = lv.shape(1)
    coarse = torch.randn((nc, 64), device="cuda").to(torch.bfloat16)
    fine = torch.randn((nf, 64), device="cuda").to(torch.bfloat16)
    ws = []
    for _ in range(2):
        net = G.Mlp(gctx, 64, 128)
        net.train([(lv, 0, coarse, fine)], steps=20, batch=100, lr=1e-3, tag=5)
        ws.append(net.get_weights())
    assert np.array_equal(ws[0], ws[1])


def test_mlp_argument_errors(gctx):
    from paper_2110_10049_amd import gosh as G
    for d, H in ((48, 64), (128, 32), (8, 64), (128, 512)):
        with pytest.raises(G.GoshError) as ei:
            G.Mlp(gctx, d, H)
        assert ei.value.status == "E_INVALID_ARG"
    sp = train_split(12, 16)
    g = G.CSR.from_numpy(sp.offsets, sp.indices)
    lv = G.gosh_coarsen(gctx, g, 64)
    net = G.Mlp(gctx, 64, 64)
    nf, _ = lv.shape(0)
    nc, _ = lv.shape(1)
    c = torch.zeros((nc, 32), device="cuda")
    f = torch.zeros((nf, 32), device="cuda")
    with pytest.raises(G.GoshError):
        G.gosh_prolong(gctx, lv, 0, c, f, mlp=net)          # d differs from the network's
    last = lv.count() - 1
    with pytest.raises(G.GoshError):
        net.train([(lv, 0, torch.zeros((nc, 64), device="cuda"), torch.zeros((nf, 64), device="cuda"))],
                  steps=1, batch=0, lr=1e-3)
    with pytest.raises(G.GoshError):
        net.adam_step(torch.zeros(net.nparams, device="cuda"), float("nan"))
    assert last >= 1


def test_prolong_full_size_sampled_rows(gctx, orc):
    # level 0 -> 1 of the scale-22 R-MAT graph (edge factor 16, isolated
    # vertices removed), d = 128, 256 hidden units, BF16 rows: the launch the
    # benchmark times; 4096 sampled rows against the reference
    from paper_2110_10049_amd import gosh as G
    from synth.rmat import drop_isolated_torch, rmat_csr_torch
    print("[mlp full size] scale 22", flush=True)
    off, idx = rmat_csr_torch(22, 16, 1, "cuda")
    off, idx, _ = drop_isolated_torch(off, idx)
    g = G.CSR(off.contiguous(), idx.contiguous())
    lv = G.gosh_coarsen(gctx, g, 100)
    d, H = 128, 256
    net = G.Mlp(gctx, d, H)
    flat = _random_weights(d, H, 21)
    net.set_weights(flat)
    n0, _ = lv.shape(0)
    n1, _ = lv.shape(1)
    gen = torch.Generator(device="cpu").manual_seed(5)
    coarse = (torch.randn((n1, d), generator=gen) * 0.3).to(torch.bfloat16).cuda()
    fine = torch.empty((n0, d), device="cuda", dtype=torch.bfloat16)
    G.gosh_prolong(gctx, lv, 0, coarse, fine, mlp=net)
    torch.cuda.synchronize()
    o, _, mp = lv.copy_out(0)
    cs = lv.cluster_sizes(0)
    rows = np.random.default_rng(8).choice(n0, 4096, replace=False)
    rows = np.concatenate([rows, [0, n0 - 1]])
    C = _rows(coarse)[mp[rows]]
    Y, scale, ferr = _reference(orc, flat, d, H, C, (o[rows + 1] - o[rows]), cs[mp[rows]], C)
    _check_close(_rows(fine[torch.from_numpy(rows).cuda()]), Y, scale, ferr, True)
