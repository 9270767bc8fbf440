"""Random-walk positive sampling (Section 3.2) on the GPU against the
reference (oracle walk_pairs / train_walks): the shuffled pairs of an epoch
are bit-exact (small graphs with isolated vertices, several levels, tags and
epochs, and the full scale-20 R-MAT train graph); sequential-mode training
matches the reference rows (FP32 and BF16, every d, k from 0 to 15) with the
exact update count; concurrent training keeps the reference's link-prediction
AUC and update count; argument errors and degenerate sizes."""
import numpy as np
import pytest
import torch

from synth import csr_from_pairs, evaluate_auc, init_rows, rmat_csr, split_edges
from tests.conftest import train_split

pytestmark = pytest.mark.gpu

SEED = 4


def _rel_rows(a, b):
    num = np.linalg.norm(a - b, axis=1)
    den = np.maximum(np.linalg.norm(b, axis=1), 1e-30)
    return float((num / den).max()) if len(a) else 0.0


def _graph(scale=9, ef=6, seed=3, extra=3):
    sp = split_edges(*rmat_csr(scale, ef, seed), seed=2)
    off = np.concatenate([sp.offsets, np.full(extra, sp.offsets[-1], sp.offsets.dtype)])
    return off, sp.indices


def _single(gctx, off, idx):
    from paper_2110_10049_amd import gosh as G
    return G.gosh_levels_single(gctx, G.CSR.from_numpy(off, idx))


@pytest.mark.parametrize("length,window,epoch,tag", [(10, 3, 0, 0), (6, 2, 5, 7), (1, 1, 1, 0), (5, 9, 2, 3),
                                                     (40, 10, 0, 1)])
def test_pairs_bit_exact(gctx, orc, length, window, epoch, tag):
    from paper_2110_10049_amd import gosh as G
    off, idx = _graph()
    print(f"[walk pairs] len={length} window={window} epoch={epoch} tag={tag}", flush=True)
    lv = _single(gctx, off, idx)
    src, pos = G.gosh_walk_pairs(gctx, lv, 0, epoch, length, window, tag)
    want_s, want_p = orc.walk_pairs(off, idx, length, window, SEED, tag=tag, epoch=epoch)
    assert np.array_equal(src.cpu().numpy(), want_s)
    assert np.array_equal(pos.cpu().numpy(), want_p)


def test_pairs_bit_exact_on_coarse_levels(gctx, orc):
    from paper_2110_10049_amd import gosh as G
    sp = train_split(12, 16)
    lv = G.gosh_coarsen(gctx, G.CSR.from_numpy(sp.offsets, sp.indices), 64)
    for level in range(lv.count()):
        off, idx, _ = lv.copy_out(level, want_map=False)
        print(f"[walk pairs] coarse level {level} n={len(off) - 1}", flush=True)
        src, pos = G.gosh_walk_pairs(gctx, lv, level, 3, 8, 3, 2)
        want_s, want_p = orc.walk_pairs(off, idx, 8, 3, SEED, level=level, tag=2, epoch=3)
        assert np.array_equal(src.cpu().numpy(), want_s) and np.array_equal(pos.cpu().numpy(), want_p)


def test_pairs_bit_exact_full_scale20(gctx, orc):
    """The scale-20 R-MAT train graph (about 1M vertices, 27M pairs per epoch
    at walk length 10 and window 3): every pair of the epoch."""
    from paper_2110_10049_amd import gosh as G
    sp = train_split(20, 16)
    print(f"[walk pairs] scale 20 n={sp.n}", flush=True)
    lv = _single(gctx, sp.offsets, sp.indices)
    src, pos = G.gosh_walk_pairs(gctx, lv, 0, 1, 10, 3)
    want_s, want_p = orc.walk_pairs(sp.offsets, sp.indices, 10, 3, SEED, epoch=1)
    assert np.array_equal(src.cpu().numpy(), want_s) and np.array_equal(pos.cpu().numpy(), want_p)


@pytest.mark.parametrize("dtype", ["f32", "bf16"])
@pytest.mark.parametrize("d,k,length,window,epochs", [(8, 1, 4, 2, 2), (16, 0, 6, 3, 2), (32, 3, 5, 2, 3),
                                                      (64, 7, 3, 1, 2), (128, 15, 4, 4, 1), (256, 2, 2, 2, 2),
                                                      (16, 1, 20, 2, 1)])
def test_deterministic_matches_reference(gctx, orc, dtype, d, k, length, window, epochs):
    from paper_2110_10049_amd import gosh as G
    off, idx = _graph(8, 5)
    n = len(off) - 1
    print(f"[walk det] {dtype} d={d} k={k} len={length} window={window} e={epochs} n={n}", flush=True)
    lv = _single(gctx, off, idx)
    f = init_rows(n, d, 3) * 8
    lr = 0.045
    cnt = torch.zeros(1, dtype=torch.int64, device="cuda")
    gctx.set_deterministic(True)
    try:
        if dtype == "f32":
            Mg = torch.from_numpy(f.copy()).cuda()
            G.gosh_train_walks(gctx, lv, 0, Mg, epochs, lr, k, length, window, updates=cnt)
            Mo = f.astype(np.float64)
            upd = orc.train_walks(off, idx, Mo, epochs, float(np.float32(lr)), k, length, window, SEED)
            torch.cuda.synchronize()
            assert _rel_rows(Mg.cpu().numpy().astype(np.float64), Mo) < 1e-4
        else:
            bits = orc.f32_to_bf16_rne(f).reshape(n, d)
            Mg = torch.from_numpy(bits.view(np.int16).copy()).view(torch.bfloat16).cuda()
            G.gosh_train_walks(gctx, lv, 0, Mg, epochs, lr, k, length, window, updates=cnt)
            Mo = bits.copy()
            upd = orc.train_walks(off, idx, Mo, epochs, float(np.float32(lr)), k, length, window, SEED)
            torch.cuda.synchronize()
            got = orc.bf16_to_f64(Mg.cpu().view(torch.int16).numpy().view(np.uint16))
            want = orc.bf16_to_f64(Mo)
            assert _rel_rows(got, want) < 2e-2
            assert np.mean(np.abs(got - want).sum(1) / np.abs(want).sum(1)) < 5e-3
    finally:
        gctx.set_deterministic(False)
    assert int(cnt.item()) == upd


def _geometric(n=4000, radius=0.03, seed=0):
    from scipy.spatial import cKDTree
    pts = np.random.default_rng(seed).random((n, 2))
    pairs = np.array(sorted(cKDTree(pts).query_pairs(radius)))
    return split_edges(*csr_from_pairs(n, pairs[:, 0], pairs[:, 1]), seed=2)


@pytest.mark.parametrize("dtype", [torch.float32, torch.bfloat16])
def test_concurrent_auc_matches_reference(gctx, orc, dtype):
    from paper_2110_10049_amd import gosh as G
    sp = _geometric()
    n, d, e, k, length, window = sp.n, 32, 10, 3, 6, 2
    f = init_rows(n, d, 3) * 20
    lv = _single(gctx, sp.offsets, sp.indices)
    Mg = torch.from_numpy(f).to(dtype).cuda()
    cnt = torch.zeros(1, dtype=torch.int64, device="cuda")
    G.gosh_train_walks(gctx, lv, 0, Mg, e, 0.045, k, length, window, updates=cnt)
    bf = dtype == torch.bfloat16
    Mo = orc.f32_to_bf16_rne(f).reshape(n, d) if bf else f.astype(np.float64)
    upd = orc.train_walks(sp.offsets, sp.indices, Mo, e, float(np.float32(0.045)), k, length, window, SEED)
    torch.cuda.synchronize()
    a_g = evaluate_auc(Mg.float().cpu().numpy(), sp, seed=5)
    a_o = evaluate_auc(orc.bf16_to_f64(Mo) if bf else Mo, sp, seed=5)
    print(f"[walk auc] {dtype}: gpu {a_g:.4f} oracle {a_o:.4f}", flush=True)
    assert int(cnt.item()) == upd
    assert a_o > 0.9
    assert abs(a_g - a_o) < 0.01


def test_zero_lr_and_degenerate_sizes(gctx):
    from paper_2110_10049_amd import gosh as G
    off, idx = _graph(8, 5)
    n = len(off) - 1
    lv = _single(gctx, off, idx)
    M = torch.from_numpy(init_rows(n, 32, 3)).cuda()
    M0 = M.clone()
    cnt = torch.zeros(1, dtype=torch.int64, device="cuda")
    G.gosh_train_walks(gctx, lv, 0, M, 2, 0.0, 3, 4, 2, updates=cnt)
    torch.cuda.synchronize()
    assert torch.equal(M, M0) and int(cnt.item()) > 0
    cnt.zero_()
    for epochs, length, window in ((0, 4, 2), (3, 0, 2), (3, 4, 0)):
        G.gosh_train_walks(gctx, lv, 0, M, epochs, 0.05, 3, length, window, updates=cnt)
    torch.cuda.synchronize()
    assert torch.equal(M, M0) and int(cnt.item()) == 0
    s, p = G.gosh_walk_pairs(gctx, lv, 0, 0, 0, 3)
    assert s.numel() == 0 and p.numel() == 0


def test_argument_errors(gctx):
    from paper_2110_10049_amd import gosh as G
    off, idx = _graph(8, 5)
    n = len(off) - 1
    lv = _single(gctx, off, idx)
    M = torch.zeros((n, 32), device="cuda")
    for kw in (dict(walk_len=1025, window=2), dict(walk_len=4, window=-1), dict(walk_len=4, window=2, k=16),
               dict(walk_len=4, window=2, lr=-1.0), dict(walk_len=4, window=2, tag=1 << 24)):
        args = dict(epochs=1, lr=0.05, k=3)
        args.update(kw)
        with pytest.raises(G.GoshError) as ei:
            G.gosh_train_walks(gctx, lv, 0, M, **args)
        assert ei.value.status == "E_INVALID_ARG"
    with pytest.raises(G.GoshError) as ei:
        G.gosh_train_walks(gctx, lv, 0, torch.zeros((n, 12), device="cuda"), 1, 0.05, 3, 4, 2)
    assert ei.value.status == "E_INVALID_ARG"
    # n * P reaches 2^32 (10^4 vertices, 524800 pairs per walk): refused
    # before any allocation
    big = _single(gctx, np.zeros(10001, np.int64), np.zeros(0, np.int32))
    with pytest.raises(G.GoshError) as ei:
        G.gosh_train_walks(gctx, big, 0, torch.zeros((10000, 8), device="cuda"), 1, 0.05, 3, 1024, 1024)
    assert ei.value.status == "E_UNSUPPORTED"
    with pytest.raises(G.GoshError):
        G.gosh_walk_pairs(gctx, lv, 1, 0, 4, 2)          # no such level
