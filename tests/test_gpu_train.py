"""TrainInGPU / UpdateEmbed / ExpandEmbedding on the GPU against the oracle.

* samples drawn on the device equal the oracle's Philox draws bit for bit;
* conflict-free update batches match within 1e-5 (FP32) and 5e-3 (BF16)
  relative per row;
* sequential-mode training equals the oracle's sequential Algorithm 3;
* copy prolongation is bit-exact.
"""
import numpy as np
import pytest
import torch

from synth import init_rows, rmat_csr
from tests.conftest import train_split

pytestmark = pytest.mark.gpu
SEED = 4


def _rel_rows(a, b):
    """max over rows of ||a - b|| / max(||b||, tiny)."""
    num = np.linalg.norm(a - b, axis=1)
    den = np.maximum(np.linalg.norm(b, axis=1), 1e-30)
    return float((num / den).max()) if len(a) else 0.0


def _bf16_bits(t: torch.Tensor) -> np.ndarray:
    return t.cpu().view(torch.int16).numpy().view(np.uint16)


def _to_dev_bf16(bits: np.ndarray) -> torch.Tensor:
    return torch.from_numpy(bits.view(np.int16).copy()).view(torch.bfloat16).cuda()


@pytest.mark.parametrize("k", [0, 1, 3, 5, 15])
def test_draw_samples_bit_exact(gctx, orc, k):
    from paper_2110_10049_amd import gosh as G
    sp = train_split(12, 16)
    print(f"[draw] k={k}", flush=True)
    g = G.CSR.from_numpy(sp.offsets, sp.indices)
    lv = G.gosh_coarsen(gctx, g, 64)
    for level in (0, lv.count() - 1):
        off, idx, _ = lv.copy_out(level, want_map=False)
        for epoch, tag in ((0, 0), (7, 3)):
            got = G.gosh_draw_samples(gctx, lv, level, epoch, k, tag).cpu().numpy()
            n = len(off) - 1
            want = np.stack([orc.draw_samples(off, idx, SEED, level, tag, epoch, s, k) for s in range(n)])
            assert np.array_equal(got, want)


def _conflict_free_batch(rng, n, nsrc, k, allow_repeat=True):
    """Sources and samples such that no row is touched by two sources."""
    perm = rng.permutation(n)
    src = perm[:nsrc]
    pool = perm[nsrc:]
    need = nsrc * (1 + k)
    assert len(pool) >= need
    samp = pool[:need].reshape(nsrc, 1 + k).astype(np.int32)
    if allow_repeat and k >= 2:
        samp[::3, 2] = samp[::3, 1]          # repeated negative within a source
        samp[1::4, 0] = samp[1::4, k]        # positive equal to a later negative
    if k >= 1:
        samp[::5, 1] = src[::5]              # negative equal to the source: skipped
    samp[2::7, 0] = -1                       # no positive (isolated source)
    return src.astype(np.int32), samp


@pytest.mark.parametrize("d", [8, 16, 32, 64, 128, 256])
@pytest.mark.parametrize("k", [0, 1, 3, 7, 15])
def test_update_batch_fp32(gctx, orc, d, k):
    from paper_2110_10049_amd import gosh as G
    rng = np.random.default_rng(100 + d + k)
    n = 4096 + 37
    nsrc = min(200, n // (2 + k) - 1)
    print(f"[update fp32] d={d} k={k} nsrc={nsrc}", flush=True)
    M0 = rng.uniform(-0.5, 0.5, size=(n, d)).astype(np.float32)
    src, samp = _conflict_free_batch(rng, n, nsrc, k)
    Mg = torch.from_numpy(M0).cuda()
    G.gosh_update_batch(gctx, Mg, torch.from_numpy(src).cuda(), torch.from_numpy(samp).cuda(), 0.05,
                        level=2, tag=1, epoch=3)
    Mo = M0.astype(np.float64)
    orc.update_batch(Mo, src, samp, float(np.float32(0.05)), SEED, 2, 1, 3)
    got = Mg.cpu().numpy().astype(np.float64)
    touched = np.unique(np.concatenate([src, samp[samp >= 0].ravel()]))
    assert _rel_rows(got[touched], Mo[touched]) < 1e-5
    untouched = np.setdiff1d(np.arange(n), touched)
    assert np.array_equal(got[untouched], M0[untouched].astype(np.float64))


@pytest.mark.parametrize("d", [8, 16, 32, 64, 128, 256])
@pytest.mark.parametrize("k", [1, 3, 15])
def test_update_batch_bf16(gctx, orc, d, k):
    from paper_2110_10049_amd import gosh as G
    rng = np.random.default_rng(200 + d + k)
    n = 3000 + 11
    nsrc = min(150, n // (2 + k) - 1)
    print(f"[update bf16] d={d} k={k} nsrc={nsrc}", flush=True)
    f = rng.uniform(-0.5, 0.5, size=(n, d)).astype(np.float32)
    bits = orc.f32_to_bf16_rne(f).reshape(n, d)
    src, samp = _conflict_free_batch(rng, n, nsrc, k)
    Mg = _to_dev_bf16(bits)
    G.gosh_update_batch(gctx, Mg, torch.from_numpy(src).cuda(), torch.from_numpy(samp).cuda(), 0.05,
                        level=1, tag=2, epoch=5)
    Mo = bits.copy()
    orc.update_batch(Mo, src, samp, float(np.float32(0.05)), SEED, 1, 2, 5)
    got = orc.bf16_to_f64(_bf16_bits(Mg))
    want = orc.bf16_to_f64(Mo)
    touched = np.unique(np.concatenate([src, samp[samp >= 0].ravel()]))
    assert _rel_rows(got[touched], want[touched]) < 5e-3
    # most elements round identically (same random bits, FP32 vs FP64 inputs)
    same = np.mean(_bf16_bits(Mg)[touched] == Mo[touched])
    assert same > 0.99
    untouched = np.setdiff1d(np.arange(n), touched)
    assert np.array_equal(_bf16_bits(Mg)[untouched], bits[untouched])


def test_update_batch_skips_out_of_range(gctx):
    from paper_2110_10049_amd import gosh as G
    M = torch.ones((10, 32), device="cuda")
    src = torch.tensor([0, 12, -3], dtype=torch.int32, device="cuda")
    samp = torch.tensor([[99, -5], [1, 2], [3, 4]], dtype=torch.int32, device="cuda")
    G.gosh_update_batch(gctx, M, src, samp, 0.1)
    torch.cuda.synchronize()
    assert torch.all(M == 1)


@pytest.mark.parametrize("dtype", ["f32", "bf16"])
@pytest.mark.parametrize("d,k", [(32, 1), (128, 3)])
def test_sequential_training_matches_oracle(gctx, orc, dtype, d, k):
    from paper_2110_10049_amd import gosh as G
    off, idx = rmat_csr(9, 6, seed=3)
    n = len(off) - 1
    epochs = 3
    print(f"[sequential train] {dtype} d={d} k={k} n={n}", flush=True)
    g = G.CSR.from_numpy(off, idx)
    lv = G.gosh_levels_single(gctx, g)
    f = init_rows(n, d, 3)
    lr = 0.045
    gctx.set_deterministic(True)
    try:
        if dtype == "f32":
            Mg = torch.from_numpy(f).cuda()
            G.gosh_train(gctx, lv, 0, Mg, epochs, lr, k)
            Mo = f.astype(np.float64)
            orc.train(off, idx, Mo, epochs, float(np.float32(lr)), k, SEED, level=0)
            got = Mg.cpu().numpy().astype(np.float64)
            assert _rel_rows(got, Mo) < 1e-4
        else:
            bits = orc.f32_to_bf16_rne(f).reshape(n, d)
            Mg = _to_dev_bf16(bits)
            G.gosh_train(gctx, lv, 0, Mg, epochs, lr, k)
            Mo = bits.copy()
            orc.train(off, idx, Mo, epochs, float(np.float32(lr)), k, SEED, level=0)
            got = orc.bf16_to_f64(_bf16_bits(Mg))
            want = orc.bf16_to_f64(Mo)
            assert _rel_rows(got, want) < 2e-2
            assert np.mean(np.abs(got - want).sum(1) / np.abs(want).sum(1)) < 5e-3
    finally:
        gctx.set_deterministic(False)


def test_update_counter(gctx, orc):
    from paper_2110_10049_amd import gosh as G
    off, idx = rmat_csr(10, 4, seed=9)          # has isolated vertices
    n = len(off) - 1
    g = G.CSR.from_numpy(off, idx)
    lv = G.gosh_levels_single(gctx, g)
    M = torch.from_numpy(init_rows(n, 64, 3)).cuda()
    cnt = torch.zeros(1, dtype=torch.int64, device="cuda")
    G.gosh_train(gctx, lv, 0, M, 4, 0.02, 3, updates=cnt)
    torch.cuda.synchronize()
    # executed updates = every positive of a vertex with neighbours + every
    # negative that is not the source itself
    want = 0
    for ep in range(4):
        s = np.stack([orc.draw_samples(off, idx, SEED, 0, 0, ep, v, 3) for v in range(n)])
        want += int((s[:, 0] >= 0).sum()) + int((s[:, 1:] != np.arange(n)[:, None]).sum())
    assert int(cnt.item()) == want


@pytest.mark.parametrize("dtype", [torch.float32, torch.bfloat16])
def test_prolong_bit_exact(gctx, orc, dtype):
    from paper_2110_10049_amd import gosh as G
    sp = train_split(12, 16)
    g = G.CSR.from_numpy(sp.offsets, sp.indices)
    lv = G.gosh_coarsen(gctx, g, 64)
    for d in (8, 128, 256):
        for i in range(lv.count() - 1):
            nf, _ = lv.shape(i)
            nc, _ = lv.shape(i + 1)
            coarse = torch.randn((nc, d), device="cuda").to(dtype)
            fine = torch.empty((nf, d), device="cuda", dtype=dtype)
            G.gosh_prolong(gctx, lv, i, coarse, fine)
            _, _, mp = lv.copy_out(i)
            want = coarse.cpu()[torch.from_numpy(mp.astype(np.int64))]
            assert torch.equal(fine.cpu(), want)


def test_train_argument_errors(gctx):
    from paper_2110_10049_amd import gosh as G
    off, idx = rmat_csr(6, 4, seed=1)
    lv = G.gosh_levels_single(gctx, G.CSR.from_numpy(off, idx))
    M = torch.zeros((64, 32), device="cuda")
    for kw in (dict(k=16), dict(k=-1), dict(lr=float("nan")), dict(lr=-1.0)):
        args = dict(epochs=1, lr=0.1, k=1)
        args.update(kw)
        with pytest.raises(G.GoshError) as ei:
            G.gosh_train(gctx, lv, 0, M, **args)
        assert ei.value.status == "E_INVALID_ARG"
    with pytest.raises(G.GoshError):
        G.gosh_train(gctx, lv, 0, torch.zeros((64, 24), device="cuda"), 1, 0.1, 1)   # d = 24
    with pytest.raises(G.GoshError):
        G.gosh_train(gctx, lv, 3, M, 1, 0.1, 1)                                      # no level 3


def test_full_scale20_bench_configuration(gctx, orc):
    """The launch the benchmark times, at full size: level 0 of the scale-20
    R-MAT train graph (614k sources), k = 3, d = 128, BF16 rows, plain
    negative stores.  The samples of 20,000 sampled sources (and the first and
    last) equal the oracle's draws bit for bit; an epoch at lr = 0 leaves every
    row bit-identical and executes exactly the oracle's update count."""
    from paper_2110_10049_amd import gosh as G
    sp = train_split(20, 16)
    n, k, d, epoch = sp.n, 3, 128, 5
    print(f"[full scale 20] n={n}", flush=True)
    lv = G.gosh_levels_single(gctx, G.CSR.from_numpy(sp.offsets, sp.indices))
    got = G.gosh_draw_samples(gctx, lv, 0, epoch, k).cpu().numpy()
    rng = np.random.default_rng(9)
    srcs = np.unique(np.concatenate([rng.integers(0, n, 20000), [0, n - 1]]))
    want = np.stack([orc.draw_samples(sp.offsets, sp.indices, SEED, 0, 0, epoch, int(s), k) for s in srcs])
    assert np.array_equal(got[srcs], want)

    M0 = torch.from_numpy(init_rows(n, d, 3)).to(torch.bfloat16).cuda()
    M = M0.clone()
    cnt = torch.zeros(1, dtype=torch.int64, device="cuda")
    gctx.set_plain_negatives(65536)
    gctx.set_plain_light_rows(65536)
    try:
        G.gosh_train(gctx, lv, 0, M, 1, 0.0, k, 0, cnt)
        torch.cuda.synchronize()
    finally:
        gctx.set_plain_negatives(0)
        gctx.set_plain_light_rows(0)
    assert torch.equal(M.view(torch.int16), M0.view(torch.int16))
    # the update count does not depend on d: the oracle runs with 8-wide rows
    upd = orc.train(sp.offsets, sp.indices, np.zeros((n, 8)), 1, 0.0, k, SEED)
    assert int(cnt.item()) == upd


def test_stream_switch_keeps_results(gctx):
    """An epoch queued on a side stream, then the context moved back to the
    default stream: the switch waits for the queued epoch, and its result
    equals the same epoch run on the default stream (deterministic mode)."""
    from paper_2110_10049_amd import gosh as G
    sp = train_split(12, 16)
    lv = G.gosh_levels_single(gctx, G.CSR.from_numpy(sp.offsets, sp.indices))
    M0 = torch.from_numpy(init_rows(sp.n, 32, 3) * 8).cuda()
    M, one = M0.clone(), M0.clone()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    gctx.set_deterministic(True)
    try:
        with torch.cuda.stream(side):
            gctx.use_current_stream()
            G.gosh_train(gctx, lv, 0, M, 1, 0.045, 3)
        gctx.use_current_stream()
        assert side.query()
        G.gosh_train(gctx, lv, 0, one, 1, 0.045, 3)
        torch.cuda.synchronize()
    finally:
        gctx.set_deterministic(False)
        gctx.use_current_stream()
    assert torch.equal(M, one)
