"""Levels whose rows fit in one workgroup's LDS trained inside that
workgroup (gosh_set_lds_levels): rows read from HBM once and written back
once, every epoch's samples drawn into an LDS table, epochs separated by
workgroup barriers.  Against the oracle and one launch per epoch: exact
update counts, lr = 0 identity, the last epoch's draws bit for bit, the
running loss, epochs in order on a chain of dependent epochs, and
end-to-end AUC within 0.01 of the oracle."""
import numpy as np
import pytest
import torch

from synth import evaluate_auc, init_rows, rmat_csr
from tests.conftest import train_split

pytestmark = pytest.mark.gpu
SEED = 4


def _rel_rows(a, b):
    num = np.linalg.norm(a - b, axis=1)
    den = np.maximum(np.linalg.norm(b, axis=1), 1e-30)
    return float((num / den).max())


@pytest.mark.parametrize("dtype", [torch.float32, torch.bfloat16])
def test_k2_chain_matches_per_epoch_launches(gctx, dtype):
    # K_2, k = 0: both sources of an epoch in one wave under either path;
    # 300 dependent epochs at lr 0.5 would drift far apart if epochs overlapped
    from paper_2110_10049_amd import gosh as G
    g = G.CSR.from_numpy(np.array([0, 1, 2], np.int64), np.array([1, 0], np.int32))
    lv = G.gosh_levels_single(gctx, g)
    f = np.random.default_rng(5).uniform(-0.05, 0.05, size=(2, 32)).astype(np.float32)
    A = torch.from_numpy(f).cuda().to(dtype)
    B = A.clone()
    gctx.set_lds_levels(1 << 20)
    try:
        G.gosh_train(gctx, lv, 0, A, 300, 0.5, 0, tag=3)
    finally:
        gctx.set_lds_levels(0)
    G.gosh_train(gctx, lv, 0, B, 300, 0.5, 0, tag=3)
    gctx.sync()
    a, b = A.float().cpu().numpy().astype(np.float64), B.float().cpu().numpy().astype(np.float64)
    assert np.abs(b).max() > 0.05
    assert _rel_rows(a, b) < (1e-4 if dtype == torch.float32 else 2e-2)


@pytest.mark.parametrize("dtype", [torch.float32, torch.bfloat16])
def test_counts_identity_draws_and_loss(gctx, orc, dtype):
    from paper_2110_10049_amd import gosh as G
    off, idx = rmat_csr(9, 6, seed=23)                  # 512 ids, some isolated
    n = len(off) - 1
    lv = G.gosh_levels_single(gctx, G.CSR.from_numpy(off, idx))
    k, d, epochs = 3, 64, 6
    gctx.set_lds_levels(1 << 20)
    try:
        M0 = torch.from_numpy(init_rows(n, d, 3)).cuda().to(dtype)
        M = M0.clone()
        cnt = torch.zeros(1, dtype=torch.int64, device="cuda")
        rec = torch.full((n, 1 + k), -9, dtype=torch.int32, device="cuda")
        gctx.set_draw_record(rec)
        try:
            G.gosh_train(gctx, lv, 0, M, epochs, 0.0, k, 0, cnt)
            gctx.sync()
        finally:
            gctx.set_draw_record(None)
        assert torch.equal(M.view(torch.int16) if dtype == torch.bfloat16 else M,
                           M0.view(torch.int16) if dtype == torch.bfloat16 else M0)
        assert int(cnt.item()) == orc.train(off, idx, np.zeros((n, 8)), epochs, 0.0, k, SEED)
        assert np.array_equal(rec.cpu().numpy(), orc.draw_all(off, idx, SEED, 0, 0, epochs - 1, k))
        f = init_rows(n, d, 3) * 40
        Mg = torch.from_numpy(f).cuda().to(dtype)
        loss = torch.zeros(epochs, dtype=torch.float64, device="cuda")
        gctx.set_loss_record(loss)
        try:
            G.gosh_train(gctx, lv, 0, Mg, epochs, 0.045, k)
            gctx.sync()
        finally:
            gctx.set_loss_record(None)
        if dtype == torch.bfloat16:
            Mo = orc.f32_to_bf16_rne(f).reshape(f.shape)
        else:
            Mo = f.astype(np.float64)
        _, want = orc.train_loss(off, idx, Mo, epochs, float(np.float32(0.045)), k, SEED)
        print(f"[lds loss] {dtype} gpu {loss.cpu().numpy()} oracle {want}", flush=True)
        np.testing.assert_allclose(loss.cpu().numpy(), want, rtol=2e-2)
    finally:
        gctx.set_lds_levels(0)


@pytest.mark.parametrize("dtype", [torch.float32, torch.bfloat16])
def test_config1_lds_levels_auc_matches_oracle(gctx, orc, dtype):
    # the coarse levels of the scale-12 hierarchy (838, 302, 83, 55 vertices
    # of 128-byte rows) fit in LDS; level 0 (3,233) does not
    from paper_2110_10049_amd import gosh as G
    from paper_2110_10049_amd.driver import EmbedConfig, embed
    sp = train_split(12, 16)
    bf = dtype == torch.bfloat16
    g = G.CSR.from_numpy(sp.offsets, sp.indices)
    cfg = EmbedConfig(d=32, epochs=200, p=0.3, lr=0.045, k=1, dtype=dtype, threshold=64)
    gctx.set_lds_levels(1 << 20)
    try:
        res = embed(gctx, g, cfg, lambda n, d: torch.from_numpy(init_rows(n, d, 3)).cuda().to(dtype))
        gctx.sync()
    finally:
        gctx.set_lds_levels(0)
    Mo, info = orc.gosh_embed(sp.offsets, sp.indices, lambda n, dd: init_rows(n, dd, 3), 32, 200, 0.3,
                              float(np.float32(0.045)), 1, seed=4, threshold=64, bf16=bf)
    Mo = orc.bf16_to_f64(Mo) if bf else Mo
    assert int(res.updates.item()) == sum(info["updates"])
    a_g = evaluate_auc(res.emb.float().cpu().numpy(), sp, seed=5)
    a_o = evaluate_auc(Mo, sp, seed=5)
    print(f"[lds e2e] {dtype} AUC gpu={a_g:.4f} oracle={a_o:.4f}", flush=True)
    assert abs(a_g - a_o) < 0.01


def test_lds_argument_errors(gctx):
    from paper_2110_10049_amd import gosh as G
    with pytest.raises(G.GoshError):
        gctx.set_lds_levels(-1)


def _geometric(n, radius, seed):
    from scipy.spatial import cKDTree
    from synth import csr_from_pairs
    pts = np.random.default_rng(seed).random((n, 2))
    pairs = np.array(sorted(cKDTree(pts).query_pairs(radius)))
    return csr_from_pairs(n, pairs[:, 0], pairs[:, 1])


@pytest.mark.parametrize("dtype", [torch.float32, torch.bfloat16])
def test_batched_lds_jobs_match_oracle(gctx, orc, dtype):
    """Batched jobs that fit in LDS train one workgroup each (the rest as
    before): exact update count, AUC of every job within 0.01 of the oracle."""
    from paper_2110_10049_amd import gosh as G
    from synth import split_edges
    splits = [split_edges(*_geometric(1100, 0.07, s), 2) for s in range(3)]
    big = split_edges(*_geometric(3000, 0.035, 7), 2)          # 3000 rows of 128 B: not in LDS
    d, k, lr, epochs = 32, 3, 0.045, 120
    jobs, want_upd = [], 0
    for j, sp in enumerate(splits + [big]):
        M = torch.from_numpy(init_rows(sp.n, d, 3 + j)).cuda().to(dtype)
        jobs.append((G.CSR.from_numpy(sp.offsets, sp.indices), M, epochs, lr, 0, j))
        want_upd += orc.train(sp.offsets, sp.indices, np.zeros((sp.n, 8)), epochs, 0.0, k, SEED, level=0, tag=j)
    cnt = torch.zeros(1, dtype=torch.int64, device="cuda")
    gctx.set_lds_levels(2000)
    try:
        G.gosh_train_batched(gctx, jobs, k, G.GOSH_BATCH_EPOCH_GRAPH, updates=cnt)
        torch.cuda.synchronize()
    finally:
        gctx.set_lds_levels(0)
    assert int(cnt.item()) == want_upd
    bf = dtype == torch.bfloat16
    for j, sp in enumerate(splits + [big]):
        f = init_rows(sp.n, d, 3 + j)
        Mo = orc.f32_to_bf16_rne(f).reshape(f.shape) if bf else f.astype(np.float64)
        orc.train(sp.offsets, sp.indices, Mo, epochs, float(np.float32(lr)), k, SEED, level=0, tag=j)
        a_g = evaluate_auc(jobs[j][1].float().cpu().numpy(), sp, seed=5)
        a_o = evaluate_auc(orc.bf16_to_f64(Mo) if bf else Mo, sp, seed=5)
        print(f"[lds batched] {dtype} job {j} n={sp.n} AUC gpu={a_g:.4f} oracle={a_o:.4f}", flush=True)
        assert a_o > 0.8
        assert abs(a_g - a_o) < 0.01
