"""All epochs of a small level in one cooperative launch with device-wide
barriers between epochs (gosh_set_resident_epochs) against one launch per
epoch and the oracle: the same samples, update counts and (where one wave
holds the whole level) bit-identical rows; epochs never overlap; AUC within
0.01 of the oracle end to end; running loss and draw record per epoch."""
import numpy as np
import pytest
import torch

from synth import evaluate_auc, init_rows, rmat_csr
from tests.conftest import train_split

pytestmark = pytest.mark.gpu
SEED = 4


def _k2(G):
    return G.CSR.from_numpy(np.array([0, 1, 2], np.int64), np.array([1, 0], np.int32))


@pytest.mark.parametrize("dtype", [torch.float32, torch.bfloat16])
def test_k2_chain_equals_per_epoch_launches(gctx, dtype):
    # two sources in one wave: the resident launch and one launch per epoch
    # run the same visits in the same order, so the rows are bit-identical;
    # 300 dependent epochs would drift apart if any two overlapped
    from paper_2110_10049_amd import gosh as G
    lv = G.gosh_levels_single(gctx, _k2(G))
    f = (np.random.default_rng(3).uniform(-0.05, 0.05, size=(2, 32))).astype(np.float32)
    A = torch.from_numpy(f).cuda().to(dtype)
    B = A.clone()
    gctx.set_resident_epochs(1 << 20)
    G.gosh_train(gctx, lv, 0, A, 300, 0.5, 2, tag=5)
    gctx.set_resident_epochs(0)
    try:
        G.gosh_train(gctx, lv, 0, B, 300, 0.5, 2, tag=5)
        gctx.sync()
    finally:
        gctx.set_resident_epochs(0)
    assert torch.equal(A.view(torch.int16) if dtype == torch.bfloat16 else A,
                       B.view(torch.int16) if dtype == torch.bfloat16 else B)
    assert A.float().abs().max().item() > 0.05


def test_counts_identity_draws_and_loss(gctx, orc):
    from paper_2110_10049_amd import gosh as G
    off, idx = rmat_csr(11, 6, seed=21)                 # 2048 ids, some isolated
    n = len(off) - 1
    lv = G.gosh_levels_single(gctx, G.CSR.from_numpy(off, idx))
    k, d, epochs = 3, 64, 5
    gctx.set_resident_epochs(1 << 20)
    try:
        # lr = 0: identity, and the update count of the per-epoch launches
        M0 = torch.from_numpy(init_rows(n, d, 3)).cuda().to(torch.bfloat16)
        M = M0.clone()
        c_res = torch.zeros(1, dtype=torch.int64, device="cuda")
        rec = torch.full((n, 1 + k), -9, dtype=torch.int32, device="cuda")
        gctx.set_draw_record(rec)
        try:
            G.gosh_train(gctx, lv, 0, M, epochs, 0.0, k, 0, c_res)
            gctx.sync()
        finally:
            gctx.set_draw_record(None)
        assert torch.equal(M.view(torch.int16), M0.view(torch.int16))
        upd = orc.train(off, idx, np.zeros((n, 8)), epochs, 0.0, k, SEED)
        assert int(c_res.item()) == upd
        # the record holds the last epoch's draws
        assert np.array_equal(rec.cpu().numpy(), orc.draw_all(off, idx, SEED, 0, 0, epochs - 1, k))
        # running loss per epoch close to the sequential oracle's
        f = init_rows(n, d, 3) * 40
        Mg = torch.from_numpy(f).cuda()
        loss = torch.zeros(epochs, dtype=torch.float64, device="cuda")
        gctx.set_loss_record(loss)
        try:
            G.gosh_train(gctx, lv, 0, Mg, epochs, 0.045, k)
            gctx.sync()
        finally:
            gctx.set_loss_record(None)
        _, want = orc.train_loss(off, idx, f.astype(np.float64), epochs, float(np.float32(0.045)), k, SEED)
        print(f"[resident loss] gpu {loss.cpu().numpy()} oracle {want}", flush=True)
        np.testing.assert_allclose(loss.cpu().numpy(), want, rtol=2e-2)
    finally:
        gctx.set_resident_epochs(0)


@pytest.mark.parametrize("dtype", [torch.float32, torch.bfloat16])
def test_config1_resident_auc_matches_oracle(gctx, orc, dtype):
    # every level of the scale-12 hierarchy (at most 3,233 vertices) resident
    from paper_2110_10049_amd import gosh as G
    from paper_2110_10049_amd.driver import EmbedConfig, embed
    sp = train_split(12, 16)
    bf = dtype == torch.bfloat16
    g = G.CSR.from_numpy(sp.offsets, sp.indices)
    cfg = EmbedConfig(d=32, epochs=200, p=0.3, lr=0.045, k=1, dtype=dtype, threshold=64)
    gctx.set_resident_epochs(1 << 20)
    try:
        res = embed(gctx, g, cfg, lambda n, d: torch.from_numpy(init_rows(n, d, 3)).cuda().to(dtype))
        gctx.sync()
    finally:
        gctx.set_resident_epochs(0)
    Mo, info = orc.gosh_embed(sp.offsets, sp.indices, lambda n, dd: init_rows(n, dd, 3), 32, 200, 0.3,
                              float(np.float32(0.045)), 1, seed=4, threshold=64, bf16=bf)
    Mo = orc.bf16_to_f64(Mo) if bf else Mo
    assert int(res.updates.item()) == sum(info["updates"])
    a_g = evaluate_auc(res.emb.float().cpu().numpy(), sp, seed=5)
    a_o = evaluate_auc(Mo, sp, seed=5)
    print(f"[resident e2e] {dtype} AUC gpu={a_g:.4f} oracle={a_o:.4f}", flush=True)
    assert abs(a_g - a_o) < 0.01


def test_resident_argument_errors(gctx):
    from paper_2110_10049_amd import gosh as G
    with pytest.raises(G.GoshError):
        gctx.set_resident_epochs(-1)
