"""End-to-end Algorithm 2 on the GPU against the oracle: link-prediction AUC on
the 20% held-out edges must agree within 0.01 (the GPU trains sources of an
epoch concurrently, the oracle in order, so only the score is compared).

The scale-20 workload (d = 128, k = 3, 600 epochs) is compared with the
oracle's stored result (tests/golden/e2e_auc_rmat20.json, written by
tests/golden/make_e2e_auc.py from oracle/ alone), in FP32 and BF16, with atomic
row updates everywhere, with the benchmark's plain negative stores and plain
light-row stores on levels of at least 262,144 vertices, and (FP32) with the
visits of hot positives grouped on level 1."""
import json
import os

import numpy as np
import pytest
import torch

from synth import csr_from_pairs, evaluate_auc, init_rows, split_edges
from synth.linkpred import auc_on_pairs, make_eval_pairs
from tests.conftest import train_split

pytestmark = pytest.mark.gpu
GOLD_C2 = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "e2e_auc_rmat20.json")
GOLD_EDGES = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "e2e_auc_rmat12_edges.json")
_PAIRS = {}


def _gpu_embed(gctx, sp, d, e, p, lr, k, threshold, dtype, orc):
    from paper_2110_10049_amd import gosh as G
    from paper_2110_10049_amd.driver import EmbedConfig, embed
    g = G.CSR.from_numpy(sp.offsets, sp.indices)

    def init(n, dd):
        f = init_rows(n, dd, 3)
        if dtype == torch.bfloat16:
            bits = orc.f32_to_bf16_rne(f).reshape(n, dd)
            return torch.from_numpy(bits.view(np.int16).copy()).view(torch.bfloat16).cuda()
        return torch.from_numpy(f).cuda()

    cfg = EmbedConfig(d=d, epochs=e, p=p, lr=lr, k=k, dtype=dtype, threshold=threshold)
    res = embed(gctx, g, cfg, init)
    torch.cuda.synchronize()
    M = res.emb.float().cpu().numpy().astype(np.float64)
    return M, res


def _oracle_embed(orc, sp, d, e, p, lr, k, threshold, bf16):
    M, info = orc.gosh_embed(sp.offsets, sp.indices, lambda n, dd: init_rows(n, dd, 3), d, e, p,
                             float(np.float32(lr)), k, seed=4, threshold=threshold, bf16=bf16)
    return (orc.bf16_to_f64(M) if bf16 else M), info


@pytest.mark.parametrize("dtype", [torch.float32, torch.bfloat16])
def test_config1_auc_matches_oracle(gctx, orc, dtype):
    # R-MAT scale 12, d=32, k=1, lr 0.045, 200 epochs, threshold 64
    sp = train_split(12, 16)
    bf = dtype == torch.bfloat16
    print(f"[e2e config1] dtype={dtype}", flush=True)
    Mg, res = _gpu_embed(gctx, sp, 32, 200, 0.3, 0.045, 1, 64, dtype, orc)
    Mo, info = _oracle_embed(orc, sp, 32, 200, 0.3, 0.045, 1, 64, bf)
    assert res.sizes == info["sizes"]
    assert list(res.schedule) == list(info["schedule"])
    assert int(res.updates.item()) == sum(info["updates"])
    a_g = evaluate_auc(Mg, sp, seed=5)
    a_o = evaluate_auc(Mo, sp, seed=5)
    print(f"[e2e config1] AUC gpu={a_g:.4f} oracle={a_o:.4f}", flush=True)
    assert abs(a_g - a_o) < 0.01


def _geometric(n=4000, radius=0.03, seed=0):
    from scipy.spatial import cKDTree
    pts = np.random.default_rng(seed).random((n, 2))
    pairs = np.array(sorted(cKDTree(pts).query_pairs(radius)))
    return csr_from_pairs(n, pairs[:, 0], pairs[:, 1])


@pytest.mark.parametrize("dtype", [torch.float32, torch.bfloat16])
def test_geometric_graph_auc_matches_oracle(gctx, orc, dtype):
    off, idx = _geometric()
    sp = split_edges(off, idx, 2)
    bf = dtype == torch.bfloat16
    print(f"[e2e geometric] dtype={dtype}", flush=True)
    Mg, _ = _gpu_embed(gctx, sp, 64, 200, 0.3, 0.045, 3, 64, dtype, orc)
    Mo, _ = _oracle_embed(orc, sp, 64, 200, 0.3, 0.045, 3, 64, bf)
    a_g = evaluate_auc(Mg, sp, seed=5)
    a_o = evaluate_auc(Mo, sp, seed=5)
    print(f"[e2e geometric] AUC gpu={a_g:.4f} oracle={a_o:.4f}", flush=True)
    assert a_o > 0.85
    assert abs(a_g - a_o) < 0.01


def test_config1_batched_small_levels_auc(gctx, orc):
    # small levels trained through the batched path keep the oracle's AUC
    from paper_2110_10049_amd import gosh as G
    from paper_2110_10049_amd.driver import EmbedConfig, embed
    sp = train_split(12, 16)
    g = G.CSR.from_numpy(sp.offsets, sp.indices)
    cfg = EmbedConfig(d=32, epochs=200, p=0.3, lr=0.045, k=1, threshold=64, batch_levels_upto=1000)
    res = embed(gctx, g, cfg, lambda n, dd: torch.from_numpy(init_rows(n, dd, 3)).cuda())
    torch.cuda.synchronize()
    Mo, info = _oracle_embed(orc, sp, 32, 200, 0.3, 0.045, 1, 64, False)
    assert int(res.updates.item()) == sum(info["updates"])
    a_g = evaluate_auc(res.emb.cpu().numpy(), sp, seed=5)
    a_o = evaluate_auc(Mo, sp, seed=5)
    print(f"[e2e batched levels] AUC gpu={a_g:.4f} oracle={a_o:.4f}", flush=True)
    assert abs(a_g - a_o) < 0.01


def test_overlapping_epochs_keep_auc(gctx, orc):
    # two epochs per launch on the larger levels (Section 6.3's suggestion):
    # the same number of updates, AUC within 0.01 of the oracle (sequential epochs)
    from paper_2110_10049_amd import gosh as G
    from paper_2110_10049_amd.driver import EmbedConfig, embed
    sp = train_split(12, 16)
    g = G.CSR.from_numpy(sp.offsets, sp.indices)
    cfg = EmbedConfig(d=32, epochs=200, p=0.3, lr=0.045, k=1, threshold=64)
    gctx.set_epoch_overlap(2, 1000)
    try:
        res = embed(gctx, g, cfg, lambda n, dd: torch.from_numpy(init_rows(n, dd, 3)).cuda())
        torch.cuda.synchronize()
    finally:
        gctx.set_epoch_overlap(1, 0)
    Mo, info = _oracle_embed(orc, sp, 32, 200, 0.3, 0.045, 1, 64, False)
    assert int(res.updates.item()) == sum(info["updates"])
    a_g = evaluate_auc(res.emb.cpu().numpy(), sp, seed=5)
    a_o = evaluate_auc(Mo, sp, seed=5)
    print(f"[e2e overlapping epochs] AUC gpu={a_g:.4f} oracle={a_o:.4f}", flush=True)
    assert abs(a_g - a_o) < 0.01


def test_overlap_with_zero_lr_is_identity(gctx):
    from paper_2110_10049_amd import gosh as G
    sp = train_split(12, 16)
    g = G.CSR.from_numpy(sp.offsets, sp.indices)
    lv = G.gosh_levels_single(gctx, g)
    M0 = torch.from_numpy(init_rows(sp.n, 64, 3)).cuda().to(torch.bfloat16)
    M = M0.clone()
    gctx.set_epoch_overlap(3, 0)
    try:
        G.gosh_train(gctx, lv, 0, M, 7, 0.0, 3)
        torch.cuda.synchronize()
    finally:
        gctx.set_epoch_overlap(1, 0)
    assert torch.equal(M, M0)
    with pytest.raises(G.GoshError):
        gctx.set_epoch_overlap(0, 0)


def test_plain_negative_stores_keep_auc_on_large_levels(gctx, orc):
    # negatives stored plainly (the paper's lock-free writes) on levels of at
    # least 8192 vertices: same update count, AUC within 0.01 of the oracle
    from paper_2110_10049_amd import gosh as G
    from paper_2110_10049_amd.driver import EmbedConfig, embed
    sp = train_split(16, 16)
    g = G.CSR.from_numpy(sp.offsets, sp.indices)
    cfg = EmbedConfig(d=32, epochs=200, p=0.3, lr=0.045, k=3, threshold=100)
    gctx.set_plain_negatives(8192)
    try:
        res = embed(gctx, g, cfg, lambda n, dd: torch.from_numpy(init_rows(n, dd, 3)).cuda())
        torch.cuda.synchronize()
    finally:
        gctx.set_plain_negatives(0)
    assert res.sizes[0] >= 8192
    Mo, info = _oracle_embed(orc, sp, 32, 200, 0.3, 0.045, 3, 100, False)
    assert int(res.updates.item()) == sum(info["updates"])
    a_g = evaluate_auc(res.emb.cpu().numpy(), sp, seed=5)
    a_o = evaluate_auc(Mo, sp, seed=5)
    print(f"[e2e plain negatives] n0={res.sizes[0]} AUC gpu={a_g:.4f} oracle={a_o:.4f}", flush=True)
    assert abs(a_g - a_o) < 0.01


@pytest.mark.parametrize("dtype", [torch.float32, torch.bfloat16])
def test_plain_negative_stores_zero_lr_is_identity(gctx, dtype):
    from paper_2110_10049_amd import gosh as G
    sp = train_split(12, 16)
    lv = G.gosh_levels_single(gctx, G.CSR.from_numpy(sp.offsets, sp.indices))
    M0 = torch.from_numpy(init_rows(sp.n, 64, 3)).cuda().to(dtype)
    M = M0.clone()
    c_plain = torch.zeros(1, dtype=torch.int64, device="cuda")
    c_atomic = torch.zeros(1, dtype=torch.int64, device="cuda")
    gctx.set_plain_negatives(1)
    try:
        G.gosh_train(gctx, lv, 0, M, 5, 0.0, 3, 0, c_plain)
        G.gosh_train_walks(gctx, lv, 0, M, 2, 0.0, 3, 4, 2)
        torch.cuda.synchronize()
    finally:
        gctx.set_plain_negatives(0)
    G.gosh_train(gctx, lv, 0, M.clone(), 5, 0.0, 3, 0, c_atomic)
    torch.cuda.synchronize()
    assert torch.equal(M, M0)
    assert int(c_plain.item()) == int(c_atomic.item())
    with pytest.raises(G.GoshError):
        gctx.set_plain_negatives(-1)


# The grouped schedule runs in FP32 only: in BF16 it moved AUC 0.004-0.009 below the ungrouped
# run's, too close to the 0.01 bar for a test that must not fail by chance; its BF16 commits
# are checked element-wise in test_gpu_grouped.py.
_C2_CASES = [(dt, *w) for dt in (torch.float32, torch.bfloat16)
             for w in ((0, 0, False), (262144, 0, False), (262144, 262144, False))] + [(torch.float32, 0, 0, True)]


@pytest.mark.parametrize("dtype,plain_min,light_min,grouped", _C2_CASES,
                         ids=[f"{'bf16' if c[0] == torch.bfloat16 else 'fp32'}-{c[1]}-{c[2]}-{c[3]}" for c in _C2_CASES])
def test_config2_auc_matches_oracle(gctx, dtype, plain_min, light_min, grouped):
    """Scale-20 R-MAT, d = 128, k = 3, 600 epochs (the benchmark's workload):
    the same levels, schedule and update count as the oracle, AUC within
    0.01 of the oracle's, and the last epoch's running loss of every level
    within 5% of the sequential oracle's; with atomic commits everywhere,
    with plain negative stores on levels of at least 262,144 vertices, with
    those plus plain stores of light rows on that level, and with atomic
    commits and the visits of hot positives grouped on the one level of
    65,536 to 262,143 vertices (hubs of at least 64 x the average degree)."""
    from paper_2110_10049_amd import gosh as G
    from paper_2110_10049_amd.driver import EmbedConfig, embed
    gold = json.load(open(GOLD_C2))
    c = gold["config"]
    ref = gold["bf16" if dtype == torch.bfloat16 else "fp64"]
    sp = train_split(c["scale"], c["edge_factor"], c["seeds"]["graph"], c["seeds"]["split"])
    if "c2" not in _PAIRS:
        _PAIRS["c2"] = make_eval_pairs(sp, c["seeds"]["eval"], c["eval"]["max_train"], c["eval"]["max_test"])
    print(f"[e2e config2] dtype={dtype} plain_min={plain_min} light_min={light_min} grouped={grouped}", flush=True)
    g = G.CSR.from_numpy(sp.offsets, sp.indices)
    cfg = EmbedConfig(d=c["d"], epochs=c["epochs"], p=c["p"], lr=c["lr"], k=c["k"], dtype=dtype,
                      threshold=c["threshold"], epoch_unit=c["epoch_unit"])
    gctx.set_plain_negatives(plain_min)
    gctx.set_plain_light_rows(light_min)
    gctx.set_grouped_positives(65536, 262143 if grouped else 0, 64.0)
    try:
        res = embed(gctx, g, cfg,
                    lambda n, d: torch.from_numpy(init_rows(n, d, c["seeds"]["init"])).cuda().to(dtype),
                    record_loss=True)
        torch.cuda.synchronize()
    finally:
        gctx.set_plain_negatives(0)
        gctx.set_plain_light_rows(0)
        gctx.set_grouped_positives(0, 0)
    assert res.sizes == ref["sizes"]
    assert list(res.schedule) == ref["schedule"]
    assert int(res.updates.item()) == ref["updates"]
    auc = auc_on_pairs(res.emb.float().cpu().numpy(), _PAIRS["c2"])
    loss = [float(res.losses[i][-1].item()) for i in range(len(res.sizes))]
    print(f"[e2e config2] AUC gpu={auc:.4f} oracle={ref['auc']:.4f}; last-epoch loss gpu={loss} "
          f"oracle={ref['last_epoch_loss']}", flush=True)
    assert abs(auc - ref["auc"]) < 0.01
    np.testing.assert_allclose(loss, ref["last_epoch_loss"], rtol=0.05)


@pytest.mark.parametrize("dtype", [torch.float32, torch.bfloat16])
def test_config1_edge_unit_auc_matches_oracle(gctx, orc, dtype):
    """The paper's epoch unit (one epoch = |E| updates, the note under Table
    3): every level's share scaled by ceil(nnz_i / (2 n_i)) passes, on the
    GPU and in the oracle: same schedule and update count as the oracle's
    run; AUC compared over eight random streams.  The small coarse levels
    then train for 700-1800 passes with a whole epoch in flight at once, and
    the method's own AUC varies by about 0.01 from stream to stream (oracle,
    FP64 0.614-0.634, BF16 0.595-0.624), so the bar is on the mean over the
    streams of the paired difference (runs of equal tag share every sample):
    |mean(GPU - oracle)| < 0.01."""
    from paper_2110_10049_amd import gosh as G
    from paper_2110_10049_amd.driver import EmbedConfig, embed
    gold = json.load(open(GOLD_EDGES))
    c = gold["config"]
    ref = gold["bf16" if dtype == torch.bfloat16 else "fp64"]
    sp = train_split(c["scale"], c["edge_factor"], c["seeds"]["graph"], c["seeds"]["split"])
    g = G.CSR.from_numpy(sp.offsets, sp.indices)
    diffs = []
    for tag, a_o in zip(c["tags"], ref):
        cfg = EmbedConfig(d=c["d"], epochs=c["epochs"], p=c["p"], lr=c["lr"], k=c["k"], dtype=dtype,
                          threshold=c["threshold"], epoch_unit=c["epoch_unit"], tag=tag)
        res = embed(gctx, g, cfg, lambda n, d: torch.from_numpy(init_rows(n, d, c["seeds"]["init"])).cuda().to(dtype))
        torch.cuda.synchronize()
        assert list(res.schedule) == gold["schedule"]
        if tag == 0:
            # the executed updates of every level at its scaled epochs (the count does not depend on the rows)
            upd = sum(orc.train(o, x, np.zeros((len(o) - 1, 8)), int(e), 0.0, c["k"], 4, level=i)
                      for i, ((o, x), e) in enumerate(zip(orc.coarsen_levels(sp.offsets, sp.indices,
                                                                             c["threshold"])[0], gold["schedule"])))
            assert int(res.updates.item()) == upd
        a_g = evaluate_auc(res.emb.float().cpu().numpy(), sp, seed=c["seeds"]["eval"])
        diffs.append(a_g - a_o)
        print(f"[e2e config1 edges] {dtype} tag {tag}: AUC gpu={a_g:.4f} oracle={a_o:.4f}", flush=True)
    mean = float(np.mean(diffs))
    print(f"[e2e config1 edges] {dtype} mean paired difference {mean:+.4f} (sd {np.std(diffs):.4f})", flush=True)
    assert abs(mean) < 0.01
