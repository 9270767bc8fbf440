"""What the learned prolongation gains, judged by link-prediction AUC on a
graph the network was not trained on, on the GPU and in the oracle:

* pairs: the scale-12 graph embedded with copy prolongation (d = 32, 600
  epochs), every fine level's trained rows with its coarse level's; the GPU
  trains its network on its pairs, the oracle (FP64 Adam, oracle/mlp.py) its
  own on the pairs of its own sequential run, both from the same stream
  initialisation and with the same minibatch draws (the GPU's initial W1 is
  compared with the oracle's bit for bit);
* evaluation: the scale-16 graph embedded with 75 epochs, expanding every
  level with the learned network: the GPU's AUC within 0.01 of the oracle's
  learned run (FP32 against FP64 rows, BF16 against BF16), and at least 0.05
  above copy prolongation at the same 75 epochs.  (On the smaller scale-14
  graph the method's own AUC in BF16 moves by up to 0.06 from one Philox
  stream to another, too much for a single-stream comparison; at scale 16 the
  oracle's spread over four streams is 0.010 in BF16 and 0.005 in FP64, with
  learned 0.87 against copy 0.60.)
"""
import numpy as np
import pytest
import torch

from synth import init_rows
from synth.linkpred import auc_on_pairs, make_eval_pairs
from tests.conftest import train_split

pytestmark = pytest.mark.gpu

D, H, K, LR, P_SMOOTH = 32, 64, 3, 0.045, 0.3
STEPS, BATCH, MLR, TAG = 400, 256, 3e-3, 11
E_PAIRS, E_EVAL, THR = 600, 75, 64
_CACHE = {}


def _oracle_network(orc):
    import oracle.mlp as OM
    if "P" not in _CACHE:
        sp = train_split(12, 16)
        levels = orc.coarsen_levels(sp.offsets, sp.indices, THR)
        graphs, maps = levels
        keep = {}
        orc.gosh_embed(sp.offsets, sp.indices, lambda n, d: init_rows(n, d, 3), D, E_PAIRS, P_SMOOTH,
                       float(np.float32(LR)), K, seed=4, threshold=THR, levels=levels, keep=keep)
        src = [OM.level_pairs(keep[i + 1], keep[i], maps[i], np.diff(graphs[i][0])) for i in range(len(graphs) - 1)]
        P = OM.init_params_stream(D, H, 4)
        losses = OM.train_pairs(P, src, STEPS, BATCH, MLR, 4, TAG)
        print(f"[oracle mlp] loss {losses[:10].mean():.4g} -> {losses[-10:].mean():.4g}", flush=True)
        _CACHE["P"] = P
    return _CACHE["P"]


def _gpu_network(gctx):
    from paper_2110_10049_amd import gosh as G
    from paper_2110_10049_amd.driver import EmbedConfig, embed
    import oracle.mlp as OM
    if "net" not in _CACHE:
        sp = train_split(12, 16)
        g = G.CSR.from_numpy(sp.offsets, sp.indices)
        cfg = EmbedConfig(d=D, epochs=E_PAIRS, p=P_SMOOTH, lr=LR, k=K, dtype=torch.float32, threshold=THR)
        res = embed(gctx, g, cfg, lambda n, d: torch.from_numpy(init_rows(n, d, 3)).cuda(), keep_levels=True)
        lv = res.levels
        net = G.Mlp(gctx, D, H)
        w1 = net.get_weights()[: H * (D + 2)]
        assert np.array_equal(w1, OM.init_params_stream(D, H, 4).W1.astype(np.float32).ravel())
        srcs = [(lv, i, res.trained[i + 1], res.trained[i]) for i in range(lv.count() - 1)]
        losses = net.train(srcs, STEPS, BATCH, MLR, tag=TAG).cpu().numpy()
        print(f"[gpu mlp] loss {losses[:10].mean():.4g} -> {losses[-10:].mean():.4g}", flush=True)
        _CACHE["net"] = (net, res, lv)
    return _CACHE["net"][0]


@pytest.mark.parametrize("dtype", [torch.float32, torch.bfloat16])
def test_learned_prolongation_auc_matches_oracle_and_beats_copy(gctx, orc, dtype):
    from paper_2110_10049_amd import gosh as G
    from paper_2110_10049_amd.driver import EmbedConfig, embed
    import oracle.mlp as OM
    bf = dtype == torch.bfloat16
    print(f"[learned auc] {dtype}", flush=True)
    net = _gpu_network(gctx)
    P = _oracle_network(orc)
    sp = train_split(16, 16)
    if "pairs" not in _CACHE:
        _CACHE["pairs"] = make_eval_pairs(sp, 5, 200_000, 1_000_000)
    pairs = _CACHE["pairs"]
    g = G.CSR.from_numpy(sp.offsets, sp.indices)
    cfg = EmbedConfig(d=D, epochs=E_EVAL, p=P_SMOOTH, lr=LR, k=K, dtype=dtype, threshold=THR)
    init = lambda n, d: torch.from_numpy(init_rows(n, d, 3)).cuda().to(dtype)
    r_l = embed(gctx, g, cfg, init, mlp=net)
    r_c = embed(gctx, g, cfg, init)
    torch.cuda.synchronize()
    a_l = auc_on_pairs(r_l.emb.float().cpu().numpy(), pairs)
    a_c = auc_on_pairs(r_c.emb.float().cpu().numpy(), pairs)

    def expand(M, i, graphs, maps):
        coarse = orc.bf16_to_f64(M) if bf else M
        fine = OM.prolong_learned(P, coarse, maps[i], np.diff(graphs[i][0]))
        return orc.f32_to_bf16_rne(fine.astype(np.float32)).reshape(fine.shape) if bf else fine

    Mo, _ = orc.gosh_embed(sp.offsets, sp.indices, lambda n, d: init_rows(n, d, 3), D, E_EVAL, P_SMOOTH,
                           float(np.float32(LR)), K, seed=4, threshold=THR, bf16=bf, prolong_fn=expand)
    a_o = auc_on_pairs(orc.bf16_to_f64(Mo) if bf else Mo, pairs)
    print(f"[learned auc] {dtype}: gpu learned {a_l:.4f}, oracle learned {a_o:.4f}, gpu copy {a_c:.4f}", flush=True)
    assert abs(a_l - a_o) < 0.01
    assert a_l > a_c + 0.05
