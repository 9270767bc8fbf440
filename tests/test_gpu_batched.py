"""Batched training (many independent jobs in one call) against per-job
training and the oracle."""
import numpy as np
import pytest
import torch

from synth import csr_from_pairs, evaluate_auc, init_rows, rmat_csr, split_edges

pytestmark = pytest.mark.gpu
MODES = ["persistent", "graph"]


def _mode(G, name):
    return {"persistent": G.GOSH_BATCH_PERSISTENT, "graph": G.GOSH_BATCH_EPOCH_GRAPH,
            "auto": G.GOSH_BATCH_AUTO}[name]


def _k2(G):
    return G.CSR.from_numpy(np.array([0, 1, 2], np.int64), np.array([1, 0], np.int32))


@pytest.mark.parametrize("mode", MODES)
def test_lr_zero_is_identity(gctx, mode):
    from paper_2110_10049_amd import gosh as G
    print(f"[batched] lr0 {mode}", flush=True)
    jobs, ref = [], []
    for s in range(6):
        off, idx = rmat_csr(8 + s % 3, 6, seed=40 + s)
        g = G.CSR.from_numpy(off, idx)
        M = torch.from_numpy(init_rows(len(off) - 1, 64, s)).cuda().to(torch.bfloat16)
        ref.append(M.clone())
        jobs.append((g, M, 5 + s, 0.0, 0, s))
    G.gosh_train_batched(gctx, jobs, 3, _mode(G, mode))
    for (_, M, *_), R in zip(jobs, ref):
        assert torch.equal(M, R)


def _rel_rows(a, b):
    num = np.linalg.norm(a - b, axis=1)
    den = np.maximum(np.linalg.norm(b, axis=1), 1e-30)
    return float((num / den).max()) if len(a) else 0.0


def _bf16_to_dev(orc, f):
    bits = orc.f32_to_bf16_rne(f).reshape(f.shape)
    return torch.from_numpy(bits.view(np.int16).copy()).view(torch.bfloat16).cuda(), bits


@pytest.mark.parametrize("dtype", [torch.float32, torch.bfloat16])
def test_deterministic_jobs_match_oracle(gctx, orc, dtype):
    """Deterministic mode: every job equals the sequential oracle (Algorithm 3
    in source order with the job's own epochs, lr, level and tag): FP32 within
    1e-4 relative per row, BF16 within 2e-2 per row; and bit for bit the rows
    of gosh_train in deterministic mode on the job's graph."""
    from paper_2110_10049_amd import gosh as G
    print(f"[batched] deterministic {dtype}", flush=True)
    bf = dtype == torch.bfloat16
    rng = np.random.default_rng(11)
    specs = []
    for j in range(12):
        off, idx = rmat_csr(6 + j % 4, 4 + j % 5, seed=300 + j)     # some with isolated vertices
        specs.append((off, idx, int(rng.integers(1, 9)), float(rng.uniform(0.01, 0.05)), j % 3, 7 * j))
    off2, idx2 = np.array([0, 1, 2], np.int64), np.array([1, 0], np.int32)
    specs.append((off2, idx2, 40, 0.5, 0, 999))                       # K_2: epochs chain strongly
    d, k = 32, 3
    jobs, inits, solo = [], [], []
    for j, (off, idx, ep, lr, level, tag) in enumerate(specs):
        n = len(off) - 1
        f = init_rows(n, d, 50 + j) * (40 if j == len(specs) - 1 else 8)
        if bf:
            M, bits = _bf16_to_dev(orc, f)
            inits.append(bits)
        else:
            M = torch.from_numpy(f).cuda()
            inits.append(f)
        jobs.append((G.CSR.from_numpy(off, idx), M, ep, lr, level, tag))
        solo.append(M.clone())
    gctx.set_deterministic(True)
    try:
        chosen = G.gosh_train_batched(gctx, jobs, k, G.GOSH_BATCH_AUTO)
        for (g, _, ep, lr, level, tag), S in zip(jobs, solo):
            # gosh_train on the job's graph: level and tag go into the Philox counter
            lv = G.gosh_levels_single(gctx, g)
            if level == 0:
                G.gosh_train(gctx, lv, 0, S, ep, lr, k, tag=tag)
        torch.cuda.synchronize()
    finally:
        gctx.set_deterministic(False)
    assert chosen[0] == G.GOSH_BATCH_PERSISTENT and chosen[2] == 0
    for j, ((off, idx, ep, lr, level, tag), J, S) in enumerate(zip(specs, jobs, solo)):
        Mo = inits[j].copy() if bf else inits[j].astype(np.float64)
        orc.train(off, idx, Mo, ep, float(np.float32(lr)), k, 4, level=level, tag=tag)
        if bf:
            got = orc.bf16_to_f64(J[1].cpu().view(torch.int16).numpy().view(np.uint16))
            want = orc.bf16_to_f64(Mo)
            assert _rel_rows(got, want) < 2e-2, j
        else:
            got = J[1].cpu().numpy().astype(np.float64)
            assert _rel_rows(got, Mo) < 1e-4, j
        if level == 0:
            assert torch.equal(J[1].view(torch.int16) if bf else J[1], S.view(torch.int16) if bf else S), j


@pytest.mark.parametrize("mode", MODES)
@pytest.mark.parametrize("dtype", [torch.float32, torch.bfloat16])
def test_k2_jobs_match_per_job_training(gctx, mode, dtype):
    # Scheduling check of the concurrent executions: each K_2 job's epochs
    # depend on the previous ones, so epochs overlapping inside one launch
    # would show up as a large difference from per-job launches (one epoch
    # per launch).  (The oracle comparison of the batched trainer is
    # test_deterministic_jobs_match_oracle.)
    from paper_2110_10049_amd import gosh as G
    print(f"[batched] k2 {mode} {dtype}", flush=True)
    g = _k2(G)
    lv = G.gosh_levels_single(gctx, g)
    rng = np.random.default_rng(7)
    jobs, refs = [], []
    for j in range(300):
        f = (rng.uniform(-0.05, 0.05, size=(2, 32))).astype(np.float32)
        epochs = int(rng.integers(5, 60))
        A = torch.from_numpy(f).cuda().to(dtype)
        B = A.clone()
        jobs.append((g, A, epochs, 0.5, 0, j))
        refs.append((B, epochs, j))
    G.gosh_train_batched(gctx, jobs, 0, _mode(G, mode))
    for B, epochs, j in refs:
        G.gosh_train(gctx, lv, 0, B, epochs, 0.5, 0, tag=j)
    torch.cuda.synchronize()
    got = torch.stack([J[1].float() for J in jobs]).cpu().numpy()
    want = torch.stack([R[0].float() for R in refs]).cpu().numpy()
    diff = np.abs(got - want).max() / np.abs(want).max()
    tol = 1e-4 if dtype == torch.float32 else 2e-2
    assert diff < tol, diff
    # and the embeddings really moved (many epochs of positives)
    assert np.abs(want).max() > 0.1


@pytest.mark.parametrize("mode", MODES)
def test_update_counter_exact(gctx, orc, mode):
    from paper_2110_10049_amd import gosh as G
    print(f"[batched] counter {mode}", flush=True)
    jobs, want = [], 0
    for s in range(5):
        off, idx = rmat_csr(9, 3, seed=60 + s)            # has isolated vertices
        n = len(off) - 1
        g = G.CSR.from_numpy(off, idx)
        M = torch.from_numpy(init_rows(n, 32, s)).cuda()
        epochs = 3 + s
        jobs.append((g, M, epochs, 0.02, 1, s))
        for ep in range(epochs):
            smp = np.stack([orc.draw_samples(off, idx, 4, 1, s, ep, v, 3) for v in range(n)])
            want += int((smp[:, 0] >= 0).sum()) + int((smp[:, 1:] != np.arange(n)[:, None]).sum())
    cnt = torch.zeros(1, dtype=torch.int64, device="cuda")
    G.gosh_train_batched(gctx, jobs, 3, _mode(G, mode), updates=cnt)
    torch.cuda.synchronize()
    assert int(cnt.item()) == want


def _geometric(n, radius, seed):
    from scipy.spatial import cKDTree
    pts = np.random.default_rng(seed).random((n, 2))
    pairs = np.array(sorted(cKDTree(pts).query_pairs(radius)))
    return csr_from_pairs(n, pairs[:, 0], pairs[:, 1])


@pytest.mark.parametrize("mode", MODES)
def test_auc_matches_oracle_per_job(gctx, orc, mode):
    from paper_2110_10049_amd import gosh as G
    print(f"[batched] auc {mode}", flush=True)
    graphs = [_geometric(3000, 0.035, s) for s in range(3)]
    splits = [split_edges(o, x, 2) for o, x in graphs]
    d, k, lr, epochs = 64, 3, 0.045, 150
    jobs = []
    for j, sp in enumerate(splits):
        g = G.CSR.from_numpy(sp.offsets, sp.indices)
        M = torch.from_numpy(init_rows(sp.n, d, 3 + j)).cuda()
        jobs.append((g, M, epochs, lr, 0, j))
    G.gosh_train_batched(gctx, jobs, k, _mode(G, mode))
    torch.cuda.synchronize()
    for j, sp in enumerate(splits):
        Mo = init_rows(sp.n, d, 3 + j).astype(np.float64)
        orc.train(sp.offsets, sp.indices, Mo, epochs, float(np.float32(lr)), k, 4, level=0, tag=j)
        a_g = evaluate_auc(jobs[j][1].cpu().numpy(), sp, seed=5)
        a_o = evaluate_auc(Mo, sp, seed=5)
        print(f"[batched] job {j} AUC gpu={a_g:.4f} oracle={a_o:.4f}", flush=True)
        assert a_o > 0.85
        assert abs(a_g - a_o) < 0.01


def test_autotune_choice_is_valid_and_cached(gctx):
    from paper_2110_10049_amd import gosh as G
    jobs = []
    for s in range(8):
        off, idx = rmat_csr(9, 8, seed=80 + s)
        g = G.CSR.from_numpy(off, idx)
        jobs.append((g, torch.from_numpy(init_rows(len(off) - 1, 16, s)).cuda(), 4, 0.03, 0, s))
    first = G.gosh_train_batched(gctx, jobs, 1, G.GOSH_BATCH_AUTO)
    assert first[0] in (G.GOSH_BATCH_PERSISTENT, G.GOSH_BATCH_EPOCH_GRAPH)
    if first[0] == G.GOSH_BATCH_PERSISTENT:
        assert first[1] in (1, 2, 4) and first[2] in (1, 4, 16)
    second = G.gosh_train_batched(gctx, jobs, 1, G.GOSH_BATCH_AUTO)
    assert second == first


def test_batched_argument_errors(gctx):
    from paper_2110_10049_amd import gosh as G
    g = _k2(G)
    M = torch.zeros((2, 32), device="cuda")
    with pytest.raises(G.GoshError):
        G.gosh_train_batched(gctx, [(g, M, 1, 0.1, 0, 1 << 24)], 1, G.GOSH_BATCH_PERSISTENT)
    with pytest.raises(G.GoshError):
        G.gosh_train_batched(gctx, [(g, M, 1, -1.0, 0, 0)], 1, G.GOSH_BATCH_PERSISTENT)
    with pytest.raises(G.GoshError):
        G.gosh_train_batched(gctx, [(g, M, 1, 0.1, 0, 0)], 16, G.GOSH_BATCH_PERSISTENT)
