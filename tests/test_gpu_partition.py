"""Partitioned embedding (Section 5) on the GPU against the reference
(oracle train_partitioned): in deterministic mode (every kernel one wave in
pool order, one kernel stream) the rows after several rounds match the
sequential reference, with part swaps, the positive cap and both row types;
in the concurrent mode link-prediction AUC matches the reference's; a memory
cap picks the part count and bounds device memory."""
import numpy as np
import pytest
import torch

from synth import csr_from_pairs, evaluate_auc, init_rows, rmat_csr, split_edges

pytestmark = pytest.mark.gpu

SEED = 4


def _rel_rows(a, b):
    num = np.linalg.norm(a - b, axis=1)
    den = np.maximum(np.linalg.norm(b, axis=1), 1e-30)
    return float((num / den).max()) if len(a) else 0.0


def _host_bf16(bits):
    return torch.from_numpy(bits.view(np.int16).copy()).view(torch.bfloat16).pin_memory()


def _bits(t):
    return t.view(torch.int16).numpy().view(np.uint16)


@pytest.mark.parametrize("dtype", ["f32", "bf16"])
# (4, 5, 7): the positive cap ends the run inside the first round
@pytest.mark.parametrize("K,B,epochs,k,d,bins,swaps", [(3, 2, 4, 2, 16, 2, True), (1, 1, 3, 3, 32, 2, False),
                                                       (4, 5, 7, 1, 8, 3, False), (2, 3, 5, 15, 64, 2, False),
                                                       (5, 1, 2, 0, 128, 2, True)])
def test_deterministic_matches_reference(gctx, orc, dtype, K, B, epochs, k, d, bins, swaps):
    from paper_2110_10049_amd import gosh as G
    sp = split_edges(*rmat_csr(9, 6, 3), seed=2)
    n = sp.n
    print(f"[partitioned det] {dtype} K={K} B={B} e={epochs} k={k} d={d} n={n}", flush=True)
    g = G.HostCSR(sp.offsets, sp.indices)
    f = init_rows(n, d, 3) * 8
    lr = 0.045
    params = G.part_params(parts=K, sub_bins=bins, pool_bins=1 + (K % 2), B=B, threads=4)
    cnt = torch.zeros(1, dtype=torch.int64, device="cuda")
    gctx.set_deterministic(True)
    try:
        if dtype == "f32":
            Mh = torch.from_numpy(f.copy()).pin_memory()
            st = G.gosh_train_partitioned(gctx, g, Mh, epochs, lr, k, level=1, tag=9, params=params, updates=cnt)
            Mo = f.astype(np.float64)
            upd, pos = orc.train_partitioned(sp.offsets, sp.indices, Mo, K, B, epochs, float(np.float32(lr)), k,
                                             SEED, level=1, tag=9)
            assert _rel_rows(Mh.numpy().astype(np.float64), Mo) < 1e-4
        else:
            bits = orc.f32_to_bf16_rne(f).reshape(n, d)
            Mh = _host_bf16(bits)
            st = G.gosh_train_partitioned(gctx, g, Mh, epochs, lr, k, level=1, tag=9, params=params, updates=cnt)
            Mo = bits.copy()
            upd, pos = orc.train_partitioned(sp.offsets, sp.indices, Mo, K, B, epochs, float(np.float32(lr)), k,
                                             SEED, level=1, tag=9)
            got, want = orc.bf16_to_f64(_bits(Mh)), orc.bf16_to_f64(Mo)
            assert _rel_rows(got, want) < 2e-2
            assert np.mean(np.abs(got - want).sum(1) / np.abs(want).sum(1)) < 5e-3
    finally:
        gctx.set_deterministic(False)
    assert st["parts"] == K and st["positives"] == pos
    assert int(cnt.item()) == upd
    assert st["part_stores"] == st["part_loads"] >= 1
    if swaps:
        assert st["part_loads"] > K          # parts left the device and came back


def _geometric(n=4000, radius=0.03, seed=0):
    from scipy.spatial import cKDTree
    pts = np.random.default_rng(seed).random((n, 2))
    pairs = np.array(sorted(cKDTree(pts).query_pairs(radius)))
    return split_edges(*csr_from_pairs(n, pairs[:, 0], pairs[:, 1]), seed=2)


@pytest.mark.parametrize("dtype", [torch.float32, torch.bfloat16])
def test_concurrent_auc_matches_reference(gctx, orc, dtype):
    from paper_2110_10049_amd import gosh as G
    sp = _geometric()
    n, d, K, B, e, k = sp.n, 32, 4, 5, 100, 3
    f = init_rows(n, d, 3) * 20
    g = G.HostCSR(sp.offsets, sp.indices)
    Mh = torch.from_numpy(f).to(dtype).pin_memory()
    st = G.gosh_train_partitioned(gctx, g, Mh, e, 0.045, k, params=G.part_params(parts=K, B=B))
    bf = dtype == torch.bfloat16
    Mo = orc.f32_to_bf16_rne(f).reshape(n, d) if bf else f.astype(np.float64)
    orc.train_partitioned(sp.offsets, sp.indices, Mo, K, B, e, float(np.float32(0.045)), k, SEED)
    a_g = evaluate_auc(Mh.float().numpy(), sp, seed=5)
    a_o = evaluate_auc(orc.bf16_to_f64(Mo) if bf else Mo, sp, seed=5)
    print(f"[partitioned auc] {dtype}: gpu {a_g:.4f} oracle {a_o:.4f} stats {st}", flush=True)
    assert a_o > 0.85
    assert abs(a_g - a_o) < 0.01


def test_memory_cap_picks_parts(gctx):
    from paper_2110_10049_amd import gosh as G
    sp = _geometric()
    n, d = sp.n, 256
    cap = 4 << 20
    ctx = G.Context(0, seed=SEED, mem_cap=cap)
    try:
        params = G.part_params(sub_bins=3, pool_bins=2, B=5)
        budget = cap - ctx.mem_in_use()
        K, need = G.gosh_partition_plan(n, d, torch.float32, budget, params)
        assert K > 3 and need <= budget
        Mh = torch.from_numpy(init_rows(n, d, 3)).pin_memory()
        M0 = Mh.clone()
        st = G.gosh_train_partitioned(ctx, G.HostCSR(sp.offsets, sp.indices), Mh, 10, 0.045, 3, params=params)
        assert st["parts"] == K
        assert st["device_bytes"] <= cap
        assert ctx.mem_in_use() <= cap
        assert torch.isfinite(Mh).all() and not torch.equal(Mh, M0)
    finally:
        ctx.close()
    tiny = G.Context(0, seed=SEED, mem_cap=512 << 10)   # below the fixed 1 MiB workspace
    try:
        with pytest.raises(G.GoshError) as ei:
            G.gosh_train_partitioned(tiny, G.HostCSR(sp.offsets, sp.indices), Mh, 10, 0.045, 3, params=params)
        assert ei.value.status == "E_CAP_EXCEEDED"
    finally:
        tiny.close()


def test_partitioned_argument_errors(gctx):
    from paper_2110_10049_amd import gosh as G
    sp = split_edges(*rmat_csr(8, 4, 1), seed=2)
    g = G.HostCSR(sp.offsets, sp.indices)
    Mh = torch.zeros((sp.n, 16))
    for bad in (dict(sub_bins=1), dict(pool_bins=0), dict(B=0), dict(B=32), dict(parts=300)):
        with pytest.raises(G.GoshError) as ei:
            G.gosh_train_partitioned(gctx, g, Mh, 2, 0.045, 3, params=G.part_params(**bad))
        assert ei.value.status == "E_INVALID_ARG"
    with pytest.raises(G.GoshError):
        G.gosh_train_partitioned(gctx, g, Mh, 2, 0.045, 16)
    with pytest.raises(G.GoshError):
        G.gosh_train_partitioned(gctx, g, torch.zeros((sp.n, 12)), 2, 0.045, 3)
    bad_off = sp.offsets.copy()
    bad_off[-1] += 1
    with pytest.raises(G.GoshError) as ei:
        G.gosh_train_partitioned(gctx, G.HostCSR(bad_off, sp.indices), Mh, 2, 0.045, 3)
    assert ei.value.status == "E_BAD_GRAPH"
    with pytest.raises(ValueError):
        G.gosh_train_partitioned(gctx, g, Mh.cuda(), 2, 0.045, 3)
