"""MultiEdgeCollapse on the GPU against the oracle (Algorithm 4): every level's
CSR and map must be bit-identical."""
import os

import numpy as np
import pytest
import torch

from synth import check_csr, csr_from_pairs, rmat_csr
from tests.conftest import train_split

pytestmark = pytest.mark.gpu
GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _compare(gctx, orc, off, idx, threshold=100, ratio=0.8, off64=False):
    from paper_2110_10049_amd import gosh as G
    print(f"[coarsen parity] n={len(off)-1} nnz={len(idx)} thr={threshold} off64={off64}", flush=True)
    g = G.CSR.from_numpy(off, idx, off64=off64)
    lv = G.gosh_coarsen(gctx, g, threshold, ratio)
    graphs, maps = orc.coarsen_levels(off, idx, threshold, ratio)
    assert lv.count() == len(graphs)
    for i, (o, x) in enumerate(graphs):
        go, gx, gm = lv.copy_out(i, want_map=i < len(maps))
        assert np.array_equal(go, o), f"offsets differ at level {i}"
        assert np.array_equal(gx, x), f"indices differ at level {i}"
        if i < len(maps):
            assert np.array_equal(gm, maps[i]), f"map differs at level {i}"
    return lv, graphs, maps


def test_hand_traces(gctx, orc):
    for line in open(os.path.join(GOLD, "coarsen_traces.txt")):
        if line.startswith("#") or not line.strip():
            continue
        _, n, edges, _, _ = [x.strip() for x in line.split("|")]
        e = np.array([[int(a) for a in p.split("-")] for p in edges.split(",")])
        off, idx = csr_from_pairs(int(n), e[:, 0], e[:, 1])
        _compare(gctx, orc, off, idx, threshold=1)


@pytest.mark.parametrize("scale,ef,seed", [(6, 2, 3), (9, 4, 1), (10, 16, 2), (11, 8, 5)])
def test_rmat_levels(gctx, orc, scale, ef, seed):
    off, idx = rmat_csr(scale, ef, seed)
    _compare(gctx, orc, off, idx, threshold=8)


def test_config1_train_graph(gctx, orc):
    sp = train_split(12, 16)
    lv, graphs, _ = _compare(gctx, orc, sp.offsets, sp.indices, threshold=64)
    assert lv.count() >= 3


def test_cluster_sizes(gctx, orc):
    from paper_2110_10049_amd import gosh as G
    off, idx = rmat_csr(11, 8, 5)
    lv = G.gosh_coarsen(gctx, G.CSR.from_numpy(off, idx), 8)
    _, maps = orc.coarsen_levels(off, idx, 8)
    for i, mp in enumerate(maps):
        nn = lv.shape(i + 1)[0]
        assert np.array_equal(lv.cluster_sizes(i), np.bincount(mp, minlength=nn))


def test_coarsen_and_single_reject_bad_graphs(gctx):
    from paper_2110_10049_amd import gosh as G
    bad = {
        "self-loop": (np.array([0, 1, 2], np.int64), np.array([0, 0], np.int32)),
        "out of range": (np.array([0, 1, 2], np.int64), np.array([1, 5], np.int32)),
        "offsets": (np.array([0, 3, 1, 2], np.int64), np.array([1, 2], np.int32)),
        "last offset": (np.array([0, 1, 1], np.int64), np.array([1, 0], np.int32)),
    }
    for name, (o, x) in bad.items():
        g = G.CSR.from_numpy(o, x)
        for fn in (lambda: G.gosh_coarsen(gctx, g, 1), lambda: G.gosh_levels_single(gctx, g)):
            with pytest.raises(G.GoshError) as ei:
                fn()
            assert ei.value.status == "E_BAD_GRAPH", name


def test_int64_offsets(gctx, orc):
    off, idx = rmat_csr(10, 8, 7)
    _compare(gctx, orc, off, idx, threshold=16, off64=True)


def test_long_chain_path(gctx, orc):
    # equal degrees along a path force one hub decision per round
    n = 300
    e = np.stack([np.arange(n - 1), np.arange(1, n)], 1)
    off, idx = csr_from_pairs(n, e[:, 0], e[:, 1])
    _compare(gctx, orc, off, idx, threshold=4)


@pytest.mark.parametrize("n,prob,seed", [(200, 1.0, 0), (500, 0.3, 1), (3000, 0.05, 2)])
def test_dense_graphs(gctx, orc, n, prob, seed):
    # average degree >= 64: hub rounds and the assignment run one wave per vertex
    rng = np.random.default_rng(seed)
    iu, ju = np.triu_indices(n, 1)
    keep = rng.random(len(iu)) < prob
    off, idx = csr_from_pairs(n, iu[keep], ju[keep])
    assert len(idx) >= 64 * n
    _compare(gctx, orc, off, idx, threshold=2)


def test_edgeless_and_isolated(gctx, orc):
    off = np.zeros(9, np.int64)
    _compare(gctx, orc, off, np.zeros(0, np.int32), threshold=2)
    e = np.array([[0, 1], [1, 2], [5, 6]])
    off, idx = csr_from_pairs(10, e[:, 0], e[:, 1])
    _compare(gctx, orc, off, idx, threshold=1)


def test_random_tiny_graphs(gctx, orc):
    rng = np.random.default_rng(30)
    for trial in range(25):
        n = int(rng.integers(2, 40))
        m = int(rng.integers(0, n * 3))
        u, v = rng.integers(0, n, m), rng.integers(0, n, m)
        off, idx = csr_from_pairs(n, u, v)
        _compare(gctx, orc, off, idx, threshold=2)


def test_validate_rejects_bad_graphs(gctx):
    from paper_2110_10049_amd import gosh as G
    good_off = np.array([0, 2, 3, 4], np.int64)
    good_idx = np.array([1, 2, 0, 0], np.int32)
    G.gosh_validate_csr(gctx, G.CSR.from_numpy(good_off, good_idx))
    cases = {
        "self-loop": (np.array([0, 1, 2], np.int64), np.array([0, 0], np.int32)),
        "out of range": (np.array([0, 1, 2], np.int64), np.array([1, 5], np.int32)),
        "unsorted": (np.array([0, 2, 3, 4], np.int64), np.array([2, 1, 0, 0], np.int32)),
        "asymmetric": (np.array([0, 1, 1], np.int64), np.array([1], np.int32)),
        "offsets": (np.array([0, 2, 1, 2], np.int64), np.array([1, 2], np.int32)),
    }
    for name, (o, x) in cases.items():
        with pytest.raises(G.GoshError) as ei:
            G.gosh_validate_csr(gctx, G.CSR.from_numpy(o, x))
        assert ei.value.status == "E_BAD_GRAPH", name


@pytest.mark.slow
def test_config2_full_size(gctx, orc):
    # scale-20 R-MAT train graph (614k vertices, 25M entries): all levels bit-exact
    sp = train_split(20, 16)
    lv, graphs, _ = _compare(gctx, orc, sp.offsets, sp.indices, threshold=100)
    sizes = lv.sizes()
    print("[coarsen parity] level sizes", sizes, flush=True)
    assert sizes[0] == sp.n and len(sizes) >= 4


def test_trim_releases_cached_blocks(gctx, orc):
    # temporaries return to the context cache; gosh_trim frees them and later
    # calls allocate again with the same results
    from paper_2110_10049_amd import gosh as G
    off, idx = rmat_csr(11, 8, 5)
    ctx = G.Context(0, seed=4)
    try:
        g = G.CSR.from_numpy(off, idx)
        lv = G.gosh_coarsen(ctx, g, 8)
        first = [lv.copy_out(i) for i in range(lv.count() - 1)]
        held = ctx.mem_in_use()
        del lv
        ctx.trim()
        assert ctx.mem_in_use() < held
        lv = G.gosh_coarsen(ctx, g, 8)
        for i, (o, x, m) in enumerate(first):
            o2, x2, m2 = lv.copy_out(i)
            assert np.array_equal(o, o2) and np.array_equal(x, x2) and np.array_equal(m, m2)
    finally:
        ctx.close()
