"""End-to-end behaviour of the oracle's Algorithm 2 driver: the multi-level
embedding learns link structure on a graph with strong locality, in FP64 and
in BF16 storage."""
import numpy as np
import pytest

from synth import csr_from_pairs, evaluate_auc, init_rows, split_edges


def _geometric(n=2000, radius=0.04, seed=0):
    from scipy.spatial import cKDTree
    pts = np.random.default_rng(seed).random((n, 2))
    pairs = np.array(sorted(cKDTree(pts).query_pairs(radius)))
    return csr_from_pairs(n, pairs[:, 0], pairs[:, 1])


@pytest.mark.parametrize("bf16", [False, True])
def test_multilevel_learns_geometric_graph(orc, bf16):
    off, idx = _geometric()
    sp = split_edges(off, idx, seed=2)
    M, info = orc.gosh_embed(sp.offsets, sp.indices, lambda n, d: init_rows(n, d, 3),
                             d=32, e=200, p=0.3, lr=0.045, k=1, seed=4, threshold=64, bf16=bf16)
    assert info["levels"] >= 3
    assert sum(info["schedule"]) == 200
    Mf = orc.bf16_to_f64(M) if bf16 else M
    assert evaluate_auc(Mf, sp, seed=5) > 0.85


def test_driver_order_and_prolongation(orc):
    # Trained coarse rows are copied to every member before the finer level
    # trains: with zero epochs on the finer levels the final rows are exactly
    # the coarsest rows expanded through all maps.
    off, idx = _geometric(600, 0.07, seed=1)
    graphs, maps = orc.coarsen_levels(off, idx, threshold=16)
    D = len(graphs)
    init = init_rows(len(graphs[-1][0]) - 1, 8, 3)
    M, info = orc.gosh_embed(off, idx, lambda n, d: init, d=8, e=0, p=0.3, lr=0.05, k=1,
                             seed=4, levels=(graphs, maps))
    want = init.astype(np.float64)
    for mp in maps[::-1]:
        want = want[mp]
    assert np.array_equal(M, want)
    # members of one cluster share their row
    mp0 = maps[0]
    for c in range(0, int(mp0.max()) + 1, 37):
        rows = M[mp0 == c]
        assert np.all(rows == rows[0])


def test_edge_epoch_unit(orc):
    # one epoch = |E| updates (the note under Table 3): a pass of Algorithm 3
    # makes n positive updates, so level i needs ceil(nnz_i / (2 n_i)) passes
    # per epoch; at least one, also for an edgeless level
    from paper_2110_10049_amd.driver import unit_epochs
    graphs = [(np.array([0, 3, 5, 8, 10]), None),      # n = 4, nnz = 10 -> ceil(10 / 8) = 2
              (np.array([0, 0, 0, 0]), None),          # n = 3, edgeless -> 1
              (np.array([0, 2, 4]), None),             # n = 2, nnz = 4 -> 1
              (np.array([0, 6, 12, 18, 24]), None)]    # n = 4, nnz = 24 (K_4 has 12) -> 3
    sched = [10, 11, 12, 13]
    want = [20, 11, 12, 39]
    assert list(orc.unit_epochs(sched, graphs, "edges")) == want
    assert list(orc.unit_epochs(sched, graphs, "passes")) == sched
    shapes = [(len(o) - 1, int(o[-1])) for o, _ in graphs]
    assert unit_epochs(sched, shapes, "edges") == want
    assert unit_epochs(sched, shapes, "passes") == sched
    with pytest.raises(ValueError):
        unit_epochs(sched, shapes, "vertices")
