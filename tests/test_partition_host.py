"""Host side of the partitioned embedding in the library (no device needed):
its sample pools equal the reference's entry for entry, its pair order is
the inside-out order, and its part count follows the memory budget."""
import numpy as np
import pytest
import torch

from synth import rmat_csr, split_edges


def _g(scale=10, ef=8, seed=1, off64=False):
    from paper_2110_10049_amd import gosh as G
    sp = split_edges(*rmat_csr(scale, ef, seed), seed=2)
    off = sp.offsets.astype(np.int64 if off64 else np.int32)
    return sp, G.HostCSR(off, sp.indices)


@pytest.mark.parametrize("K,i,j,B,threads,off64", [(1, 0, 0, 1, 1, False), (3, 2, 0, 5, 4, False),
                                                    (4, 1, 1, 5, 3, True), (5, 4, 2, 7, 8, False),
                                                    (7, 6, 3, 2, 16, True)])
def test_pools_equal_reference(orc, K, i, j, B, threads, off64):
    from paper_2110_10049_amd import gosh as G
    sp, g = _g(off64=off64)
    for rnd in (0, 3):
        a = G.gosh_partition_pool(g, K, i, j, B, seed=0x1234567890AB, level=3, tag=77, round=rnd, threads=threads)
        b = orc.pool(sp.offsets, sp.indices, K, i, j, B, seed=0x1234567890AB, level=3, tag=77, round=rnd)
        for x, y in zip(a, b):
            assert np.array_equal(x, y)


def test_inside_out_matches_reference(orc):
    from paper_2110_10049_amd import gosh as G
    for K in (1, 2, 3, 6, 11, 40):
        assert G.gosh_inside_out(K) == orc.inside_out(K)


def test_plan_picks_smallest_fitting_part_count():
    from paper_2110_10049_amd import gosh as G
    p = G.part_params(sub_bins=3, pool_bins=2, B=5)
    n, d = 37_500_000, 128
    K, need = G.gosh_partition_plan(n, d, torch.bfloat16, 16 << 30, p)
    assert K > 3 and need <= 16 << 30
    _, more = G.gosh_partition_plan(n, d, torch.bfloat16, 16 << 30, G.part_params(parts=K - 1))
    assert K == 4 or more > 16 << 30
    K2, _ = G.gosh_partition_plan(n, d, torch.bfloat16, 6 << 30, p)
    assert K2 > K
    assert G.gosh_partition_plan(1000, 64, torch.float32, 1 << 30, G.part_params(parts=2))[0] == 2
    with pytest.raises(G.GoshError):
        G.gosh_partition_plan(n, d, torch.bfloat16, 1 << 20, p)
    with pytest.raises(G.GoshError):
        G.gosh_partition_plan(n, d, torch.bfloat16, 16 << 30, G.part_params(sub_bins=1))


def test_pool_rejects_bad_requests():
    from paper_2110_10049_amd import gosh as G
    _, g = _g(8, 4)
    for args in ((0, 0, 0, 5), (3, 3, 0, 5), (3, 0, 0, 0), (3, 0, 0, 32)):
        with pytest.raises(G.GoshError):
            G.gosh_partition_pool(g, *args, seed=1)
