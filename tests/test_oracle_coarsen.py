"""Pins of the oracle's MultiEdgeCollapse (Algorithm 4, Section 4) and of the
epoch distribution (Section 3): hand traces, a brute-force fixed-point
characterisation on tiny graphs, structural invariants and stop rule."""
import itertools
import os

import numpy as np
import pytest

from synth import check_csr, csr_from_pairs, rmat_csr

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _traces():
    out = []
    for line in open(os.path.join(GOLD, "coarsen_traces.txt")):
        if line.startswith("#") or not line.strip():
            continue
        name, n, edges, mp, nn = [x.strip() for x in line.split("|")]
        e = [tuple(int(a) for a in p.split("-")) for p in edges.split(",")]
        out.append(pytest.param(int(n), e, [int(x) for x in mp.split()], int(nn), id=name))
    return out


@pytest.mark.parametrize("n,edges,want,nn", _traces())
def test_hand_traces(orc, n, edges, want, nn):
    e = np.array(edges)
    off, idx = csr_from_pairs(n, e[:, 0], e[:, 1])
    mp, got_nn, _ = orc.coarsen_map(off, idx)
    assert list(mp) == want and got_nn == nn


def _brute_force_map(n, adj):
    """Hub set as the unique H with: v in H  <=>  no eligible neighbour of v
    in H precedes v (found by enumerating all 2^n subsets); members go to
    their earliest eligible hub neighbour; hubs are numbered in order."""
    deg = np.array([len(a) for a in adj])
    nnz = int(deg.sum())
    order = sorted(range(n), key=lambda v: (-deg[v], v))
    rank = {v: r for r, v in enumerate(order)}
    elig = [[u for u in adj[v] if deg[v] * n <= nnz or deg[u] * n <= nnz] for v in range(n)]
    sols = []
    for mask in range(1 << n):
        H = {v for v in range(n) if mask >> v & 1}
        ok = all((v in H) == (not any(h in H and rank[h] < rank[v] for h in elig[v]))
                 for v in range(n))
        if ok:
            sols.append(H)
    assert len(sols) == 1
    H = sols[0]
    hub_ids = {h: i for i, h in enumerate(sorted(H, key=lambda v: rank[v]))}
    mp = []
    for v in range(n):
        if v in H:
            mp.append(hub_ids[v])
        else:
            h = min((h for h in elig[v] if h in H), key=lambda h: rank[h])
            mp.append(hub_ids[h])
    return mp


def test_brute_force_tiny_graphs(orc):
    rng = np.random.default_rng(20)
    for trial in range(150):
        n = int(rng.integers(1, 12))
        p = rng.uniform(0.1, 0.7)
        pairs = [(a, b) for a, b in itertools.combinations(range(n), 2) if rng.random() < p]
        if pairs:
            e = np.array(pairs)
            off, idx = csr_from_pairs(n, e[:, 0], e[:, 1])
        else:
            off, idx = np.zeros(n + 1, np.int64), np.zeros(0, np.int32)
        adj = [list(idx[off[v]:off[v + 1]]) for v in range(n)]
        mp, nn, _ = orc.coarsen_map(off, idx)
        assert list(mp) == _brute_force_map(n, adj)
        assert nn == max(mp) + 1 if n else nn == 0


def _check_level(off, idx, mp, nn, coff, cidx):
    n = len(off) - 1
    deg = np.diff(off)
    nnz = int(off[-1])
    # partition with contiguous ids
    assert mp.min() == 0 and mp.max() == nn - 1
    assert len(np.unique(mp)) == nn
    src = np.repeat(np.arange(n), deg)
    elig = (deg[src] * n <= nnz) | (deg[idx] * n <= nnz)
    # hubs = first vertex of each cluster in (-deg, id) order
    order = np.lexsort((np.arange(n), -deg))
    first = np.full(nn, -1)
    for v in order:
        if first[mp[v]] < 0:
            first[mp[v]] = v
    hub = np.zeros(n, bool)
    hub[first] = True
    # hubs form an independent set in the eligible graph ...
    assert not np.any(hub[src] & hub[idx] & elig)
    # ... every non-hub is eligible-adjacent to its own hub
    members = np.nonzero(~hub)[0]
    for v in members:
        nb = idx[off[v]:off[v + 1]]
        e = elig[off[v]:off[v + 1]]
        assert first[mp[v]] in set(nb[e])
    # cluster ids ascend with the hubs' processing order
    rank = np.empty(n, np.int64)
    rank[order] = np.arange(n)
    assert np.all(np.diff(rank[first]) > 0)
    # coarse graph = distinct mapped pairs without loops, simple and symmetric
    check_csr(coff, cidx)
    a, b = mp[src].astype(np.int64), mp[idx].astype(np.int64)
    keep = a != b
    want = np.unique(a[keep] * nn + b[keep])
    csrc = np.repeat(np.arange(nn), np.diff(coff))
    assert np.array_equal(want, csrc * nn + cidx)


@pytest.mark.parametrize("scale,ef,seed", [(9, 4, 1), (10, 16, 2), (11, 8, 3)])
def test_invariants_rmat(orc, scale, ef, seed):
    off, idx = rmat_csr(scale, ef, seed)
    graphs, maps = orc.coarsen_levels(off, idx, threshold=16)
    for i, mp in enumerate(maps):
        (o, x), (co, cx) = graphs[i], graphs[i + 1]
        _check_level(o, x, mp, len(co) - 1, co, cx)
    sizes = [len(g[0]) - 1 for g in graphs]
    # stop rule: every level but the last passed the continue test
    for a, b in zip(sizes[:-2], sizes[1:-1]):
        assert b >= 16 and b <= 0.8 * a
    assert sizes[-1] < 16 or sizes[-1] > 0.8 * sizes[-2]


def test_complete_graph_collapses_without_loops(orc):
    # Table 5's last level (823 vertices, density 822 = complete graph) implies
    # coarse graphs carry neither self-loops nor duplicate edges: two cliques
    # joined by every cross edge collapse to K_2 with nnz 2, not more.
    n = 10
    pairs = np.array([(a, b) for a in range(n) for b in range(a + 1, n)])
    off, idx = csr_from_pairs(n, pairs[:, 0], pairs[:, 1])
    mp, nn, _ = orc.coarsen_map(off, idx)
    assert nn == 1
    coff, cidx = orc.coarse_graph(off, idx, mp, nn)
    assert coff.tolist() == [0, 0]
    # star of stars: K_{1,4} centres, each with 3 leaves
    edges = [(0, c) for c in (1, 2, 3, 4)] + [(c, 5 + 3 * (c - 1) + j) for c in (1, 2, 3, 4) for j in range(3)]
    e = np.array(edges)
    off, idx = csr_from_pairs(17, e[:, 0], e[:, 1])
    mp, nn, _ = orc.coarsen_map(off, idx)
    coff, cidx = orc.coarse_graph(off, idx, mp, nn)
    check_csr(coff, cidx)


def test_empty_and_edgeless(orc):
    graphs, maps = orc.coarsen_levels(np.zeros(1, np.int64), np.zeros(0, np.int32))
    assert len(graphs) == 1 and maps == []
    off = np.zeros(6, np.int64)
    graphs, maps = orc.coarsen_levels(off, np.zeros(0, np.int32), threshold=2)
    assert len(graphs) == 2 and list(maps[0]) == [0, 1, 2, 3, 4]


# ---------------------------------------------------------------- schedule
def _schedules():
    out = []
    for line in open(os.path.join(GOLD, "epoch_schedule.txt")):
        if line.startswith("#") or not line.strip():
            continue
        a, b = line.split("|")
        e, p, D = a.split()
        out.append((int(e), float(p), int(D), [int(x) for x in b.split()]))
    return out


@pytest.mark.parametrize("e,p,D,want", _schedules())
def test_schedule_worked_examples(orc, e, p, D, want):
    assert list(orc.epoch_schedule(e, p, D)) == want


def test_schedule_properties(orc):
    for e in (1, 7, 100, 600, 1000):
        for p in (0.0, 0.1, 0.3, 0.5, 1.0):
            for D in (1, 2, 5, 11):
                s = orc.epoch_schedule(e, p, D)
                assert s.sum() == e
                assert np.all(np.diff(s) >= 0) or p == 1.0
    # p = 0: purely geometric, e_i proportional to 2^i
    s = orc.epoch_schedule(31 * 8, 0.0, 5)
    assert list(s) == [8, 16, 32, 64, 128]
    with pytest.raises(ValueError):
        orc.epoch_schedule(10, 1.5, 3)
