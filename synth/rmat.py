"""Seeded R-MAT graphs (Chakrabarti, Zhan, Faloutsos, SDM 2004).

Each draw i picks, for every bit level l (most significant first), one of the
four quadrants with probabilities (a, b, c, d): a -> (0,0), b -> (0,1),
c -> (1,0), d -> (1,1) for the (row, column) bit.  The uniform value that picks
the quadrant is a counter-based hash of (seed, i, l): SplitMix64's output
function (Steele, Lea, Flood, OOPSLA 2014) applied to
``(seed << 40) ^ (i << 6) ^ l``, top 32 bits.  The graph is therefore a pure
function of (scale, draws, seed) and can be regenerated in chunks.

Undirected "edge factor" ``ef`` means ``ef * n`` draws; self-loops are dropped,
both directions are stored and duplicates removed, so the CSR average degree
is at most ``2 * ef`` (density |E|/|V| as in Table 2 of the paper).
"""
from __future__ import annotations

import numpy as np

RMAT_ABCD = (0.57, 0.19, 0.19, 0.05)

_M64 = np.uint64(0xFFFFFFFFFFFFFFFF)
_GOLD = np.uint64(0x9E3779B97F4A7C15)
_MIX1 = np.uint64(0xBF58476D1CE4E5B9)
_MIX2 = np.uint64(0x94D049BB133111EB)


def _splitmix_u32(z: np.ndarray) -> np.ndarray:
    """Top 32 bits of SplitMix64's output function of ``z + golden``."""
    with np.errstate(over="ignore"):
        z = z + _GOLD
        z = (z ^ (z >> np.uint64(30))) * _MIX1
        z = (z ^ (z >> np.uint64(27))) * _MIX2
        z = z ^ (z >> np.uint64(31))
    return (z >> np.uint64(32)).astype(np.uint32)


def _thresholds(abcd):
    a, b, c, _ = abcd
    t = np.array([a, a + b, a + b + c], dtype=np.float64) * 4294967296.0
    return np.floor(t).astype(np.uint64)


def rmat_pairs(scale: int, first: int, count: int, seed: int,
               abcd=RMAT_ABCD) -> tuple[np.ndarray, np.ndarray]:
    """Draws ``first .. first+count-1`` of the R-MAT stream: (row, col) int64."""
    ta, tab, tabc = _thresholds(abcd)
    idx = np.arange(first, first + count, dtype=np.uint64)
    base = (np.uint64(seed) << np.uint64(40)) ^ (idx << np.uint64(6))
    row = np.zeros(count, dtype=np.int64)
    col = np.zeros(count, dtype=np.int64)
    for lvl in range(scale):
        r = _splitmix_u32(base ^ np.uint64(lvl)).astype(np.uint64)
        bit = np.int64(1) << np.int64(scale - 1 - lvl)
        rbit = r >= tab                      # quadrants c, d
        cbit = ((r >= ta) & (r < tab)) | (r >= tabc)   # quadrants b, d
        row += rbit * bit
        col += cbit * bit
    return row, col


def csr_from_pairs(n: int, u: np.ndarray, v: np.ndarray):
    """Simple undirected CSR from (u, v) pairs: loops dropped, both
    directions stored, duplicates removed, rows sorted ascending."""
    u = np.asarray(u, dtype=np.int64)
    v = np.asarray(v, dtype=np.int64)
    keep = u != v
    u, v = u[keep], v[keep]
    key = np.concatenate([u * n + v, v * n + u])
    key = np.unique(key)
    src = key // n
    dst = (key - src * n).astype(np.int32)
    offsets = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(np.bincount(src, minlength=n), out=offsets[1:])
    return offsets, dst


def rmat_csr(scale: int, edge_factor: float, seed: int, n: int | None = None,
             abcd=RMAT_ABCD, chunk: int = 1 << 24):
    """R-MAT graph with ``m = round(edge_factor * n)`` draws.

    ``n`` defaults to ``2**scale``.  A non-power-of-two ``n`` draws at scale
    ``ceil(log2 n)`` and rejects pairs with an endpoint ``>= n`` until ``m``
    pairs are accepted (draw order is preserved).
    Returns (offsets int64[n+1], indices int32[nnz]).
    """
    if n is None:
        n = 1 << scale
    m = int(round(edge_factor * n))
    us, vs = [], []
    have = 0
    first = 0
    while have < m:
        cnt = min(chunk, max(m - have, 1) * (1 if n == (1 << scale) else 2) + 1024)
        r, c = rmat_pairs(scale, first, cnt, seed, abcd)
        first += cnt
        if n != (1 << scale):
            ok = (r < n) & (c < n)
            r, c = r[ok], c[ok]
        take = min(len(r), m - have)
        us.append(r[:take])
        vs.append(c[:take])
        have += take
    u = np.concatenate(us) if us else np.zeros(0, np.int64)
    v = np.concatenate(vs) if vs else np.zeros(0, np.int64)
    return csr_from_pairs(n, u, v)


def check_csr(offsets: np.ndarray, indices: np.ndarray) -> None:
    """Raise ValueError unless (offsets, indices) is a simple symmetric CSR
    with sorted rows and no self-loops."""
    n = len(offsets) - 1
    if offsets[0] != 0 or np.any(np.diff(offsets) < 0) or offsets[-1] != len(indices):
        raise ValueError("offsets not monotone from 0 to nnz")
    if len(indices) and (indices.min() < 0 or indices.max() >= n):
        raise ValueError("index out of range")
    src = np.repeat(np.arange(n, dtype=np.int64), np.diff(offsets))
    if np.any(src == indices):
        raise ValueError("self-loop")
    d = np.diff(indices.astype(np.int64))
    rowstart = np.zeros(len(indices), dtype=bool)
    rowstart[offsets[:-1][np.diff(offsets) > 0]] = True
    if np.any((d <= 0) & ~rowstart[1:]):
        raise ValueError("row not strictly ascending")
    fwd = np.sort(src * n + indices)
    bwd = np.sort(indices.astype(np.int64) * n + src)
    if not np.array_equal(fwd, bwd):
        raise ValueError("not symmetric")


# --------------------------------------------------------------------------- torch port
def _s64(c: int) -> int:
    """uint64 constant as the int64 with the same bits."""
    return c - (1 << 64) if c >= (1 << 63) else c


def _lsr(z, k: int):
    """Logical right shift of int64 tensors holding uint64 bit patterns."""
    return (z >> k) & ((1 << (64 - k)) - 1)


def rmat_pairs_torch(scale: int, first: int, count: int, seed: int, device, abcd=RMAT_ABCD):
    """The same draws as rmat_pairs, computed with torch int64 arithmetic
    (wrapping multiplication has the uint64 bit pattern) on `device`."""
    import torch
    ta, tab, tabc = (int(x) for x in _thresholds(abcd))
    idx = torch.arange(first, first + count, dtype=torch.int64, device=device)
    base = (seed << 40) ^ (idx << 6)
    row = torch.zeros(count, dtype=torch.int64, device=device)
    col = torch.zeros(count, dtype=torch.int64, device=device)
    gold, m1, m2 = _s64(0x9E3779B97F4A7C15), _s64(0xBF58476D1CE4E5B9), _s64(0x94D049BB133111EB)
    for lvl in range(scale):
        z = (base ^ lvl) + gold
        z = (z ^ _lsr(z, 30)) * m1
        z = (z ^ _lsr(z, 27)) * m2
        z = z ^ _lsr(z, 31)
        r = _lsr(z, 32)
        bit = 1 << (scale - 1 - lvl)
        row += (r >= tab).to(torch.int64) * bit
        col += (((r >= ta) & (r < tab)) | (r >= tabc)).to(torch.int64) * bit
    return row, col


def rmat_csr_torch(scale: int, edge_factor: float, seed: int, device, n: int | None = None,
                   abcd=RMAT_ABCD, chunk: int = 1 << 26, offsets_dtype=None):
    """rmat_csr on `device`: returns torch (offsets, indices int32); offsets are
    int64 unless offsets_dtype says otherwise.  Same graph as rmat_csr."""
    import torch
    if n is None:
        n = 1 << scale
    m = int(round(edge_factor * n))
    keys = []
    have = 0
    first = 0
    while have < m:
        cnt = min(chunk, max(m - have, 1) * (1 if n == (1 << scale) else 2) + 1024)
        r, c = rmat_pairs_torch(scale, first, cnt, seed, device, abcd)
        first += cnt
        if n != (1 << scale):
            ok = (r < n) & (c < n)
            r, c = r[ok], c[ok]
        take = min(r.numel(), m - have)
        r, c = r[:take], c[:take]
        keep = r != c
        r, c = r[keep], c[keep]
        keys.append(torch.unique(torch.cat([r * n + c, c * n + r])))
        have += take
        del r, c
    key = torch.unique(torch.cat(keys)) if keys else torch.zeros(0, dtype=torch.int64, device=device)
    del keys
    src = torch.div(key, n, rounding_mode="floor")
    dst = (key - src * n).to(torch.int32)
    del key
    offsets = torch.zeros(n + 1, dtype=torch.int64, device=device)
    offsets[1:] = torch.cumsum(torch.bincount(src, minlength=n), 0)
    if offsets_dtype is not None:
        offsets = offsets.to(offsets_dtype)
    return offsets, dst


def drop_isolated_torch(offsets, indices):
    """Removes vertices without neighbours and relabels the rest in ascending
    old id (torch tensors on any device).  Returns (offsets, indices, old_id)."""
    import torch
    deg = offsets[1:] - offsets[:-1]
    keep = deg > 0
    old_id = torch.nonzero(keep).flatten()
    newid = torch.full((deg.numel(),), -1, dtype=torch.int64, device=offsets.device)
    newid[old_id] = torch.arange(old_id.numel(), device=offsets.device)
    new_off = torch.zeros(old_id.numel() + 1, dtype=offsets.dtype, device=offsets.device)
    new_off[1:] = torch.cumsum(deg[keep], 0).to(offsets.dtype)
    new_idx = newid[indices.long()].to(torch.int32)
    return new_off, new_idx, old_id
