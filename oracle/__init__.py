"""GOSH CPU oracle -- test infrastructure only.

A plain FP64 reference of the method of "Boosting Graph Embedding on a Single
GPU" (arXiv 2110.10049), used by the tests and the smoke check to check the
HIP path, and timed by the benchmark's CPU-baseline leg.  The product path
never imports it.  The arithmetic is in ``gosh_oracle.c`` (loaded with ctypes);
this module adds numpy marshalling and the parts that are plain definitions:

  * coarsening levels with the stop rule of Algorithm 4
  * copy prolongation (ExpandEmbedding of Algorithm 2): M_i[v] = M_{i+1}[map_i[v]]
  * the multi-level driver of Algorithm 2, trained from the coarsest level
    down to level 0
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

_i64p = np.ctypeslib.ndpointer(dtype=np.int64, flags="C_CONTIGUOUS")
_i32p = np.ctypeslib.ndpointer(dtype=np.int32, flags="C_CONTIGUOUS")
_u32p = np.ctypeslib.ndpointer(dtype=np.uint32, flags="C_CONTIGUOUS")


class _Emb(C.Structure):
    _fields_ = [("rows", C.c_void_p), ("bf16", C.c_int32), ("d", C.c_int32)]


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            from .build import build
            build()
        L = C.CDLL(_LIB_PATH)
        L.orc_philox4x32_10.argtypes = [_u32p, _u32p, _u32p]
        L.orc_philox_many.argtypes = [_u32p, C.c_int64, _u32p, _u32p]
        L.orc_philox_many.restype = None
        L.orc_stream_block.argtypes = [C.c_uint64, C.c_int32, C.c_uint32, C.c_int32, C.c_int64,
                                       C.c_uint32, C.c_uint32, C.c_uint32, _u32p]
        L.orc_draw_samples.argtypes = [_i64p, _i32p, C.c_int64, C.c_uint64, C.c_int32, C.c_uint32,
                                       C.c_int32, C.c_int64, C.c_int32, _i32p]
        L.orc_sr_bits.argtypes = [C.c_uint64, C.c_int32, C.c_uint32, C.c_int32, C.c_int64,
                                  C.c_uint32, C.c_int32, C.c_int32]
        L.orc_sr_bits.restype = C.c_uint32
        L.orc_bf16_sr.argtypes = [C.c_float, C.c_uint32]
        L.orc_bf16_sr.restype = C.c_uint16
        L.orc_bf16_rne.argtypes = [C.c_float]
        L.orc_bf16_rne.restype = C.c_uint16
        L.orc_bf16_to_f64.argtypes = [C.c_uint16]
        L.orc_bf16_to_f64.restype = C.c_double
        L.orc_sigmoid.argtypes = [C.c_double]
        L.orc_sigmoid.restype = C.c_double
        L.orc_loss.argtypes = [C.c_double, C.c_int]
        L.orc_loss.restype = C.c_double
        L.orc_visit.argtypes = [C.POINTER(_Emb), C.c_int64, _i32p, C.c_int32, C.c_double,
                                C.c_uint64, C.c_int32, C.c_uint32, C.c_int32]
        L.orc_visit.restype = C.c_int32
        L.orc_update_batch.argtypes = [C.POINTER(_Emb), C.c_int64, _i32p, _i32p, C.c_int32,
                                       C.c_double, C.c_uint64, C.c_int32, C.c_uint32, C.c_int32]
        L.orc_update_batch.restype = C.c_int64
        L.orc_train.argtypes = [_i64p, _i32p, C.c_int64, C.POINTER(_Emb), C.c_int32, C.c_double,
                                C.c_int32, C.c_uint64, C.c_int32, C.c_uint32, C.c_int64, C.c_int64]
        L.orc_train.restype = C.c_int64
        L.orc_train_loss.argtypes = [_i64p, _i32p, C.c_int64, C.POINTER(_Emb), C.c_int32, C.c_double,
                                     C.c_int32, C.c_uint64, C.c_int32, C.c_uint32,
                                     np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")]
        L.orc_train_loss.restype = C.c_int64
        L.orc_train_hogwild.argtypes = [_i64p, _i32p, C.c_int64, C.POINTER(_Emb), C.c_int32, C.c_double,
                                        C.c_int32, C.c_uint64, C.c_int32, C.c_uint32, C.c_int32]
        L.orc_train_hogwild.restype = C.c_int64
        L.orc_draw_all.argtypes = [_i64p, _i32p, C.c_int64, C.c_uint64, C.c_int32, C.c_uint32, C.c_int32,
                                   C.c_int32, _i32p]
        L.orc_draw_all.restype = None
        L.orc_coarsen_map.argtypes = [_i64p, _i32p, C.c_int64, _i32p, C.c_void_p]
        L.orc_coarsen_map.restype = C.c_int64
        L.orc_coarse_graph.argtypes = [_i64p, _i32p, C.c_int64, _i32p, C.c_int64, _i64p, _i32p]
        L.orc_coarse_graph.restype = C.c_int64
        L.orc_epoch_schedule.argtypes = [C.c_int32, C.c_double, C.c_int32, _i32p]
        L.orc_epoch_schedule.restype = C.c_int32
        L.orc_part_starts.argtypes = [C.c_int64, C.c_int32, _i64p]
        L.orc_inside_out.argtypes = [C.c_int32, _i32p]
        L.orc_inside_out.restype = C.c_int64
        L.orc_pool.argtypes = [_i64p, _i32p, C.c_int64, C.c_int32, C.c_int32, C.c_int32, C.c_int32,
                               C.c_uint64, C.c_int32, C.c_uint32, C.c_int32, C.c_void_p, C.c_void_p,
                               C.c_void_p]
        L.orc_pool.restype = C.c_int64
        L.orc_train_partitioned.argtypes = [_i64p, _i32p, C.c_int64, C.POINTER(_Emb), C.c_int32, C.c_int32,
                                            C.c_int32, C.c_double, C.c_int32, C.c_uint64, C.c_int32,
                                            C.c_uint32, C.POINTER(C.c_int64)]
        L.orc_train_partitioned.restype = C.c_int64
        L.orc_walk.argtypes = [_i64p, _i32p, C.c_uint64, C.c_int32, C.c_uint32, C.c_int32, C.c_int64, C.c_int32,
                               _i32p]
        L.orc_walk.restype = C.c_int32
        L.orc_walk_offsets.argtypes = [C.c_int32, C.c_int32, C.c_void_p, C.c_void_p]
        L.orc_walk_offsets.restype = C.c_int32
        L.orc_walk_keys.argtypes = [C.c_int64, C.c_uint64, C.c_int32, C.c_uint32, C.c_int32, _u32p]
        L.orc_walk_keys.restype = None
        L.orc_walk_order.argtypes = [C.c_int64, C.c_int32, C.c_uint64, C.c_int32, C.c_uint32, C.c_int32, _i64p]
        L.orc_walk_order.restype = C.c_int64
        L.orc_walk_pairs.argtypes = [_i64p, _i32p, C.c_int64, C.c_uint64, C.c_int32, C.c_uint32, C.c_int32,
                                     C.c_int32, C.c_int32, _i32p, _i32p]
        L.orc_walk_pairs.restype = C.c_int64
        L.orc_train_walks.argtypes = [_i64p, _i32p, C.c_int64, C.POINTER(_Emb), C.c_int32, C.c_double, C.c_int32,
                                      C.c_int32, C.c_int32, C.c_uint64, C.c_int32, C.c_uint32]
        L.orc_train_walks.restype = C.c_int64
        _lib = L
    return _lib


def _csr(offsets, indices):
    return (np.ascontiguousarray(offsets, dtype=np.int64),
            np.ascontiguousarray(indices, dtype=np.int32))


# --------------------------------------------------------------------------- random stream
def philox4x32_10(ctr, key) -> np.ndarray:
    out = np.zeros(4, np.uint32)
    lib().orc_philox4x32_10(np.asarray(ctr, np.uint32), np.asarray(key, np.uint32), out)
    return out


def philox_many(ctr, key) -> np.ndarray:
    """Philox4x32-10 of every row of ctr ([m, 4] uint32) under one key: [m, 4]."""
    ctr = np.ascontiguousarray(ctr, np.uint32).reshape(-1, 4)
    out = np.zeros_like(ctr)
    lib().orc_philox_many(ctr.reshape(-1), len(ctr), np.asarray(key, np.uint32), out.reshape(-1))
    return out


def stream_block(seed, level, tag, epoch, src, kind, slot, block) -> np.ndarray:
    out = np.zeros(4, np.uint32)
    lib().orc_stream_block(seed, level, tag, epoch, src, kind, slot, block, out)
    return out


def draw_samples(offsets, indices, seed, level, tag, epoch, src, k) -> np.ndarray:
    offsets, indices = _csr(offsets, indices)
    out = np.zeros(1 + k, np.int32)
    lib().orc_draw_samples(offsets, indices, len(offsets) - 1, seed, level, tag, epoch, src, k, out)
    return out


def draw_all(offsets, indices, seed, level, tag, epoch, k) -> np.ndarray:
    """[n, 1+k] samples of every source for one epoch."""
    offsets, indices = _csr(offsets, indices)
    n = len(offsets) - 1
    out = np.zeros((max(n, 1), 1 + k), np.int32)
    lib().orc_draw_all(offsets, indices, n, seed, level, tag, epoch, k, out.reshape(-1))
    return out[:n]


def sr_bits(seed, level, tag, epoch, src, slot, e, d) -> int:
    return int(lib().orc_sr_bits(seed, level, tag, epoch, src, slot, e, d))


def bf16_sr(x: float, r16: int) -> int:
    return int(lib().orc_bf16_sr(x, r16))


def bf16_rne(x: float) -> int:
    return int(lib().orc_bf16_rne(x))


def f32_to_bf16_rne(a: np.ndarray) -> np.ndarray:
    """Vectorised round-to-nearest-even FP32 -> BF16 bits (finite inputs)."""
    u = np.ascontiguousarray(a, dtype=np.float32).view(np.uint32).astype(np.uint64)
    lsb = (u >> np.uint64(16)) & np.uint64(1)
    return ((u + np.uint64(0x7FFF) + lsb) >> np.uint64(16)).astype(np.uint16)


def bf16_to_f64(h: np.ndarray) -> np.ndarray:
    return (np.asarray(h, np.uint16).astype(np.uint32) << np.uint32(16)).view(np.float32).astype(np.float64)


def sigmoid(x: float) -> float:
    return float(lib().orc_sigmoid(x))


def loss(x: float, b: int) -> float:
    return float(lib().orc_loss(x, b))


# --------------------------------------------------------------------------- updates
def _emb(M: np.ndarray) -> _Emb:
    if not M.flags.c_contiguous or M.ndim != 2:
        raise ValueError("embedding must be a C-contiguous [n, d] array")
    if M.dtype == np.float64:
        bf = 0
    elif M.dtype == np.uint16:
        bf = 1
    else:
        raise ValueError("oracle rows are float64 or uint16 (BF16 bits)")
    return _Emb(M.ctypes.data, bf, M.shape[1])


def visit(M, src, samples, lr, seed=0, level=0, tag=0, epoch=0) -> int:
    s = np.ascontiguousarray(samples, np.int32)
    e = _emb(M)
    return int(lib().orc_visit(C.byref(e), src, s, len(s) - 1, lr, seed, level, tag, epoch))


def update_batch(M, src, samples, lr, seed=0, level=0, tag=0, epoch=0) -> int:
    src = np.ascontiguousarray(src, np.int32)
    samples = np.ascontiguousarray(samples, np.int32)
    k = samples.shape[1] - 1
    e = _emb(M)
    return int(lib().orc_update_batch(C.byref(e), len(src), src, samples.reshape(-1), k, lr,
                                      seed, level, tag, epoch))


def train(offsets, indices, M, epochs, lr, k, seed, level=0, tag=0, src_lo=0, src_hi=None) -> int:
    offsets, indices = _csr(offsets, indices)
    n = len(offsets) - 1
    if M.shape[0] != n:
        raise ValueError("embedding rows != |V|")
    if not 0 <= k <= 15:
        raise ValueError("k out of range")
    e = _emb(M)
    hi = n if src_hi is None else src_hi
    return int(lib().orc_train(offsets, indices, n, C.byref(e), epochs, lr, k, seed, level, tag,
                               src_lo, hi))


def train_loss(offsets, indices, M, epochs, lr, k, seed, level=0, tag=0):
    """Sequential Algorithm 3 (as train) over all sources; returns (updates,
    float64 [epochs] running loss of each epoch: the Section 2 objective
    summed over the epoch's executed updates, each taken before its update)."""
    offsets, indices = _csr(offsets, indices)
    n = len(offsets) - 1
    if M.shape[0] != n:
        raise ValueError("embedding rows != |V|")
    if not 0 <= k <= 15:
        raise ValueError("k out of range")
    e = _emb(M)
    out = np.zeros(max(epochs, 1), np.float64)
    u = lib().orc_train_loss(offsets, indices, n, C.byref(e), epochs, lr, k, seed, level, tag, out)
    return int(u), out[:epochs]


def train_hogwild(offsets, indices, M, epochs, lr, k, seed, threads, level=0, tag=0) -> int:
    """Algorithm 3 on FP64 rows with each epoch's sources spread over
    `threads` OpenMP threads without locks (timing of the oracle on all host
    cores; the rows depend on thread timing).  Returns the executed updates."""
    offsets, indices = _csr(offsets, indices)
    n = len(offsets) - 1
    if M.shape[0] != n or M.dtype != np.float64:
        raise ValueError("FP64 embedding with one row per vertex")
    if not 0 <= k <= 15 or threads < 1:
        raise ValueError("k or threads out of range")
    e = _emb(M)
    return int(lib().orc_train_hogwild(offsets, indices, n, C.byref(e), epochs, lr, k, seed, level, tag, threads))


# --------------------------------------------------------------------------- coarsening
def coarsen_map(offsets, indices):
    """(map int32[n], n_next, order int32[n]) of one MultiEdgeCollapse level."""
    offsets, indices = _csr(offsets, indices)
    n = len(offsets) - 1
    mp = np.zeros(max(n, 1), np.int32)
    order = np.zeros(max(n, 1), np.int32)
    nn = lib().orc_coarsen_map(offsets, indices, n, mp, order.ctypes.data)
    return mp[:n], int(nn), order[:n]


def coarse_graph(offsets, indices, mp, n_next):
    offsets, indices = _csr(offsets, indices)
    n = len(offsets) - 1
    off = np.zeros(n_next + 1, np.int64)
    idx = np.zeros(max(int(offsets[-1]), 1), np.int32)
    nnz = lib().orc_coarse_graph(offsets, indices, n, np.ascontiguousarray(mp, np.int32),
                                 n_next, off, idx)
    if nnz < 0:
        raise MemoryError("oracle coarse graph")
    return off, idx[:nnz].copy()


def coarsen_levels(offsets, indices, threshold=100, ratio=0.8, max_levels=128):
    """Algorithm 4's level loop: returns (graphs [(offsets, indices)], maps).

    A level is appended before the exit test (do-while); coarsening continues
    while |V_{i+1}| >= threshold and |V_{i+1}| <= ratio * |V_i|.  An empty
    input graph has nothing to coarsen and yields only G_0."""
    offsets, indices = _csr(offsets, indices)
    graphs, maps = [(offsets, indices)], []
    if len(offsets) - 1 == 0:
        return graphs, maps
    while len(graphs) < max_levels:
        off, idx = graphs[-1]
        n = len(off) - 1
        mp, nn, _ = coarsen_map(off, idx)
        graphs.append(coarse_graph(off, idx, mp, nn))
        maps.append(mp)
        if not (nn >= threshold and nn <= ratio * n):
            break
    return graphs, maps


def epoch_schedule(e, p, D) -> np.ndarray:
    out = np.zeros(D, np.int32)
    if lib().orc_epoch_schedule(e, p, D, out) != 0:
        raise ValueError("bad schedule arguments")
    return out


def prolong(coarse: np.ndarray, mp: np.ndarray) -> np.ndarray:
    """ExpandEmbedding: fine row v is the coarse row of its super vertex."""
    return np.ascontiguousarray(coarse[np.asarray(mp, np.int64)])


def lr_at(lr: float, j: int, e_i: int) -> float:
    return lr * max(1.0 - j / e_i, 1e-4)


def unit_epochs(sched, graphs, unit="passes"):
    """Epochs of each level in Algorithm 3 passes for an epoch unit.

    "passes": one epoch is one pass of Algorithm 3 (every vertex a source
    once), the schedule as it is.  "edges": the unit of the paper's
    experiments, one epoch = |E| updates (the note under Table 3): level i
    has nnz_i / 2 undirected edges and a pass visits n_i sources, so its
    share e_i becomes e_i * ceil(nnz_i / (2 n_i)) passes (at least one pass
    per epoch, also for an edgeless level)."""
    if unit == "passes":
        return np.asarray(sched, np.int32)
    if unit != "edges":
        raise ValueError(f"unknown epoch unit {unit!r}")
    out = []
    for e_i, (off, _) in zip(sched, graphs):
        n_i, nnz_i = len(off) - 1, int(off[-1])
        mult = max(1, -(-nnz_i // (2 * n_i))) if n_i > 0 else 1
        out.append(int(e_i) * mult)
    return np.asarray(out, np.int32)


def gosh_embed(offsets, indices, init_fn, d, e, p, lr, k, seed, threshold=100,
               ratio=0.8, bf16=False, tag=0, levels=None, epoch_unit="passes", losses=None,
               prolong_fn=None, keep=None):
    """Algorithm 2: coarsen, initialise the coarsest rows with
    ``init_fn(n_coarsest, d)`` (float32), train levels D-1 .. 0 with their
    epoch share (in the given epoch unit, see unit_epochs), expanding each
    trained level to the next finer one.  Returns (M_0, info) with M_0
    float64 or BF16 bits.  With a dict `losses`, losses[i] receives level
    i's per-epoch running loss (train_loss).  prolong_fn(M, i, graphs,
    maps) expands trained level i+1 onto level i in place of the copy, in
    the rows' storage (FP64, or BF16 bits); a dict `keep` receives every
    level's trained rows."""
    if levels is None:
        graphs, maps = coarsen_levels(offsets, indices, threshold, ratio)
    else:
        graphs, maps = levels
    D = len(graphs)
    sched = unit_epochs(epoch_schedule(e, p, D), graphs, epoch_unit)
    init = np.asarray(init_fn(len(graphs[-1][0]) - 1, d), dtype=np.float32)
    M = f32_to_bf16_rne(init).reshape(init.shape) if bf16 else init.astype(np.float64)
    updates = []
    for i in range(D - 1, -1, -1):
        off, idx = graphs[i]
        if losses is not None:
            u, losses[i] = train_loss(off, idx, M, int(sched[i]), lr, k, seed, level=i, tag=tag)
            updates.append(u)
        else:
            updates.append(train(off, idx, M, int(sched[i]), lr, k, seed, level=i, tag=tag))
        if keep is not None:
            keep[i] = M.copy()
        if i > 0:
            if prolong_fn is not None:
                M = np.ascontiguousarray(prolong_fn(M, i - 1, graphs, maps), dtype=M.dtype)
            else:
                M = prolong(M, maps[i - 1])
    return M, {"levels": D, "schedule": sched, "sizes": [len(g[0]) - 1 for g in graphs],
               "updates": updates[::-1]}


# --------------------------------------------------------------------------- partitioned embedding
def part_starts(n: int, K: int) -> np.ndarray:
    out = np.zeros(K + 1, np.int64)
    lib().orc_part_starts(n, K, out)
    return out


def inside_out(K: int) -> list:
    buf = np.zeros(K * (K + 1), np.int32)
    m = lib().orc_inside_out(K, buf)
    return [(int(buf[2 * j]), int(buf[2 * j + 1])) for j in range(m)]


def pool(offsets, indices, K, i, j, B, seed, level=0, tag=0, round=0):
    """Entries (src, pos, b) of pool S_{i,j} of a round, in pool order."""
    offsets, indices = _csr(offsets, indices)
    n = len(offsets) - 1
    L = lib()
    cnt = L.orc_pool(offsets, indices, n, K, i, j, B, seed, level, tag, round, None, None, None)
    src = np.zeros(max(cnt, 1), np.int32)
    pos = np.zeros(max(cnt, 1), np.int32)
    bb = np.zeros(max(cnt, 1), np.int32)
    L.orc_pool(offsets, indices, n, K, i, j, B, seed, level, tag, round, src.ctypes.data, pos.ctypes.data,
               bb.ctypes.data)
    return src[:cnt], pos[:cnt], bb[:cnt]


def train_partitioned(offsets, indices, M, K, B, epochs, lr, k, seed, level=0, tag=0):
    """Sequential Section-5 training in place on M; returns (updates, positives)."""
    offsets, indices = _csr(offsets, indices)
    n = len(offsets) - 1
    if M.shape[0] != n:
        raise ValueError("embedding rows != |V|")
    if not 0 <= k <= 15:
        raise ValueError("k out of range")
    e = _emb(M)
    pos = C.c_int64()
    upd = lib().orc_train_partitioned(offsets, indices, n, C.byref(e), K, B, epochs, lr, k, seed, level, tag,
                                      C.byref(pos))
    return int(upd), int(pos.value)


# --------------------------------------------------------------------------- random-walk sampling
def walk(offsets, indices, v, length, seed, level=0, tag=0, epoch=0) -> np.ndarray:
    offsets, indices = _csr(offsets, indices)
    out = np.zeros(length + 1, np.int32)
    m = lib().orc_walk(offsets, indices, seed, level, tag, epoch, v, length, out)
    return out[:m]


def walk_offsets(length, window):
    """The pair offsets (a, b) of a walk, in pair-number order."""
    L = lib()
    P = L.orc_walk_offsets(length, window, None, None)
    a = np.zeros(max(P, 1), np.int32)
    b = np.zeros(max(P, 1), np.int32)
    L.orc_walk_offsets(length, window, a.ctypes.data, b.ctypes.data)
    return a[:P], b[:P]


def walk_keys(m, seed, level=0, tag=0, epoch=0) -> np.ndarray:
    """Shuffle keys of pair numbers 0..m-1."""
    out = np.zeros(max(m, 1), np.uint32)
    lib().orc_walk_keys(m, seed, level, tag, epoch, out)
    return out[:m]


def walk_order(n, P, seed, level=0, tag=0, epoch=0) -> np.ndarray:
    out = np.zeros(max(n * P, 1), np.int64)
    lib().orc_walk_order(n, P, seed, level, tag, epoch, out)
    return out[:n * P]


def walk_pairs(offsets, indices, length, window, seed, level=0, tag=0, epoch=0):
    """The (source, positive) pairs of one epoch in visiting order (-1 for void)."""
    offsets, indices = _csr(offsets, indices)
    n = len(offsets) - 1
    m = n * len(walk_offsets(length, window)[0])
    src = np.zeros(max(m, 1), np.int32)
    pos = np.zeros(max(m, 1), np.int32)
    lib().orc_walk_pairs(offsets, indices, n, seed, level, tag, epoch, length, window, src, pos)
    return src[:m], pos[:m]


def train_walks(offsets, indices, M, epochs, lr, k, length, window, seed, level=0, tag=0) -> int:
    offsets, indices = _csr(offsets, indices)
    n = len(offsets) - 1
    if M.shape[0] != n:
        raise ValueError("embedding rows != |V|")
    if not 0 <= k <= 15:
        raise ValueError("k out of range")
    e = _emb(M)
    return int(lib().orc_train_walks(offsets, indices, n, C.byref(e), epochs, lr, k, length, window, seed, level,
                                     tag))
