"""Algorithm 2 (Section 3) over the C ABI: coarsen, initialise the coarsest
rows, train every level from the coarsest to the original graph with its
share of the epochs, and expand each trained level onto the next finer one.

Orchestration only: coarsening, training and expansion run in libgosh.so.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import torch

from . import gosh as G


@dataclass
class EmbedConfig:
    d: int = 128
    epochs: int = 600          # e: total epochs over all levels (Algorithm 3 passes)
    p: float = 0.3             # smoothing ratio of the epoch distribution
    lr: float = 0.045
    k: int = 3                 # negatives per source (n_s)
    dtype: torch.dtype = torch.float32
    threshold: int = 100
    max_ratio: float = 0.8
    tag: int = 0
    # levels with at most this many vertices train through the batched
    # (single persistent launch) path instead of one launch per epoch; 0 = off
    batch_levels_upto: int = 0
    batch_mode: int = G.GOSH_BATCH_AUTO
    # positive sampling: "edge" (one uniform neighbour per source and epoch,
    # Algorithm 3) or "walk" (every pair within `window` steps of one walk of
    # `walk_len` steps per vertex and epoch, shuffled; Section 3.2)
    sampler: str = "edge"
    walk_len: int = 10
    window: int = 3
    # epoch unit of the schedule: "passes" (one epoch = one pass of
    # Algorithm 3, every vertex a source once) or "edges" (the unit of the
    # paper's experiments, one epoch = |E| updates: level i's share e_i
    # becomes e_i * ceil(nnz_i / (2 n_i)) passes)
    epoch_unit: str = "passes"


@dataclass
class EmbedResult:
    emb: torch.Tensor
    sizes: list
    schedule: list
    updates: int = 0
    levels: object = None
    timings: dict = field(default_factory=dict)
    # trained rows of every level (level -> tensor), when asked for with keep_levels
    trained: dict = field(default_factory=dict)
    # executed UpdateEmbed calls of each level (level -> int64 device tensor)
    level_updates: dict = field(default_factory=dict)
    # running loss of every epoch of each level (level -> float64 device tensor), with record_loss
    losses: dict = field(default_factory=dict)


def unit_epochs(sched, shapes, unit):
    """Epochs of each level in Algorithm 3 passes (see EmbedConfig.epoch_unit);
    shapes[i] = (n_i, nnz_i)."""
    if unit == "passes":
        return list(sched)
    if unit != "edges":
        raise ValueError(f"unknown epoch unit {unit!r}")
    return [int(e) * (max(1, -(-nnz // (2 * n))) if n > 0 else 1) for e, (n, nnz) in zip(sched, shapes)]


def embed(ctx: G.Context, g0: G.CSR, cfg: EmbedConfig, init_fn, levels: G.Levels | None = None,
          coarsen: bool = True, level_events: bool = False, mlp: G.Mlp | None = None,
          keep_levels: bool = False, record_loss: bool = False) -> EmbedResult:
    """init_fn(n, d) -> device tensor [n, d] of cfg.dtype for the coarsest level.

    With level_events, timings["train_events"][i] holds a (start, end) pair
    of events recorded on the context stream around level i's training, and
    with the walk sampler timings["walk_level0"] holds the device time of
    level 0's sampling and update launches (the call waits for level 0).
    mlp: expand with the learned prolongation instead of the copy.
    keep_levels: keep every level's trained rows in result.trained (the
    (coarse, fine) pairs the prolongation network is trained on).
    record_loss: record every epoch's running loss of the per-epoch trainer
    (result.losses).  With level_events, timings["coarsen_events"] holds
    events around the coarsening."""
    if cfg.sampler not in ("edge", "walk"):
        raise ValueError(f"unknown sampler {cfg.sampler!r}")
    ev_c = None
    if levels is None:
        if level_events:
            ev_c = (torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
            ev_c[0].record(ctx.stream)
        levels = G.gosh_coarsen(ctx, g0, cfg.threshold, cfg.max_ratio) if coarsen else G.gosh_levels_single(ctx, g0)
        if level_events:
            ev_c[1].record(ctx.stream)
    D = levels.count()
    sizes = levels.sizes()
    shapes = [levels.shape(i) for i in range(D)]
    sched = unit_epochs(G.gosh_epoch_schedule(cfg.epochs, cfg.p, D), shapes, cfg.epoch_unit)
    dev = f"cuda:{ctx.device}"
    M = init_fn(sizes[-1], cfg.d)
    if M.dtype != cfg.dtype or tuple(M.shape) != (sizes[-1], cfg.d):
        raise ValueError("init_fn returned a wrong shape or dtype")
    counters = torch.zeros(D, dtype=torch.int64, device=dev)
    events = {}
    events_walk = None
    trained = {}
    losses = {}
    for i in range(D - 1, -1, -1):
        counter = counters[i:i + 1]
        if level_events:
            ev = (torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
            ev[0].record(ctx.stream)
        if cfg.sampler == "walk":
            tm = G.gosh_train_walks(ctx, levels, i, M, sched[i], cfg.lr, cfg.k, cfg.walk_len, cfg.window, cfg.tag,
                                    counter, timing=level_events and i == 0)
            if tm is not None:
                events_walk = tm
        elif cfg.batch_levels_upto and sizes[i] <= cfg.batch_levels_upto:
            G.gosh_train_batched(ctx, [(levels.csr(i), M, sched[i], cfg.lr, i, cfg.tag)], cfg.k,
                                 cfg.batch_mode, updates=counter)
        elif record_loss:
            losses[i] = torch.zeros(max(sched[i], 1), dtype=torch.float64, device=dev)
            ctx.set_loss_record(losses[i])
            try:
                G.gosh_train(ctx, levels, i, M, sched[i], cfg.lr, cfg.k, cfg.tag, counter)
            finally:
                ctx.set_loss_record(None)
        else:
            G.gosh_train(ctx, levels, i, M, sched[i], cfg.lr, cfg.k, cfg.tag, counter)
        if level_events:
            ev[1].record(ctx.stream)
            events[i] = ev
        if keep_levels:
            trained[i] = M
        if i > 0:
            fine = torch.empty((sizes[i - 1], cfg.d), dtype=cfg.dtype, device=dev)
            G.gosh_prolong(ctx, levels, i - 1, M, fine, mlp=mlp)
            M = fine
    return EmbedResult(emb=M, sizes=sizes, schedule=sched, updates=counters.sum().reshape(1), levels=levels,
                       timings={"train_events": events, "walk_level0": events_walk, "coarsen_events": ev_c},
                       trained=trained, level_updates={i: counters[i] for i in range(D)}, losses=losses)
