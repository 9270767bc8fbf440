"""ctypes binding of libgosh.so (the C ABI in include/gosh.h).

Argument marshalling only: torch device tensors are passed by data_ptr(),
the current torch stream is handed to the context, and every status code
other than GOSH_OK raises GoshError with the library's message.  There is no
fallback: if libgosh.so is missing or cannot be loaded, every call raises.
"""
from __future__ import annotations

import ctypes as C
import os

import torch

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libgosh.so")

GOSH_F32, GOSH_BF16 = 0, 1
STATUS = {0: "OK", 1: "E_INVALID_ARG", 2: "E_BAD_GRAPH", 3: "E_OOM", 4: "E_CAP_EXCEEDED",
          5: "E_UNSUPPORTED", 6: "E_DEVICE"}


class GoshError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{STATUS.get(code, code)}: {msg}")
        self.code = code
        self.status = STATUS.get(code, str(code))


class gosh_walk_timing(C.Structure):
    _fields_ = [("sample_ms", C.c_double), ("train_ms", C.c_double), ("epochs", C.c_int32)]


class gosh_csr(C.Structure):
    _fields_ = [("n", C.c_int64), ("nnz", C.c_int64), ("offsets", C.c_void_p),
                ("offsets_is_i64", C.c_int32), ("indices", C.c_void_p)]


class gosh_job(C.Structure):
    _fields_ = [("g", gosh_csr), ("emb", C.c_void_p), ("epochs", C.c_int32), ("lr", C.c_float),
                ("level", C.c_int32), ("tag", C.c_uint32)]


GOSH_BATCH_AUTO, GOSH_BATCH_PERSISTENT, GOSH_BATCH_EPOCH_GRAPH = 0, 1, 2
GOSH_COARSEN_EXACT, GOSH_COARSEN_LOCK_SKIP = 0, 1


class gosh_part_params(C.Structure):
    _fields_ = [("parts", C.c_int32), ("sub_bins", C.c_int32), ("pool_bins", C.c_int32), ("B", C.c_int32),
                ("threads", C.c_int32)]


class gosh_part_stats(C.Structure):
    _fields_ = [("parts", C.c_int32), ("rounds", C.c_int32), ("positives", C.c_int64),
                ("pool_entries", C.c_int64), ("part_loads", C.c_int64), ("part_stores", C.c_int64),
                ("kernels", C.c_int64), ("h2d_bytes", C.c_double), ("d2h_bytes", C.c_double),
                ("seconds", C.c_double), ("sample_seconds", C.c_double), ("kernel_seconds", C.c_double),
                ("device_bytes", C.c_uint64)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class gosh_mlp_batch(C.Structure):
    _fields_ = [("rows", C.c_int64), ("coarse", C.c_void_p), ("deg", C.c_void_p), ("clsz", C.c_void_p),
                ("target", C.c_void_p)]


class gosh_mlp_source(C.Structure):
    _fields_ = [("lv", C.c_void_p), ("level", C.c_int32), ("coarse", C.c_void_p), ("fine", C.c_void_p)]


_lib = None

# (name, restype, argtypes) of every exported entry point
_P = C.c_void_p
_SIGNATURES = [
    ("gosh_ctx_create", C.c_int, [C.c_int, C.c_uint64, _P, C.c_uint64, C.POINTER(_P)]),
    ("gosh_ctx_destroy", C.c_int, [_P]),
    ("gosh_set_stream", C.c_int, [_P, _P]),
    ("gosh_sync", C.c_int, [_P]),
    ("gosh_last_error", C.c_char_p, [_P]),
    ("gosh_mem_in_use", C.c_int, [_P, C.POINTER(C.c_uint64)]),
    ("gosh_set_deterministic", C.c_int, [_P, C.c_int]),
    ("gosh_set_epoch_overlap", C.c_int, [_P, C.c_int32, C.c_int64]),
    ("gosh_set_plain_negatives", C.c_int, [_P, C.c_int64]),
    ("gosh_set_plain_light_rows", C.c_int, [_P, C.c_int64]),
    ("gosh_set_grouped_positives", C.c_int, [_P, C.c_int64, C.c_int64, C.c_double]),
    ("gosh_set_loss_record", C.c_int, [_P, _P, C.c_int64]),
    ("gosh_set_resident_epochs", C.c_int, [_P, C.c_int64]),
    ("gosh_set_lds_levels", C.c_int, [_P, C.c_int64]),
    ("gosh_set_draw_record", C.c_int, [_P, _P, C.c_int64]),
    ("gosh_trim", C.c_int, [_P]),
    ("gosh_set_coarsen_mode", C.c_int, [_P, C.c_int, C.c_int64]),
    ("gosh_validate_csr", C.c_int, [_P, C.POINTER(gosh_csr), C.c_int]),
    ("gosh_coarsen", C.c_int, [_P, C.POINTER(gosh_csr), C.c_int64, C.c_double, C.POINTER(_P)]),
    ("gosh_levels_single", C.c_int, [_P, C.POINTER(gosh_csr), C.POINTER(_P)]),
    ("gosh_levels_destroy", C.c_int, [_P]),
    ("gosh_levels_count", C.c_int, [_P, C.POINTER(C.c_int32)]),
    ("gosh_level_shape", C.c_int, [_P, C.c_int32, C.POINTER(C.c_int64), C.POINTER(C.c_int64)]),
    ("gosh_level_csr", C.c_int, [_P, C.c_int32, C.POINTER(gosh_csr)]),
    ("gosh_level_map", C.c_int, [_P, C.c_int32, C.POINTER(_P), C.POINTER(_P)]),
    ("gosh_level_copy_out", C.c_int, [_P, _P, C.c_int32, _P, _P, _P, _P]),
    ("gosh_epoch_schedule", C.c_int, [C.c_int32, C.c_double, C.c_int32, C.POINTER(C.c_int32)]),
    ("gosh_train", C.c_int, [_P, _P, C.c_int32, _P, C.c_int, C.c_int32, C.c_int32, C.c_float,
                             C.c_int32, C.c_uint32, _P]),
    ("gosh_train_walks", C.c_int, [_P, _P, C.c_int32, _P, C.c_int, C.c_int32, C.c_int32, C.c_float,
                                   C.c_int32, C.c_int32, C.c_int32, C.c_uint32, _P, C.POINTER(gosh_walk_timing)]),
    ("gosh_walk_pairs", C.c_int, [_P, _P, C.c_int32, C.c_int32, C.c_int32, C.c_int32, C.c_uint32, _P, _P,
                                  C.c_int64, C.POINTER(C.c_int64)]),
    ("gosh_train_batched", C.c_int, [_P, C.POINTER(gosh_job), C.c_int32, C.c_int, C.c_int32, C.c_int32,
                                     C.c_int, _P, C.POINTER(C.c_int32)]),
    ("gosh_train_batched_noalloc", C.c_int, [_P, C.POINTER(gosh_job), C.c_int32, C.c_int, C.c_int32, C.c_int32,
                                             _P]),
    ("gosh_prolong", C.c_int, [_P, _P, C.c_int32, _P, _P, C.c_int, C.c_int32, _P]),
    ("gosh_train_partitioned", C.c_int, [_P, C.POINTER(gosh_csr), _P, C.c_int, C.c_int32, C.c_int32, C.c_float,
                                         C.c_int32, C.c_int32, C.c_uint32, C.POINTER(gosh_part_params), _P,
                                         C.POINTER(gosh_part_stats)]),
    ("gosh_partition_plan", C.c_int, [C.c_int64, C.c_int32, C.c_int, C.c_uint64, C.POINTER(gosh_part_params),
                                      C.POINTER(C.c_int32), C.POINTER(C.c_uint64)]),
    ("gosh_inside_out", C.c_int, [C.c_int32, _P]),
    ("gosh_partition_pool", C.c_int, [C.POINTER(gosh_csr), C.c_int32, C.c_int32, C.c_int32, C.c_int32, C.c_uint64,
                                      C.c_int32, C.c_uint32, C.c_int32, C.c_int32, C.POINTER(C.c_int64), _P, _P, _P,
                                      C.c_int64]),
    ("gosh_mlp_create", C.c_int, [_P, C.c_int32, C.c_int32, C.POINTER(_P)]),
    ("gosh_mlp_destroy", C.c_int, [_P]),
    ("gosh_mlp_num_params", C.c_int, [_P, C.POINTER(C.c_int64)]),
    ("gosh_mlp_set_weights", C.c_int, [_P, _P, _P]),
    ("gosh_mlp_get_weights", C.c_int, [_P, _P, _P]),
    ("gosh_mlp_grad", C.c_int, [_P, _P, C.c_int, C.POINTER(gosh_mlp_batch), _P, _P]),
    ("gosh_mlp_adam_step", C.c_int, [_P, _P, _P, C.c_float]),
    ("gosh_mlp_train", C.c_int, [_P, _P, C.c_int, C.POINTER(gosh_mlp_source), C.c_int32, C.c_int32, C.c_int32,
                                 C.c_float, C.c_uint32, _P]),
    ("gosh_draw_samples", C.c_int, [_P, _P, C.c_int32, C.c_int32, C.c_int32, C.c_uint32, _P]),
    ("gosh_update_batch", C.c_int, [_P, _P, C.c_int, C.c_int32, C.c_int64, C.c_int32, _P, _P,
                                    C.c_int32, C.c_float, C.c_int32, C.c_uint32, C.c_int32]),
]
EXPORTS = [s[0] for s in _SIGNATURES]


def lib():
    """Loads libgosh.so; raises if it is not built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_2110_10049_amd/build.py")
        L = C.CDLL(LIB_PATH)
        for name, res, args in _SIGNATURES:
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _dtype_code(t: torch.Tensor) -> int:
    if t.dtype == torch.float32:
        return GOSH_F32
    if t.dtype == torch.bfloat16:
        return GOSH_BF16
    raise TypeError("embeddings are float32 or bfloat16")


def _dev(t: torch.Tensor, dtype=None, name="tensor"):
    if not t.is_cuda:
        raise ValueError(f"{name} must be a device tensor")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if dtype is not None and t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}")
    return C.c_void_p(t.data_ptr())


class Context:
    """A gosh_ctx bound to one device and (by default) torch's current stream."""

    def __init__(self, device: int = 0, seed: int = 0, mem_cap: int = 0, stream=None):
        self._L = lib()
        self.device = device
        h = C.c_void_p()
        if stream is None:
            stream = torch.cuda.current_stream(device)
        self._check_raw(self._L.gosh_ctx_create(device, seed, C.c_void_p(stream.cuda_stream), mem_cap,
                                                C.byref(h)), None)
        self.h = h
        self.stream = stream

    def _check_raw(self, st, h):
        if st != 0:
            msg = self._L.gosh_last_error(h).decode() if h is not None else "context creation failed"
            raise GoshError(st, msg)

    def check(self, st):
        if st != 0:
            raise GoshError(st, self._L.gosh_last_error(self.h).decode())

    def use_current_stream(self):
        s = torch.cuda.current_stream(self.device)
        self.check(self._L.gosh_set_stream(self.h, C.c_void_p(s.cuda_stream)))
        self.stream = s

    def sync(self):
        self.check(self._L.gosh_sync(self.h))

    def mem_in_use(self) -> int:
        v = C.c_uint64()
        self.check(self._L.gosh_mem_in_use(self.h, C.byref(v)))
        return v.value

    def set_deterministic(self, on: bool):
        self.check(self._L.gosh_set_deterministic(self.h, 1 if on else 0))

    def set_epoch_overlap(self, epochs_in_flight: int, min_vertices: int = 0):
        """Concurrent epochs on levels of at least min_vertices vertices (1 = off)."""
        self.check(self._L.gosh_set_epoch_overlap(self.h, epochs_in_flight, min_vertices))

    def trim(self):
        """Release the device blocks cached by the context."""
        self.check(self._L.gosh_trim(self.h))

    def set_coarsen_mode(self, mode: int, batch: int = 0):
        """GOSH_COARSEN_EXACT (default) or GOSH_COARSEN_LOCK_SKIP with `batch` vertices per launch."""
        self.check(self._L.gosh_set_coarsen_mode(self.h, mode, batch))

    def set_plain_negatives(self, min_vertices: int):
        """Plain stores for negative rows on levels of at least min_vertices vertices (0 = off)."""
        self.check(self._L.gosh_set_plain_negatives(self.h, min_vertices))

    def set_grouped_positives(self, min_vertices: int, max_vertices: int, hot_factor: float = 64.0):
        """Group the visits of hot positives on levels with min <= n <= max (max 0 = off)."""
        self.check(self._L.gosh_set_grouped_positives(self.h, min_vertices, max_vertices, hot_factor))

    def set_plain_light_rows(self, min_vertices: int):
        """Plain stores for rows of at most average degree on levels of at least min_vertices vertices (0 = off)."""
        self.check(self._L.gosh_set_plain_light_rows(self.h, min_vertices))

    def set_resident_epochs(self, max_vertices: int):
        """All epochs of a level of at most max_vertices vertices in one launch (0 = off)."""
        self.check(self._L.gosh_set_resident_epochs(self.h, max_vertices))

    def set_lds_levels(self, max_vertices: int):
        """Levels of at most max_vertices vertices whose rows fit in LDS train in one workgroup (0 = off)."""
        self.check(self._L.gosh_set_lds_levels(self.h, max_vertices))

    def set_loss_record(self, loss: "torch.Tensor | None"):
        """Running loss per epoch of later gosh_train calls, added to a float64
        device tensor (the caller zeroes it); None turns recording off."""
        if loss is None:
            self.check(self._L.gosh_set_loss_record(self.h, None, 0))
        else:
            self.check(self._L.gosh_set_loss_record(self.h, _dev(loss, torch.float64, "loss"), loss.numel()))
        self._loss_buf = loss   # keep alive while recording

    def set_draw_record(self, samples: "torch.Tensor | None"):
        """Samples drawn inside gosh_train, written to an int32 device tensor
        [n, 1+k] (test hook); None turns it off."""
        if samples is None:
            self.check(self._L.gosh_set_draw_record(self.h, None, 0))
        else:
            self.check(self._L.gosh_set_draw_record(self.h, _dev(samples, torch.int32, "samples"),
                                                    samples.numel()))
        self._draw_buf = samples

    def close(self):
        if getattr(self, "h", None) is not None and self.h.value:
            self._L.gosh_ctx_destroy(self.h)
            self.h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class CSR:
    """Keeps device tensors alive behind a gosh_csr view."""

    def __init__(self, offsets: torch.Tensor, indices: torch.Tensor):
        if offsets.dtype not in (torch.int32, torch.int64):
            raise TypeError("offsets must be int32 or int64")
        _dev(offsets, name="offsets")
        _dev(indices, torch.int32, "indices")
        self.offsets, self.indices = offsets, indices
        self.view = gosh_csr(offsets.numel() - 1, indices.numel(), offsets.data_ptr(),
                             1 if offsets.dtype == torch.int64 else 0, indices.data_ptr())

    @classmethod
    def from_numpy(cls, offsets, indices, device="cuda", off64=False):
        o = torch.as_tensor(offsets, dtype=torch.int64 if off64 else torch.int32).to(device)
        i = torch.as_tensor(indices, dtype=torch.int32).to(device)
        return cls(o.contiguous(), i.contiguous())


class Levels:
    """A gosh_levels hierarchy; keeps the level-0 CSR alive."""

    def __init__(self, ctx: Context, handle: C.c_void_p, g0: CSR):
        self.ctx, self.h, self.g0 = ctx, handle, g0

    def count(self) -> int:
        D = C.c_int32()
        self.ctx.check(lib().gosh_levels_count(self.h, C.byref(D)))
        return D.value

    def shape(self, level: int):
        n, nnz = C.c_int64(), C.c_int64()
        self.ctx.check(lib().gosh_level_shape(self.h, level, C.byref(n), C.byref(nnz)))
        return n.value, nnz.value

    def sizes(self):
        return [self.shape(i)[0] for i in range(self.count())]

    def csr(self, level: int) -> gosh_csr:
        out = gosh_csr()
        self.ctx.check(lib().gosh_level_csr(self.h, level, C.byref(out)))
        return out

    def copy_out(self, level: int, want_map=True):
        import numpy as np
        n, nnz = self.shape(level)
        off = np.zeros(n + 1, np.int64)
        idx = np.zeros(max(nnz, 1), np.int32)
        mp = np.zeros(max(n, 1), np.int32) if want_map else None
        self.ctx.check(lib().gosh_level_copy_out(
            self.ctx.h, self.h, level, off.ctypes.data, idx.ctypes.data,
            mp.ctypes.data if mp is not None else None, None))
        return off, idx[:nnz], (mp[:n] if mp is not None else None)

    def cluster_sizes(self, level: int):
        """Sizes of the clusters of `level` that form the vertices of level+1."""
        import numpy as np
        nn, _ = self.shape(level + 1)
        cs = np.zeros(max(nn, 1), np.int32)
        self.ctx.check(lib().gosh_level_copy_out(self.ctx.h, self.h, level, None, None, None, cs.ctypes.data))
        return cs[:nn]

    def close(self):
        if getattr(self, "h", None) is not None and self.h.value:
            lib().gosh_levels_destroy(self.h)
            self.h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ------------------------------------------------------------------ entry points
def gosh_validate_csr(ctx: Context, g: CSR, check_symmetry: bool = True):
    ctx.check(lib().gosh_validate_csr(ctx.h, C.byref(g.view), 1 if check_symmetry else 0))


def gosh_coarsen(ctx: Context, g0: CSR, threshold: int = 100, max_ratio: float = 0.8) -> Levels:
    h = C.c_void_p()
    ctx.check(lib().gosh_coarsen(ctx.h, C.byref(g0.view), threshold, max_ratio, C.byref(h)))
    return Levels(ctx, h, g0)


def gosh_levels_single(ctx: Context, g0: CSR) -> Levels:
    h = C.c_void_p()
    ctx.check(lib().gosh_levels_single(ctx.h, C.byref(g0.view), C.byref(h)))
    return Levels(ctx, h, g0)


def gosh_epoch_schedule(e: int, p: float, D: int):
    out = (C.c_int32 * D)()
    st = lib().gosh_epoch_schedule(e, p, D, out)
    if st != 0:
        raise GoshError(st, "bad schedule arguments")
    return list(out)


def gosh_train(ctx: Context, lv: Levels, level: int, emb: torch.Tensor, epochs: int, lr: float, k: int,
               tag: int = 0, updates: torch.Tensor | None = None):
    n, _ = lv.shape(level)
    if emb.dim() != 2 or emb.shape[0] != n:
        raise ValueError(f"embedding must be [{n}, d]")
    e = _dev(emb, name="emb")
    u = _dev(updates, torch.int64, "updates") if updates is not None else None
    ctx.check(lib().gosh_train(ctx.h, lv.h, level, e, _dtype_code(emb), emb.shape[1], epochs, lr, k, tag, u))


def gosh_train_walks(ctx: Context, lv: Levels, level: int, emb: torch.Tensor, epochs: int, lr: float, k: int,
                     walk_len: int, window: int, tag: int = 0, updates: torch.Tensor | None = None,
                     timing: bool = False):
    """Random-walk positive sampling (Section 3.2) on one level; see gosh.h.
    With timing, waits and returns {"sample_ms", "train_ms", "epochs"}."""
    n, _ = lv.shape(level)
    if emb.dim() != 2 or emb.shape[0] != n:
        raise ValueError(f"embedding must be [{n}, d]")
    e = _dev(emb, name="emb")
    u = _dev(updates, torch.int64, "updates") if updates is not None else None
    t = gosh_walk_timing() if timing else None
    ctx.check(lib().gosh_train_walks(ctx.h, lv.h, level, e, _dtype_code(emb), emb.shape[1], epochs, lr, k,
                                     walk_len, window, tag, u, C.byref(t) if timing else None))
    if timing:
        return {"sample_ms": t.sample_ms, "train_ms": t.train_ms, "epochs": t.epochs}
    return None


def gosh_walk_pairs(ctx: Context, lv: Levels, level: int, epoch: int, walk_len: int, window: int,
                    tag: int = 0) -> tuple[torch.Tensor, torch.Tensor]:
    """The (source, positive) pairs of one walk epoch in visiting order (-1 for void)."""
    cnt = C.c_int64()
    ctx.check(lib().gosh_walk_pairs(ctx.h, lv.h, level, epoch, walk_len, window, tag, None, None, 0,
                                    C.byref(cnt)))
    m = cnt.value
    dev = f"cuda:{ctx.device}"
    src = torch.empty(max(m, 1), dtype=torch.int32, device=dev)
    pos = torch.empty(max(m, 1), dtype=torch.int32, device=dev)
    ctx.check(lib().gosh_walk_pairs(ctx.h, lv.h, level, epoch, walk_len, window, tag, _dev(src), _dev(pos), m,
                                    C.byref(cnt)))
    return src[:m], pos[:m]


def gosh_prolong(ctx: Context, lv: Levels, fine_level: int, coarse: torch.Tensor, fine: torch.Tensor,
                 mlp: "Mlp | None" = None):
    nf, _ = lv.shape(fine_level)
    nc, _ = lv.shape(fine_level + 1)
    if coarse.shape != (nc, fine.shape[1]) or fine.shape[0] != nf or coarse.dtype != fine.dtype:
        raise ValueError("prolong shapes/dtypes do not match the levels")
    ctx.check(lib().gosh_prolong(ctx.h, lv.h, fine_level, _dev(coarse, name="coarse"), _dev(fine, name="fine"),
                                 _dtype_code(fine), fine.shape[1], mlp.h if mlp is not None else None))


class Mlp:
    """A gosh_mlp prolongation network (library-owned weights)."""

    def __init__(self, ctx: Context, d: int, hidden: int):
        self.ctx, self.d, self.hidden = ctx, d, hidden
        h = C.c_void_p()
        ctx.check(lib().gosh_mlp_create(ctx.h, d, hidden, C.byref(h)))
        self.h = h
        n = C.c_int64()
        ctx.check(lib().gosh_mlp_num_params(self.h, C.byref(n)))
        self.nparams = n.value

    def split(self, flat):
        """Views (W1 [H, d+2], b1 [H], W2 [d, H], b2 [d]) of a flat parameter vector."""
        d, H = self.d, self.hidden
        a = H * (d + 2)
        return (flat[:a].reshape(H, d + 2), flat[a:a + H], flat[a + H:a + H + d * H].reshape(d, H),
                flat[a + H + d * H:])

    def set_weights(self, flat):
        import numpy as np
        w = np.ascontiguousarray(flat, dtype=np.float32).ravel()
        if w.size != self.nparams:
            raise ValueError(f"expected {self.nparams} parameters")
        self.ctx.check(lib().gosh_mlp_set_weights(self.ctx.h, self.h, w.ctypes.data))

    def get_weights(self):
        import numpy as np
        w = np.zeros(self.nparams, np.float32)
        self.ctx.check(lib().gosh_mlp_get_weights(self.ctx.h, self.h, w.ctypes.data))
        return w

    def grad(self, coarse: torch.Tensor, deg: torch.Tensor, clsz: torch.Tensor, target: torch.Tensor):
        """(gradient [P] float32 device tensor, loss float) of the MSE on an explicit batch."""
        B = coarse.shape[0]
        if coarse.shape != (B, self.d) or target.shape != coarse.shape or target.dtype != coarse.dtype:
            raise ValueError("coarse and target must be [rows, d] of one dtype")
        if deg.numel() != B or clsz.numel() != B:
            raise ValueError("deg and clsz need one entry per row")
        b = gosh_mlp_batch(B, _dev(coarse, name="coarse").value, _dev(deg, torch.int32, "deg").value,
                           _dev(clsz, torch.int32, "clsz").value, _dev(target, name="target").value)
        g = torch.empty(self.nparams, dtype=torch.float32, device=coarse.device)
        loss = torch.empty(1, dtype=torch.float32, device=coarse.device)
        self.ctx.check(lib().gosh_mlp_grad(self.ctx.h, self.h, _dtype_code(coarse), C.byref(b), _dev(g),
                                           _dev(loss)))
        return g, float(loss.item())

    def adam_step(self, grads: torch.Tensor, lr: float):
        if grads.numel() != self.nparams:
            raise ValueError(f"expected {self.nparams} gradients")
        self.ctx.check(lib().gosh_mlp_adam_step(self.ctx.h, self.h, _dev(grads, torch.float32, "grads"), lr))

    def train(self, sources, steps: int, batch: int, lr: float, tag: int = 0, losses: bool = True):
        """sources: list of (Levels, level, coarse rows, fine rows).  Returns the
        per-step minibatch losses (a float32 device tensor) or None."""
        arr = (gosh_mlp_source * len(sources))()
        dtype = None
        for i, (lv, level, coarse, fine) in enumerate(sources):
            dtype = coarse.dtype if dtype is None else dtype
            if coarse.dtype != dtype or fine.dtype != dtype:
                raise ValueError("all sources need one dtype")
            nf, _ = lv.shape(level)
            nc, _ = lv.shape(level + 1)
            if coarse.shape != (nc, self.d) or fine.shape != (nf, self.d):
                raise ValueError("source shapes do not match the levels")
            arr[i] = gosh_mlp_source(lv.h.value, level, _dev(coarse, name="coarse").value,
                                     _dev(fine, name="fine").value)
        out = None
        if losses and steps > 0:
            out = torch.empty(steps, dtype=torch.float32, device=f"cuda:{self.ctx.device}")
        code = _dtype_code(sources[0][2]) if sources else GOSH_F32
        self.ctx.check(lib().gosh_mlp_train(self.ctx.h, self.h, code, arr, len(sources), steps, batch, lr, tag,
                                            _dev(out) if out is not None else None))
        return out

    def close(self):
        if getattr(self, "h", None) is not None and self.h.value:
            lib().gosh_mlp_destroy(self.h)
            self.h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def gosh_draw_samples(ctx: Context, lv: Levels, level: int, epoch: int, k: int, tag: int = 0) -> torch.Tensor:
    n, _ = lv.shape(level)
    out = torch.empty((n, 1 + k), dtype=torch.int32, device=f"cuda:{ctx.device}")
    ctx.check(lib().gosh_draw_samples(ctx.h, lv.h, level, epoch, k, tag, _dev(out)))
    return out


def gosh_update_batch(ctx: Context, emb: torch.Tensor, src: torch.Tensor, samples: torch.Tensor, lr: float,
                      level: int = 0, tag: int = 0, epoch: int = 0):
    if samples.dim() != 2 or samples.shape[0] != src.numel():
        raise ValueError("samples must be [nsrc, 1+k]")
    k = samples.shape[1] - 1
    ctx.check(lib().gosh_update_batch(ctx.h, _dev(emb, name="emb"), _dtype_code(emb), emb.shape[1], emb.shape[0],
                                      src.numel(), _dev(src, torch.int32, "src"),
                                      _dev(samples, torch.int32, "samples"), k, lr, level, tag, epoch))


def gosh_train_batched(ctx: Context, jobs, k: int, mode: int = GOSH_BATCH_AUTO,
                       updates: torch.Tensor | None = None):
    """jobs: list of (CSR or gosh_csr view, emb tensor, epochs, lr, level, tag).
    Returns the execution used: (mode, blocks per CU, chunk length)."""
    if not jobs:
        return (0, 0, 0)
    arr, code, d = _job_array(jobs)
    chosen = (C.c_int32 * 3)()
    u = _dev(updates, torch.int64, "updates") if updates is not None else None
    ctx.check(lib().gosh_train_batched(ctx.h, arr, len(jobs), code, d, k, mode, u, chosen))
    return tuple(chosen)


def _job_array(jobs):
    """(gosh_job array, dtype code, d) of a list of (CSR or gosh_csr view, emb,
    epochs, lr, level, tag)."""
    arr = (gosh_job * max(len(jobs), 1))()
    if not jobs:
        return arr, GOSH_F32, 8
    dtype = jobs[0][1].dtype
    d = jobs[0][1].shape[1]
    for i, (g, emb, epochs, lr, level, tag) in enumerate(jobs):
        view = g.view if isinstance(g, CSR) else g
        if emb.dtype != dtype or emb.dim() != 2 or emb.shape[1] != d or emb.shape[0] != view.n:
            raise ValueError("every job needs a [n, d] embedding of the same dtype and d")
        arr[i] = gosh_job(view, _dev(emb, name="emb").value, epochs, lr, level, tag)
    return arr, _dtype_code(jobs[0][1]), d


def gosh_train_batched_noalloc(ctx: Context, jobs, k: int, updates: torch.Tensor | None = None):
    """gosh_train_batched without any device allocation by the library (its
    tables live in a static device array); jobs as gosh_train_batched."""
    arr, code, d = _job_array(jobs)
    u = _dev(updates, torch.int64, "updates") if updates is not None else None
    ctx.check(lib().gosh_train_batched_noalloc(ctx.h, arr, len(jobs), code, d, k, u))


# ------------------------------------------------------------------ partitioned embedding (Section 5)
def part_params(parts=0, sub_bins=3, pool_bins=2, B=5, threads=0) -> gosh_part_params:
    return gosh_part_params(parts, sub_bins, pool_bins, B, threads)


class HostCSR:
    """A gosh_csr view of HOST numpy arrays (kept alive here)."""

    def __init__(self, offsets, indices):
        import numpy as np
        self.offsets = np.ascontiguousarray(offsets)
        if self.offsets.dtype not in (np.int32, np.int64):
            self.offsets = self.offsets.astype(np.int64)
        self.indices = np.ascontiguousarray(indices, dtype=np.int32)
        self.view = gosh_csr(len(self.offsets) - 1, len(self.indices), self.offsets.ctypes.data,
                             1 if self.offsets.dtype == np.int64 else 0, self.indices.ctypes.data)


def _raise_host(st, what):
    if st != 0:
        raise GoshError(st, what)


def gosh_inside_out(K: int):
    import numpy as np
    buf = np.zeros(max(K * (K + 1), 2), np.int32)
    _raise_host(lib().gosh_inside_out(K, buf.ctypes.data), "bad part count")
    return [(int(buf[2 * q]), int(buf[2 * q + 1])) for q in range(K * (K + 1) // 2)]


def gosh_partition_plan(n: int, d: int, dtype: torch.dtype, budget: int, params: gosh_part_params):
    K = C.c_int32()
    b = C.c_uint64()
    code = GOSH_BF16 if dtype == torch.bfloat16 else GOSH_F32
    _raise_host(lib().gosh_partition_plan(n, d, code, budget, C.byref(params), C.byref(K), C.byref(b)),
                "no plan fits")
    return K.value, b.value


def gosh_partition_pool(g: HostCSR, K: int, i: int, j: int, B: int, seed: int, level: int = 0, tag: int = 0,
                        round: int = 0, threads: int = 0):
    """Pool S_{i,j} of a round as the library builds it: (src, pos, b) arrays."""
    import numpy as np
    cnt = C.c_int64()
    _raise_host(lib().gosh_partition_pool(C.byref(g.view), K, i, j, B, seed, level, tag, round, threads,
                                          C.byref(cnt), None, None, None, 0), "bad pool request")
    m = cnt.value
    src, pos, bb = (np.zeros(max(m, 1), np.int32) for _ in range(3))
    _raise_host(lib().gosh_partition_pool(C.byref(g.view), K, i, j, B, seed, level, tag, round, threads,
                                          C.byref(cnt), src.ctypes.data, pos.ctypes.data, bb.ctypes.data, m),
                "bad pool request")
    return src[:m], pos[:m], bb[:m]


def gosh_train_partitioned(ctx: Context, g: HostCSR, emb: torch.Tensor, epochs: int, lr: float, k: int,
                           level: int = 0, tag: int = 0, params: gosh_part_params | None = None,
                           updates: torch.Tensor | None = None) -> dict:
    """Section 5 on a host graph and HOST rows (a CPU tensor, pinned for
    asynchronous copies), updated in place; returns the run's statistics."""
    if emb.is_cuda or not emb.is_contiguous() or emb.dim() != 2 or emb.shape[0] != g.view.n:
        raise ValueError("emb must be a contiguous host tensor [n, d]")
    params = params or part_params()
    st = gosh_part_stats()
    u = _dev(updates, torch.int64, "updates") if updates is not None else None
    ctx.check(lib().gosh_train_partitioned(ctx.h, C.byref(g.view), C.c_void_p(emb.data_ptr()), _dtype_code(emb),
                                           emb.shape[1], epochs, lr, k, level, tag, C.byref(params), u,
                                           C.byref(st)))
    return st.as_dict()
