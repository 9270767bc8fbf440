"""Seeded initial embedding rows.

The paper only says the coarsest matrix is initialised randomly (Algorithm 2,
Section 3); the workloads here use U[-0.5/d, 0.5/d], drawn with numpy's PCG64
from a fixed seed and handed identically to the oracle and to the HIP path.
"""
from __future__ import annotations

import numpy as np


def init_rows(n: int, d: int, seed: int) -> np.ndarray:
    """float32 [n, d] uniform in [-0.5/d, 0.5/d]."""
    rng = np.random.default_rng(seed)
    h = 0.5 / d
    return rng.uniform(-h, h, size=(n, d)).astype(np.float32)
