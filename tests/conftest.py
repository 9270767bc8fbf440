import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (HIP device) and the built libgosh.so")
    config.addinivalue_line("markers", "slow: long-running CPU test")


@pytest.fixture(scope="session")
def orc():
    import oracle
    oracle.lib()
    return oracle


@pytest.fixture(scope="session")
def gctx():
    """A library context on cuda:0 bound to torch's current stream."""
    import torch
    from paper_2110_10049_amd import gosh as G
    if not torch.cuda.is_available():
        pytest.fail("GPU test run without a HIP device")
    ctx = G.Context(0, seed=4)
    yield ctx
    ctx.close()


_GRAPHS = {}


def train_split(scale, ef, seed=1, split_seed=2):
    """Link-prediction train graph of an R-MAT graph (cached per session)."""
    key = (scale, ef, seed, split_seed)
    if key not in _GRAPHS:
        from synth import rmat_csr, split_edges
        off, idx = rmat_csr(scale, ef, seed)
        _GRAPHS[key] = split_edges(off, idx, split_seed)
    return _GRAPHS[key]
