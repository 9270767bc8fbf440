"""Seeded synthetic inputs shared by the CPU oracle and the HIP path.

The paper's datasets (SNAP/KONECT graphs, Table 2) are not available, so every
graph used here is a seeded R-MAT graph with the shape of those workloads.
This package holds input preparation and the downstream link-prediction
evaluator only; none of the embedding method's arithmetic (coarsening,
sampling, updates, prolongation) lives here.

  rmat      R-MAT edge draws -> simple undirected CSR (both directions stored)
  linkpred  80/20 edge split of Section 6.1, negative pairs, LR + AUCROC evaluator
  rows      seeded initial embedding rows, U[-0.5/d, 0.5/d]
"""
from .rmat import rmat_csr, rmat_pairs, csr_from_pairs, check_csr
from .linkpred import LinkSplit, split_edges, evaluate_auc
from .rows import init_rows

__all__ = [
    "rmat_csr", "rmat_pairs", "csr_from_pairs", "check_csr",
    "LinkSplit", "split_edges", "evaluate_auc", "init_rows",
]
