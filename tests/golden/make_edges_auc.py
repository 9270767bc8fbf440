"""Writes tests/golden/e2e_auc_rmat12_edges.json: the FP64 oracle's link-
prediction AUC on the scale-12 R-MAT workload trained in the paper's epoch
unit (one epoch = |E| updates, the note under Table 3), for eight random
streams (tag 0..7) in FP64 and BF16 storage.  The GPU test compares the mean
over the eight streams of (GPU AUC - oracle AUC), pairing runs of equal tag,
which share every sample draw.

Only oracle/ and synth/ are called.  Workload: R-MAT scale 12, edge factor
16, graph seed 1, split seed 2, init seed 3, Philox seed 4, d = 32, k = 1,
lr 0.045 (as float32), e = 200, p = 0.3, threshold 64, evaluator seed 5.

Usage: python tests/golden/make_edges_auc.py   (about a minute on 8 cores)
"""
from __future__ import annotations

import json
import os
import sys
from concurrent.futures import ProcessPoolExecutor

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

OUT = os.path.join(HERE, "e2e_auc_rmat12_edges.json")
CONFIG = {"scale": 12, "edge_factor": 16, "d": 32, "k": 1, "lr": 0.045, "epochs": 200, "p": 0.3, "threshold": 64,
          "epoch_unit": "edges", "tags": list(range(8)),
          "seeds": {"graph": 1, "split": 2, "init": 3, "philox": 4, "eval": 5}}


def run(args):
    bf16, tag = args
    import oracle
    from synth import evaluate_auc, init_rows, rmat_csr, split_edges
    c = CONFIG
    s = c["seeds"]
    sp = split_edges(*rmat_csr(c["scale"], c["edge_factor"], s["graph"]), s["split"])
    M, info = oracle.gosh_embed(sp.offsets, sp.indices, lambda n, d: init_rows(n, d, s["init"]), c["d"], c["epochs"],
                                c["p"], float(np.float32(c["lr"])), c["k"], seed=s["philox"],
                                threshold=c["threshold"], bf16=bf16, tag=tag, epoch_unit=c["epoch_unit"])
    emb = oracle.bf16_to_f64(M) if bf16 else M
    return bf16, tag, round(evaluate_auc(emb, sp, s["eval"]), 6), [int(x) for x in info["schedule"]]


def main():
    jobs = [(b, t) for b in (False, True) for t in CONFIG["tags"]]
    with ProcessPoolExecutor(min(8, os.cpu_count() or 1)) as ex:
        res = list(ex.map(run, jobs))
    out = {"generated_by": "tests/golden/make_edges_auc.py (oracle/ and synth/ only)", "config": CONFIG,
           "schedule": res[0][3],
           "fp64": [a for b, t, a, _ in res if not b], "bf16": [a for b, t, a, _ in res if b]}
    with open(OUT, "w") as f:
        json.dump(out, f, indent=1)
        f.write("\n")
    print(json.dumps(out))


if __name__ == "__main__":
    main()
