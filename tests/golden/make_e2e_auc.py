"""Writes tests/golden/e2e_auc_rmat20.json: the FP64 oracle's end-to-end
result on the scale-20 R-MAT workload (Algorithm 2 over MultiEdgeCollapse
levels, Algorithm 3 run sequentially), which the GPU tests and bench.py
compare against.

Only the oracle (oracle/) and the shared input generators and evaluator
(synth/) are called; nothing here touches the HIP path.

Workload: R-MAT scale 20, edge factor 16 (a,b,c,d = 0.57,0.19,0.19,0.05),
graph seed 1, 80/20 link-prediction split with seed 2 (Section 6.1), rows
initialised U[-0.5/d, 0.5/d] with seed 3, Philox seed 4, d = 128, k = 3,
lr = 0.045 (as float32), e = 600 epochs in Algorithm 3 passes, p = 0.3,
threshold 100.  Rows in FP64, and again stored as BF16 with stochastic
rounding.  AUC: logistic regression on Hadamard features, classifier
trained on 200,000 sampled labelled pairs and scored on 1,000,000 sampled
test pairs (evaluator seed 5).  The running loss (the Section 2 objective
summed over each epoch's executed updates) of every level's last epoch is
stored beside it.

Usage: python tests/golden/make_e2e_auc.py   (about 10 minutes on 2 cores)
"""
from __future__ import annotations

import json
import os
import sys
import time
from concurrent.futures import ProcessPoolExecutor

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

OUT = os.path.join(HERE, "e2e_auc_rmat20.json")
CONFIG = {"scale": 20, "edge_factor": 16, "d": 128, "k": 3, "lr": 0.045, "epochs": 600, "p": 0.3,
          "threshold": 100, "epoch_unit": "passes",
          "seeds": {"graph": 1, "split": 2, "init": 3, "philox": 4, "eval": 5},
          "eval": {"max_train": 200_000, "max_test": 1_000_000}}


def run(bf16: bool) -> dict:
    import oracle
    from synth import init_rows, rmat_csr, split_edges
    from synth.linkpred import auc_on_pairs, make_eval_pairs

    c = CONFIG
    s = c["seeds"]
    sp = split_edges(*rmat_csr(c["scale"], c["edge_factor"], s["graph"]), s["split"])
    t = time.time()
    losses = {}
    M, info = oracle.gosh_embed(sp.offsets, sp.indices, lambda n, d: init_rows(n, d, s["init"]), c["d"],
                                c["epochs"], c["p"], float(np.float32(c["lr"])), c["k"], seed=s["philox"],
                                threshold=c["threshold"], bf16=bf16, epoch_unit=c["epoch_unit"], losses=losses)
    train_s = time.time() - t
    emb = oracle.bf16_to_f64(M) if bf16 else M
    pairs = make_eval_pairs(sp, s["eval"], c["eval"]["max_train"], c["eval"]["max_test"])
    auc = auc_on_pairs(emb, pairs)
    D = len(info["sizes"])
    return {"auc": round(auc, 6), "sizes": [int(x) for x in info["sizes"]],
            "schedule": [int(x) for x in info["schedule"]],
            "updates": int(sum(info["updates"])),
            "last_epoch_loss": [float(losses[i][-1]) if len(losses[i]) else None for i in range(D)],
            "oracle_seconds": round(train_s, 1)}


def main():
    with ProcessPoolExecutor(2) as ex:
        f32 = ex.submit(run, False)
        b16 = ex.submit(run, True)
        res = {"fp64": f32.result(), "bf16": b16.result()}
    out = {"generated_by": "tests/golden/make_e2e_auc.py (oracle/ and synth/ only)", "config": CONFIG, **res}
    with open(OUT, "w") as f:
        json.dump(out, f, indent=1)
        f.write("\n")
    print(json.dumps(out))


if __name__ == "__main__":
    main()
