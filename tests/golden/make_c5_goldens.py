"""Writes tests/golden/c5_oracle_solves.json: two FP64 oracle solves on the n=20,000 x p=2,000,000
workload (10 GB packed, 100 causal SNPs, 5 covariates + intercept unpenalised), the reference that
the GPU's FP64 and int8 matrix-core solves of the same traits are compared with.

Calls only the oracle (oracle/) and the seeded input generator; nothing from the device path. Each
oracle solve takes many minutes on a few host cores (one gradient pass decodes all 10 GB).

usage: python tests/golden/make_c5_goldens.py [--out PATH]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import oracle  # noqa: E402
from paper_1608_01398_amd import synth  # noqa: E402

SEED = 2
# (trait seed or None for the workload's own trait, k): the workload's trait at the number of effects,
# and a further trait of the same generator above it
SOLVES = [(None, 100), (700, 150)]


def c5_traits(prob):
    out = {}
    for ts, _ in SOLVES:
        if ts is None:
            out[ts] = prob["y"]
        else:
            y, *_ = synth.make_trait(prob["bed"], prob["n"], prob["q"], 100, (0.05, 0.3), seed=ts, Z=prob["Z"],
                                     intercept=1.0)
            out[ts] = y
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=os.path.join(os.path.dirname(os.path.abspath(__file__)), "c5_oracle_solves.json"))
    args = ap.parse_args()
    t0 = time.time()
    prob = synth.make_problem("c5", SEED)
    print(f"generated n={prob['n']} p={prob['p']} in {time.time() - t0:.0f} s", flush=True)
    traits = c5_traits(prob)
    rows = []
    for ts, k in SOLVES:
        t1 = time.time()
        ref = oracle.fit(prob["bed"], prob["n"], traits[ts], k, Z=prob["Z"], intercept=True)
        dt = time.time() - t1
        print(f"trait seed {ts} k={k}: status {ref['status']} iterations {ref['n_iter']} in {dt:.0f} s", flush=True)
        rows.append(dict(trait_seed=ts, k=k, status=int(ref["status"]), n_iter=int(ref["n_iter"]),
                         support=[int(x) for x in ref["support"]], beta_S=[float(x) for x in ref["beta_S"]],
                         beta_cov=[float(x) for x in ref["beta_cov"]],
                         loss_trace=[float(x) for x in ref["loss_trace"]], oracle_seconds=round(dt, 1)))
    doc = dict(workload="n=20,000 x p=2,000,000 packed 2-bit PLINK, 1% missing, 100 causal SNPs with effects "
                        "+-U(0.05,0.3), 5 N(0,1) FP32 covariates + intercept 1.0, unpenalised; FP64 oracle, "
                        "default options (tol 1e-10, c 0.01, shrink 0.5, max_backtrack 50, max_iter 200)",
               generator=dict(cfg="c5", seed=SEED), threads=int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1)),
               solves=rows)
    with open(args.out, "w") as f:
        json.dump(doc, f, indent=1)
    print(f"wrote {args.out} in {time.time() - t0:.0f} s", flush=True)


if __name__ == "__main__":
    main()
