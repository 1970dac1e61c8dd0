"""Launch only the gradient passes of the benchmark workload, for hardware-counter runs.

Builds the n=5000 x p=500,000 matrix with the benchmark's generator (seed 1), one subject set (all
subjects), and launches through the C ABI either the single-trait pass (3 x FP64, 3 x FP32) or the
batched matrix-core pass for 108 random residual rows (3 launches). Example:

  rocprofv3 --pmc SQ_WAVES SQ_BUSY_CYCLES -d out -o run --output-format csv -- \
      python3 paper_1608_01398_amd/profile_passes.py single

usage: python3 paper_1608_01398_amd/profile_passes.py {single,batched} [--reps R]
"""
from __future__ import annotations

import argparse
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("which", choices=["single", "batched"])
    ap.add_argument("--reps", type=int, default=3)
    ap.add_argument("--solves", type=int, default=108)
    args = ap.parse_args()

    import torch

    from paper_1608_01398_amd import iht, synth

    if not torch.cuda.is_available():
        raise SystemExit("profile_passes.py needs a HIP device")
    prob = synth.make_problem("c2", 1, workers=1)
    n, p = prob["n"], prob["p"]
    geno = iht.Geno(prob["bed"], n)
    stats = iht.Stats(geno)
    torch.cuda.synchronize()
    if args.which == "single":
        r = torch.from_numpy(prob["y"]).cuda()
        g = torch.empty(p, dtype=torch.float64, device="cuda")
        for precision in (iht.FP64, iht.FP32):
            for _ in range(args.reps):
                iht.gradient(geno, stats, r, precision, out=g)
    else:
        T = args.solves
        R = torch.randn((T, n), dtype=torch.float64, device="cuda", generator=torch.Generator("cuda").manual_seed(1))
        G = torch.empty((T, p), dtype=torch.float64, device="cuda")
        for _ in range(args.reps):
            iht.gradient_batch(geno, [stats] * T, R, out=G)
    torch.cuda.synchronize()
    print(f"profile_passes: {args.which} done", flush=True)


if __name__ == "__main__":
    main()
