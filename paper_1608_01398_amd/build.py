"""Build libiht.so (HIP for gfx950) in-tree with hipcc.

Usage: python -m paper_1608_01398_amd.build [--isa DIR]   (--isa keeps the gfx950 assembly)
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
SOURCES = [os.path.join(CSRC, f) for f in ("iht_pass.hip", "iht_device.hip", "iht_batch.hip", "iht_solve.hip", "iht_engine.hip", "iht_api.hip", "iht_serve.hip", "iht_noalloc.hip")]
LIB = os.path.join(HERE, "libiht.so")
ARCH = "gfx950"

FLAGS = [
    "-O3", "-std=c++17", "-fPIC", "-shared", f"--offload-arch={ARCH}",
    # keep every rounding step as written (products and sums rounded separately, as the oracle does)
    "-ffp-contract=off",
    # no packed FP32 instructions in any generated code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I", os.path.join(ROOT, "include"), "-I", CSRC,
]


def build(isa_dir: str | None = None, verbose: bool = False) -> str:
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    tmp = LIB + ".tmp"
    cmd = [hipcc] + FLAGS + ["-o", tmp] + SOURCES
    if isa_dir:
        os.makedirs(isa_dir, exist_ok=True)
        cmd += ["-save-temps=cwd"]
        cwd = isa_dir
    else:
        cwd = HERE
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, cwd=cwd, capture_output=True, text=True)
    err = "\n".join(l for l in r.stderr.splitlines() if "packed-fp32-ops" not in l and l.strip())
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed ({r.returncode}):\n{err}")
    if err and verbose:
        print(err, file=sys.stderr)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    isa = None
    if "--isa" in sys.argv:
        isa = sys.argv[sys.argv.index("--isa") + 1]
    print(build(isa_dir=isa, verbose=True))
