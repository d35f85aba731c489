"""Runs the library's autotuner (h2_autotune) on a named workload and writes
the tuning cache.

  python -m paper_1705_04601_amd.autotune [--workload cube1m] [--out PATH] [--precisions fp64,mixed]

The H^2 matrix is built as the benchmark builds it (seeded synthetic points);
for each precision the autotuner measures every built GEMM tile variant the
sparsification, ILU(0) factorisation, preconditioner application and FP64
product plan, and the Schur knobs, with the workload's right-hand-side count,
and saves the fastest under this GPU's architecture (other architectures'
entries in the file are kept).  The default output is tune.json beside the
library, which the library reads at start-up.
"""

from __future__ import annotations

import argparse
import json
import os
import time

import h2inputs
import paper_1705_04601_amd as P


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--workload", default="cube1m", choices=sorted(h2inputs.WORKLOADS))
    ap.add_argument("--out", default=os.path.join(os.path.dirname(os.path.abspath(__file__)), "tune.json"))
    # knobs shared by both precisions (the Schur and solve work lists) keep the
    # value of the last precision tuned: the mixed path, the one measured
    ap.add_argument("--precisions", default="fp64,mixed")
    ap.add_argument("--nrhs", type=int, default=0, help="right-hand sides (default: the workload's)")
    a = ap.parse_args(argv)
    import torch
    torch.cuda.set_device(0)
    wl = h2inputs.WORKLOADS[a.workload]
    n = wl["n"]
    x = h2inputs.points(wl["kind"], n, wl["seed"])
    kern = P.H2_KERNEL_EXP if wl.get("kernel") == "exp" else P.H2_KERNEL_INVDIST
    h = P.h2_build(x, h2inputs.kernel_scale(wl["scale"], n), wl.get("diag", 1.0), wl["leaf"], wl["cheb"],
                   wl["tol"], wl["rank_cap"], kernel=kern)
    nrhs = a.nrhs or wl["nrhs"]
    P.h2_tune_clear()  # start from the built-in defaults
    for name in a.precisions.split(","):
        prec = {"mixed": P.H2_MIXED, "fp64": P.H2_FP64}[name]
        t0 = time.perf_counter()
        P.h2_autotune(h, prec, nrhs, a.out)
        print(f"autotune {a.workload} {name} nrhs {nrhs}: {time.perf_counter() - t0:.1f} s", flush=True)
    with open(a.out) as f:
        print(json.dumps(json.load(f), indent=1))


if __name__ == "__main__":
    main()
