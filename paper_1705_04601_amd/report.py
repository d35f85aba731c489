"""Storage study of the sparse factorization A = U S V^T (Sections 5.1-5.2).

  python -m paper_1705_04601_amd.report [--max-n N] [--fill-max-n N] [--kernels inv,exp] [--dims 2,3]

For each kernel (inverse distance of Example 5.1, the exp core of Example 5.2),
each dimension (uniform points in the unit square or cube) and N doubling
from 2048 to --max-n, the H^2 matrix is built on the host and planned
without device work.  One line per case: nonzeros per row of S, and the
storage in MB (8-byte entries) of the dense matrix, the H^2 matrix, the
factors U + S + V (U and V counted separately, as the paper sums them; the
library stores the orthogonal blocks once and the upper block triangle of S,
since A is symmetric) and of S alone.  Up to --fill-max-n the exact mode's
filled S (upper triangle) and its Schur flops are added.

H^2 settings per dimension reach the paper's accuracy 1e-6 (relative error
of products with random vectors, both kernels): leaf 64 and recompression
tolerance 1e-7 in both; in 2D 6 Chebyshev nodes per axis and the
admissibility dist >= diam, in 3D 4 nodes per axis (the library's limit of
64 nodes per cluster) and the stronger dist >= 2 diam.
"""

from __future__ import annotations

import argparse
import time

import numpy as np

import h2inputs
import paper_1705_04601_amd as P

SETTINGS = {2: dict(leaf=64, cheb=6, tol=1e-7, eta=1.0), 3: dict(leaf=64, cheb=4, tol=1e-7, eta=2.0)}
KERNELS = {"inv": (P.H2_KERNEL_INVDIST, 1.0, 0.0), "exp": (P.H2_KERNEL_EXP, 1.0, 3.0)}


def case(kernel: str, dim: int, n: int, with_fill: bool, seed: int = 11) -> dict:
    kind = "square" if dim == 2 else "cube"
    x = h2inputs.points(kind, n, seed)
    kern, scale, diag = KERNELS[kernel]
    st = SETTINGS[dim]
    t0 = time.perf_counter()
    h = P.h2_build(x, scale, diag, st["leaf"], st["cheb"], st["tol"], 0, st["eta"], kernel=kern)
    t1 = time.perf_counter()
    r = P.h2_plan_report(h, with_fill=with_fill)
    r["build_s"] = t1 - t0
    r["plan_s"] = time.perf_counter() - t1
    r["kernel"], r["dim"] = kernel, dim
    return r


def line(r: dict) -> str:
    mb = 8 / 2**20
    n = r["n"]
    usv = 2 * r["q_entries"] + r["s_entries"]
    diag = 2 * r["s_upper_entries"] - r["s_entries"]  # entries of the diagonal blocks
    fill = (f"{(2 * r['filled_entries'] - diag) / n:9.1f} {r['exact_flops'] / 1e9:10.2f}"
            if r["filled_entries"] >= 0 else f"{'-':>9s} {'-':>10s}")
    return (f"{r['kernel']:4s} {r['dim']}D {n:8d} {r['s_entries'] / n:9.1f} {r['h2_close_entries'] / n:9.1f} "
            f"{n * n * mb:11.1f} {r['h2_entries'] * mb:9.1f} {usv * mb:9.1f} {r['s_entries'] * mb:9.1f} "
            f"{fill} {r['build_s']:7.1f} {r['plan_s']:7.1f}")


HEADER = (f"{'core':4s} dim {'N':>8s} {'nnz/row':>9s} {'close/row':>9s} {'dense MB':>11s} {'H2 MB':>9s} {'U+S+V MB':>9s} "
          f"{'S MB':>9s} {'fill/row':>9s} {'exact GF':>10s} {'build s':>7s} {'plan s':>7s}")


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--max-n", type=int, default=1 << 20)
    ap.add_argument("--fill-max-n", type=int, default=1 << 17)
    ap.add_argument("--kernels", default="inv,exp")
    ap.add_argument("--dims", default="2,3")
    a = ap.parse_args(argv)
    print(HEADER, flush=True)
    for kernel in a.kernels.split(","):
        for dim in (int(d) for d in a.dims.split(",")):
            n = 2048
            while n <= a.max_n:
                print(line(case(kernel, dim, n, n <= a.fill_max_n)), flush=True)
                n *= 2


if __name__ == "__main__":
    main()
