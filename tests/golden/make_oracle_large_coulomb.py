"""Writes tests/golden/oracle_large_coulomb_2049.json from the CPU oracle only.

The benchmark workload (2049^2 nodes, h = 0.25, E = 2, QD with the automatic
|Re lambda0|, V(1,1) red-black over 9 levels, FP64 FGMRES(40), x0 = 0):

  * fgmres_1e8: the oracle's own solve to a 1e-8 true relative residual --
    iterations, restarts, final residual, wall time and thread count (the
    iteration count scales the CPU baseline of the benchmark);
  * solution_1e12: the oracle's solution at a 1e-12 true residual, sampled
    at every `stride`-th node of each axis (x fastest, the nodes i, j in
    0, stride, ..., n-1), with the largest |x| over all nodes and the 2-norm,
    the reference for the relative error of GPU solutions at full size.

Run from the repository root:  python tests/golden/make_oracle_large_coulomb.py
(about an hour on 8 cores).  Nothing else writes this file.
"""
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_1012_4307_amd import workloads as W  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "oracle_large_coulomb_2049.json")
STRIDE = 32


def main():
    w = W.large_coulomb(n=2049)
    P = oracle.Problem(w.dim, w.n, w.lo, w.hi, w.ecs, w.k2, w.nlev)
    lam0 = P.set_operator("qd", 0.0)
    P.set_cycle("rbgs", 1.0)
    b = w.rhs[0]
    out = dict(workload="large_coulomb(n=2049): h = 0.25, E = 2, QD (automatic |Re lambda0|), V(1,1) red-black, "
                        "9 levels, FGMRES(40), x0 = 0", lam0=lam0, threads=oracle.num_threads())
    t0 = time.perf_counter()
    _, st = P.solve(b, "fgmres", 40, 1e-8, 20000)
    out["fgmres_1e8"] = dict(st, seconds=round(time.perf_counter() - t0, 1))
    print("1e-8:", out["fgmres_1e8"], flush=True)
    t0 = time.perf_counter()
    x, st = P.solve(b, "fgmres", 40, 1e-12, 40000)
    assert st["status"] == 0, st
    sl = slice(0, None, STRIDE)
    xs = x[sl, sl]
    out["solution_1e12"] = dict(stats=dict(st, seconds=round(time.perf_counter() - t0, 1)), stride=STRIDE,
                                max_abs=float(np.abs(x).max()), norm2=float(np.linalg.norm(x)),
                                re=[float(v) for v in xs.real.ravel()], im=[float(v) for v in xs.imag.ravel()])
    print("1e-12:", out["solution_1e12"]["stats"], flush=True)
    with open(OUT, "w") as fh:
        json.dump(out, fh, indent=0)


if __name__ == "__main__":
    main()
