"""Benchmark: time to a 1e-8 true relative residual and V-cycle HBM bandwidth on
the 2049^2 ECS grid (soft-Coulomb wavenumber, E = 2, h = 0.25 so k h ~ 0.5,
ECS beyond 80% of the half width at theta = pi/6; QD preconditioner inverted by
one V(1,1) red-black Gauss-Seidel cycle over 9 levels; flexible GMRES(40) in
FP64), mixed precision versus FP64.

One step = one complete solve from x = 0 to ||b - A x|| <= 1e-8 ||b|| with the
mixed-precision form (complex-FP32 cycle inside FP64 flexible GMRES).  The
FP64 form is timed the same way for the comparison.  Inputs are resident in
HBM before the timed region.  Prints one JSON line.

    python bench.py [--steps K] [--warmup W] [--gpus 1] [--no-cpu]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=int, default=2049)
    ap.add_argument("--inner", type=int, default=-1, help="FP32 inner Bi-CGSTAB iterations (mixed form); -1: default")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--vcycles", type=int, default=20, help="cycles timed for the V-cycle bandwidth")
    return ap.parse_args()


def level_nodes(n, nlev, dim=2):
    out = []
    for _ in range(nlev):
        out.append(n ** dim)
        n = (n - 1) // 2 + 1
    return out


def vcycle_algorithmic_bytes(n, nlev, real_bytes):
    """Minimum HBM traffic of one V(1,1) red-black cycle from a zero guess, per
    level l < coarsest: down pass reads b (2 reals), k^2 (1) and writes u (2)
    and the coarse residual (2/4); up pass reads u (2), the coarse correction
    (2/4), b (2), k^2 (1) and writes u (2): 13 reals per node."""
    nodes = level_nodes(n, nlev)
    per_node = (5.5 + 7.5) * real_bytes
    return sum(nodes[:-1]) * per_node


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}); the solver is single-GPU in this build",
              file=sys.stderr)
        sys.exit(2)
    import torch
    import paper_1012_4307_amd as E
    from paper_1012_4307_amd import workloads as W

    if not os.path.exists(E.LIB_PATH):
        from paper_1012_4307_amd import build as B
        B.build()
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    w = W.large_coulomb(n=args.n)
    k2 = torch.from_numpy(w.k2).to(dev)
    b = torch.from_numpy(w.rhs[0]).to(dev)
    inner = 0 if args.inner < 0 else args.inner

    def make(dt, inner_it):
        pc = E.Precond(kind="qd", re_lambda0=0.0, smoother="rbgs", omega=1.0, nu1=1, nu2=1, gamma_f=1, gamma_c=1,
                       coarsest_nodes=9, vcycle_dtype=dt)
        kr = E.Krylov(method="fgmres", restart=40, rtol=1e-8, maxit=20000, inner=inner_it)
        return E.Solver(2, w.n, w.lo, w.hi, w.ecs, k2, pc, kr)

    S64 = make("f64", 0)
    S32 = make("f32", inner)
    nlev = S64.nlev

    def timed_solves(S, k, timers=()):
        for cls in timers:
            S.timing(cls, True)
        times, stats, x = [], None, None
        for _ in range(k):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            x, st = S.solve(b)
            torch.cuda.synchronize()
            times.append(time.perf_counter() - t0)
            stats = st
            if st["status"] != 0:
                raise RuntimeError(f"solve did not converge: {st}")
        out = {}
        for cls in timers:
            out[cls] = S.timing_read(cls)
            S.timing(cls, False)
        return times, stats, x, out

    for _ in range(args.warmup):
        S32.solve(b)
        S64.solve(b)
    classes = ("smooth", "mdot", "apply_A", "coarse", "mupdate", "restrict", "prolong", "down", "up")
    t32, st32, x32, ktim = timed_solves(S32, args.steps, classes)
    t64, st64, x64, ktim64 = timed_solves(S64, args.steps, classes)
    rel_diff = float((x32 - x64).abs().max() / x64.abs().max())

    # V-cycle bandwidth (algorithmic bytes of a V(1,1) RB cycle / cycle time)
    def vcycle_rate(S, real_bytes):
        v = b.clone()
        for _ in range(3):
            S.vcycle(v)
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        ev0.record()
        for _ in range(args.vcycles):
            S.vcycle(v)
        ev1.record()
        torch.cuda.synchronize()
        ms = ev0.elapsed_time(ev1) / args.vcycles
        by = vcycle_algorithmic_bytes(args.n, nlev, real_bytes)
        return ms, by / (ms * 1e-3) / 1e9

    vc64_ms, vc64_gbs = vcycle_rate(S64, 8)
    vc32_ms, vc32_gbs = vcycle_rate(S32, 4)

    kernels = {}
    for cls, (nl, ms, by) in ktim.items():
        if nl:
            kernels[cls] = dict(launches=nl, total_ms=round(ms, 3), avg_us=round(1e3 * ms / nl, 2),
                                gbs=round(by / (ms * 1e-3) / 1e9, 1) if ms > 0 else None)
    dom = max((c for c in kernels if c != "coarse"), key=lambda c: kernels[c]["total_ms"])
    nl, ms, by = ktim[dom]
    achieved = by / (ms * 1e-3) / 1e9
    roofline = dict(bound="hbm", kernel=dom, achieved=round(achieved, 1), peak=HBM_PEAK_GBS, unit="GB/s",
                    frac=round(achieved / HBM_PEAK_GBS, 4), traffic=None,
                    bytes_per_launch=round(by / nl), avg_launch_us=round(1e3 * ms / nl, 2))

    cpu = None
    if not args.no_cpu:
        cpu = cpu_baseline(w, st64["iterations"])

    value = float(np.median(t32))
    line = {
        "metric": "time-to-1e-8 residual + V-cycle HBM GB/s, 2049^2 ECS grid, mixed vs FP64",
        "value": round(value, 4),
        "unit": "s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(1e3 * float(np.mean(t32)), 2),
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64",
        "data": "synthetic",
        "config": {"workload": f"soft-Coulomb ECS Helmholtz {args.n}^2, h=0.25, E=2, QD, V(1,1) RB-GS, "
                               f"{nlev} levels, FGMRES(40) to 1e-8",
                   "grid": args.n, "h": 0.25, "E": 2.0, "theta": "pi/6", "levels": nlev, "restart": 40,
                   "inner_fp32_iterations": inner},
        "mixed": dict(seconds=round(value, 4), iterations=st32["iterations"], vcycles=st32["vcycles"],
                      rel_residual=st32["rel_residual"], rel_diff_vs_fp64_solution=rel_diff),
        "fp64": dict(seconds=round(float(np.median(t64)), 4), iterations=st64["iterations"],
                     vcycles=st64["vcycles"], rel_residual=st64["rel_residual"]),
        "speedup_mixed_vs_fp64": round(float(np.median(t64)) / value, 3),
        "vcycle": {"fp64_ms": round(vc64_ms, 4), "fp64_gbs": round(vc64_gbs, 1),
                   "fp32_ms": round(vc32_ms, 4), "fp32_gbs": round(vc32_gbs, 1),
                   "model": "algorithmic bytes of a V(1,1) RB cycle, 13 reals/node/level"},
        "kernels_mixed": kernels,
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


def cpu_baseline(w, gpu_iterations):
    """The CPU oracle (plain FP64 C, OpenMP) on a bounded sample: one restart
    cycle (40 FGMRES iterations, 40 V-cycles) of the same solve on the same
    inputs, timed, then scaled by the GPU FP64 iteration count to an estimated
    time-to-1e-8."""
    import oracle
    P = oracle.Problem(w.dim, w.n, w.lo, w.hi, w.ecs, w.k2, w.nlev)
    P.set_operator("qd")
    P.set_cycle("rbgs", 1.0)
    sample = 40
    t0 = time.perf_counter()
    _, st = P.solve(w.rhs[0], "fgmres", 40, 1e-8, sample)
    dt = time.perf_counter() - t0
    per_it = dt / max(1, st["iterations"])
    return dict(value=round(per_it * gpu_iterations, 2), unit="s", cores=oracle.num_threads(), kind="oracle",
                sample=f"{st['iterations']} FGMRES(40) iterations of the same {w.n[0]}^2 solve in {dt:.1f} s "
                       f"({per_it:.3f} s/iteration), scaled by the {gpu_iterations} iterations the FP64 solve needs")


if __name__ == "__main__":
    main()
