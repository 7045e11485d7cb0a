"""Benchmark: time to a 1e-8 true relative residual and V-cycle HBM bandwidth on
the 2049^2 ECS grid, mixed precision versus FP64.

Workload: soft-Coulomb wavenumber k^2 = 2(E + 1/sqrt(r^2+1)), E = 2, h = 0.25
(k h ~ 0.5) on [-256, 256]^2, ECS beyond |x|, |y| = 204.8 at theta = pi/6,
right-hand side phi0 * V; QD preconditioner (|Re lambda0| = max k^2) inverted
by one V(1,1) red-black Gauss-Seidel cycle over 9 levels (coarsest 9^2);
flexible GMRES(40) in FP64.

One step = one complete solve from x = 0 to ||b - A x|| <= 1e-8 ||b||, timed
with inputs already resident in HBM.  `value` is the mixed-precision solve:
FP64 FGMRES(40) whose preconditioner is a few iterations of complex-FP32
Bi-CGSTAB around the complex-FP32 V-cycle (Arnoldi, Hessenberg least squares
and the true residual stay FP64 on the GPU).  Reported beside it: the plain
FP64 solve (FGMRES(40), FP64 cycle) timed the same way, the FP32-cycle-only
FGMRES(40), FP64 Bi-CGSTAB, V-cycle bandwidth, per-kernel timings of the
dominant kernel measured with HIP events inside the timed region (and, as a
cross-check, from an in-process kernel trace of one more solve), and the CPU
oracle on a bounded sample.  Prints one JSON line.

    python bench.py [--steps K] [--warmup W] [--gpus 1] [--no-cpu] [--no-trace]
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
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic.json")
# kernel classes are timed with HIP events on one launch in this many: each
# timed launch costs a few microseconds of event overhead on the stream
TIMED_ONE_IN = 8

def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=int, default=2049)
    ap.add_argument("--restart", type=int, default=40)
    ap.add_argument("--inner", type=int, default=16, help="FP32 inner Bi-CGSTAB iterations per FGMRES step")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-context", action="store_true", help="skip the context solves (FP32-cycle FGMRES, "
                                                               "FP64 Bi-CGSTAB)")
    ap.add_argument("--vcycles", type=int, default=20, help="cycles timed for the V-cycle bandwidth")
    ap.add_argument("--no-trace", action="store_true",
                    help="skip the in-process kernel trace of one more mixed solve (for runs under rocprofv3)")
    ap.add_argument("--config", default="mixed2049",
                    choices=["mixed2049", "batched", "persistent_probe", "adjoint", "cube", "coulomb513", "small65",
                             "paper_mp", "coupled"],
                    help="mixed2049 (default): the headline line; the others report the secondary workloads")
    ap.add_argument("--batch-count", type=int, default=96)
    ap.add_argument("--batch-streams", type=int, default=32, help="HIP streams the batched systems are spread over")
    ap.add_argument("--batch-cycle", choices=("f64", "f32"), default="f64",
                    help="dtype of the multigrid cycle of the batched systems (the Krylov vectors stay FP64)")
    return ap.parse_args()


def level_nodes(n, nlev, dim=2):
    out = []
    for _ in range(nlev):
        out.append(n ** dim)
        n = (n - 1) // 2 + 1
    return out


# Algorithmic bytes per node of one level's passes of the V(1,1) red-black
# cycle from a zero guess, in reals of the cycle's dtype.  "method": the
# passes as the method states them -- the down pass reads b and k^2 and writes
# the pre-smoothed iterate u and the coarse residual (2 + 1 + 2 + 2/4 = 5.5),
# the up pass reads u, the coarse correction, b and k^2 and writes u
# (2 + 2/4 + 2 + 1 + 2 = 7.5).  "kernel": what the fused kernels must move,
# since the up kernel recomputes the pre-smoothed iterate from b instead of
# reading it (down 3.5, up 5.5).
PASS_REALS = {"method": {"down": 5.5, "up": 7.5}, "kernel": {"down": 3.5, "up": 5.5}}


def vcycle_algorithmic_bytes(n, nlev, real_bytes, model="method"):
    """Algorithmic HBM bytes of one V(1,1) cycle: (down + up) reals per node of
    every level above the coarsest."""
    nodes = level_nodes(n, nlev)
    per = PASS_REALS[model]["down"] + PASS_REALS[model]["up"]
    return sum(nodes[:-1]) * per * real_bytes


def trace_dominant_us(run, cls, PS):
    """Average duration (us) of the finest-grid launches of kernel class `cls`
    in a kernel trace of run(), or None when the class has no pattern or the
    tracer records nothing."""
    import tempfile
    import torch
    from torch.profiler import ProfilerActivity, profile
    if cls not in dict(PS.CLASSES):
        return None
    with profile(activities=[ProfilerActivity.CUDA]) as prof:
        run()
        torch.cuda.synchronize()
    fd, path = tempfile.mkstemp(suffix=".json")
    os.close(fd)
    try:
        prof.export_chrome_trace(path)
        with open(path) as f:
            events = json.load(f).get("traceEvents", [])
    finally:
        os.remove(path)
    return PS.trace_class_avg(events, cls)


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU (got --gpus {args.gpus}): the solver runs on a single GPU and has no "
              f"multi-GPU path (a split into horizontal slabs with halo exchange is not implemented)", file=sys.stderr)
        sys.exit(2)
    import torch
    import paper_1012_4307_amd as E
    from paper_1012_4307_amd import profile_summary as PS
    from paper_1012_4307_amd import workloads as W

    if not os.path.exists(E.LIB_PATH):
        from paper_1012_4307_amd import build as B
        B.build()
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    if args.config != "mixed2049":
        from paper_1012_4307_amd import bench_workloads
        bench_workloads.run(args)
        return
    w = W.large_coulomb(n=args.n)
    k2 = torch.from_numpy(w.k2).to(dev)
    b = torch.from_numpy(w.rhs[0]).to(dev)

    def make(dt, method, inner, orth="dcgs2"):
        pc = E.Precond(kind="qd", re_lambda0=0.0, smoother="rbgs", omega=1.0, nu1=1, nu2=1, gamma_f=1, gamma_c=1,
                       coarsest_nodes=9, vcycle_dtype=dt)
        kr = E.Krylov(method=method, restart=args.restart, rtol=1e-8, maxit=20000, inner=inner, orth=orth)
        return E.Solver(2, w.n, w.lo, w.hi, w.ecs, k2, pc, kr)

    Smix = make("f32", "fgmres", args.inner)
    S64 = make("f64", "fgmres", 0)
    nlev = S64.nlev

    timed_classes = ("down", "up", "down_p", "down_s", "mdot", "mupdate", "apply_A")

    def timed_solves(S, k, timers=()):
        for cls in timers:
            S.timing(cls, True, every=TIMED_ONE_IN)
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
        Smix.solve(b)
        S64.solve(b)
    tmix, stmix, xmix, ktim = timed_solves(Smix, args.steps, timed_classes)
    # the comparison solves take longer: at most 5 timed runs each
    t64, st64, x64, _ = timed_solves(S64, min(args.steps, 5))
    rel_diff = float((xmix - x64).abs().max() / x64.abs().max())
    # the same nested algorithm with the FP64 cycle and FP64 inner Bi-CGSTAB:
    # the mixed form's factor over it is the precision's share of the speedup
    Sn64 = make("f64", "fgmres", args.inner)
    Sn64.solve(b)
    tn64, stn64, xn64, _ = timed_solves(Sn64, min(args.steps, 5))
    del Sn64
    # the cycle's levels below the finest (every kernel of the chain, the tail
    # included), timed in one more mixed solve outside the headline's runs
    _, stc, _, ctim = timed_solves(Smix, 1, ("coarse",))
    nlc, msc, _ = ctim["coarse"]
    coarse_chain = dict(launches_timed=nlc, avg_launch_us=round(1e3 * msc / nlc, 2) if nlc else None,
                        per_cycle_us=round(1e3 * msc * TIMED_ONE_IN / stc["vcycles"], 1),
                        launches_per_cycle=round(nlc * TIMED_ONE_IN / stc["vcycles"], 2))

    context = {}
    if not args.no_context:
        for name, (dt, method, inner, orth) in {
                "fgmres_fp32_cycle": ("f32", "fgmres", 0, "dcgs2"),
                "fgmres_fp64_cgs1": ("f64", "fgmres", 0, "cgs1"),
                "fgmres_fp64_cgs2": ("f64", "fgmres", 0, "cgs2"),
                "fgmres_fp64_cgs2_selective": ("f64", "fgmres", 0, "cgs2_selective"),
                "mixed_cgs1": ("f32", "fgmres", args.inner, "cgs1"),
                "mixed_cgs2_selective": ("f32", "fgmres", args.inner, "cgs2_selective"),
                "bicgstab_fp64": ("f64", "bicgstab", 0, "dcgs2")}.items():
            S = make(dt, method, inner, orth)
            S.solve(b)
            tt, st, _, _ = timed_solves(S, 1)
            context[name] = dict(seconds=round(tt[0], 4), iterations=st["iterations"], vcycles=st["vcycles"],
                                 rel_residual=st["rel_residual"], second_gram_schmidt_passes=st["reorthogonalisations"])
            del S

    # V-cycle rate (algorithmic bytes of a V(1,1) RB cycle / cycle time), on
    # vectors in the cycle's dtype: warm (back to back) and cold (a 512 MiB
    # write between cycles evicts the 256 MB last-level cache)
    flush = torch.empty(512 << 20, dtype=torch.uint8, device=dev)

    def vcycle_rate(S, real_bytes):
        v = b.to(S.cycle_dtype)
        for _ in range(3):
            S.vcycle_native(v)
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        ev0.record()
        for _ in range(args.vcycles):
            S.vcycle_native(v)
        ev1.record()
        torch.cuda.synchronize()
        ms = ev0.elapsed_time(ev1) / args.vcycles
        cold = []
        for _ in range(5):
            E.copy_probe(flush, flush)
            ev0.record()
            S.vcycle_native(v)
            ev1.record()
            torch.cuda.synchronize()
            cold.append(ev0.elapsed_time(ev1))
        cms = float(np.median(cold))
        out = {"ms": round(ms, 4), "cold_ms": round(cms, 4)}
        for model in ("method", "kernel"):
            by = vcycle_algorithmic_bytes(args.n, nlev, real_bytes, model)
            for tag, t in (("warm", ms), ("cold", cms)):
                gbs = by / (t * 1e-3) / 1e9
                out[f"{model}_{tag}_gbs"] = round(gbs, 1)
                out[f"{model}_{tag}_frac"] = round(gbs / HBM_PEAK_GBS, 4)
        return out

    vc64 = vcycle_rate(S64, 8)
    vc32 = vcycle_rate(Smix, 4)
    del flush

    # copy probe (plain device copy of 512 MiB): the practical HBM rate, and
    # the reference dispatch that scales the FETCH_SIZE / WRITE_SIZE counters
    src = torch.empty(512 << 20, dtype=torch.uint8, device=dev)
    dst = torch.empty_like(src)
    for _ in range(2):
        E.copy_probe(src, dst)
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    ev0.record()
    for _ in range(5):
        E.copy_probe(src, dst)
    ev1.record()
    torch.cuda.synchronize()
    copy_gbs = 2 * src.numel() / (ev0.elapsed_time(ev1) / 5 * 1e-3) / 1e9
    del src, dst
    # the same rates as fractions of the copy probe (the practical HBM rate)
    for vc in (vc64, vc32):
        for key in [k for k in vc if k.endswith("_gbs")]:
            vc[key[:-4] + "_frac_of_copy"] = round(vc[key] / copy_gbs, 4)

    kernels = {}
    for cls, (nl, ms, by) in ktim.items():
        if nl:
            kernels[cls] = dict(launches=nl, total_ms=round(ms, 3), avg_us=round(1e3 * ms / nl, 2),
                                algo_gbs=round(by / (ms * 1e-3) / 1e9, 1) if ms > 0 else None)
    dom = max(kernels, key=lambda c: kernels[c]["total_ms"])
    nl, ms, by = ktim[dom]
    # a timed duration runs from the kernel's dispatch to its completion, the
    # same span rocprofv3's kernel trace reports; `achieved` uses it as is.
    # The duration of an empty timed launch is reported beside it (the fixed
    # part of every launch), and the rate net of it for reference.
    overhead_us = Smix.timing_calibrate(200)
    raw_us = 1e3 * ms / nl
    net_us = max(raw_us - overhead_us, 1e-3)
    # the timers carry the kernel model's bytes; the method's bytes of the same
    # launch follow from the finest grid's node count (classes "up"/"down" are
    # finest-level launches of the FP32 cycle)
    kernel_bytes = by / nl
    if dom in ("up", "down"):
        method_bytes = args.n * args.n * PASS_REALS["method"][dom] * 4
        model = f"{dom} pass as the method states it: {PASS_REALS['method'][dom]} FP32 reals per fine node"
    else:
        method_bytes, model = kernel_bytes, "the kernel's own minimum traffic"
    achieved = method_bytes / (raw_us * 1e-6) / 1e9
    traffic = None
    try:
        with open(TRAFFIC_FILE) as f:
            tr = json.load(f)
        if tr.get("sources_digest") == PS.sources_digest() and dom in tr.get("kernels", {}):
            traffic = tr["kernels"][dom]["hbm_bytes_per_launch"]
    except (OSError, ValueError):
        traffic = None
    roofline = dict(bound="hbm", achieved=round(achieved, 1), peak=HBM_PEAK_GBS, unit="GB/s",
                    frac=round(achieved / HBM_PEAK_GBS, 4), traffic=traffic, kernel=dom,
                    bytes_model=model, algo_bytes_per_launch=round(method_bytes), avg_launch_us=round(raw_us, 2),
                    kernel_model=dict(bytes_per_launch=round(kernel_bytes),
                                      achieved=round(kernel_bytes / (raw_us * 1e-6) / 1e9, 1),
                                      frac=round(kernel_bytes / (raw_us * 1e-6) / 1e9 / HBM_PEAK_GBS, 4)),
                    counters=None if traffic is None else dict(
                        hbm_bytes_per_launch=traffic, achieved=round(traffic / (raw_us * 1e-6) / 1e9, 1),
                        frac=round(traffic / (raw_us * 1e-6) / 1e9 / HBM_PEAK_GBS, 4)),
                    frac_of_copy_probe=round(achieved / copy_gbs, 4),
                    empty_kernel_us=round(overhead_us, 2),
                    achieved_net_of_empty=round(method_bytes / (net_us * 1e-6) / 1e9, 1), launches=nl,
                    timed_one_launch_in=TIMED_ONE_IN)

    # cross-check of the dominant kernel's duration: an in-process kernel trace
    # (the ROCm tracer behind torch.profiler) of one more mixed solve.  Its
    # durations are the kernels' own execution, as in rocprofv3's kernel
    # trace; a launch timed with HIP events also spans the dispatch of the
    # kernel and the completion of its stop event.
    if not args.no_trace:
        tr_us = trace_dominant_us(lambda: Smix.solve(b), dom, PS)
        if tr_us:
            roofline["trace"] = dict(
                avg_launch_us=round(tr_us, 2), achieved=round(method_bytes / (tr_us * 1e-6) / 1e9, 1),
                frac=round(method_bytes / (tr_us * 1e-6) / 1e9 / HBM_PEAK_GBS, 4),
                kernel_model_frac=round(kernel_bytes / (tr_us * 1e-6) / 1e9 / HBM_PEAK_GBS, 4),
                source="in-process kernel trace (torch.profiler) of one more mixed solve: the dominant class's "
                       "finest-grid launches")

    cpu = None
    if not args.no_cpu:
        cpu = cpu_baseline(w, st64["iterations"], args.restart,
                           {"mixed": xmix.cpu().numpy(), "fp64": x64.cpu().numpy(),
                            "nested_fp64": xn64.cpu().numpy()})

    value = float(np.median(tmix))
    line = {
        "metric": "time-to-1e-8 residual + V-cycle HBM GB/s, 2049^2 ECS grid, mixed vs FP64",
        "value": round(value, 4),
        "unit": "s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(1e3 * float(np.mean(tmix)), 2),
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64",
        "data": "synthetic",
        "config": {"workload": f"soft-Coulomb ECS Helmholtz {args.n}^2 nodes, h=0.25, E=2, theta=pi/6, QD + "
                               f"V(1,1) RB-GS over {nlev} levels, FP64 FGMRES({args.restart}) to 1e-8 with "
                               f"{args.inner} FP32 Bi-CGSTAB inner iterations per step",
                   "grid": args.n, "h": 0.25, "E": 2.0, "levels": nlev, "restart": args.restart,
                   "inner_fp32_iterations": args.inner,
                   "arnoldi": "classical Gram-Schmidt, second pass delayed by one step"},
        "mixed": dict(seconds=round(value, 4), iterations=stmix["iterations"],
                      inner_iterations=stmix["inner_iterations"], vcycles=stmix["vcycles"],
                      rel_residual=stmix["rel_residual"], rel_diff_vs_fp64_solution=rel_diff,
                      second_gram_schmidt_passes=stmix["reorthogonalisations"],
                      inner_runs_cut_short=stmix["inner_breakdowns"]),
        "fp64": dict(seconds=round(float(np.median(t64)), 4), iterations=st64["iterations"],
                     vcycles=st64["vcycles"], rel_residual=st64["rel_residual"],
                     second_gram_schmidt_passes=st64["reorthogonalisations"]),
        "nested_fp64": dict(seconds=round(float(np.median(tn64)), 4), iterations=stn64["iterations"],
                            inner_iterations=stn64["inner_iterations"], vcycles=stn64["vcycles"],
                            rel_residual=stn64["rel_residual"],
                            second_gram_schmidt_passes=stn64["reorthogonalisations"],
                            inner_runs_cut_short=stn64["inner_breakdowns"]),
        "speedup_mixed_vs_fp64": round(float(np.median(t64)) / value, 3),
        "speedup_mixed_vs_nested_fp64": round(float(np.median(tn64)) / value, 3),
        "context_solves": context,
        "vcycle": {"fp64": vc64, "fp32": vc32,
                   "bytes_models": {"method": "13 reals/node/level above the coarsest (down 5.5, up 7.5)",
                                    "kernel": "9 reals/node/level (down 3.5, up 5.5: the iterate is recomputed)"},
                   "cold": "a 512 MiB write before each cycle evicts the 256 MB last-level cache",
                   "vectors": "in the cycle's dtype (no conversion passes)"},
        "copy_probe_gbs": round(copy_gbs, 1),
        "kernels_in_timed_region": kernels,
        "coarse_chain": coarse_chain,
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


GOLDEN_ORACLE = os.path.join(ROOT, "tests", "golden", "oracle_large_coulomb_2049.json")


def cpu_baseline(w, gpu_iterations, restart, solutions):
    """The CPU oracle (plain FP64 C with OpenMP) on a bounded sample of the same
    solve, on the same 2049^2 inputs:
      * all threads: one complete restart cycle of its FGMRES(restart) (every
        basis size 0 .. restart-1, one FP64 V-cycle each), timed once;
      * the first 4 iterations, timed three times at all threads and three
        times at one thread (medians): the one-thread restart cycle is the
        all-thread one scaled by the ratio of the two short samples.
    The per-iteration time of a restart cycle is scaled to the iterations the
    oracle's own solve needs to reach 1e-8 (stored by the oracle-only script
    tests/golden/make_oracle_large_coulomb.py; the FP64 GPU solve's count when
    that file is absent).  The first cycle also pays the first touch of the
    basis (about 2.7 GB), which later cycles do not.  The same leg recomputes
    the true relative residual of each GPU solution with the oracle's operator
    and, with the stored samples of the oracle's 1e-12 solution, its relative
    error."""
    import oracle
    P = oracle.Problem(w.dim, w.n, w.lo, w.hi, w.ecs, w.k2, w.nlev)
    P.set_operator("qd")
    P.set_cycle("rbgs", 1.0)
    b = w.rhs[0]
    bi = np.zeros_like(b)
    bi[1:-1, 1:-1] = b[1:-1, 1:-1]
    golden = None
    if os.path.exists(GOLDEN_ORACLE):
        with open(GOLDEN_ORACLE) as fh:
            golden = json.load(fh)
    checks = {}
    for name, x in solutions.items():
        c = dict(rel_residual_oracle=float(np.linalg.norm(bi - P.apply(x)) / np.linalg.norm(bi)))
        if golden is not None:
            g = golden["solution_1e12"]
            st = g["stride"]
            ref = (np.array(g["re"]) + 1j * np.array(g["im"])).reshape(x[::st, ::st].shape)
            c["rel_error_vs_oracle_sampled"] = float(np.abs(x[::st, ::st] - ref).max() / g["max_abs"])
            c["samples"] = int(ref.size)
        checks[name] = c
    allc = oracle.num_threads()
    SHORT = 4

    def run(threads, k):
        oracle.set_threads(threads)
        t0 = time.perf_counter()
        P.solve(b, "fgmres", restart, 1e-8, k)
        return time.perf_counter() - t0

    t_cycle = run(allc, restart)
    short_all = [run(allc, SHORT) for _ in range(3)]
    short_one = [run(1, SHORT) for _ in range(3)]
    oracle.set_threads(allc)
    m_all, m_one = float(np.median(short_all)), float(np.median(short_one))
    per_all = t_cycle / restart
    per_one = per_all * m_one / m_all
    iters = golden["fgmres_1e8"]["iterations"] if golden else gpu_iterations
    src = "the oracle's own FGMRES(40) solve to 1e-8" if golden else "the FP64 GPU solve (no stored oracle count)"
    out = dict(value=round(per_all * iters, 2), unit="s", cores=allc, kind="oracle",
               sample=f"one restart cycle ({restart} iterations) of the oracle's FP64 FGMRES({restart}) on the same "
                      f"{w.n[0]}^2 inputs at {allc} threads ({t_cycle:.1f} s), scaled to the {iters} iterations of "
                      f"{src}; one thread: the same scaled by the medians of 3 runs of the first {SHORT} "
                      f"iterations at 1 and at {allc} threads ({m_one:.2f} / {m_all:.2f} s)",
               one_thread=dict(value=round(per_one * iters, 2), cores=1, seconds_per_iteration=round(per_one, 4),
                               short_runs_s=[round(t, 3) for t in short_one]),
               all_threads=dict(value=round(per_all * iters, 2), cores=allc, seconds_per_iteration=round(per_all, 4),
                                restart_cycle_s=round(t_cycle, 3), short_runs_s=[round(t, 3) for t in short_all]),
               oracle_iterations=iters, solution_checks=checks)
    if golden:
        out["oracle_full_solve_reference"] = dict(seconds=golden["fgmres_1e8"]["seconds"],
                                                  threads=golden["threads"],
                                                  note="the whole oracle solve, timed once where the stored "
                                                       "file was written (not this host)")
    return out


if __name__ == "__main__":
    main()
