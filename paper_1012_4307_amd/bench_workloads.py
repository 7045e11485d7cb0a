"""Secondary measurements behind ``bench.py --config ...`` (the headline line is
the 2049^2 mixed-precision solve).  Each prints one JSON line.

batched     many independent systems (grids 257^2 / 513^2 / 1025^2, E, theta
            and 1-8 right-hand sides per system, seeded) in one batched
            Bi-CGSTAB call, each system on its own stream with its right-hand
            sides solved together, cycle schedule autotuned per grid; aggregate
            right-hand sides solved per second, beside the same batch with the
            right-hand sides one at a time and the same systems solved one call
            at a time.
adjoint     the differentiable solve on 1025^2 (E = 2): forward and backward
            (adjoint) time, gradient of L = 1/2 ||M u - d||^2 against central
            differences (eps = 1e-6) on 50 random interior nodes and on 5 nodes
            with large gradients.
cube        3D 7-point 129^3 forward solve at constant k = 12 (QD, V(1,1)
            red-black, FGMRES(30)).
coulomb513  soft-Coulomb QD problems on 513^2, E in {0.5, 1, 2, 4}, Bi-CGSTAB.
small65     the 65^2 constant-k problem (CSL, omega-Jacobi, GMRES(30)) for both
            right-hand sides and both signs of the complex shift.
coupled     the coupled block system of Sec. 2 (4 soft-Coulomb channels on
            513^2 with thresholds and short-range couplings, channel 0
            driven): FGMRES(30) to 1e-8 with the block-diagonal
            preconditioner, blocks solved by the batched Bi-CGSTAB driver to
            1e-3 (FP32 cycles, one stream per block), and with one cycle per
            block instead.
persistent_probe
            the two persistent organisations of the batched solve that the
            library does not use, measured by the probes of
            include/ecsmg_probe.h: the memory rate of red-black sweeps with one
            workgroup per independent grid (257^2, 513^2, 1025^2; 1, 32, 256
            grids at once), and the cost of a device-wide phase barrier among a
            group of workgroups (8 to 256 workgroups, with and without 64 KiB
            written per workgroup and phase).
paper_mp    the model problems of Sec. 5 (Tables 1-4: MP1 k = 160 on 385^2,
            MP2 on 641^2, MP3 k = 2 on 641^2 and k = 4 on 897^2), each with the
            CSL, CSG and QD set-ups of its table: stand-alone multigrid on
            M x = f (cycles to a 1e-6 residual reduction; mg-conv = geometric
            mean of the residual ratios over all cycles, with the mean of the
            last 5 beside it) and right preconditioned Bi-CGSTAB on A u = f to
            1e-6, FP64 throughout; also the warm start of Sec. 5 (stand-alone
            multigrid to 1e-2 as Bi-CGSTAB's initial guess).
"""
from __future__ import annotations

import json
import math
import time

import numpy as np


def _emit(d):
    print(json.dumps(d), flush=True)


def _solver(w, vcycle_dtype="f64", krylov=None, stream=None):
    import torch
    from . import solver_for
    if stream is None:
        return solver_for(w, vcycle_dtype=vcycle_dtype, krylov=krylov)
    with torch.cuda.stream(stream):
        return solver_for(w, vcycle_dtype=vcycle_dtype, krylov=krylov)


def _timed(fn):
    import torch
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    out = fn()
    torch.cuda.synchronize()
    return out, time.perf_counter() - t0


def batched(args):
    import torch
    from . import Krylov, batch_solve
    from . import workloads as W
    from .autotune import autotune_group
    descs = W.batch_systems(count=args.batch_count)
    kr = Krylov(method="bicgstab", rtol=1e-8, maxit=20000)
    streams = [torch.cuda.Stream() for _ in range(max(1, args.batch_streams))]
    solvers, rhs = [], []
    for q, d in enumerate(descs):
        w = W.batch_inputs(d)
        solvers.append(_solver(w, args.batch_cycle, kr, streams[q % len(streams)]))
        rhs.append(torch.stack([torch.from_numpy(b).to("cuda") for b in w.rhs]))
    torch.cuda.synchronize()
    # one schedule per grid size, tuned for the throughput of concurrent
    # cycles (the systems of that size on their own streams)
    groups = {}
    for q, d in enumerate(descs):
        groups.setdefault((d["n"], args.batch_cycle), []).append(solvers[q])
    tuned = {key: autotune_group(group) for key, group in groups.items()}
    torch.cuda.synchronize()
    total = sum(int(b.shape[0]) for b in rhs)
    # the same batch with each system's right-hand sides one at a time (the
    # per-system launches serve one right-hand side each)
    batch_solve(solvers, rhs, kr, group=1)
    (_, stats1), secs1 = _timed(lambda: batch_solve(solvers, rhs, kr, group=1))
    batch_solve(solvers, rhs, kr)   # warm-up (also fills the graph caches)
    (xs, stats), secs = _timed(lambda: batch_solve(solvers, rhs, kr))
    ok = all(s["status"] == 0 for s in stats) and all(s["status"] == 0 for s in stats1)
    worst = max(s["rel_residual"] for s in stats)
    # the same work one call at a time (sequential solves, one stream)
    seq_sample = min(len(solvers), 12)
    (_, seq_secs) = _timed(lambda: [solvers[q].solve(rhs[q][r], krylov=kr)
                                    for q in range(seq_sample) for r in range(rhs[q].shape[0])])
    seq_total = sum(int(rhs[q].shape[0]) for q in range(seq_sample))
    by_size = {}
    for q, d in enumerate(descs):
        e = by_size.setdefault(d["n"], dict(systems=0, rhs=0, iterations=0))
        e["systems"] += 1
        e["rhs"] += int(rhs[q].shape[0])
        e["iterations"] += stats[q]["iterations"]
    _emit(dict(metric="batched ECS Helmholtz solves to 1e-8 (Bi-CGSTAB, QD V(1,1) RB-GS)", unit="solves/s",
               value=round(total / secs, 3), higher_is_better=True, systems=len(descs), right_hand_sides=total,
               seconds=round(secs, 3), all_converged=ok, worst_rel_residual=worst,
               one_rhs_at_a_time=dict(solves_per_s=round(total / secs1, 3), seconds=round(secs1, 3)),
               multi_rhs_speedup=round(secs1 / secs, 3),
               sequential_solves_per_s=round(seq_total / seq_secs, 3), sequential_sample_rhs=seq_total,
               speedup_vs_sequential=round((total / secs) / (seq_total / seq_secs), 3),
               tuning={f"{k[0]}_{k[1]}": v for k, v in tuned.items()}, by_size=by_size,
               dtype="f64" if args.batch_cycle == "f64" else "f32 cycle + f64 Krylov", data="synthetic"))


def adjoint(args):
    import torch
    from . import Krylov
    from . import workloads as W
    from .autograd import helmholtz_solve
    n = 1025
    w, k2_true, idx, rng = W.adjoint_case(n=n)
    fwd = Krylov(method="bicgstab", rtol=1e-8, maxit=20000)
    # the finite-difference check needs solves far below the FD step: 1e-12
    # by FGMRES (Bi-CGSTAB's true residual stalls just above 1e-13 here)
    tight = Krylov(method="fgmres", restart=40, rtol=1e-12, maxit=40000)
    S = _solver(w, "f64", tight)
    f = torch.from_numpy(w.rhs[0]).to("cuda")
    k2 = torch.from_numpy(w.k2).to("cuda")
    ii = torch.as_tensor(idx, device="cuda")
    from . import solver_for
    wt = W.Workload(w.name, 2, w.n, w.lo, w.hi, w.ecs, k2_true, w.rhs, w.precond, w.cycle, w.krylov, w.nlev)
    St = solver_for(wt, krylov=tight)
    ut, _ = St.solve(f)
    d = ut[ii][:, ii]
    del St

    def loss(k2v, kr):
        u = helmholtz_solve(S, k2v, f, krylov=kr, adjoint_krylov=kr)
        r = u[ii][:, ii] - d
        return 0.5 * (r.real ** 2 + r.imag ** 2).sum()

    kg = k2.clone().requires_grad_(True)
    L = loss(kg, fwd)
    torch.autograd.grad(loss(kg, fwd), kg)   # warm-up of both directions
    reps = [_timed(lambda: torch.autograd.grad(loss(kg, fwd), kg))[1] for _ in range(3)]
    t_fwd_bwd = float(np.median(reps))
    S.solve(f, krylov=fwd)
    t_fwd = float(np.median([_timed(lambda: S.solve(f, krylov=fwd))[1] for _ in range(3)]))
    kg = k2.clone().requires_grad_(True)
    (gt,) = torch.autograd.grad(loss(kg, tight), kg)
    gt = gt.cpu().numpy()
    x = W.real_nodes(n, -10.0, 10.0)
    inner = np.flatnonzero((np.abs(x) <= 8))
    # 50 random interior nodes (|x|, |y| <= 8) at eps = 1e-6; and 5 nodes
    # among those whose gradient is at least 1e-2 times the largest, at
    # eps = 1e-6 and 1e-3.  With gradients ~1e-7 and the loss known to ~1e-15 from
    # 1e-12 solves, eps = 1e-6 leaves ~1e-3 relative noise in the quotient;
    # eps = 1e-3 brings it below 1e-5 while the truncation error stays
    # O((eps / k^2)^2) ~ 1e-8
    rand_cells = [(int(rng.choice(inner)), int(rng.choice(inner))) for _ in range(50)]
    big = np.flatnonzero(np.abs(gt).ravel() >= 1e-2 * np.abs(gt).max())
    big_cells = [(int(t // n), int(t % n)) for t in rng.choice(big, size=5, replace=False)]
    gscale = float(np.abs(gt).max())

    def fd(j, i, eps):
        kp = k2.clone(); kp[j, i] += eps
        km = k2.clone(); km[j, i] -= eps
        return (float(loss(kp, tight)) - float(loss(km, tight))) / (2 * eps)

    with torch.no_grad():
        rand_err = [abs(fd(j, i, 1e-6) - gt[j, i]) / gscale for (j, i) in rand_cells]
        big = []
        for (j, i) in big_cells:
            f6, f3 = fd(j, i, 1e-6), fd(j, i, 1e-3)
            big.append(dict(cell=[j, i], grad=float(gt[j, i]), fd_1e6=f6, fd_1e3=f3,
                            err_1e6_rel=abs(f6 - gt[j, i]) / abs(gt[j, i]),
                            err_1e3_rel=abs(f3 - gt[j, i]) / abs(gt[j, i])))
    _emit(dict(metric="adjoint gradient of a 1025^2 ECS solve", unit="s", value=round(t_fwd_bwd, 4),
               higher_is_better=False, forward_seconds=round(t_fwd, 4),
               forward_plus_backward_seconds=round(t_fwd_bwd, 4), loss=float(L),
               fd_random_cells=len(rand_cells),
               fd_random_max_err_rel_to_max_grad=float(max(rand_err)),
               fd_random_median_err_rel_to_max_grad=float(np.median(rand_err)),
               fd_large_grad_max_err_eps1e3_rel=max(e["err_1e3_rel"] for e in big),
               fd_large_grad_cells=big, dtype="f64", data="synthetic"))


def cube(args):
    import torch
    from . import Krylov
    from . import workloads as W
    w = W.cube_constant_k(n=129, k=12.0)
    kr = Krylov(method="fgmres", restart=30, rtol=1e-8, maxit=5000)
    S = _solver(w, "f64", kr)
    f = torch.from_numpy(w.rhs[0]).to("cuda")
    S.solve(f)
    (x, st), secs = _timed(lambda: S.solve(f))
    # the same solve with the other Arnoldi variants
    others = {}
    for orth in ("cgs2_selective", "cgs1"):
        k1 = Krylov(method="fgmres", restart=30, rtol=1e-8, maxit=5000, orth=orth)
        S.solve(f, krylov=k1)
        (_, st1), secs1 = _timed(lambda: S.solve(f, krylov=k1))
        others[orth] = dict(seconds=round(secs1, 4), iterations=st1["iterations"],
                            second_passes=st1["reorthogonalisations"], rel_residual=st1["rel_residual"])
    _emit(dict(metric="3D 129^3 ECS Helmholtz solve to 1e-8 (k = 12, QD, V(1,1) RB-GS, FGMRES(30))", unit="s",
               value=round(secs, 4), higher_is_better=False, iterations=st["iterations"], vcycles=st["vcycles"],
               second_passes=st["reorthogonalisations"], rel_residual=st["rel_residual"], status=st["status"],
               other_arnoldi=others, dtype="f64", data="synthetic"))


def coulomb513(args):
    import torch
    from . import workloads as W
    rows = []
    for E_ in (0.5, 1.0, 2.0, 4.0):
        w = W.coulomb(E=E_, n=513)
        S = _solver(w, "f64")
        f = torch.from_numpy(w.rhs[0]).to("cuda")
        S.solve(f)
        (x, st), secs = _timed(lambda: S.solve(f))
        rows.append(dict(E=E_, seconds=round(secs, 4), iterations=st["iterations"], rel_residual=st["rel_residual"]))
    _emit(dict(metric="513^2 soft-Coulomb QD Bi-CGSTAB solves to 1e-8", unit="s",
               value=round(sum(r["seconds"] for r in rows), 4), higher_is_better=False, runs=rows, dtype="f64",
               data="synthetic"))


def small65(args):
    import torch
    from . import workloads as W
    rows = []
    for beta2 in (0.5, -0.5):
        w = W.small_constant_k(beta2=beta2)
        S = _solver(w, "f64")
        for q, b in enumerate(w.rhs):
            f = torch.from_numpy(b).to("cuda")
            S.solve(f)
            (x, st), secs = _timed(lambda: S.solve(f))
            rows.append(dict(beta2=beta2, rhs=["gaussian", "random"][q], seconds=round(secs, 5),
                             iterations=st["iterations"], rel_residual=st["rel_residual"]))
    _emit(dict(metric="65^2 constant-k CSL GMRES(30) solves to 1e-8", unit="s",
               value=round(sum(r["seconds"] for r in rows), 4), higher_is_better=False, runs=rows, dtype="f64",
               data="synthetic"))


def _standalone_mg(S, f, rtol=1e-6, maxcycles=200):
    """Stand-alone multigrid on M x = f from x = 0 (``ecs_mg_solve``).  Returns
    (cycles, average reduction per cycle over all cycles, geometric mean of the
    last 5 ratios, seconds, final reduction)."""
    S.mg_solve(f, rtol=rtol, maxcycles=maxcycles)
    (x, st, hist), secs = _timed(lambda: S.mg_solve(f, rtol=rtol, maxcycles=maxcycles))
    ratios = [hist[i + 1] / hist[i] for i in range(len(hist) - 1)]
    last = ratios[-5:]
    last5 = math.exp(sum(math.log(q) for q in last) / len(last)) if last else 0.0
    cycles = st["iterations"]
    conv = (hist[-1] / hist[0]) ** (1.0 / cycles) if cycles else 0.0
    return cycles, conv, last5, secs, hist[-1] / hist[0]


# Printed results of Tables 1-4 (Sec. 5), per set-up: mg-conv, # stand-alone
# cycles, Bi-CGSTAB iterations, Bi-CGSTAB cputime in seconds (the authors'
# machine; context only).
PAPER_TABLES = {
    ("T1 MP1 k=160", "csl"): (0.43, 17, 60, 131), ("T1 MP1 k=160", "csg"): (0.39, 15, 62, 122),
    ("T1 MP1 k=160", "qd"): (0.09, 6, 170, 339),
    ("T2 MP2 nu=7 k=4", "csl"): (0.53, 22, 137, 454), ("T2 MP2 nu=7 k=4", "csg"): (0.53, 22, 143, 456),
    ("T2 MP2 nu=7 k=4", "qd"): (0.15, 8, 357, 1180),
    ("T3 MP3 k=2", "csl"): (0.32, 13, 60, 189), ("T3 MP3 k=2", "csg"): (0.32, 13, 61, 190),
    ("T3 MP3 k=2", "qd"): (0.17, 8, 164, 540),
    ("T4 MP3 k=4", "csl"): (0.32, 13, 210, 1100), ("T4 MP3 k=4", "csg"): (0.31, 12, 160, 854),
    ("T4 MP3 k=4", "qd"): (0.13, 7, 545, 2800),
}


def paper_mp(args):
    import torch
    from . import Krylov, Precond, Solver
    from . import workloads as W
    tables = (("T1 MP1 k=160", W.paper_mp1), ("T2 MP2 nu=7 k=4", W.paper_mp2),
              ("T3 MP3 k=2", lambda: W.paper_mp3(2.0)), ("T4 MP3 k=4", lambda: W.paper_mp3(4.0, 75.0, 768)))
    rows = []
    total = 0.0
    for label, make in tables:
        w, setups = make()
        k2 = torch.from_numpy(w.k2).to("cuda")
        f = torch.from_numpy(w.rhs[0]).to("cuda")
        kr = Krylov(method="bicgstab", rtol=1e-6, maxit=5000)
        for name, p, cyc in setups:
            pc = Precond(kind=p["kind"], beta1=p.get("beta1", -1.0), beta2=p.get("beta2", -0.5),
                         theta_alpha=p.get("theta_alpha", math.pi / 13), re_lambda0=p.get("lam0", 0.0),
                         smoother=cyc["smoother"], omega=cyc["omega"], nu1=cyc["nu1"], nu2=cyc["nu2"],
                         gamma_f=cyc["gamma_f"], gamma_c=cyc["gamma_c"], coarsest_nodes=cyc["coarsest"],
                         vcycle_dtype="f64")
            S = Solver(w.dim, w.n, w.lo, w.hi, w.ecs, k2, pc, kr)
            cycles, conv, last5, mg_secs, red = _standalone_mg(S, f)
            S.solve(f)
            (x, st), secs = _timed(lambda: S.solve(f))
            total += secs

            # warm start (Sec. 5, MP1): the preconditioner's own solution to 1e-2 as the guess
            def warm():
                x0, st0, _ = S.mg_solve(f, rtol=1e-2, maxcycles=50)
                return S.solve(f, x0=x0), st0["iterations"]
            warm()
            ((_, stw), wcyc), wsecs = _timed(warm)
            rows.append(dict(table=label, grid=w.n[0], precond=name, cycle=f"F{cyc['gamma_f']}^{cyc['gamma_c']}"
                             if cyc["gamma_c"] > 1 else "V", smoother=cyc["smoother"], omega=cyc["omega"],
                             mg_conv=round(conv, 3), mg_conv_last5=round(last5, 3), mg_cycles=cycles, mg_seconds=round(mg_secs, 4),
                             mg_reduction=red, bicgstab_iterations=st["iterations"], vcycles=st["vcycles"],
                             seconds=round(secs, 4), rel_residual=st["rel_residual"], status=st["status_name"],
                             warm_mg_cycles=wcyc, warm_bicgstab_iterations=stw["iterations"],
                             warm_seconds=round(wsecs, 4),
                             paper=dict(zip(("mg_conv", "mg_cycles", "bicgstab_iterations", "seconds"),
                                            PAPER_TABLES[(label, name)]))))
            print(json.dumps(rows[-1]), flush=True)
            del S
    _emit(dict(metric="Sec. 5 model problems: Bi-CGSTAB solves to 1e-6, all 12 set-ups", unit="s",
               value=round(total, 4), higher_is_better=False, runs=rows, dtype="f64", data="synthetic"))


def coupled(args):
    import torch
    from . import Krylov, coupled_solve
    from . import workloads as W
    nb, n = 4, 513
    blocks, k2c, rhs = W.coupled_blocks(nb=nb, n=n)
    streams = [torch.cuda.Stream() for _ in range(nb)]
    solvers = [_solver(w, "f32", stream=streams[i]) for i, w in enumerate(blocks)]
    kc = torch.from_numpy(k2c).to("cuda")
    b = torch.from_numpy(rhs).to("cuda")
    outer = Krylov(method="fgmres", restart=30, rtol=1e-8, maxit=500)
    inner = Krylov(method="bicgstab", rtol=1e-3, maxit=100)
    outer_sel = Krylov(method="fgmres", restart=30, rtol=1e-8, maxit=500, orth="cgs2_selective")
    outer_cgs1 = Krylov(method="fgmres", restart=30, rtol=1e-8, maxit=500, orth="cgs1")
    rows = {}
    for mode in ("batched_bicgstab_1e-3", "one_cycle_per_block", "one_cycle_per_block_cgs2_selective",
                 "one_cycle_per_block_cgs1"):
        only = mode.startswith("one_cycle_per_block")
        ko = outer_cgs1 if mode.endswith("cgs1") else outer_sel if mode.endswith("selective") else outer
        coupled_solve(solvers, kc, b, outer=ko, inner=inner, cycles_only=only)
        (x, st), secs = _timed(lambda: coupled_solve(solvers, kc, b, outer=ko, inner=inner, cycles_only=only))
        rows[mode] = dict(seconds=round(secs, 4), outer_iterations=st["iterations"],
                          inner_iterations=st["inner_iterations"], vcycles=st["vcycles"],
                          second_passes=st.get("reorthogonalisations"), rel_residual=st["rel_residual"],
                          status=st["status_name"])
    best = min(r["seconds"] for m, r in rows.items() if not m.endswith(("cgs1", "selective")))
    _emit(dict(metric=f"coupled block system, {nb} channels on {n}^2, FGMRES(30) to 1e-8", unit="s", value=best,
               higher_is_better=False, runs=rows, dtype="f64 outer / f32 cycles", data="synthetic"))


def persistent_probe(args):
    import ctypes
    from . import lib
    L = lib()
    L.ecs_probe_item_sweeps.argtypes = [ctypes.c_int] * 4 + [ctypes.POINTER(ctypes.c_double)]
    L.ecs_probe_group_barrier.argtypes = [ctypes.c_int] * 3 + [ctypes.POINTER(ctypes.c_double)] * 2
    sweeps, rows = 4, []
    for n in (257, 513, 1025):
        for g in (1, 32, 256):
            ms = ctypes.c_double()
            rc = L.ecs_probe_item_sweeps(n, g, g, sweeps, ctypes.byref(ms))
            if rc != 0:
                raise RuntimeError(f"ecs_probe_item_sweeps({n}, {g}) returned {rc}")
            # per sweep and node: read u, b, k^2 once, write u once (56 B in FP64)
            gbs = g * n * n * 56.0 * sweeps / (ms.value * 1e-3) / 1e9
            rows.append(dict(n=n, workgroups=g, ms_per_sweep=round(ms.value / sweeps, 4), gbs=round(gbs, 1),
                             gbs_per_workgroup=round(gbs / g, 2)))
            print(f"item sweeps n={n} workgroups={g}: {gbs:.0f} GB/s", flush=True)
    bars = []
    for blocks in (8, 32, 64, 256):
        for nbytes in (0, 65536):
            ub, ul = ctypes.c_double(), ctypes.c_double()
            rc = L.ecs_probe_group_barrier(blocks, 2000, nbytes, ctypes.byref(ub), ctypes.byref(ul))
            if rc != 0:
                raise RuntimeError(f"ecs_probe_group_barrier({blocks}, {nbytes}) returned {rc}")
            bars.append(dict(workgroups=blocks, bytes_per_workgroup=nbytes, us_per_phase=round(ub.value, 3),
                             us_per_phase_local=round(ul.value, 3), barrier_us=round(ub.value - ul.value, 3)))
            print(f"group barrier {blocks} workgroups, {nbytes} B: {ub.value - ul.value:.2f} us", flush=True)
    _emit(dict(metric="persistent batched-solve organisations: one-workgroup-per-grid sweep rate and phase "
                      "barrier cost", unit="GB/s", value=max(r["gbs"] for r in rows), higher_is_better=True,
               item_sweeps=rows, group_barrier=bars, sweep_bytes_per_node=56, dtype="f64", data="synthetic"))


def run(args):
    {"batched": batched, "persistent_probe": persistent_probe, "adjoint": adjoint, "cube": cube, "coulomb513": coulomb513, "small65": small65,
     "paper_mp": paper_mp, "coupled": coupled}[args.config](args)
