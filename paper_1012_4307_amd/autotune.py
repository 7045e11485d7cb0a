"""Autotuner of the fused V(1,1) cycle's launch schedule.

It times the cycle under every candidate schedule -- tile heights of the
fused down / up kernels, the grid size below which short tiles are used, the
size below which levels run in the single-workgroup tail kernel, and the
size below which levels run two per kernel -- and keeps the fastest.  Two
objectives:

- ``autotune(solver)``: the latency of one cycle of one solver (HIP events),
  for single solves;
- ``autotune_group(solvers)``: the throughput of cycles of several systems of
  the same size, each on its own stream (wall clock around a device-wide
  synchronisation), for batched solves.  There the host issues the launches
  of all systems from one thread and the device overlaps them, so fewer,
  longer launches (two levels per kernel, taller tiles) that win for one
  cycle can lose.

Results are cached in a JSON file keyed by GPU architecture, grid, dtype and
objective (``$ECSMG_TUNING_CACHE``, default ``~/.cache/ecsmg/tuning.json``),
so a batch of systems of the same size pays the search once.  The schedule
does not change the method's arithmetic; which kernel kind runs a level can
change the rounding of the cycle (kernels order some floating-point operations
differently), so the objective is time per cycle, not time per solve.
"""
from __future__ import annotations

import itertools
import json
import os
import time
from typing import Dict

# fuse_updates does not change a cycle (only how a Bi-CGSTAB feeds it) and
# keeps its default
DEFAULT = dict(down_rows=4, up_rows=8, small_grid=513, tail_nodes=33, pair_grid=129, fuse_updates=1)


def cache_path() -> str:
    return os.environ.get("ECSMG_TUNING_CACHE", os.path.join(os.path.expanduser("~"), ".cache", "ecsmg",
                                                             "tuning.json"))


def _key(solver) -> str:
    import torch
    arch = torch.cuda.get_device_properties(solver.device).gcnArchName.split(":")[0]
    return f"{arch}|{solver.dim}d|{'x'.join(str(v) for v in solver.n)}|{solver.precond.vcycle_dtype}"


def candidates(dtype: str):
    downs = (2, 4, 6, 8, 16) if dtype == "f32" else (2, 4, 6, 8)
    tails = (17, 33, 65) if dtype == "f32" else (17, 33)   # FP32 cycles have a wide tail up to 65^2
    for d, u, sg, tn, pg in itertools.product(downs, (4, 8, 16), (257, 513), tails, (0, 129, 513)):
        yield dict(down_rows=d, up_rows=u, small_grid=sg, tail_nodes=tn, pair_grid=pg, fuse_updates=1)


def time_cycles(solver, v, reps: int = 10) -> float:
    """Mean milliseconds of one V-cycle: HIP events on the solver's own stream,
    where its cycles run (a solver made under another stream than the current
    one would otherwise be timed by events that bracket only the host's
    launches), on a preallocated output."""
    import torch
    from . import _ptr, lib
    L = lib()
    z = torch.empty_like(v)
    torch.cuda.synchronize()
    for _ in range(2):
        solver._check(L.ecs_vcycle(solver._h, _ptr(v), _ptr(z)))
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(solver.stream)
    for _ in range(reps):
        solver._check(L.ecs_vcycle(solver._h, _ptr(v), _ptr(z)))
    e1.record(solver.stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def _fused_schedule(solver) -> bool:
    """Only the fused 2D V(1,1) red-black cycle has a launch schedule."""
    p = solver.precond
    return solver.dim == 2 and p.smoother == "rbgs" and p.nu1 == 1 and p.nu2 == 1 and p.gamma_f == 1 \
        and p.gamma_c == 1


def _load_cache(path):
    if os.path.exists(path):
        try:
            with open(path) as f:
                return json.load(f)
        except (OSError, ValueError):
            pass
    return {}


def _search(apply, time_one, dtype, key, use_cache):
    """Time every candidate schedule (apply(cand), then time_one()), apply the
    fastest and cache it under `key`."""
    path = cache_path()
    cache = _load_cache(path) if use_cache else {}
    if use_cache and key in cache:
        best = cache[key]["tuning"]
        apply(best)
        return best
    results = []
    for cand in candidates(dtype):
        apply(cand)
        results.append((time_one(), cand))
    results.sort(key=lambda r: r[0])
    best_ms, best = results[0]
    apply(best)
    if use_cache:
        cache[key] = dict(tuning=best, cycle_ms=best_ms,
                          default_ms=next(ms for ms, c in results if c == DEFAULT) if DEFAULT in
                          [c for _, c in results] else None)
        os.makedirs(os.path.dirname(path), exist_ok=True)
        tmp = path + ".tmp"
        with open(tmp, "w") as f:
            json.dump(cache, f, indent=1, sort_keys=True)
        os.replace(tmp, path)
    return best


def autotune(solver, use_cache: bool = True, reps: int = 10) -> Dict[str, int]:
    """Pick and apply the schedule with the fastest single cycle of `solver`;
    returns it."""
    import torch
    if not _fused_schedule(solver):
        return solver.get_tuning()
    g = torch.Generator(device=solver.device).manual_seed(0)
    v = torch.randn(solver.shape, dtype=torch.complex128, device=solver.device, generator=g)
    return _search(lambda c: solver.set_tuning(**c), lambda: time_cycles(solver, v, reps),
                   solver.precond.vcycle_dtype, _key(solver), use_cache)


def time_group_cycles(solvers, vs, zs, reps: int = 3) -> float:
    """Wall-clock milliseconds per cycle when every solver of the group runs
    `reps` cycles, each on its own context's stream, issued round-robin from
    this thread."""
    import torch
    from . import _ptr, lib
    L = lib()

    def one_round():
        for S, v, z in zip(solvers, vs, zs):
            S._check(L.ecs_vcycle(S._h, _ptr(v), _ptr(z)))

    one_round()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        one_round()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) * 1e3 / (reps * len(solvers))


def autotune_group(solvers, use_cache: bool = True, reps: int = 3, max_group: int = 16) -> Dict[str, int]:
    """Pick the schedule with the highest cycle throughput over a group of
    solvers of one grid size and dtype (each with its own stream), apply it
    to all of them and return it.  At most `max_group` of them are timed."""
    import torch
    s0 = solvers[0]
    key = _key(s0)
    if any(_key(S) != key for S in solvers):
        raise ValueError("autotune_group: solvers differ in grid, dimension or cycle dtype")
    if not _fused_schedule(s0):
        return s0.get_tuning()
    timed = list(solvers[:max_group])
    g = torch.Generator(device=s0.device).manual_seed(0)
    vs = [torch.randn(S.shape, dtype=torch.complex128, device=S.device, generator=g) for S in timed]
    zs = [torch.empty_like(v) for v in vs]
    torch.cuda.synchronize()

    def apply(c):
        for S in solvers:
            S.set_tuning(**c)

    return _search(apply, lambda: time_group_cycles(timed, vs, zs, reps), s0.precond.vcycle_dtype,
                   key + f"|group{len(timed)}", use_cache)
