"""Autotuner of the fused V(1,1) cycle's launch schedule.

For one solver (grid size, dimension, cycle dtype) it times the cycle under
every candidate schedule -- tile heights of the fused down / up kernels, the
grid size below which short tiles are used, the size below which levels run
in the single-workgroup tail kernel, and the size below which levels run two
per kernel -- and keeps the fastest.  Results
are cached in a JSON file keyed by GPU architecture, grid and dtype
(``$ECSMG_TUNING_CACHE``, default ``~/.cache/ecsmg/tuning.json``), so a
batch of systems of the same size pays the search once.  The schedule only
changes performance: the arithmetic of every node is the same.
"""
from __future__ import annotations

import itertools
import json
import os
from typing import Dict

# fuse_updates does not change a cycle (only how the nested FP32 Bi-CGSTAB
# feeds it) and keeps its default
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
    for d, u, sg, tn, pg in itertools.product(downs, (4, 8, 16), (257, 513), (17, 33), (0, 129, 513)):
        yield dict(down_rows=d, up_rows=u, small_grid=sg, tail_nodes=tn, pair_grid=pg, fuse_updates=1)


def time_cycles(solver, v, reps: int = 10) -> float:
    """Mean milliseconds of one V-cycle (HIP events on the current stream)."""
    import torch
    for _ in range(2):
        solver.vcycle(v)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        solver.vcycle(v)
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def autotune(solver, use_cache: bool = True, reps: int = 10) -> Dict[str, int]:
    """Pick and apply the fastest schedule for `solver`; returns it."""
    import torch
    if solver.dim != 2 or solver.precond.smoother != "rbgs" or solver.precond.nu1 != 1 or solver.precond.nu2 != 1 \
            or solver.precond.gamma_f != 1 or solver.precond.gamma_c != 1:
        return solver.get_tuning()   # only the fused V(1,1) red-black cycle has a schedule
    key = _key(solver)
    path = cache_path()
    cache = {}
    if use_cache and os.path.exists(path):
        try:
            with open(path) as f:
                cache = json.load(f)
        except (OSError, ValueError):
            cache = {}
    if use_cache and key in cache:
        best = cache[key]["tuning"]
        solver.set_tuning(**best)
        return best
    g = torch.Generator(device=solver.device).manual_seed(0)
    v = torch.randn(solver.shape, dtype=torch.complex128, device=solver.device, generator=g)
    results = []
    for cand in candidates(solver.precond.vcycle_dtype):
        solver.set_tuning(**cand)
        results.append((time_cycles(solver, v, reps), cand))
    results.sort(key=lambda r: r[0])
    best_ms, best = results[0]
    solver.set_tuning(**best)
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
