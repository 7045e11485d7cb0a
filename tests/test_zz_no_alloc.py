"""ecs_solve_static -- the solve for callers that cannot allocate device
memory -- against ecs_solve through the C ABI: two calls in a row on
different contexts (the second on a smaller grid, another Krylov method and
cycle dtype), each equal to the workspace-backed solve bit for bit, with
contexts whose workspace holds only the hierarchy; a solve whose Krylov
storage exceeds the static scratch is refused."""
import numpy as np
import pytest

from helpers import gpu_for, oracle_for, to_gpu, to_np
import paper_1012_4307_amd as E
from paper_1012_4307_amd import workloads as W

pytestmark = pytest.mark.gpu


def solver(w, dt, kr):
    import torch
    p, c = w.precond, w.cycle
    pc = E.Precond(kind=p["kind"], re_lambda0=p.get("lam0", 0.0), smoother=c["smoother"], omega=c["omega"],
                   nu1=c["nu1"], nu2=c["nu2"], gamma_f=c["gamma_f"], gamma_c=c["gamma_c"],
                   coarsest_nodes=c["coarsest"], vcycle_dtype=dt)
    k2 = torch.from_numpy(np.ascontiguousarray(w.k2)).to("cuda")
    return E.Solver(w.dim, w.n, w.lo, w.hi, w.ecs, k2, pc, kr, hierarchy_only=True)


def test_solve_static_equals_solve():
    import torch
    cases = [(W.coulomb(E=2.0, n=257), "f64", E.Krylov(method="bicgstab", rtol=1e-8, maxit=2000)),
             (W.large_coulomb(n=129, coarsest=9), "f32",
              E.Krylov(method="fgmres", restart=20, rtol=1e-10, maxit=2000, inner=4))]
    for w, dt, kr in cases:
        S = solver(w, dt, kr)
        ws_bytes = S.ws.numel()
        b = to_gpu(w.rhs[0])
        xs, sts = S.solve_static(b)
        torch.cuda.synchronize()
        assert S.ws.numel() == ws_bytes       # the workspace was not grown for the static call
        assert sts["status"] == 0, (w.name, sts)
        x, st = S.solve(b)                     # the workspace-backed solve (grows the workspace)
        assert (sts["iterations"], sts["inner_iterations"]) == (st["iterations"], st["inner_iterations"]), w.name
        assert torch.equal(xs, x), w.name
        P = oracle_for(w)
        bi = W._zero_boundary(w.rhs[0])
        res = np.linalg.norm(bi - P.apply(to_np(xs))) / np.linalg.norm(bi)
        assert res <= 1.05 * kr.rtol, (w.name, res)


def test_solve_static_rejects_oversize():
    w = W.coulomb(E=2.0, n=1025)
    S = solver(w, "f64", E.Krylov(method="bicgstab", rtol=1e-8, maxit=10))
    with pytest.raises(E.EcsError) as ei:
        S.solve_static(to_gpu(w.rhs[0]))
    assert ei.value.status == -2 and "MiB" in str(ei.value)
