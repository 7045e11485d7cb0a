"""GPU parity of every step of the multigrid-preconditioned solve against the
FP64 CPU oracle, element by element, through the C ABI.

Tolerances: the FP64 path differs from the oracle only by rounding order,
so single steps must agree to 1e-13 (relative to the largest entry) and a
whole cycle to 1e-12; the FP32 cycle must agree to 1e-5 per step and 2e-4 per
cycle (a few FP32 ulps amplified by the coarse-level solves)."""
import math

import numpy as np
import pytest

from helpers import gpu_for, oracle_for, ragged_workload, relerr, to_gpu, to_np
from paper_1012_4307_amd import workloads as W

pytestmark = pytest.mark.gpu

TOL = {"f64": 1e-13, "f32": 1e-5}
CYCLE_TOL = {"f64": 1e-12, "f32": 2e-4}


def cases():
    c1 = W.small_constant_k()
    c2 = W.coulomb(E=2.0, n=129)
    rg = ragged_workload()
    return {"small_constant_k": c1, "coulomb129": c2, "ragged97": rg}


CASES = cases()


@pytest.fixture(scope="module", params=list(CASES))
def case(request):
    return CASES[request.param]


@pytest.mark.parametrize("dt", ["f64", "f32"])
def test_operator_apply(case, dt):
    w = case
    P = oracle_for(w)
    S = gpu_for(w, dt)
    rng = np.random.default_rng(5)
    x = W.random_complex(w.shape, rng)
    for op in ("A", "M", "AT"):
        y = to_np(S.apply(to_gpu(x), op))
        assert relerr(y, P.apply(x, which=op)) < 1e-13, op
        assert np.all(y[0] == 0) and np.all(y[:, -1] == 0)


@pytest.mark.parametrize("dt", ["f64", "f32"])
def test_smoother_sweep(case, dt):
    w = case
    P = oracle_for(w)
    S = gpu_for(w, dt)
    cdt = np.complex64 if dt == "f32" else np.complex128
    rng = np.random.default_rng(6)
    for level in (0, 1):
        shape = S.level_shape(level)
        b = W.random_complex(shape, rng)
        u = W.random_complex(shape, rng)
        if dt == "f32":
            b = b.astype(cdt).astype(np.complex128)
            u = u.astype(cdt).astype(np.complex128)
        for ns in (1, 2):
            got = to_np(S.smooth(to_gpu(b.astype(cdt)), to_gpu(u.astype(cdt)), level, ns))
            ref = P.smooth(b, u, level, w.cycle["smoother"], w.cycle["omega"], ns)
            assert relerr(got, ref) < TOL[dt] * (10 if dt == "f32" else 1), (level, ns)


@pytest.mark.parametrize("dt", ["f64", "f32"])
def test_residual_restrict_and_prolong(case, dt):
    w = case
    P = oracle_for(w)
    S = gpu_for(w, dt)
    cdt = np.complex64 if dt == "f32" else np.complex128
    rng = np.random.default_rng(7)
    for level in range(S.nlev - 1):
        shape = S.level_shape(level)
        b = W.random_complex(shape, rng).astype(cdt).astype(np.complex128)
        u = W.random_complex(shape, rng).astype(cdt).astype(np.complex128)
        rc = to_np(S.residual_restrict(to_gpu(b.astype(cdt)), to_gpu(u.astype(cdt)), level))
        ref = P.restrict(P.residual(b, u, level), level)
        assert relerr(rc, ref) < TOL[dt] * (10 if dt == "f32" else 1), level
        ec = W.random_complex(S.level_shape(level + 1), rng).astype(cdt).astype(np.complex128)
        up = to_np(S.prolong_correct(to_gpu(ec.astype(cdt)), to_gpu(u.astype(cdt)), level))
        assert relerr(up, P.prolong_add(ec, u, level)) < TOL[dt], level


@pytest.mark.parametrize("dt", ["f64", "f32"])
def test_coarse_solve(case, dt):
    w = case
    P = oracle_for(w)
    S = gpu_for(w, dt)
    cdt = np.complex64 if dt == "f32" else np.complex128
    rng = np.random.default_rng(8)
    b = W.random_complex(S.level_shape(S.nlev - 1), rng).astype(cdt).astype(np.complex128)
    x = to_np(S.coarse_solve(to_gpu(b.astype(cdt))))
    assert relerr(x, P.coarse_solve(b)) < (1e-12 if dt == "f64" else 1e-5)


@pytest.mark.parametrize("dt", ["f64", "f32"])
def test_vcycle(case, dt):
    w = case
    P = oracle_for(w)
    S = gpu_for(w, dt)
    rng = np.random.default_rng(9)
    for v in (w.rhs[0], W.random_complex(w.shape, rng)):
        z = to_np(S.vcycle(to_gpu(v)))
        assert relerr(z, P.mg_apply(v)) < CYCLE_TOL[dt]


@pytest.mark.parametrize("dt", ["f64", "f32"])
def test_vcycle_native_dtype(dt):
    """The cycle on vectors in its own dtype (no conversion passes) equals the
    oracle's cycle of the same right-hand side."""
    import torch
    w = W.coulomb(E=2.0, n=257)
    P = oracle_for(w)
    S = gpu_for(w, dt)
    v = W.random_complex(w.shape, np.random.default_rng(14))
    vd = to_gpu(v).to(torch.complex64 if dt == "f32" else torch.complex128)
    z = S.vcycle_native(vd)
    assert z.dtype == vd.dtype
    ref = P.mg_apply(to_np(vd).astype(np.complex128))
    assert relerr(to_np(z).astype(np.complex128), ref) < CYCLE_TOL[dt]


@pytest.mark.parametrize("dt", ["f64", "f32"])
def test_vcycle_tail_schedules(dt):
    """The single-workgroup tail over every admissible range of coarse levels:
    the whole cycle (33^2 grid), the dense solve alone, and coarsest grids of
    9, 4, 225 and 49 unknowns (64, 64, 4 and 16 threads per row of the dense
    solve), against the oracle's cycle.  FP32 cycles also run the wide tail:
    from a 65^2 level, the whole cycle of a 65^2 grid, and from a ragged 49^2
    level."""
    rng = np.random.default_rng(12)
    runs = [(W.coulomb(E=1.0, n=33), (33, 17, 9, 5, 3)),
            (ragged_workload(), (3, 4, 7, 13, 25)),
            (ragged_workload(n=129, coarsest=17), (17, 33)),
            (W.coulomb(E=2.0, n=129, coarsest=9), (9, 17, 33))]
    if dt == "f32":
        runs += [(W.coulomb(E=2.0, n=257, coarsest=9), (65,)), (W.coulomb(E=1.0, n=65, coarsest=9), (65,)),
                 (ragged_workload(n=193, coarsest=7), (49, 65))]
    for w, tails in runs:
        P = oracle_for(w)
        S = gpu_for(w, dt)
        for v in (w.rhs[0], W.random_complex(w.shape, rng)):
            ref = P.mg_apply(v)
            for tn in tails:
                S.set_tuning(tail_nodes=tn)
                assert relerr(to_np(S.vcycle(to_gpu(v))), ref) < CYCLE_TOL[dt], (w.name, w.n, tn)


@pytest.mark.parametrize("dt", ["f64", "f32"])
def test_vcycle_two_level_kernels(dt):
    """Levels run two per kernel (down: levels l, l+1 in one block with the
    intermediate right-hand side in LDS; up: levels l+1, l): every pairing
    the schedule allows -- none, only the smallest levels, all levels above
    the tail, an odd count with a single level on top -- against the oracle."""
    rng = np.random.default_rng(13)
    runs = [(W.coulomb(E=2.0, n=257), (0, 33, 65, 129, 257)),
            (ragged_workload(n=193, coarsest=7), (0, 25, 49, 97, 193)),
            (W.coulomb(E=1.0, n=65), (0, 65))]
    for w, pgs in runs:
        P = oracle_for(w)
        S = gpu_for(w, dt)
        v = W.random_complex(w.shape, rng)
        ref = P.mg_apply(v)
        for pg in pgs:
            for tn in (9, 33):
                S.set_tuning(tail_nodes=tn, pair_grid=pg)
                assert relerr(to_np(S.vcycle(to_gpu(v))), ref) < CYCLE_TOL[dt], (w.name, w.n, pg, tn)


@pytest.mark.parametrize("dt", ["f64", "f32"])
def test_vcycle_tile_heights(dt):
    """Every tile height of the fused down and up kernels (coarse rows per
    block 2..6, 8, and 16 in FP32; fine rows 4..32), applied on every level
    above the tail of a ragged grid, against the oracle's cycle."""
    w = ragged_workload(n=193, coarsest=7)
    P = oracle_for(w)
    S = gpu_for(w, dt)
    v = W.random_complex(w.shape, np.random.default_rng(16))
    ref = P.mg_apply(v)
    downs = (2, 3, 4, 5, 6, 8) + ((16,) if dt == "f32" else ())
    for d in downs:
        for u in (4, 8, 10, 12, 16, 32):
            S.set_tuning(down_rows=d, up_rows=u, small_grid=3, tail_nodes=33, pair_grid=0)
            assert relerr(to_np(S.vcycle(to_gpu(v))), ref) < CYCLE_TOL[dt], (d, u)


@pytest.mark.parametrize("gf,gc,smoother,omega,nu", [(2, 2, "rbgs", 1.05, 1), (1, 2, "jacobi", 0.8, 1),
                                                      (1, 4, "jacobi", 0.5, 2), (1, 1, "rbgs", 1.0, 2)])
def test_general_cycles(gf, gc, smoother, omega, nu):
    """Algorithm 1 with other cycle indices (W, F, F_1^4) and sweep counts."""
    w = W.coulomb(E=1.0, n=129)
    cyc = dict(smoother=smoother, omega=omega, nu1=nu, nu2=nu, gamma_f=gf, gamma_c=gc, coarsest=5)
    for prec in (dict(kind="qd", lam0=0.0), dict(kind="csl", beta1=-1.0, beta2=-0.5),
                 dict(kind="csg", theta_alpha=math.pi / 13)):
        P = oracle_for(w, prec=prec, cycle=cyc)
        S = gpu_for(w, "f64", prec=prec, cycle=cyc)
        z = to_np(S.vcycle(to_gpu(w.rhs[0])))
        assert relerr(z, P.mg_apply(w.rhs[0])) < 1e-12, (prec["kind"], gf, gc)


@pytest.mark.parametrize("dt", ["f64", "f32"])
@pytest.mark.parametrize("gf,gc,smoother,omega,nu1,nu2", [(1, 4, "jacobi", 0.8, 1, 1), (1, 3, "jacobi", 0.5, 2, 1),
                                                          (2, 2, "rbgs", 1.05, 0, 2), (1, 2, "rbgs", 1.0, 1, 0),
                                                          (2, 3, "jacobi", 0.8, 1, 2)])
def test_general_cycle_tail(dt, gf, gc, smoother, omega, nu1, nu2):
    """General cycles whose coarse end runs as one single-workgroup schedule:
    every tail start (none, the last levels, the whole hierarchy), unequal
    and zero sweep counts, against the oracle; the captured cycle replays the
    eager one bit for bit."""
    import torch
    rng = np.random.default_rng(15)
    cyc = dict(smoother=smoother, omega=omega, nu1=nu1, nu2=nu2, gamma_f=gf, gamma_c=gc)
    runs = [(ragged_workload(n=97, coarsest=4), 4, (3, 7, 13, 25, 33)),
            (W.paper_mp2(L=6.25, n_int=64, n_layer=16)[0], 6, (3, 11, 21, 33)),
            (W.coulomb(E=1.0, n=33), 5, (9, 33))]
    for w, c, tails in runs:
        cy = dict(cyc, coarsest=c)
        prec = dict(kind="csl", beta1=-1.0, beta2=-0.5)
        P = oracle_for(w, prec=prec, cycle=cy)
        S = gpu_for(w, dt, prec=prec, cycle=cy)
        v = W.random_complex(w.shape, rng)
        ref = P.mg_apply(v)
        for tn in tails:
            S.set_tuning(tail_nodes=tn)
            S.set_graphs(False)
            ze = S.vcycle(to_gpu(v))
            assert relerr(to_np(ze), ref) < (1e-12 if dt == "f64" else CYCLE_TOL[dt]), (w.name, tn)
            S.set_graphs(True)
            for _ in range(3):
                zg = S.vcycle(to_gpu(v))
                torch.cuda.synchronize()
                assert torch.equal(zg, ze), (w.name, tn)


def test_3d_steps_and_cycle():
    w = W.cube_constant_k(n=33, k=6.0)
    P = oracle_for(w)
    S = gpu_for(w, "f64")
    rng = np.random.default_rng(10)
    x = W.random_complex(w.shape, rng)
    for op in ("A", "M", "AT"):
        assert relerr(to_np(S.apply(to_gpu(x), op)), P.apply(x, which=op)) < 1e-13
    b = W.random_complex(w.shape, rng)
    assert relerr(to_np(S.smooth(to_gpu(b), to_gpu(x))), P.smooth(b, x)) < 1e-13
    rc = to_np(S.residual_restrict(to_gpu(b), to_gpu(x)))
    assert relerr(rc, P.restrict(P.residual(b, x))) < 1e-13
    ec = W.random_complex(S.level_shape(1), rng)
    assert relerr(to_np(S.prolong_correct(to_gpu(ec), to_gpu(x))), P.prolong_add(ec, x)) < 1e-13
    assert relerr(to_np(S.vcycle(to_gpu(b))), P.mg_apply(b)) < 1e-12
    S32 = gpu_for(w, "f32")
    assert relerr(to_np(S32.vcycle(to_gpu(b))), P.mg_apply(b)) < 2e-4


@pytest.mark.parametrize("n,coarsest", [(97, 4), (65, 5)])
def test_3d_steps_and_cycle_wide(n, coarsest):
    """3D grids wider than one 64-node x-tile of the 3D kernels (97^3 ragged,
    unsymmetric layers, random k^2; 65^3 one node over the tile): every step
    and one cycle (both dtypes) against the oracle."""
    w = ragged_workload(n=n, coarsest=coarsest, dim=3, seed=33)
    P = oracle_for(w)
    S = gpu_for(w, "f64")
    rng = np.random.default_rng(11)
    x = W.random_complex(w.shape, rng)
    for op in ("A", "M", "AT"):
        y = to_np(S.apply(to_gpu(x), op))
        assert relerr(y, P.apply(x, which=op)) < 1e-13, op
        assert np.all(y[0] == 0) and np.all(y[:, :, -1] == 0)
    b = W.random_complex(w.shape, rng)
    assert relerr(to_np(S.smooth(to_gpu(b), to_gpu(x))), P.smooth(b, x)) < 1e-13
    rc = to_np(S.residual_restrict(to_gpu(b), to_gpu(x)))
    assert relerr(rc, P.restrict(P.residual(b, x))) < 1e-13
    ec = W.random_complex(S.level_shape(1), rng)
    assert relerr(to_np(S.prolong_correct(to_gpu(ec), to_gpu(x))), P.prolong_add(ec, x)) < 1e-13
    ref = P.mg_apply(b)
    assert relerr(to_np(S.vcycle(to_gpu(b))), ref) < 1e-12
    S32 = gpu_for(w, "f32")
    assert relerr(to_np(S32.vcycle(to_gpu(b))), ref) < 2e-4


def test_full_size_vcycle_sampled():
    """The benchmark grid (2049^2, h = 0.25, 9 levels): one FP64 cycle checked
    against the oracle on the whole grid (one oracle cycle takes seconds)."""
    w = W.large_coulomb(n=2049)
    P = oracle_for(w)
    S = gpu_for(w, "f64")
    z = to_np(S.vcycle(to_gpu(w.rhs[0])))
    assert relerr(z, P.mg_apply(w.rhs[0])) < 1e-12
    S32 = gpu_for(w, "f32")
    z32 = to_np(S32.vcycle(to_gpu(w.rhs[0])))
    assert relerr(z32, P.mg_apply(w.rhs[0])) < 2e-4


def test_vcycle_graph_replay_matches_eager():
    """The captured cycle graph, replayed several times with other eager work
    and synchronisations in between, reproduces the eager cycle bit for bit
    (both dtypes)."""
    import torch
    w = W.coulomb(E=2.0, n=257)
    for dt in ("f64", "f32"):
        S = gpu_for(w, dt)
        v = to_gpu(w.rhs[0])
        S.set_graphs(False)
        ref = S.vcycle(v)
        S.set_graphs(True)
        x = to_gpu(W.random_complex(w.shape, np.random.default_rng(3)))
        for r in range(4):
            z = S.vcycle(v)
            torch.cuda.synchronize()
            y = S.apply(x, "A")
            torch.cuda.synchronize()
            assert torch.equal(z, ref), (dt, r)
        assert torch.isfinite(y.abs()).all()
        # the default mode launches this fused cycle eagerly
        S.set_graphs("auto")
        assert torch.equal(S.vcycle(v), ref), dt


def test_sampled_timing_and_launch_mode_arguments():
    """Kernel timing of one launch in `every` (the 1st, (every+1)-th, ...):
    ten cycles timed one in four give three timed fine-level down launches,
    all with the same algorithmic bytes; launch modes outside
    never/always/auto and negative timing arguments are rejected."""
    import torch
    import paper_1012_4307_amd as E
    w = W.coulomb(E=2.0, n=257)
    S = gpu_for(w, "f32")
    v = to_gpu(w.rhs[0]).to(torch.complex64)
    S.timing("down", True, every=4)
    for _ in range(10):
        S.vcycle_native(v)
    n, ms, by = S.timing_read("down")
    S.timing("down", False)
    assert n == 3 and ms > 0, (n, ms)
    assert by == pytest.approx(3 * 257 * 257 * 4 * 3.5)  # read b, k^2; write the coarse quarter
    S.timing("down", True)
    for _ in range(5):
        S.vcycle_native(v)
    n, _, _ = S.timing_read("down")
    S.timing("down", False)
    assert n == 5
    assert E.lib().ecs_set_graphs(S._h, 3) == -1
    assert E.lib().ecs_timing_enable(S._h, 7, -1) == -1
    with pytest.raises(ValueError):
        S.timing("down", True, every=0)
