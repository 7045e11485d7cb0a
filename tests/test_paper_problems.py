"""The model problems of Sec. 5 (Tables 1-4): grids and sources of the
synthetic inputs, the stand-alone multigrid iteration used to report mg-conv,
and GPU parity on reduced-size versions of MP1 and MP2 with the tables'
CSL / CSG / QD set-ups (F cycles with omega-Jacobi, V(1,1) red-black)."""
import json
import math
import os

import numpy as np
import pytest

from helpers import gpu_for, oracle_for, relerr, to_gpu, to_np
from paper_1012_4307_amd import workloads as W


def test_paper_grids():
    """Cell counts of the table captions: MP1 256 interior + 64 per side on all
    four sides over [0,1]; MP2/MP3 512 (768) interior cells of [0,50] ([0,75])
    plus 128 layer cells on the east and north sides."""
    w1, _ = W.paper_mp1()
    assert w1.n == (385, 385) and w1.lo == (-0.25, -0.25) and w1.hi == (1.25, 1.25)
    assert w1.ecs[0] == ((0.0, math.pi / 6), (1.0, math.pi / 6)) and w1.ecs[1] == w1.ecs[0]
    x = W.real_nodes(385, -0.25, 1.25)
    assert x[64] == 0.0 and abs(x[320] - 1.0) < 1e-15 and abs(x[1] - x[0] - 1 / 256) < 1e-15
    w2, _ = W.paper_mp2()
    assert w2.n == (641, 641) and w2.lo == (0.0, 0.0) and w2.hi == (62.5, 62.5)
    assert w2.ecs[0] == (None, (50.0, math.pi / 6))
    w4, _ = W.paper_mp3(4.0, 75.0, 768)
    assert w4.n == (897, 897) and w4.hi == (87.5, 87.5)
    for w, c in ((w1, 4), (w2, 6), (w4, 8)):
        assert w.cycle["coarsest"] == c and w.nlev == 8
        assert (w.n[0] - 1) == (c - 1) * 2 ** (w.nlev - 1)


def test_paper_sources_and_wavenumbers():
    w1, s1 = W.paper_mp1()
    f = w1.rhs[0]
    assert f[192, 192] == 1.0 and np.count_nonzero(f) == 1
    assert np.all(w1.k2 == 160.0 ** 2)
    w2, _ = W.paper_mp2()
    assert w2.k2[0, 0] == 16.0 + 14.0               # k^2 + nu (1 + 1) at the origin
    assert abs(w2.k2[-1, -1] - 16.0) < 1e-12        # the Gaussians vanish far out
    assert np.all(np.abs(w2.rhs[0][0, :]) == 0) and np.all(np.abs(w2.rhs[0][:, -1]) == 0)
    assert abs(w2.rhs[0][1, 1] - math.exp(-2 * (50 / 512) ** 2)) < 1e-15
    w3, s3 = W.paper_mp3(2.0)
    assert np.all(np.isfinite(w3.k2))
    h = 50 / 512
    assert abs(w3.k2[3, 5] - (4.0 + 1 / (5 * h) + 1 / (3 * h))) < 1e-12
    # table parameters
    names = [s[0] for s in s1]
    assert names == ["csl", "csg", "qd"]
    assert s1[0][2]["gamma_c"] == 4 and s1[1][2]["gamma_c"] == 3 and s1[2][2]["gamma_c"] == 1
    assert s3[2][1]["lam0"] == -4.19 and s3[2][2]["omega"] == 1.05


def test_qd_uses_magnitude_of_re_lambda0():
    """Sec. 5 prints Re(lambda0) < 0 while the QD operator divides by its
    magnitude: both signs give the same operator."""
    w, _ = W.paper_mp2(L=6.25, n_int=64, n_layer=16)
    P = oracle_for(w, prec=dict(kind="qd", lam0=-16.88))
    Q = oracle_for(w, prec=dict(kind="qd", lam0=16.88))
    rng = np.random.default_rng(3)
    v = W.random_complex(w.shape, rng)
    assert np.array_equal(P.apply(v, which="M"), Q.apply(v, which="M"))
    assert P.lam0 == 16.88


PROBLEMS = {
    "mp1": W.paper_mp1,
    "mp2": W.paper_mp2,
    "mp3k2": lambda: W.paper_mp3(2.0),
    "mp3k4": lambda: W.paper_mp3(4.0, 75.0, 768),
}


def standalone_mg(step, apply_m, f, rtol=1e-6, maxcycles=60):
    """x_{m+1} = x_m + MG(f - M x_m) from x_0 = 0 until ||f - M x|| <= rtol ||f||;
    returns the residual norms (interior nodes; the boundary of f is zero)."""
    x = np.zeros_like(f)
    hist = [np.linalg.norm(f)]
    while len(hist) <= maxcycles and hist[-1] > rtol * hist[0]:
        x = x + step(W._zero_boundary(f - apply_m(x)))
        hist.append(np.linalg.norm(W._zero_boundary(f - apply_m(x))))
    return np.array(hist)


def test_tables_standalone_multigrid():
    """The oracle's operators and Algorithm 1 on the full-size model problems
    with each table row's cycle set-up: the number of stand-alone cycles to a
    1e-6 residual reduction equals the printed # cycles in all 12 rows, and
    the average reduction per cycle, (||r_N|| / ||r_0||)^(1/N), is within
    0.01 of the printed mg-conv.  (The geometric mean of only the last 5 ratios
    runs 0.03-0.05 above the printed CSL/CSG factors; the mean over all
    cycles is the figure that reproduces the tables.)"""
    with open(os.path.join(os.path.dirname(__file__), "golden", "sec5_tables.json")) as fh:
        rows = json.load(fh)["rows"]
    built = {}
    for row in rows:
        if row["problem"] not in built:
            built[row["problem"]] = PROBLEMS[row["problem"]]()
        w, setups = built[row["problem"]]
        _, p, c = next(s for s in setups if s[0] == row["precond"])
        P = oracle_for(w, prec=p, cycle=c)
        h = standalone_mg(P.mg_apply, lambda x: P.apply(x, which="M"), w.rhs[0])
        cycles = len(h) - 1
        conv = (h[-1] / h[0]) ** (1.0 / cycles)
        assert cycles == row["cycles"], (row, cycles)
        assert abs(conv - row["mg_conv"]) <= 0.01, (row, conv)


def _reduced_mp1():
    """MP1 on 32 + 2 x 8 cells at k = 20 (k h as in Table 1 up to a factor 0.6),
    with Re(lambda0) scaled like the table's -2.6e4 ~ -k^2."""
    w, setups = W.paper_mp1(k=20.0, n_int=32, n_layer=8)
    setups[2][1]["lam0"] = -400.0
    return w, setups


REDUCED = {
    "mp1": _reduced_mp1,
    "mp2": lambda: W.paper_mp2(L=6.25, n_int=64, n_layer=16),
}


@pytest.mark.parametrize("prob", sorted(REDUCED))
@pytest.mark.parametrize("which", [0, 1, 2])
def test_cycle_with_guess_is_correction(prob, which):
    """The stand-alone multigrid iteration is run as x += MG(f - M x) with the
    zero-guess cycle: Algorithm 1 is linear in (b, u), so a cycle started from
    u equals u plus the zero-guess cycle of the residual.  Checked on the
    oracle for every set-up (omega-Jacobi F cycles and red-black V cycles)."""
    w, setups = REDUCED[prob]()
    _, p, c = setups[which]
    P = oracle_for(w, prec=p, cycle=c)
    rng = np.random.default_rng(11)
    u = W.random_complex(w.shape, rng)
    b = w.rhs[0]
    lhs = P.mg_cycle(b, u)
    r = b - P.apply(u, which="M")
    r = W._zero_boundary(r)
    rhs = u + P.mg_apply(r)
    assert relerr(lhs, rhs) < 1e-12


def _history(step, apply_m, f, cycles):
    x = np.zeros_like(f)
    hist = [np.linalg.norm(f)]
    for _ in range(cycles):
        x = x + step(W._zero_boundary(f - apply_m(x)))
        hist.append(np.linalg.norm(W._zero_boundary(f - apply_m(x))))
    return np.array(hist), x


@pytest.mark.gpu
@pytest.mark.parametrize("prob", sorted(REDUCED))
@pytest.mark.parametrize("which", [0, 1, 2])
def test_paper_setups_match_oracle(prob, which):
    """Reduced MP1 / MP2 with each table set-up: 8 stand-alone cycles (residual
    history and iterate) and the Bi-CGSTAB solution against the oracle."""
    import paper_1012_4307_amd as E
    w, setups = REDUCED[prob]()
    name, p, c = setups[which]
    P = oracle_for(w, prec=p, cycle=c)
    S = gpu_for(w, "f64", prec=p, cycle=c, krylov=E.Krylov(method="bicgstab", rtol=1e-11, maxit=3000))
    f = w.rhs[0]
    ho, xo = _history(P.mg_apply, lambda x: P.apply(x, which="M"), f, 8)
    xg, stg, hg = S.mg_solve(to_gpu(f), rtol=0.0, maxcycles=8)
    assert stg["iterations"] == 8 and stg["status_name"] == "not_converged", stg
    print(prob, name, "oracle factors", ho[1:] / ho[:-1])
    # relative agreement, down to the rounding floor of a residual norm (~1e-16 ||f|| times the operator's size)
    assert np.all(np.abs(hg * ho[0] - ho) <= 1e-9 * ho + 1e-14 * ho[0])
    assert relerr(to_np(xg), xo) < 1e-10
    # started from a guess (no cycle): the residual of the oracle's 8th iterate
    xg3, _, hg3 = S.mg_solve(to_gpu(f), x0=to_gpu(xo), rtol=0.0, maxcycles=0)
    assert abs(hg3[0] * ho[0] - ho[-1]) <= 1e-9 * ho[-1] + 1e-12 * ho[0]
    x, st = S.solve(to_gpu(f))
    assert st["status"] == 0, st
    xs, _ = P.solve(f, "fgmres", 30, 1e-13, 5000)
    assert relerr(to_np(x), xs) < 1e-8


@pytest.mark.gpu
def test_tables_on_gpu():
    """Full-size model problems on the GPU with every table row's set-up: the
    stand-alone cycle count equals the printed # cycles, and right
    preconditioned Bi-CGSTAB reaches 1e-6 within 15% of the printed iteration
    count (the Bi-CGSTAB variant and its stopping norm are not printed, so
    counts are compared loosely)."""
    import paper_1012_4307_amd as E
    with open(os.path.join(os.path.dirname(__file__), "golden", "sec5_tables.json")) as fh:
        rows = json.load(fh)["rows"]
    built = {}
    for row in rows:
        if row["problem"] not in built:
            built[row["problem"]] = PROBLEMS[row["problem"]]()
        w, setups = built[row["problem"]]
        _, p, c = next(s for s in setups if s[0] == row["precond"])
        S = gpu_for(w, "f64", prec=p, cycle=c, krylov=E.Krylov(method="bicgstab", rtol=1e-6, maxit=2000))
        f = to_gpu(w.rhs[0])
        _, stm, h = S.mg_solve(f, rtol=1e-6, maxcycles=60)
        x, st = S.solve(f)
        print(row, "gpu cycles", stm["iterations"], "gpu iterations", st["iterations"], flush=True)
        assert stm["status"] == 0 and stm["iterations"] == row["cycles"] == len(h) - 1, (row, stm)
        assert abs((h[-1] / h[0]) ** (1.0 / len(h[1:])) - row["mg_conv"]) <= 0.01, row
        assert st["status"] == 0 and abs(st["iterations"] - row["bicgstab"]) <= 0.15 * row["bicgstab"], (row, st)
        del S


@pytest.mark.gpu
def test_warm_start_from_preconditioner_solution():
    """Sec. 5 (MP1) feeds the preconditioner's solution at 1e-2 to the Krylov
    method as its initial guess: the stand-alone solve stops at the first
    cycle below 1e-2, and Bi-CGSTAB from that guess meets the tolerance.  For
    CSL (M close to A in scale) the guess does not cost iterations; the saving
    of 50 iterations that Sec. 5 reports is not reproduced (counts stay within
    a few iterations, see the bench), so only the mechanism is asserted."""
    import paper_1012_4307_amd as E
    w, setups = W.paper_mp1()
    for which in (0, 2):
        _, p, c = setups[which]
        S = gpu_for(w, "f64", prec=p, cycle=c, krylov=E.Krylov(method="bicgstab", rtol=1e-6, maxit=2000))
        f = to_gpu(w.rhs[0])
        _, cold = S.solve(f)
        x0, st0, h0 = S.mg_solve(f, rtol=1e-2, maxcycles=50)
        assert st0["status"] == 0 and h0[-1] <= 1e-2 < h0[-2]
        x, warm = S.solve(f, x0=x0)
        print(p["kind"], "cold", cold["iterations"], "warm", warm["iterations"], "mg cycles", st0["iterations"])
        assert warm["status"] == 0 and warm["rel_residual"] <= 1.05e-6
        if p["kind"] == "csl":
            assert warm["iterations"] <= cold["iterations"] + 3


@pytest.mark.gpu
@pytest.mark.parametrize("which", [0, 2])
def test_warm_start_matches_oracle(which):
    """Sec. 5's warm start on MP1 (CSL F-cycle and QD V-cycle set-ups of
    Table 1) against the oracle doing the same: the stand-alone multigrid
    iterate at 1e-2 (oracle: its own cycles from zero), then Bi-CGSTAB from
    that guess.  The guesses agree to rounding, and so do the warm-started
    solutions, both driven well below the table's tolerance."""
    import paper_1012_4307_amd as E
    w, setups = W.paper_mp1()
    _, p, c = setups[which]
    P = oracle_for(w, prec=p, cycle=c)
    f = w.rhs[0]
    step = P.mg_apply
    x0o = np.zeros_like(f)
    h = [np.linalg.norm(f)]
    while h[-1] > 1e-2 * h[0]:
        x0o = x0o + step(W._zero_boundary(f - P.apply(x0o, which="M")))
        h.append(np.linalg.norm(W._zero_boundary(f - P.apply(x0o, which="M"))))
    S = gpu_for(w, "f64", prec=p, cycle=c, krylov=E.Krylov(method="bicgstab", rtol=1e-10, maxit=5000))
    x0g, st0, hg = S.mg_solve(to_gpu(f), rtol=1e-2, maxcycles=50)
    assert st0["status"] == 0 and st0["iterations"] == len(h) - 1, (st0, len(h) - 1)
    assert relerr(to_np(x0g), x0o) < 1e-10
    x, st = S.solve(to_gpu(f), x0=x0g)
    assert st["status"] == 0, st
    xo, sto = P.solve(f, "bicgstab", rtol=1e-12, maxit=20000, x0=x0o)
    assert sto["status"] == 0, sto
    err = relerr(to_np(x), xo)
    print(p["kind"], "guess cycles", len(h) - 1, "warm iterations gpu", st["iterations"], "oracle",
          sto["iterations"], "relerr", err, flush=True)
    assert err <= 1e-8

