"""Seeded synthetic workloads of the ECS Helmholtz solver.

This module only produces inputs -- node coordinates of the real grid, the
wavenumber field k^2 at those nodes, right-hand sides and solver settings --
for the model problems the solver is exercised on.  It contains none of the
method's arithmetic (no complex contour, stencil, smoother or Krylov step), so
both the GPU library and the CPU oracle can be fed from it with identical
bytes.

Workloads (sizes are nodes per axis including both Dirichlet end nodes):

* ``small_constant_k`` -- 65^2 nodes on [-1,1]^2 (h = 1/32), ECS layers from
  |x|, |y| = 0.75 at theta = pi/6 on all four sides, constant k = 8; unit
  Gaussian source (sigma = 0.05) and a seeded random complex RHS; CSL
  preconditioner -Lap - (1 - 0.5i) k^2 with V(1,1) omega-Jacobi (0.8), coarsest
  5x5, GMRES(30) to 1e-8.
* ``coulomb(E, n)`` -- soft-Coulomb wavenumber k^2 = 2(E + 1/sqrt(r^2+1)) on
  [-10,10]^2, ECS in the outer 20% (|x| > 8) at pi/6, RHS phi0 * V with the
  Gaussian ground state phi0 = pi^-1/2 exp(-r^2/2) and V = -1/sqrt(r^2+1);
  QD preconditioner, V(1,1) red-black Gauss-Seidel.
* ``large_coulomb(n, h)`` -- the same operator family at k h ~ 0.5: h = 0.25,
  domain [-(n-1)h/2, (n-1)h/2]^2, ECS beyond 80% of the half width, E = 2;
  at n = 2049 this is the 2049^2 mixed-precision benchmark grid.
* ``batch_systems()`` -- the 96-system batch: grids {257, 513, 1025}^2,
  E ~ U[0.5, 4], theta in {pi/8, pi/6, pi/4}, 1-8 random complex RHS each.
* ``adjoint_case(n)`` -- soft-Coulomb E = 2 on [-10,10]^2 with a 64x64
  sampling sub-grid and data from a +5% Gaussian bump of k^2.
* ``cube_constant_k(n)`` -- 3D [-1,1]^3, ECS from 0.75 at pi/6, k = 12,
  Gaussian source.
* ``coupled_blocks(nb, n)`` -- a coupled block system of the kind Sec. 2
  derives from the partial-wave expansion: nb soft-Coulomb channels on
  [-10,10]^2 (ECS from 8 at pi/6) with thresholds, k^2_ii = 2(E - eps_i +
  1/sqrt(r^2+1)), eps_i = 0.5 i, coupled by short-range symmetric potentials
  k^2_ij = 2 c_ij exp(-r^2/2), c_ij ~ U[0.1, 0.3] (seeded); the entrance
  channel 0 is driven by phi0 V, the others start empty.
* ``paper_mp1`` / ``paper_mp2`` / ``paper_mp3`` -- the model problems of
  Sec. 5 with the grids of Tables 1-4: MP1 (-Lap - k^2, k = 160, unit
  source at the centre node, interior [0,1]^2 with 64-cell layers on all
  four sides); MP2 (k^2 = 16 + 7 (exp(-x^2) + exp(-y^2)), [0,50]^2 with
  128-cell layers on the east and north sides, Dirichlet at x = 0 and y = 0);
  MP3 (k^2 = k0^2 + 1/x + 1/y on [0,50]^2 or [0,75]^2, same layers).  The
  sources of MP2/MP3 are exp(-(x^2 + y^2)).  Each comes with the three
  preconditioner set-ups of its table (CSL, CSG, QD).
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Tuple

import numpy as np

SEED_RANDOM_RHS = 1012
SEED_BATCH = 20101012
SEED_ADJOINT = 4307
SEED_COUPLED = 1012430


@dataclasses.dataclass
class Workload:
    name: str
    dim: int
    n: Tuple[int, ...]                 # nodes per axis (x first)
    lo: Tuple[float, ...]
    hi: Tuple[float, ...]
    # per axis: (lo_side, hi_side), each None (plain Dirichlet) or (layer start, theta)
    ecs: Tuple[Tuple[Optional[Tuple[float, float]], Optional[Tuple[float, float]]], ...]
    k2: np.ndarray                     # float64, shape reversed(n)
    rhs: List[np.ndarray]              # complex128, shape reversed(n)
    precond: dict                      # kind + parameters
    cycle: dict                        # smoother, omega, nu1, nu2, gamma_f, gamma_c, coarsest
    krylov: dict                       # method, m, rtol, maxit
    nlev: int = 0                      # multigrid levels (finest = 0)

    @property
    def shape(self):
        return tuple(reversed(self.n))

    @property
    def nodes(self):
        return int(np.prod(self.n))


def real_nodes(n: int, lo: float, hi: float) -> np.ndarray:
    """Real node coordinates x_i = lo + i (hi - lo)/(n - 1), i = 0..n-1."""
    return lo + np.arange(n, dtype=np.float64) * ((hi - lo) / (n - 1))


def levels_to(n: int, coarsest: int) -> int:
    """Number of levels when halving n-1 until n == coarsest."""
    lev = 1
    while n > coarsest:
        if (n - 1) % 2:
            raise ValueError(f"{n} nodes cannot be coarsened to {coarsest}")
        n = (n - 1) // 2 + 1
        lev += 1
    if n != coarsest:
        raise ValueError("coarsest size not reachable")
    return lev


def _grid2(n, lo, hi):
    x = real_nodes(n, lo, hi)
    X, Y = np.meshgrid(x, x, indexing="xy")   # shape (ny, nx), x fastest
    return X, Y


def _zero_boundary(v: np.ndarray) -> np.ndarray:
    v = v.copy()
    if v.ndim == 2:
        v[0, :] = v[-1, :] = 0
        v[:, 0] = v[:, -1] = 0
    else:
        v[0] = v[-1] = 0
        v[:, 0] = v[:, -1] = 0
        v[:, :, 0] = v[:, :, -1] = 0
    return v


def random_complex(shape, rng: np.random.Generator, dtype=np.complex128) -> np.ndarray:
    v = rng.standard_normal(shape) + 1j * rng.standard_normal(shape)
    return _zero_boundary(v.astype(dtype))


def soft_coulomb_k2(X, Y, E, Z=1.0):
    return 2.0 * (E + Z / np.sqrt(X * X + Y * Y + 1.0))


def ground_state_source(X, Y):
    r2 = X * X + Y * Y
    phi0 = np.exp(-0.5 * r2) / math.sqrt(math.pi)
    V = -1.0 / np.sqrt(r2 + 1.0)
    return _zero_boundary((phi0 * V).astype(np.complex128))


def small_constant_k(n: int = 65, beta2: float = 0.5) -> Workload:
    lo, hi = -1.0, 1.0
    X, Y = _grid2(n, lo, hi)
    k = 8.0
    k2 = np.full((n, n), k * k)
    sig = 0.05
    f1 = _zero_boundary(np.exp(-(X * X + Y * Y) / (2 * sig * sig)).astype(np.complex128))
    rng = np.random.default_rng(SEED_RANDOM_RHS)
    f2 = random_complex((n, n), rng)
    th = math.pi / 6
    side = ((-0.75, th), (0.75, th))
    # -Lap - (1 - 0.5 i) k^2 = -Lap + (b1 + i b2) k^2 with b1 = -1, b2 = +0.5
    return Workload("small_constant_k", 2, (n, n), (lo, lo), (hi, hi), (side, side), k2, [f1, f2],
                    dict(kind="csl", beta1=-1.0, beta2=beta2),
                    dict(smoother="jacobi", omega=0.8, nu1=1, nu2=1, gamma_f=1, gamma_c=1, coarsest=5),
                    dict(method="gmres", m=30, rtol=1e-8, maxit=2000), levels_to(n, 5))


def coulomb(E: float = 1.0, n: int = 513, L: float = 10.0, theta: float = math.pi / 6,
            coarsest: int = 5, method: str = "bicgstab") -> Workload:
    lo, hi = -L, L
    X, Y = _grid2(n, lo, hi)
    k2 = soft_coulomb_k2(X, Y, E)
    f = ground_state_source(X, Y)
    s = 0.8 * L
    side = ((-s, theta), (s, theta))
    return Workload(f"coulomb_E{E:g}_n{n}", 2, (n, n), (lo, lo), (hi, hi), (side, side), k2, [f],
                    dict(kind="qd", lam0=0.0),
                    dict(smoother="rbgs", omega=1.0, nu1=1, nu2=1, gamma_f=1, gamma_c=1, coarsest=coarsest),
                    dict(method=method, m=40, rtol=1e-8, maxit=5000), levels_to(n, coarsest))


def large_coulomb(n: int = 2049, h: float = 0.25, E: float = 2.0, coarsest: int = 9,
                  method: str = "fgmres", m: int = 40) -> Workload:
    half = 0.5 * (n - 1) * h
    w = coulomb(E=E, n=n, L=half, coarsest=coarsest, method=method)
    w.name = f"large_coulomb_n{n}_h{h:g}"
    w.krylov = dict(method=method, m=m, rtol=1e-8, maxit=20000)
    return w


def batch_systems(count: int = 96, sizes=(257, 513, 1025), seed: int = SEED_BATCH):
    """System descriptions of the batched workload (inputs are generated lazily
    by ``batch_inputs`` so that a caller can scale the batch down)."""
    rng = np.random.default_rng(seed)
    thetas = (math.pi / 8, math.pi / 6, math.pi / 4)
    out = []
    for s in range(count):
        n = sizes[s % len(sizes)]
        E = float(rng.uniform(0.5, 4.0))
        th = thetas[(s // 3) % 3]
        nrhs = int(rng.integers(1, 9))
        rhs_f32 = (s % 2 == 0)
        out.append(dict(index=s, n=n, E=E, theta=th, nrhs=nrhs, rhs_f32=rhs_f32, rhs_seed=int(rng.integers(0, 2**31 - 1))))
    return out


def batch_inputs(desc: dict) -> Workload:
    w = coulomb(E=desc["E"], n=desc["n"], theta=desc["theta"], method="bicgstab")
    rng = np.random.default_rng(desc["rhs_seed"])
    rhs = []
    for _ in range(desc["nrhs"]):
        v = random_complex(w.shape, rng)
        if desc["rhs_f32"]:
            v = v.astype(np.complex64).astype(np.complex128)   # an FP32 RHS upcast exactly
        rhs.append(v)
    w.rhs = rhs
    w.name = f"batch{desc['index']}"
    return w


def adjoint_case(n: int = 1025, E: float = 2.0, seed: int = SEED_ADJOINT):
    """Returns (workload at the unperturbed k^2, k^2_true, sampler (rows, cols))."""
    w = coulomb(E=E, n=n, method="bicgstab")
    X, Y = _grid2(n, -10.0, 10.0)
    rng = np.random.default_rng(seed)
    cx, cy = rng.uniform(-4.0, 4.0, size=2)
    bump = np.exp(-((X - cx) ** 2 + (Y - cy) ** 2) / (2 * 1.0 ** 2))
    k2_true = w.k2 * (1.0 + 0.05 * bump)
    # 64 x 64 sampling nodes covering the same physical patch at every size
    # (fewer on grids too coarse to hold 64 distinct nodes there)
    count = min(64, (n - 1) // 2)
    s = max(1, (n - 1) // 128)
    i0 = (n - 1) // 4
    idx = i0 + s * np.arange(count)
    fd_rng = np.random.default_rng(seed)
    w.name = f"adjoint_n{n}"
    return w, k2_true, idx, fd_rng


def cube_constant_k(n: int = 129, k: float = 12.0, coarsest: int = 5) -> Workload:
    lo, hi = -1.0, 1.0
    x = real_nodes(n, lo, hi)
    Z, Y, X = np.meshgrid(x, x, x, indexing="ij")   # shape (nz, ny, nx)
    k2 = np.full((n, n, n), k * k)
    sig = 0.05
    f = _zero_boundary(np.exp(-(X * X + Y * Y + Z * Z) / (2 * sig * sig)).astype(np.complex128))
    th = math.pi / 6
    side = ((-0.75, th), (0.75, th))
    return Workload(f"cube_n{n}", 3, (n, n, n), (lo,) * 3, (hi,) * 3, (side, side, side), k2, [f],
                    dict(kind="qd", lam0=0.0),
                    dict(smoother="rbgs", omega=1.0, nu1=1, nu2=1, gamma_f=1, gamma_c=1, coarsest=coarsest),
                    dict(method="fgmres", m=30, rtol=1e-8, maxit=3000), levels_to(n, coarsest))


# ------------------------------------------------------------------ Sec. 5
def _paper_grid(n_int: int, n_layer: int, L: float, sides: str):
    """Nodes of an interior [0, L] split into n_int cells plus n_layer cells of
    the same width in each ECS layer (sides 'both': layers below 0 and above L;
    'hi': above L only)."""
    h = L / n_int
    lo = -n_layer * h if sides == "both" else 0.0
    n = n_int + (2 if sides == "both" else 1) * n_layer + 1
    return n, lo, lo + (n - 1) * h


def _coarsest(n: int) -> int:
    """Coarsest grid reached by halving n - 1 down to its odd part (>= 3 nodes)."""
    m = n - 1
    while m % 2 == 0 and m > 2:
        m //= 2
    return m + 1


def _paper_setups(csl, csg, qd, cyc_csl, cyc_csg, om_jac, om_rb, coarsest):
    """The three preconditioners of one table: (name, precond, cycle)."""
    def jac(gc):
        return dict(smoother="jacobi", omega=om_jac, nu1=1, nu2=1, gamma_f=1, gamma_c=gc, coarsest=coarsest)
    return [("csl", dict(kind="csl", beta1=csl[0], beta2=csl[1]), jac(cyc_csl)),
            ("csg", dict(kind="csg", theta_alpha=csg), jac(cyc_csg)),
            ("qd", dict(kind="qd", lam0=qd),
             dict(smoother="rbgs", omega=om_rb, nu1=1, nu2=1, gamma_f=1, gamma_c=1, coarsest=coarsest))]


def _paper_workload(name, n, lo, hi, side, k2, f, coarsest):
    return Workload(name, 2, (n, n), (lo, lo), (hi, hi), (side, side), k2, [f],
                    dict(kind="qd", lam0=0.0),
                    dict(smoother="rbgs", omega=1.0, nu1=1, nu2=1, gamma_f=1, gamma_c=1, coarsest=coarsest),
                    dict(method="bicgstab", rtol=1e-6, maxit=5000), levels_to(n, coarsest))


def paper_mp1(k: float = 160.0, n_int: int = 256, n_layer: int = 64):
    """MP1 of Table 1: -Lap - k^2 on the interior [0,1]^2 with ECS layers on
    all four sides and a unit value at the centre node as the source."""
    n, lo, hi = _paper_grid(n_int, n_layer, 1.0, "both")
    th = math.pi / 6
    k2 = np.full((n, n), k * k)
    f = np.zeros((n, n), np.complex128)
    f[n // 2, n // 2] = 1.0
    c = _coarsest(n)
    w = _paper_workload("paper_mp1", n, lo, hi, ((0.0, th), (1.0, th)), k2, f, c)
    return w, _paper_setups((-1.0, -0.3), math.pi / 14, -2.6e4, 4, 3, 0.8, 1.0, c)


def _paper_mp23(k2_of, L, n_int, n_layer, name):
    n, lo, hi = _paper_grid(n_int, n_layer, L, "hi")
    X, Y = _grid2(n, lo, hi)
    k2 = k2_of(X, Y)
    f = _zero_boundary(np.exp(-(X * X + Y * Y)).astype(np.complex128))
    return _paper_workload(name, n, lo, hi, (None, (L, math.pi / 6)), k2, f, _coarsest(n))


def paper_mp2(nu: float = 7.0, k: float = 4.0, L: float = 50.0, n_int: int = 512, n_layer: int = 128):
    """MP2 of Table 2: k^2(x, y) = k^2 + nu (exp(-x^2) + exp(-y^2)) on the
    interior [0, L]^2, ECS layers on the east and north sides."""
    w = _paper_mp23(lambda X, Y: k * k + nu * (np.exp(-X * X) + np.exp(-Y * Y)), L, n_int, n_layer, "paper_mp2")
    return w, _paper_setups((-1.0, -0.4), math.pi / 17, -16.88, 3, 3, 0.5, 1.0, w.cycle["coarsest"])


def paper_mp3(k: float = 2.0, L: float = 50.0, n_int: int = 512, n_layer: int = 128):
    """MP3 of Tables 3 (k = 2, [0,50]^2) and 4 (k = 4, [0,75]^2):
    k^2(x, y) = k^2 + 1/x + 1/y (the Dirichlet nodes x = 0, y = 0 carry 0)."""
    def k2_of(X, Y):
        with np.errstate(divide="ignore"):
            v = k * k + 1.0 / X + 1.0 / Y
        v[~np.isfinite(v)] = 0.0
        return v
    w = _paper_mp23(k2_of, L, n_int, n_layer, f"paper_mp3_k{k:g}")
    c = w.cycle["coarsest"]
    if k == 2.0:
        return w, _paper_setups((-1.0, -0.6), math.pi / 13, -4.19, 2, 2, 0.8, 1.05, c)
    return w, _paper_setups((-1.0, -0.6), math.pi / 13, -16.18, 4, 3, 0.8, 1.05, c)


# ------------------------------------------------------------ coupled blocks
def coupled_blocks(nb: int = 4, n: int = 257, E: float = 2.0, L: float = 10.0, coarsest: int = 5,
                   seed: int = SEED_COUPLED):
    """(blocks, k2c, rhs): nb channel workloads (QD, V(1,1) red-black), the
    coupling potentials k2c[i, j] (nb x nb x shape, symmetric, zero diagonal)
    and the stacked right-hand side (nb x shape)."""
    rng = np.random.default_rng(seed)
    X, Y = _grid2(n, -L, L)
    r2 = X * X + Y * Y
    blocks = []
    for i in range(nb):
        w = coulomb(E=E - 0.5 * i, n=n, L=L, coarsest=coarsest)
        w.name = f"channel{i}"
        blocks.append(w)
    c = rng.uniform(0.1, 0.3, size=(nb, nb))
    c = np.triu(c, 1)
    c = c + c.T
    g = np.exp(-r2 / 2.0)
    k2c = np.zeros((nb, nb) + X.shape)
    for i in range(nb):
        for j in range(nb):
            if i != j:
                k2c[i, j] = 2.0 * c[i, j] * g
    rhs = np.zeros((nb,) + X.shape, np.complex128)
    rhs[0] = blocks[0].rhs[0]
    return blocks, k2c, rhs
