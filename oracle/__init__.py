"""Plain FP64 CPU oracle for the ECS Helmholtz solve -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  The product library never loads it, and
it shares no code with the GPU path: the C source ``ecs_oracle.c`` restates
the method of bin Zubair, Reps and Vanroose (Sec. 3.1-3.2 discretisation,
Sec. 4 preconditioners and Algorithm 1, Sec. 5 Krylov outer solvers) as plain
loops.  This module marshals numpy arrays through ctypes, and assembles the
coupled block system of Sec. 2 densely from the per-block operators for small
grids (``coupled_dense``).

Arrays are numpy ``complex128`` (vectors) or ``float64`` (k^2), C-contiguous,
shaped ``(n1, n0)`` in 2D and ``(n2, n1, n0)`` in 3D (x fastest).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "ecs_oracle.c")
_LIB = os.path.join(_HERE, "libecs_oracle.so")
_lib = None

KIND = {"A": 0, "none": 0, "laplace": 1, "csl": 2, "csg": 3, "qd": 4}
SMOOTHER = {"jacobi": 0, "rbgs": 1}
KRYLOV = {"gmres": 0, "fgmres": 1, "bicgstab": 2}
WHICH = {"A": 0, "M": 1, "AT": 2}


def build() -> str:
    """Compile the oracle with gcc (C11, OpenMP).  Returns the library path."""
    cmd = ["gcc", "-std=c11", "-O2", "-fopenmp", "-fPIC", "-shared", "-o", _LIB + ".tmp", _SRC, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(_LIB + ".tmp", _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB):
        build()
    lib = ctypes.CDLL(_LIB)
    P = ctypes.c_void_p
    D = ctypes.c_double
    Ii = ctypes.c_int
    lib.ora_zmap.argtypes = [Ii, D, D, Ii, D, D, Ii, D, D, P]
    lib.ora_zmap.restype = None
    lib.ora_create.argtypes = [Ii, P, P, P, P, P, Ii]
    lib.ora_create.restype = P
    lib.ora_destroy.argtypes = [P]
    lib.ora_set_operator.argtypes = [P, Ii, D, D]
    lib.ora_set_operator.restype = D
    lib.ora_set_cycle.argtypes = [P, Ii, D, Ii, Ii, Ii, Ii]
    lib.ora_mg_apply.argtypes = [P, P, P]
    lib.ora_mg_cycle.argtypes = [P, P, P]
    lib.ora_get_visits.argtypes = [P, P]
    lib.ora_reset_visits.argtypes = [P]
    lib.ora_apply.argtypes = [P, Ii, Ii, P, P]
    lib.ora_residual.argtypes = [P, Ii, P, P, P]
    lib.ora_smooth.argtypes = [P, Ii, Ii, D, Ii, P, P]
    lib.ora_restrict.argtypes = [P, Ii, P, P]
    lib.ora_prolong_add.argtypes = [P, Ii, P, P]
    lib.ora_coarse_solve.argtypes = [P, P, P]
    lib.ora_level_nodes.argtypes = [P, Ii, P]
    lib.ora_level_nodes.restype = Ii
    lib.ora_weights.argtypes = [P, Ii, Ii, P, P, P]
    lib.ora_get_k2.argtypes = [P, Ii, P]
    lib.ora_solve.argtypes = [P, Ii, Ii, Ii, Ii, D, Ii, P, P, P]
    lib.ora_solve.restype = Ii
    lib.ora_num_threads.restype = Ii
    lib.ora_set_threads.argtypes = [Ii]
    lib.ora_set_threads.restype = None
    _lib = lib
    return lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def num_threads() -> int:
    return int(_load().ora_num_threads())


def set_threads(n: int) -> None:
    """Threads of the oracle's parallel loops (timing only)."""
    _load().ora_set_threads(int(n))


def zmap(n: int, lo: float, hi: float, ecs_lo=None, ecs_hi=None) -> np.ndarray:
    """Complex node coordinates of one axis (Sec. 3.1).

    ``ecs_lo`` / ``ecs_hi`` are ``None`` (Dirichlet end, no layer) or a pair
    ``(start, theta)``: beyond ``start`` the contour is rotated by ``theta``.
    """
    out = np.zeros(2 * n, dtype=np.float64)
    fl, sl, tl = (1, ecs_lo[0], ecs_lo[1]) if ecs_lo else (0, 0.0, 0.0)
    fh, sh, th = (1, ecs_hi[0], ecs_hi[1]) if ecs_hi else (0, 0.0, 0.0)
    _load().ora_zmap(int(n), float(lo), float(hi), fl, float(sl), float(tl), fh, float(sh), float(th), _ptr(out))
    return out[0::2] + 1j * out[1::2]


class Problem:
    """A discretised ECS Helmholtz problem with its multigrid hierarchy.

    dim      2 or 3
    n        nodes per axis including both boundary nodes (tuple of dim ints)
    lo, hi   real interval per axis
    ecs      per axis a pair (lo_side, hi_side), each None or (start, theta)
    k2       float64 array of k^2 at the real node coordinates
    nlev     number of multigrid levels (finest = 0)
    """

    def __init__(self, dim, n, lo, hi, ecs, k2, nlev):
        lib = _load()
        self.dim = int(dim)
        self.n = tuple(int(v) for v in n)
        self.shape = tuple(reversed(self.n))
        self.z = []
        for a in range(self.dim):
            elo, ehi = ecs[a]
            self.z.append(zmap(self.n[a], lo[a], hi[a], elo, ehi))
        zs = [np.ascontiguousarray(np.stack([z.real, z.imag], axis=1).ravel()) for z in self.z]
        while len(zs) < 3:
            zs.append(np.zeros(2, dtype=np.float64))
        self._zs = zs
        k2 = np.ascontiguousarray(k2, dtype=np.float64)
        assert k2.shape == self.shape, (k2.shape, self.shape)
        narr = np.array(list(self.n) + [1] * (3 - self.dim), dtype=np.int32)
        self._h = lib.ora_create(self.dim, _ptr(narr), _ptr(zs[0]), _ptr(zs[1]), _ptr(zs[2]), _ptr(k2), int(nlev))
        if not self._h:
            raise ValueError("oracle: bad hierarchy request")
        self.nlev = int(nlev)
        self.lam0 = 0.0

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            _load().ora_destroy(h)
            self._h = None

    # -- configuration --------------------------------------------------
    def set_operator(self, kind: str, p1: float = 0.0, p2: float = 0.0) -> float:
        """Preconditioner operator (Sec. 5): 'A', 'laplace', 'csl' (p1=b1, p2=b2),
        'csg' (p1=theta_alpha), 'qd' (p1=Re lambda0, its magnitude is used; 0 means max k^2)."""
        self.lam0 = float(_load().ora_set_operator(self._h, KIND[kind], float(p1), float(p2)))
        return self.lam0

    def set_cycle(self, smoother="rbgs", omega=1.0, nu1=1, nu2=1, gamma_f=1, gamma_c=1):
        _load().ora_set_cycle(self._h, SMOOTHER[smoother], float(omega), int(nu1), int(nu2), int(gamma_f), int(gamma_c))

    # -- helpers --------------------------------------------------------
    def level_shape(self, level: int):
        out = np.zeros(3, dtype=np.int32)
        if _load().ora_level_nodes(self._h, int(level), _ptr(out)) != 0:
            raise IndexError(level)
        return tuple(int(v) for v in reversed(out[: self.dim]))

    def _vec(self, x, level=0):
        x = np.ascontiguousarray(x, dtype=np.complex128)
        assert x.shape == self.level_shape(level), (x.shape, self.level_shape(level))
        return x

    def zeros(self, level=0):
        return np.zeros(self.level_shape(level), dtype=np.complex128)

    def weights(self, level: int, axis: int):
        n = self.level_shape(level)[self.dim - 1 - axis]
        am = np.zeros(2 * n); ap = np.zeros(2 * n); w = np.zeros(2 * n)
        _load().ora_weights(self._h, int(level), int(axis), _ptr(am), _ptr(ap), _ptr(w))
        c = lambda v: v[0::2] + 1j * v[1::2]
        return c(am), c(ap), c(w)

    def k2(self, level: int):
        out = np.zeros(self.level_shape(level), dtype=np.float64)
        _load().ora_get_k2(self._h, int(level), _ptr(out))
        return out

    # -- per-step operations -------------------------------------------
    def apply(self, x, level=0, which="A"):
        x = self._vec(x, level)
        y = self.zeros(level)
        _load().ora_apply(self._h, int(level), WHICH[which], _ptr(x), _ptr(y))
        return y

    def residual(self, b, u, level=0):
        b = self._vec(b, level); u = self._vec(u, level)
        r = self.zeros(level)
        _load().ora_residual(self._h, int(level), _ptr(b), _ptr(u), _ptr(r))
        return r

    def smooth(self, b, u, level=0, smoother="rbgs", omega=1.0, nsweeps=1):
        b = self._vec(b, level)
        u = self._vec(u, level).copy()
        _load().ora_smooth(self._h, int(level), SMOOTHER[smoother], float(omega), int(nsweeps), _ptr(b), _ptr(u))
        return u

    def restrict(self, rf, level=0):
        rf = self._vec(rf, level)
        rc = self.zeros(level + 1)
        _load().ora_restrict(self._h, int(level), _ptr(rf), _ptr(rc))
        return rc

    def prolong_add(self, ec, uf, level=0):
        ec = self._vec(ec, level + 1)
        uf = self._vec(uf, level).copy()
        _load().ora_prolong_add(self._h, int(level), _ptr(ec), _ptr(uf))
        return uf

    def coarse_solve(self, b):
        b = self._vec(b, self.nlev - 1)
        x = self.zeros(self.nlev - 1)
        _load().ora_coarse_solve(self._h, _ptr(b), _ptr(x))
        return x

    def mg_apply(self, v):
        """z = MG(0, M_0, v, 0, ...): one preconditioner application from zero."""
        v = self._vec(v)
        z = self.zeros()
        _load().ora_mg_apply(self._h, _ptr(v), _ptr(z))
        return z

    def mg_cycle(self, b, u):
        b = self._vec(b); u = self._vec(u).copy()
        _load().ora_mg_cycle(self._h, _ptr(b), _ptr(u))
        return u

    def visits(self):
        out = np.zeros(self.nlev, dtype=np.int64)
        _load().ora_get_visits(self._h, _ptr(out))
        return out

    def reset_visits(self):
        _load().ora_reset_visits(self._h)

    def solve(self, b, krylov="gmres", m=30, rtol=1e-8, maxit=2000, precond=True, transpose=False, x0=None):
        """Solve A x = b (or A^T x = b) on the finest grid; returns (x, stats)."""
        b = self._vec(b)
        x = self.zeros() if x0 is None else self._vec(x0).copy()
        st = np.zeros(5, dtype=np.float64)
        _load().ora_solve(self._h, 2 if transpose else 0, KRYLOV[krylov], 1 if precond else 0, int(m),
                          float(rtol), int(maxit), _ptr(b), _ptr(x), _ptr(st))
        stats = dict(iterations=int(st[0]), restarts=int(st[1]), precond_applications=int(st[2]),
                     rel_residual=float(st[3]), status=int(st[4]))
        return x, stats

    def dense(self, which="A", level=0):
        """Dense matrix of an operator on the interior unknowns (small grids only),
        assembled column by column from ``apply``; returns (matrix, interior mask)."""
        shape = self.level_shape(level)
        mask = np.zeros(shape, dtype=bool)
        sl = tuple(slice(1, s - 1) for s in shape)
        mask[sl] = True
        idx = np.flatnonzero(mask.ravel())
        nu = idx.size
        A = np.zeros((nu, nu), dtype=np.complex128)
        e = np.zeros(int(np.prod(shape)), dtype=np.complex128)
        for c, p in enumerate(idx):
            e[:] = 0
            e[p] = 1
            y = self.apply(e.reshape(shape), level, which).ravel()
            A[:, c] = y[idx]
        return A, mask


def coupled_dense(problems, k2c):
    """Dense matrix of the coupled block system of Sec. 2 (the blocked
    Helmholtz operator): diagonal blocks A_ii from each problem's operator on
    the interior unknowns, off-diagonal blocks -diag(k2c[i, j]) at the same
    unknowns.  Small grids only.  Returns (matrix, interior mask)."""
    nb = len(problems)
    blocks = [P.dense("A") for P in problems]
    mask = blocks[0][1]
    nu = blocks[0][0].shape[0]
    A = np.zeros((nb * nu, nb * nu), dtype=np.complex128)
    for i in range(nb):
        A[i * nu:(i + 1) * nu, i * nu:(i + 1) * nu] = blocks[i][0]
        for j in range(nb):
            if j != i and k2c is not None:
                A[i * nu:(i + 1) * nu, j * nu:(j + 1) * nu] = -np.diag(np.asarray(k2c[i, j])[mask])
    return A, mask


def coupled_solve_dense(problems, k2c, b):
    """Solution of the coupled system by a dense direct solve (stacked
    (nb, *shape) arrays, zero on the boundary)."""
    A, mask = coupled_dense(problems, k2c)
    nb = len(problems)
    rhs = np.concatenate([np.asarray(b[i])[mask] for i in range(nb)])
    sol = np.linalg.solve(A, rhs)
    x = np.zeros((nb,) + mask.shape, dtype=np.complex128)
    nu = int(mask.sum())
    for i in range(nb):
        x[i][mask] = sol[i * nu:(i + 1) * nu]
    return x
