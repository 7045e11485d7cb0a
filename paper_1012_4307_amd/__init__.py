"""MI355X-native multigrid-preconditioned Krylov solver for the exterior-
complex-scaled (ECS) Helmholtz problem  (-Lap - k^2(x)) u = f.

Method: bin Zubair, Reps, Vanroose, "A preconditioned iterative solver for the
scattering solutions of the Schroedinger equation" -- ECS discretisation
(Sec. 3), CSL / CSG / QD preconditioners inverted by one multigrid cycle
(Sec. 4, Algorithm 1), right-preconditioned Krylov outer solve (Sec. 5).

This module is a thin ctypes binding of the C ABI in ``include/ecsmg.h``
(``libecsmg.so``, built from ``csrc/*.hip``).  It only marshals arguments:
tensors must be contiguous CUDA (HIP) tensors; every arithmetic step runs in
the library's HIP kernels on the tensors' device and the current torch
stream.  There is no CPU fallback: if the library is missing the binding
raises.
"""
from __future__ import annotations

import ctypes
import dataclasses
import math
import os
from dataclasses import dataclass, field
from typing import Optional

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libecsmg.so")

# enums of ecsmg.h
F64, F32 = 0, 1
DIRICHLET, ECS = 0, 1
PREC = {"none": 0, "laplace": 1, "csl": 2, "csg": 3, "qd": 4}
SMOOTHER = {"jacobi": 0, "rbgs": 1}
KRYLOV = {"gmres": 0, "fgmres": 1, "bicgstab": 2}
ORTH = {"dcgs2": 0, "cgs2": 1, "cgs1": 2, "cgs2_selective": 3}


def _code(table, name, what):
    """The ABI code of an option name; ValueError naming the choices otherwise."""
    try:
        return table[name]
    except KeyError:
        raise ValueError(f"unknown {what} {name!r}: one of {', '.join(sorted(table))}") from None


OP = {"A": 0, "AT": 1, "M": 2}
STATUS = {0: "ok", 1: "not_converged", -1: "einval", -2: "enomem", -3: "edevice", -4: "ebreakdown", -5: "estate"}
TIMER = {"smooth": 0, "mdot": 1, "apply_A": 2, "coarse": 3, "mupdate": 4, "restrict": 5, "prolong": 6, "down": 7,
         "up": 8, "empty": 9, "down_p": 10, "down_s": 11}


class EcsError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


class PrecDesc(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int), ("beta1", ctypes.c_double), ("beta2", ctypes.c_double),
                ("theta_alpha", ctypes.c_double), ("re_lambda0", ctypes.c_double), ("smoother", ctypes.c_int),
                ("omega", ctypes.c_double), ("nu1", ctypes.c_int), ("nu2", ctypes.c_int), ("gamma_f", ctypes.c_int),
                ("gamma_c", ctypes.c_int), ("coarsest_nodes", ctypes.c_int), ("vcycle_dtype", ctypes.c_int)]


class SolveDesc(ctypes.Structure):
    _fields_ = [("krylov", ctypes.c_int), ("restart", ctypes.c_int), ("rtol", ctypes.c_double),
                ("maxit", ctypes.c_int), ("x_is_guess", ctypes.c_int), ("inner", ctypes.c_int),
                ("history", ctypes.POINTER(ctypes.c_double)), ("history_len", ctypes.c_int),
                ("orth", ctypes.c_int), ("nrhs", ctypes.c_int)]


class Tuning(ctypes.Structure):
    _fields_ = [("down_rows", ctypes.c_int), ("up_rows", ctypes.c_int), ("small_grid", ctypes.c_int),
                ("tail_nodes", ctypes.c_int), ("pair_grid", ctypes.c_int), ("fuse_updates", ctypes.c_int)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class Stats(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int), ("restarts", ctypes.c_int), ("vcycles", ctypes.c_int64),
                ("inner_iterations", ctypes.c_int64), ("rel_residual", ctypes.c_double),
                ("seconds", ctypes.c_double), ("status", ctypes.c_int), ("reorthogonalisations", ctypes.c_int64),
                ("inner_breakdowns", ctypes.c_int64)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_lib = None


def lib():
    """Load libecsmg.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_1012_4307_amd.build`")
    L = ctypes.CDLL(LIB_PATH)
    P, I, D, Z = ctypes.c_void_p, ctypes.c_int, ctypes.c_double, ctypes.c_size_t
    pP = ctypes.POINTER(ctypes.c_void_p)
    sig = {
        "ecs_create": [pP, I, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(D), ctypes.POINTER(D), P],
        "ecs_set_ecs": [P, I, I, I, D, D],
        "ecs_set_k2": [P, P, I],
        "ecs_set_precond": [P, ctypes.POINTER(PrecDesc)],
        "ecs_workspace_size": [P, ctypes.POINTER(SolveDesc), ctypes.POINTER(Z)],
        "ecs_set_workspace": [P, P, Z],
        "ecs_solve": [P, ctypes.POINTER(SolveDesc), P, P, ctypes.POINTER(Stats)],
        "ecs_solve_static": [P, ctypes.POINTER(SolveDesc), P, P, ctypes.POINTER(Stats)],
        "ecs_solve_adjoint": [P, ctypes.POINTER(SolveDesc), P, P, ctypes.POINTER(Stats)],
        "ecs_grad_k2": [P, P, P, P],
        "ecs_apply": [P, I, P, P],
        "ecs_vcycle": [P, P, P],
        "ecs_smooth": [P, I, P, P, I],
        "ecs_residual_restrict": [P, I, P, P, P],
        "ecs_prolong_correct": [P, I, P, P],
        "ecs_coarse_solve": [P, P, P],
        "ecs_level_info": [P, I, ctypes.POINTER(I), ctypes.POINTER(ctypes.c_int64)],
        "ecs_timing_enable": [P, I, I],
        "ecs_timing_read": [P, I, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(D), ctypes.POINTER(D)],
        "ecs_batch_solve": [I, pP, ctypes.POINTER(ctypes.POINTER(SolveDesc)), pP, pP, ctypes.POINTER(I),
                            ctypes.POINTER(Stats)],
        "ecs_copy_probe": [P, P, Z, P],
        "ecs_timing_calibrate": [P, I],
        "ecs_vcycle_native": [P, P, P],
        "ecs_mg_solve": [P, P, P, D, I, I, ctypes.POINTER(D), I, ctypes.POINTER(Stats)],
        "ecs_coupled_workspace_size": [I, pP, ctypes.POINTER(SolveDesc), ctypes.POINTER(Z)],
        "ecs_coupled_solve": [I, pP, P, ctypes.POINTER(SolveDesc), ctypes.POINTER(SolveDesc), P, Z, P, P,
                              ctypes.POINTER(Stats)],
        "ecs_set_graphs": [P, I],
        "ecs_set_tuning": [P, ctypes.POINTER(Tuning)],
        "ecs_get_tuning": [P, ctypes.POINTER(Tuning)],
    }
    for name, args in sig.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = ctypes.c_int
    L.ecs_last_error.argtypes = [P]
    L.ecs_last_error.restype = ctypes.c_char_p
    L.ecs_destroy.argtypes = [P]
    L.ecs_destroy.restype = None
    _lib = L
    return L


EXPORTED = ["ecs_create", "ecs_set_ecs", "ecs_set_k2", "ecs_set_precond", "ecs_workspace_size", "ecs_set_workspace",
            "ecs_solve", "ecs_solve_adjoint", "ecs_grad_k2", "ecs_apply", "ecs_vcycle", "ecs_smooth",
            "ecs_residual_restrict", "ecs_prolong_correct", "ecs_coarse_solve", "ecs_level_info",
            "ecs_timing_enable", "ecs_timing_read", "ecs_batch_solve", "ecs_copy_probe", "ecs_last_error",
            "ecs_destroy", "ecs_set_graphs", "ecs_set_tuning", "ecs_get_tuning", "ecs_timing_calibrate",
            "ecs_vcycle_native", "ecs_mg_solve", "ecs_coupled_workspace_size", "ecs_coupled_solve",
            "ecs_solve_static"]


def _torch():
    import torch
    return torch


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr())


def _stream_ptr(device):
    torch = _torch()
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


class _StreamOrder:
    """Orders the library's streams (each context enqueues on the stream that
    was current when it was made) with the caller's current stream around one
    call: before it, each of them waits for the caller's stream, so inputs
    written there are complete when the library reads them; after it, the
    caller's stream waits for each of them, so outputs can be used there, and
    the outputs' memory is marked in use on them, so torch's allocator does not
    hand it out again before they are done.  Nothing happens for a context on
    the caller's current stream."""

    def __init__(self, streams, outs=()):
        self.streams = list(streams)
        self.outs = outs

    def __enter__(self):
        torch = _torch()
        self.cur = torch.cuda.current_stream(self.streams[0].device) if self.streams else None
        for st in self.streams:
            if st != self.cur:
                st.wait_stream(self.cur)
        return self

    def __exit__(self, exc_type, exc, tb):
        if exc_type is None:
            for st in self.streams:
                if st != self.cur:
                    for t in self.outs:
                        t.record_stream(st)
                    self.cur.wait_stream(st)
        return False


@dataclass
class Precond:
    """Preconditioner and cycle (Sec. 4-5).  kind: none | laplace | csl | csg | qd."""
    kind: str = "qd"
    beta1: float = -1.0
    beta2: float = -0.5
    theta_alpha: float = math.pi / 13
    re_lambda0: float = 0.0            # QD: Re(lambda0) (its magnitude is used); 0 -> max k^2
    smoother: str = "rbgs"
    omega: float = 1.0
    nu1: int = 1
    nu2: int = 1
    gamma_f: int = 1
    gamma_c: int = 1
    coarsest_nodes: int = 5
    vcycle_dtype: str = "f64"          # f64 | f32

    def to_c(self):
        return PrecDesc(_code(PREC, self.kind, "preconditioner kind"), self.beta1, self.beta2, self.theta_alpha,
                        self.re_lambda0, _code(SMOOTHER, self.smoother, "smoother"), self.omega, self.nu1,
                        self.nu2, self.gamma_f, self.gamma_c,
                        self.coarsest_nodes, F32 if self.vcycle_dtype == "f32" else F64)


@dataclass
class Krylov:
    method: str = "gmres"      # gmres | fgmres | bicgstab
    restart: int = 30
    rtol: float = 1e-8
    maxit: int = 2000
    inner: int = 0             # nested Bi-CGSTAB iterations (cycle dtype) per FGMRES step
    orth: str = "dcgs2"        # Arnoldi Gram-Schmidt: dcgs2 | cgs2_selective | cgs2 | cgs1
    nrhs: int = 0              # Bi-CGSTAB workspace for the batched solve: right-hand sides at once (0: none)

    def to_c(self, x_is_guess=False, history=None):
        d = SolveDesc(_code(KRYLOV, self.method, "Krylov method"), self.restart, self.rtol, self.maxit,
                      1 if x_is_guess else 0, self.inner, None, 0, _code(ORTH, self.orth, "orthogonalisation"),
                      self.nrhs)
        if history is not None:
            d.history = history.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
            d.history_len = history.size
        return d


class Solver:
    """One ECS Helmholtz problem on one GPU.

    dim, n, lo, hi : grid (nodes per axis incl. both Dirichlet ends)
    ecs            : per axis (lo_side, hi_side), each None or (layer start, theta)
    k2             : float64 or float32 CUDA tensor of k^2 at the nodes, shape
                     reversed(n) (float32 is widened once, at set-up)
    precond        : Precond
    krylov         : Krylov settings used to size the workspace (larger ones
                     reallocate it on demand)
    hierarchy_only : size the workspace for the hierarchy alone (enough for
                     the single-step calls and solve_static)
    """

    def __init__(self, dim, n, lo, hi, ecs, k2, precond: Precond, krylov: Optional[Krylov] = None,
                 hierarchy_only: bool = False):
        torch = _torch()
        L = lib()
        self.dim = int(dim)
        self.n = tuple(int(v) for v in n)
        self.shape = tuple(reversed(self.n))
        self.device = None
        self._k2_dtype(k2)
        self.device = k2.device
        self.k2 = k2
        self.precond = precond
        self.krylov = krylov or Krylov()
        h = ctypes.c_void_p()
        nodes = (ctypes.c_int64 * 3)(*(list(self.n) + [1] * (3 - self.dim)))
        lo3 = (ctypes.c_double * 3)(*(list(lo) + [0.0] * (3 - self.dim)))
        hi3 = (ctypes.c_double * 3)(*(list(hi) + [1.0] * (3 - self.dim)))
        # the context enqueues all its work on the stream current at creation
        self.stream = torch.cuda.current_stream(self.device)
        with torch.cuda.device(self.device):
            self._check(L.ecs_create(ctypes.byref(h), self.dim, nodes, lo3, hi3,
                                     ctypes.c_void_p(self.stream.cuda_stream)), None)
        self._h = h
        for a in range(self.dim):
            for side in (0, 1):
                spec = ecs[a][side]
                if spec is not None:
                    self._check(L.ecs_set_ecs(h, a, side, ECS, float(spec[0]), float(spec[1])))
        self._check(L.ecs_set_k2(h, _ptr(k2), self._k2_dtype(k2)))
        self._pd = precond.to_c()
        self._check(L.ecs_set_precond(h, ctypes.byref(self._pd)))
        self.nlev = self.level_count()
        self.ws = None
        self._ensure_workspace(None if hierarchy_only else self.krylov)

    # ------------------------------------------------------------------
    def _check(self, rc, h="self"):
        if rc == 0:
            return 0
        msg = ""
        hh = self._h if h == "self" else h
        if hh is not None:
            msg = lib().ecs_last_error(hh).decode()
        raise EcsError(rc, msg)

    def __del__(self):
        h = getattr(self, "_h", None)
        L = _lib  # None once the interpreter is tearing the module down
        if h is not None and h.value and L is not None:
            L.ecs_destroy(h)
            self._h = None

    def _k2_dtype(self, k2):
        """The library's dtype code of a k^2 tensor; raises ValueError unless it
        is a contiguous float64 / float32 CUDA tensor of the grid's shape on the
        solver's device."""
        torch = _torch()
        ok = (isinstance(k2, torch.Tensor) and k2.is_cuda and k2.dtype in (torch.float64, torch.float32)
              and k2.is_contiguous() and tuple(k2.shape) == self.shape
              and (self.device is None or k2.device == self.device))
        if not ok:
            desc = f"{k2.dtype} {tuple(k2.shape)} on {k2.device}" if isinstance(k2, torch.Tensor) else type(k2).__name__
            raise ValueError(f"k2 must be a contiguous float64 or float32 CUDA tensor of shape {self.shape}"
                             f"{'' if self.device is None else ' on ' + str(self.device)}, got {desc}")
        return F64 if k2.dtype == torch.float64 else F32

    def _set_workspace(self, ws, nbytes):
        """Hand `ws` to the library, which builds the hierarchy in it on the
        context's stream: that stream first waits for the caller's, so memory
        the caller's stream used before (torch may hand out a block freed
        there) is not overwritten early."""
        base = ws.data_ptr()
        off = (-base) % 256
        with _StreamOrder([self.stream], (ws,)):
            self._check(lib().ecs_set_workspace(self._h, ctypes.c_void_p(base + off), nbytes - off))

    def _ensure_workspace(self, kr: Optional[Krylov]):
        torch = _torch()
        L = lib()
        need = ctypes.c_size_t()
        d = kr.to_c() if kr is not None else None
        self._check(L.ecs_workspace_size(self._h, ctypes.byref(d) if d is not None else None, ctypes.byref(need)))
        if self.ws is not None and self.ws.numel() >= need.value:
            return
        self.ws = torch.empty(need.value + 256, dtype=torch.uint8, device=self.device)
        self._set_workspace(self.ws, self.ws.numel())

    def reset_k2(self, k2):
        """Replace k^2 (same shape and device; float64 or float32) and rebuild
        the hierarchy."""
        code = self._k2_dtype(k2)
        L = lib()
        with _StreamOrder([self.stream]):
            self._check(L.ecs_set_k2(self._h, _ptr(k2), code))
        self.k2 = k2
        need = ctypes.c_size_t()
        self._check(L.ecs_workspace_size(self._h, None, ctypes.byref(need)))
        if self.ws.numel() < need.value + 256:   # an FP32 field needs room for its FP64 copy
            self.ws = None
            self._ensure_workspace(self.krylov)
        else:
            self._set_workspace(self.ws, self.ws.numel())

    def level_count(self):
        nl = ctypes.c_int()
        self._check(lib().ecs_level_info(self._h, 0, ctypes.byref(nl), None))
        return nl.value

    def level_shape(self, level):
        nodes = (ctypes.c_int64 * 3)()
        nl = ctypes.c_int()
        self._check(lib().ecs_level_info(self._h, level, ctypes.byref(nl), nodes))
        return tuple(reversed([int(nodes[a]) for a in range(self.dim)]))

    def _vec(self, t, dtype=None, shape=None):
        torch = _torch()
        dtype = dtype or torch.complex128
        shape = shape or self.shape
        if not (t.is_cuda and t.dtype == dtype and t.is_contiguous() and tuple(t.shape) == tuple(shape)):
            raise ValueError(f"expected contiguous {dtype} CUDA tensor of shape {shape}, got {t.dtype} {tuple(t.shape)}")
        return t

    @property
    def cycle_dtype(self):
        torch = _torch()
        return torch.complex64 if self.precond.vcycle_dtype == "f32" else torch.complex128

    # ------------------------------------------------------------ solves
    def solve(self, b, x0=None, krylov: Optional[Krylov] = None, history=None):
        """Solve A x = b; returns (x, stats dict)."""
        torch = _torch()
        kr = krylov or self.krylov
        self._ensure_workspace(kr)
        b = self._vec(b)
        x = x0.clone() if x0 is not None else torch.empty_like(b)
        st = Stats()
        d = kr.to_c(x0 is not None, history)
        with _StreamOrder([self.stream], (x,)):
            rc = lib().ecs_solve(self._h, ctypes.byref(d), _ptr(b), _ptr(x), ctypes.byref(st))
        if rc < 0:
            self._check(rc)
        out = st.as_dict()
        out["status_name"] = STATUS.get(rc, rc)
        return x, out

    def solve_static(self, b, x0=None, krylov: Optional[Krylov] = None, history=None):
        """Solve A x = b through ecs_solve_static: the Krylov vectors live in
        the library's static device scratch, so the call allocates nothing on
        the device beyond the output tensor (the workspace is not grown);
        returns (x, stats dict)."""
        torch = _torch()
        kr = krylov or self.krylov
        b = self._vec(b)
        x = x0.clone() if x0 is not None else torch.empty_like(b)
        st = Stats()
        d = kr.to_c(x0 is not None, history)
        with _StreamOrder([self.stream], (x,)):
            rc = lib().ecs_solve_static(self._h, ctypes.byref(d), _ptr(b), _ptr(x), ctypes.byref(st))
        if rc < 0:
            self._check(rc)
        out = st.as_dict()
        out["status_name"] = STATUS.get(rc, rc)
        return x, out

    def mg_solve(self, b, x0=None, rtol=1e-6, maxcycles=100):
        """Stand-alone multigrid on the preconditioner, M x = b: x <- x + MG(b - M x)
        until ||b - M x|| <= rtol ||b|| (Sec. 5).  Returns (x, stats dict, history of
        ||b - M x_m|| / ||b||, m = 0 .. cycles)."""
        import numpy as np
        torch = _torch()
        self._ensure_workspace(self.krylov)
        b = self._vec(b)
        x = x0.clone() if x0 is not None else torch.empty_like(b)
        hist = np.zeros(maxcycles + 1)
        st = Stats()
        with _StreamOrder([self.stream], (x,)):
            rc = lib().ecs_mg_solve(self._h, _ptr(b), _ptr(x), float(rtol), int(maxcycles),
                                    1 if x0 is not None else 0, hist.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                    hist.size, ctypes.byref(st))
        if rc < 0:
            self._check(rc)
        out = st.as_dict()
        out["status_name"] = STATUS.get(rc, rc)
        return x, out, hist[: out["iterations"] + 1]

    def solve_adjoint(self, g, krylov: Optional[Krylov] = None):
        """Solve A^T lam = g (no conjugation); returns (lam, stats dict)."""
        torch = _torch()
        kr = krylov or self.krylov
        self._ensure_workspace(kr)
        g = self._vec(g)
        lam = torch.empty_like(g)
        st = Stats()
        d = kr.to_c()
        with _StreamOrder([self.stream], (lam,)):
            rc = lib().ecs_solve_adjoint(self._h, ctypes.byref(d), _ptr(g), _ptr(lam), ctypes.byref(st))
        if rc < 0:
            self._check(rc)
        out = st.as_dict()
        out["status_name"] = STATUS.get(rc, rc)
        return lam, out

    def grad_k2(self, lam, u):
        torch = _torch()
        lam = self._vec(lam)
        u = self._vec(u)
        g = torch.empty(self.shape, dtype=torch.float64, device=self.device)
        with _StreamOrder([self.stream], (g,)):
            self._check(lib().ecs_grad_k2(self._h, _ptr(lam), _ptr(u), _ptr(g)))
        return g

    # ------------------------------------------------------- single steps
    def apply(self, x, op="A"):
        torch = _torch()
        x = self._vec(x)
        y = torch.empty_like(x)
        with _StreamOrder([self.stream], (y,)):
            self._check(lib().ecs_apply(self._h, OP[op], _ptr(x), _ptr(y)))
        return y

    def vcycle(self, v):
        """z = MG(v): complex128 in and out (converted around an FP32 cycle)."""
        torch = _torch()
        v = self._vec(v)
        z = torch.empty_like(v)
        with _StreamOrder([self.stream], (z,)):
            self._check(lib().ecs_vcycle(self._h, _ptr(v), _ptr(z)))
        return z

    def vcycle_native(self, v):
        """z = MG(v) on vectors in the cycle's own dtype (complex64 for an FP32
        cycle), without conversion passes."""
        torch = _torch()
        v = self._vec(v, self.cycle_dtype)
        z = torch.empty_like(v)
        with _StreamOrder([self.stream], (z,)):
            self._check(lib().ecs_vcycle_native(self._h, _ptr(v), _ptr(z)))
        return z

    def smooth(self, b, u, level=0, nsweeps=1):
        shape = self.level_shape(level)
        b = self._vec(b, self.cycle_dtype, shape)
        u = self._vec(u, self.cycle_dtype, shape).clone()
        with _StreamOrder([self.stream], (u,)):
            self._check(lib().ecs_smooth(self._h, level, _ptr(b), _ptr(u), nsweeps))
        return u

    def residual_restrict(self, b, u, level=0):
        torch = _torch()
        shape = self.level_shape(level)
        b = self._vec(b, self.cycle_dtype, shape)
        u = self._vec(u, self.cycle_dtype, shape)
        rc = torch.empty(self.level_shape(level + 1), dtype=self.cycle_dtype, device=self.device)
        with _StreamOrder([self.stream], (rc,)):
            self._check(lib().ecs_residual_restrict(self._h, level, _ptr(b), _ptr(u), _ptr(rc)))
        return rc

    def prolong_correct(self, ec, u, level=0):
        ec = self._vec(ec, self.cycle_dtype, self.level_shape(level + 1))
        u = self._vec(u, self.cycle_dtype, self.level_shape(level)).clone()
        with _StreamOrder([self.stream], (u,)):
            self._check(lib().ecs_prolong_correct(self._h, level, _ptr(ec), _ptr(u)))
        return u

    def coarse_solve(self, b):
        torch = _torch()
        shape = self.level_shape(self.nlev - 1)
        b = self._vec(b, self.cycle_dtype, shape)
        x = torch.empty_like(b)
        with _StreamOrder([self.stream], (x,)):
            self._check(lib().ecs_coarse_solve(self._h, _ptr(b), _ptr(x)))
        return x

    def set_tuning(self, down_rows=4, up_rows=8, small_grid=513, tail_nodes=33, pair_grid=129, fuse_updates=1):
        """Launch schedule of the fused V(1,1) cycle, and whether the nested
        FP32 Bi-CGSTAB forms its updates inside the finest down kernel
        (performance only)."""
        t = Tuning(down_rows, up_rows, small_grid, tail_nodes, pair_grid, int(fuse_updates))
        self._check(lib().ecs_set_tuning(self._h, ctypes.byref(t)))

    def get_tuning(self):
        t = Tuning()
        self._check(lib().ecs_get_tuning(self._h, ctypes.byref(t)))
        return t.as_dict()

    def set_graphs(self, mode):
        """Launch mode of the cycle: True (HIP graph replay), False (eager) or
        "auto" (the default: graphs for general cycles, eager launches for
        the fused 2D V(1,1) red-black cycle)."""
        code = {False: 0, True: 1, "auto": 2}[mode]
        self._check(lib().ecs_set_graphs(self._h, code))

    # ----------------------------------------------------------- timing
    def timing(self, kclass: str, enable: bool = True, every: int = 1):
        """Time launches of one kernel class with HIP events: every launch, or
        one in ``every``."""
        if every < 1:
            raise ValueError("every must be >= 1")
        self._check(lib().ecs_timing_enable(self._h, TIMER[kclass], every if enable else 0))

    def timing_calibrate(self, launches: int = 200) -> float:
        """Mean timed duration (us) of an empty kernel: the fixed part of every
        timed duration."""
        self._check(lib().ecs_timing_calibrate(self._h, launches))
        n, ms, _ = self.timing_read("empty")
        return 1e3 * ms / max(n, 1)

    def timing_read(self, kclass: str):
        """(launches, total ms, algorithmic bytes) of one kernel class since the last read."""
        n = ctypes.c_int64()
        ms = ctypes.c_double()
        by = ctypes.c_double()
        self._check(lib().ecs_timing_read(self._h, TIMER[kclass], ctypes.byref(n), ctypes.byref(ms),
                                          ctypes.byref(by)))
        return n.value, ms.value, by.value


def batch_solve(solvers, rhs, krylov, x0=None, group=8):
    """Solve every right-hand side of every system by Bi-CGSTAB: rhs[s] is a
    contiguous complex128 CUDA tensor of shape (nrhs_s, *solvers[s].shape) on
    that solver's device; krylov is one Krylov for all systems or a list with
    one per system; x0 (optional) a list with each system's initial guesses
    (a tensor like rhs[s], or None for zero guesses); group: right-hand sides
    of a system solved at once (1..8; the fused 2D V(1,1) red-black cycle,
    else one at a time).  Returns (solutions, stats)."""
    torch = _torch()
    n = len(solvers)
    krs = list(krylov) if isinstance(krylov, (list, tuple)) else [krylov] * n
    x0s = list(x0) if x0 is not None else [None] * n
    if len(rhs) != n or len(krs) != n or len(x0s) != n:
        raise ValueError(f"{n} solvers need {n} right-hand side tensors, Krylov settings and guesses "
                         f"(got {len(rhs)}, {len(krs)} and {len(x0s)})")
    if len({id(S) for S in solvers}) != n:
        raise ValueError("a solver appears twice in the batch")
    for q, (S, b, kr) in enumerate(zip(solvers, rhs, krs)):
        if kr.method != "bicgstab":
            raise ValueError(f"system {q}: the batched solve uses Bi-CGSTAB, got {kr.method}")
        if not (isinstance(b, torch.Tensor) and b.is_cuda and b.dtype == torch.complex128 and b.is_contiguous()
                and b.dim() == len(S.shape) + 1 and tuple(b.shape[1:]) == S.shape and b.device == S.device):
            desc = f"{b.dtype} {tuple(b.shape)}" if isinstance(b, torch.Tensor) else type(b).__name__
            raise ValueError(f"system {q}: rhs must be a contiguous complex128 CUDA tensor of shape "
                             f"(nrhs, {', '.join(map(str, S.shape))}) on {S.device}, got {desc}")
        g = x0s[q]
        if g is not None and not (isinstance(g, torch.Tensor) and g.is_cuda and g.dtype == torch.complex128
                                  and g.is_contiguous() and tuple(g.shape) == tuple(b.shape) and g.device == b.device):
            raise ValueError(f"system {q}: x0 must be a contiguous complex128 CUDA tensor like its rhs")
    if not 1 <= int(group) <= 8:
        raise ValueError("group must be in [1, 8]")
    for S, kr, b in zip(solvers, krs, rhs):
        # the fused 2D V(1,1) red-black cycle solves up to 8 right-hand sides at once
        fused = (S.dim == 2 and S.precond.smoother == "rbgs" and S.precond.nu1 == 1 and S.precond.nu2 == 1
                 and S.precond.gamma_f == 1 and S.precond.gamma_c == 1 and S.nlev > 1)
        S._ensure_workspace(dataclasses.replace(kr, nrhs=max(1, min(int(b.shape[0]), int(group))) if fused else 1))
    xs = [torch.empty_like(b) if g is None else g.clone() for b, g in zip(rhs, x0s)]
    ctxs = (ctypes.c_void_p * n)(*[S._h.value for S in solvers])
    bs = (ctypes.c_void_p * n)(*[b.data_ptr() for b in rhs])
    xp = (ctypes.c_void_p * n)(*[x.data_ptr() for x in xs])
    nr = (ctypes.c_int * n)(*[int(b.shape[0]) for b in rhs])
    st = (Stats * n)()
    descs = [dataclasses.replace(kr, nrhs=int(group)).to_c(g is not None) for kr, g in zip(krs, x0s)]
    dp = (ctypes.POINTER(SolveDesc) * n)(*[ctypes.pointer(d) for d in descs])
    with _StreamOrder([S.stream for S in solvers], tuple(xs)):
        rc = lib().ecs_batch_solve(n, ctxs, dp, bs, xp, nr, st)
    if rc < 0:
        msg = "; ".join(lib().ecs_last_error(S._h).decode() for S in solvers if lib().ecs_last_error(S._h))
        raise EcsError(rc, msg or "batched solve failed")
    return xs, [s.as_dict() for s in st]


def coupled_solve(solvers, k2c, b, x0=None, outer: Optional[Krylov] = None, inner: Optional[Krylov] = None,
                  cycles_only: bool = False):
    """Solve the coupled block system sum_j A_ij x_j = b_i (A_ii: solver i's
    operator, A_ij = -k2c[i, j]) by FGMRES with the block-diagonal preconditioner
    (Sec. 2): every block solved by its solver through the batched Bi-CGSTAB
    driver to ``inner.rtol`` (or one multigrid cycle each with ``cycles_only``).
    k2c: float64 CUDA tensor (nb, nb, *shape) or None; b: complex128 CUDA tensor
    (nb, *shape).  Returns (x, stats dict)."""
    torch = _torch()
    nb = len(solvers)
    outer = outer or Krylov(method="fgmres", restart=30, rtol=1e-8, maxit=500)
    inner = inner or Krylov(method="bicgstab", rtol=1e-3, maxit=200)
    shape = tuple(solvers[0].shape)
    if not (b.is_cuda and b.dtype == torch.complex128 and b.is_contiguous() and tuple(b.shape) == (nb,) + shape):
        raise ValueError(f"b must be a contiguous complex128 CUDA tensor of shape {(nb,) + shape}")
    if k2c is not None and not (k2c.is_cuda and k2c.dtype == torch.float64 and k2c.is_contiguous()
                                and tuple(k2c.shape) == (nb, nb) + shape):
        raise ValueError(f"k2c must be a contiguous float64 CUDA tensor of shape {(nb, nb) + shape}")
    for S in solvers:
        S._ensure_workspace(dataclasses.replace(inner, nrhs=1))   # one right-hand side per block solve
    hs = (ctypes.c_void_p * nb)(*[S._h.value for S in solvers])
    do = outer.to_c(x0 is not None)
    di = inner.to_c()
    need = ctypes.c_size_t()
    L = lib()
    rc = L.ecs_coupled_workspace_size(nb, hs, ctypes.byref(do), ctypes.byref(need))
    if rc != 0:
        raise EcsError(rc, L.ecs_last_error(solvers[0]._h).decode())
    ws = torch.empty(need.value + 256, dtype=torch.uint8, device=b.device)
    off = (-ws.data_ptr()) % 256
    x = x0.clone() if x0 is not None else torch.empty_like(b)
    st = Stats()
    with _StreamOrder([S.stream for S in solvers], (x, ws)):
        rc = L.ecs_coupled_solve(nb, hs, _ptr(k2c) if k2c is not None else None, ctypes.byref(do),
                                 None if cycles_only else ctypes.byref(di), ctypes.c_void_p(ws.data_ptr() + off),
                                 need.value + 256 - off, _ptr(b), _ptr(x), ctypes.byref(st))
    if rc < 0:
        raise EcsError(rc, L.ecs_last_error(solvers[0]._h).decode())
    out = st.as_dict()
    out["status_name"] = STATUS.get(rc, rc)
    return x, out


def copy_probe(src, dst):
    torch = _torch()
    nbytes = src.numel() * src.element_size()
    rc = lib().ecs_copy_probe(_ptr(src), _ptr(dst), nbytes, _stream_ptr(src.device))
    if rc != 0:
        raise EcsError(rc, "copy probe failed")


def solver_for(workload, device="cuda", vcycle_dtype="f64", krylov: Optional[Krylov] = None, precond=None):
    """Build a Solver from a workloads.Workload (inputs copied to the GPU)."""
    torch = _torch()
    w = workload
    k2 = torch.from_numpy(w.k2).to(device)
    p = w.precond
    cyc = w.cycle
    pc = precond or Precond(kind=p["kind"], beta1=p.get("beta1", -1.0), beta2=p.get("beta2", -0.5),
                            theta_alpha=p.get("theta_alpha", math.pi / 13), re_lambda0=p.get("lam0", 0.0),
                            smoother=cyc["smoother"], omega=cyc["omega"], nu1=cyc["nu1"], nu2=cyc["nu2"],
                            gamma_f=cyc["gamma_f"], gamma_c=cyc["gamma_c"], coarsest_nodes=cyc["coarsest"],
                            vcycle_dtype=vcycle_dtype)
    kr = krylov or Krylov(method=w.krylov["method"], restart=w.krylov.get("m", 30), rtol=w.krylov["rtol"],
                          maxit=w.krylov["maxit"])
    return Solver(w.dim, w.n, w.lo, w.hi, w.ecs, k2, pc, kr)
