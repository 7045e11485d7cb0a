"""CPU checks of the C ABI boundary: the HIP library loads, exports every
entry point declared in include/ecsmg.h, and validates arguments on the host
before touching a device.  No compute call is made."""
import ctypes
import os
import re

import pytest

import paper_1012_4307_amd as E

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "ecsmg.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = set(re.findall(r"\b(ecs_[a-z0-9_]+)\s*\(", src))
    return sorted(names)


def test_header_declares_the_binding_surface():
    names = declared_functions()
    assert set(names) == set(E.EXPORTED), set(names) ^ set(E.EXPORTED)


def test_library_exports_every_declared_symbol():
    lib = E.lib()
    for name in declared_functions():
        assert hasattr(lib, name), name


def test_create_rejects_bad_arguments_without_a_device():
    lib = E.lib()
    h = ctypes.c_void_p()
    nodes = (ctypes.c_int64 * 3)(65, 65, 1)
    lo = (ctypes.c_double * 3)(-1, -1, 0)
    hi = (ctypes.c_double * 3)(1, 1, 1)
    assert lib.ecs_create(ctypes.byref(h), 4, nodes, lo, hi, None) == -1
    assert lib.ecs_create(ctypes.byref(h), 1, nodes, lo, hi, None) == -1
    bad = (ctypes.c_int64 * 3)(2, 65, 1)
    assert lib.ecs_create(ctypes.byref(h), 2, bad, lo, hi, None) == -1
    flip = (ctypes.c_double * 3)(1, -1, 0)
    assert lib.ecs_create(ctypes.byref(h), 2, nodes, flip, hi, None) == -1
    assert lib.ecs_create(None, 2, nodes, lo, hi, None) == -1


def test_null_context_is_rejected():
    lib = E.lib()
    assert lib.ecs_set_k2(None, None, 0) == -1
    assert lib.ecs_apply(None, 0, None, None) == -1
    assert lib.ecs_solve(None, None, None, None, None) == -1
    assert lib.ecs_last_error(None) == b"null context"
    lib.ecs_destroy(None)


def test_probe_header_symbols_are_exported_and_check_arguments():
    """The measurement probes (include/ecsmg_probe.h) are exported and refuse
    out-of-range arguments before any device call."""
    src = open(os.path.join(ROOT, "include", "ecsmg_probe.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = sorted(set(re.findall(r"\b(ecs_[a-z0-9_]+)\s*\(", src)))
    assert names == ["ecs_probe_group_barrier", "ecs_probe_item_sweeps"]
    lib = E.lib()
    for name in names:
        assert hasattr(lib, name), name
    ms = ctypes.c_double()
    f = lib.ecs_probe_item_sweeps
    f.argtypes = [ctypes.c_int] * 4 + [ctypes.POINTER(ctypes.c_double)]
    assert f(4, 1, 1, 1, ctypes.byref(ms)) == -1          # grid too small
    assert f(65, 2, 3, 1, ctypes.byref(ms)) == -1         # more workgroups than grids
    assert f(65, 1, 1, 65, ctypes.byref(ms)) == -1        # too many sweeps
    assert f(4097, 4096, 1, 1, ctypes.byref(ms)) == -1    # more than 64 GiB
    assert f(65, 1, 1, 1, None) == -1
    g = lib.ecs_probe_group_barrier
    g.argtypes = [ctypes.c_int] * 3 + [ctypes.POINTER(ctypes.c_double)] * 2
    ub, ul = ctypes.c_double(), ctypes.c_double()
    assert g(0, 10, 0, ctypes.byref(ub), ctypes.byref(ul)) == -1
    assert g(8, 0, 0, ctypes.byref(ub), ctypes.byref(ul)) == -1
    assert g(8, 10, (1 << 20) + 8, ctypes.byref(ub), ctypes.byref(ul)) == -1
    assert g(8, 10, 0, None, ctypes.byref(ul)) == -1
