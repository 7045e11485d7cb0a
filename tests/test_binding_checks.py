"""CPU checks of the Python binding's argument validation: inputs that the C
side cannot size-check (device pointers) are refused with ValueError before
any library call, so a wrong dtype, shape, device or count never reaches a
kernel.  No GPU is needed: the checks run before the first device access."""
import types

import pytest
import torch

import paper_1012_4307_amd as E


def fake_solver(shape=(9, 9), device=torch.device("cuda", 0)):
    # just the attributes the validation reads
    S = types.SimpleNamespace(shape=shape, device=device, _h=None)
    S._k2_dtype = types.MethodType(E.Solver._k2_dtype, S)
    return S


def test_k2_dtype_device_shape_are_checked():
    S = fake_solver()
    for bad in (torch.zeros((9, 9), dtype=torch.float64),                # host memory
                torch.zeros((9, 9), dtype=torch.float16),                # neither float64 nor float32
                torch.zeros((9, 9), dtype=torch.complex128),
                torch.zeros((9, 8), dtype=torch.float64),
                torch.zeros((9, 18), dtype=torch.float64)[:, ::2],       # not contiguous
                "k2"):
        with pytest.raises(ValueError):
            S._k2_dtype(bad)


def test_solver_refuses_host_k2_before_creating_a_context():
    k2 = torch.zeros((9, 9), dtype=torch.float64)
    with pytest.raises(ValueError):
        E.Solver(2, (9, 9), (-1, -1), (1, 1), ((None, None), (None, None)), k2, E.Precond())


def test_reset_k2_validates_before_the_library():
    S = fake_solver()
    with pytest.raises(ValueError):
        E.Solver.reset_k2(S, torch.zeros((9, 9), dtype=torch.float32))   # host tensor


def test_batch_solve_validates_every_rhs():
    kr = E.Krylov(method="bicgstab")
    S0, S1 = fake_solver(), fake_solver((17, 17))
    cpu = torch.zeros((1, 9, 9), dtype=torch.complex128)
    with pytest.raises(ValueError, match="right-hand side"):
        E.batch_solve([S0, S1], [cpu], kr)                 # short list
    with pytest.raises(ValueError):
        E.batch_solve([S0], [cpu], kr)                     # host tensor
    with pytest.raises(ValueError):
        E.batch_solve([S0], [torch.zeros((2, 9, 9), dtype=torch.complex64)], kr)
    with pytest.raises(ValueError):
        E.batch_solve([S0], [torch.zeros((9, 9), dtype=torch.complex128)], kr)   # no rhs axis
    with pytest.raises(ValueError):
        E.batch_solve([S0, S0], [cpu, cpu], kr)            # the same system twice
    with pytest.raises(ValueError):
        E.batch_solve([S0], [cpu], [kr, kr])               # one Krylov per system
    with pytest.raises(ValueError):
        E.batch_solve([S0], [cpu], E.Krylov(method="gmres"))


def test_option_names_are_checked():
    """Unknown option names raise ValueError naming the choices (no library
    call is made to build a descriptor)."""
    with pytest.raises(ValueError, match="orthogonalisation"):
        E.Krylov(method="fgmres", orth="mgs").to_c()
    with pytest.raises(ValueError, match="Krylov method"):
        E.Krylov(method="cg").to_c()
    with pytest.raises(ValueError, match="smoother"):
        E.Precond(smoother="gs").to_c()
    with pytest.raises(ValueError, match="preconditioner kind"):
        E.Precond(kind="ilu").to_c()
    assert E.Krylov().to_c().orth == E.ORTH["dcgs2"] == 0
