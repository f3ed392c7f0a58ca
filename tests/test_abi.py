"""CPU checks of the boundary: the HIP library loads without a GPU and exports
every function that include/nysipm.h declares; the Python binding has the
same names and refuses to run without a GPU (no CPU fallback)."""

import ctypes
import os
import re

import pytest
import torch

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "nysipm.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:int|const char\*)\s+(\w+)\s*\(", text, flags=re.M)))


def test_header_declares_the_entry_points():
    names = declared_functions()
    for n in ("nys_normal_apply", "nys_sketch", "nys_precond_apply", "nys_pcg_solve", "ipm_solve",
              "ipm_adjoint", "nys_create", "nys_destroy", "nys_last_error"):
        assert n in names


def test_library_exports_every_declared_symbol():
    from paper_2404_14524_amd import nysipm
    lib = nysipm.load_library()
    for name in declared_functions():
        assert hasattr(lib, name), name
        assert isinstance(getattr(lib, name), ctypes._CFuncPtr)
    assert sorted(nysipm.EXPORTS) == declared_functions()


def test_binding_names_match_the_abi():
    import paper_2404_14524_amd as pkg
    for name in ("nys_normal_apply", "nys_sketch", "nys_precond_apply", "nys_pcg_solve",
                 "nys_newton_solve", "ipm_solve", "ipm_adjoint", "nys_test_matrix"):
        assert callable(getattr(pkg, name))


@pytest.mark.skipif(torch.cuda.is_available(), reason="checks the no-GPU refusal")
def test_no_cpu_fallback():
    import paper_2404_14524_amd as pkg
    A = torch.zeros((2, 3), dtype=torch.float64)
    with pytest.raises((RuntimeError, ValueError)):
        pkg.nys_normal_apply(A, torch.ones(3, dtype=torch.float64), 1.0, torch.ones(2, dtype=torch.float64))


def test_create_rejects_bad_device_without_gpu_work():
    from paper_2404_14524_amd import nysipm
    lib = nysipm.load_library()
    h = ctypes.c_void_p()
    assert lib.nys_create(ctypes.byref(h), -1, None) == nysipm.NYS_EINVAL
    assert lib.nys_create(None, 0, None) == nysipm.NYS_EINVAL
