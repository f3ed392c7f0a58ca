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


# ---------------------------------------------------------------- host logic of the IP-PMM driver

def _rule_cases(seed, count):
    import numpy as np
    rng = np.random.default_rng(seed)
    for _ in range(count):
        rule = int(rng.integers(0, 3))
        ell_min = int(rng.integers(1, 60))
        ell_max = int(rng.integers(ell_min, 6000))
        if rng.random() < 0.3:                       # exact products c * d_hat
            d_hat = float(rng.integers(0, 3000)) / 2.0
        else:
            d_hat = float(np.exp(rng.uniform(-3, np.log(5000))))
        mu = float(np.exp(rng.uniform(-20, 2)))
        r = rng.random()
        lam_last = mu if r < 0.1 else float(mu * np.exp(rng.uniform(-5, 5)))
        c_ell = float(rng.choice([0.5, 1.0, 2.0, 3.7]))
        yield (rule, d_hat, lam_last, mu, int(rng.integers(0, 80)), int(rng.integers(1, 3000)), ell_min,
               ell_max, c_ell)


def test_sketch_size_rule_matches_oracle():
    """nys_sketch_size_rule against the oracle's rule, bit-exact, on seeded
    inputs that include exact products c_ell d_hat and lambda_hat_ell = mu."""
    from oracle import adaptive
    from paper_2404_14524_amd import nysipm
    lib = nysipm.load_library()
    for case in _rule_cases(21, 4000):
        got = lib.nys_sketch_size_rule(*case)
        assert got == adaptive.sketch_size_rule(*case), case
    # documented edge behaviour: non-finite d_hat gives ell_max; bad clamps / rule fail
    assert lib.nys_sketch_size_rule(1, float("nan"), 1.0, 1.0, 0, 10, 4, 77, 2.0) == 77
    assert lib.nys_sketch_size_rule(1, float("inf"), 1.0, 1.0, 0, 10, 4, 77, 2.0) == 77
    assert lib.nys_sketch_size_rule(1, 3.0, 1.0, 1.0, 0, 10, 9, 8, 2.0) == nysipm.NYS_EINVAL
    assert lib.nys_sketch_size_rule(7, 3.0, 1.0, 1.0, 0, 10, 1, 8, 2.0) == nysipm.NYS_EINVAL
    assert lib.nys_sketch_size_rule(1, 3.0, 1.0, 1.0, 0, 10, 1, 8, 0.0) == nysipm.NYS_EINVAL


def test_rebuild_rule_matches_oracle():
    import numpy as np
    from oracle import adaptive
    from paper_2404_14524_amd import nysipm
    lib = nysipm.load_library()
    rng = np.random.default_rng(22)
    for _ in range(4000):
        k = int(rng.integers(0, 60))
        k_build = int(rng.integers(-1, k + 1))
        pcg_ref = int(rng.integers(0, 500))
        pcg_prev = int(pcg_ref * rng.choice([0.5, 1.0, 1.5, 2.0]) + rng.integers(-2, 3)) if rng.random() < 0.5 \
            else int(rng.integers(0, 1000))
        max_age = int(rng.integers(-1, 6))
        growth = float(rng.choice([1.0, 1.5, 2.0, 1.25]))
        case = (k, k_build, pcg_prev, pcg_ref, max_age, growth)
        assert bool(lib.nys_precond_rebuild_due(*case)) == adaptive.rebuild_due(*case), case


# ---------------------------------------------------------------- argument checks of the binding

def test_binding_refuses_views_the_kernels_would_read_past():
    """Row-major views with overlapping rows (expanded, broadcast) or a
    non-unit column stride are refused before any library call; so are 2-D
    arguments and preconditioner parts that are not dense row-major blocks."""
    from paper_2404_14524_amd import nysipm as b
    A = torch.zeros(6, 5, dtype=torch.float64)
    assert b._rows_ok(A) and b._rows_ok(A[:, 1:4]) and b._rows_ok(A[2:3])
    assert not b._rows_ok(torch.zeros(1, 5).expand(6, 5))     # row stride 0
    assert not b._rows_ok(A.t())                              # column stride 6
    assert b._rows_ok(torch.zeros(6, 1).expand(6, 1)) and b._rows_ok(torch.zeros(1, 5))
    dev = A.device
    b._mat64(A, 6, 5, "A", dev)
    for bad in (A[:, :4], A.float(), A.t().contiguous(), torch.zeros(1, 5, dtype=torch.float64).expand(6, 5)):
        with pytest.raises(ValueError):
            b._mat64(bad, 6, 5, "A", dev)
    U = torch.zeros(6, 2, dtype=torch.float64)
    b.Precond(U, torch.zeros(2, dtype=torch.float64)).c()
    with pytest.raises(ValueError):
        b.Precond(torch.zeros(1, 2, dtype=torch.float64).expand(6, 2), torch.zeros(2, dtype=torch.float64)).c()
    with pytest.raises(ValueError):
        b.Precond(U, torch.zeros(3, dtype=torch.float64)).c()
    i32 = torch.int32
    P = b.PChol(torch.zeros(2, dtype=i32), torch.zeros(6, dtype=i32), U, torch.zeros(2, 2, dtype=torch.float64),
                torch.zeros(6, dtype=torch.float64))
    P.c()
    P.pos = torch.zeros(6, dtype=torch.int64)
    with pytest.raises(ValueError):
        P.c()


def test_binding_sets_the_stream_only_when_it_changes(monkeypatch):
    """nys_set_stream waits for the handle's previous stream, so the binding
    calls it only when torch's current stream changes (a fake library and
    fake torch stream stand in for the GPU)."""
    from paper_2404_14524_amd import nysipm as b
    calls = []

    class FakeLib:
        def nys_create(self, h, idx, stream):
            return 0

        def nys_set_stream(self, h, stream):
            calls.append(stream.value)
            return 0

    class FakeStream:
        def __init__(self, ptr):
            self.cuda_stream = ptr

    current = [FakeStream(0)]
    monkeypatch.setattr(b, "load_library", lambda: FakeLib())
    monkeypatch.setattr(b, "_handles", {})
    monkeypatch.setattr(b, "_streams", {})
    monkeypatch.setattr(torch.cuda, "is_available", lambda: True)
    monkeypatch.setattr(torch.cuda, "current_stream", lambda idx=None: current[0])
    dev = torch.device("cuda", 0)
    for _ in range(3):
        b._handle(dev)
    assert calls == [None]                   # the null stream, once (ctypes maps 0 to None)
    current[0] = FakeStream(1234)
    b._handle(dev)
    b._handle(dev)
    assert calls == [None, 1234]
