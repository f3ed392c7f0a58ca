"""GPU check of the allocation-free PCG entry point (nys_pcg_solve_noalloc)
through the C ABI: on the same inputs it returns what nys_pcg_solve returns,
bit for bit, over two calls in a row whose second is smaller (so the fixed
scratch holds the first call's values when the second starts), with and
without a transposed copy and a preconditioner; sizes beyond the scratch are
refused before anything runs."""

import numpy as np
import pytest
import torch

from instances import make_instance
from oracle import normal_eq

pytestmark = pytest.mark.gpu

DEV = "cuda"


@pytest.fixture(scope="module")
def nys():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2404_14524_amd as pkg
    return pkg


def _t(a, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device=DEV)


def _case(nys, m, n, rank, seed, ell, transposed, dtype):
    inst = make_instance("lowrank_5000x20000", seed=seed, m=m, n=n, rank=rank)
    A = inst.A.to(dtype)
    rng = np.random.default_rng(seed)
    d = _t(rng.uniform(0.01, 5.0, n))
    xi = _t(rng.standard_normal(m))
    Ad = A.to(DEV)
    A_t = nys.nys_transpose(Ad) if transposed else None
    P = nys.nys_sketch(Ad, d, ell, seed=seed) if ell else None
    return A.double().numpy(), Ad, A_t, d, xi, P


@pytest.mark.parametrize("first,second", [
    ((1500, 6000, 30, 11, 60, True, torch.float32), (700, 2500, 20, 12, 40, False, torch.float64)),
    ((1200, 5000, 30, 13, 0, False, torch.float64), (600, 3000, 20, 14, 30, True, torch.float32)),
])
def test_noalloc_matches_pcg_solve_on_two_calls(nys, first, second):
    delta = 1e-3
    for case in (first, second):
        m, n, rank, seed, ell, transposed, dtype = case
        print(f"noalloc pcg m={m} n={n} ell={ell} transposed={transposed} {dtype}", flush=True)
        A64, Ad, A_t, d, xi, P = _case(nys, m, n, rank, seed, ell, transposed, dtype)
        y_ref, info_ref = nys.nys_pcg_solve(Ad, d, delta, xi, P=P, A_t=A_t, rtol=1e-10, maxit=4000)
        y = torch.zeros(m, dtype=torch.float64, device=DEV)
        y_out, info = nys.nys_pcg_solve_noalloc(Ad, d, delta, xi, y, P=P, A_t=A_t, rtol=1e-10, maxit=4000)
        torch.cuda.synchronize()
        assert y_out.data_ptr() == y.data_ptr()
        assert info_ref.status == 0 and info.status == 0
        assert info.iters == info_ref.iters
        assert info.true_res == info_ref.true_res
        assert torch.equal(y, y_ref), float((y - y_ref).abs().max())
        # and the solution itself, against a dense FP64 solve of the same system
        M = normal_eq.normal_matrix(A64, d.cpu().numpy(), delta)
        xin = xi.cpu().numpy()
        assert np.linalg.norm(xin - M @ y.cpu().numpy()) <= 1.01e-10 * np.linalg.norm(xin) + 1e-14


def test_noalloc_warm_start_matches(nys):
    """A non-zero initial guess (the first step is a true residual) gives the
    same iterates through both entry points."""
    A64, Ad, A_t, d, xi, P = _case(nys, 900, 4000, 20, 21, 40, True, torch.float32)
    y0 = _t(np.random.default_rng(3).standard_normal(900) * 1e-2)
    y_ref, info_ref = nys.nys_pcg_solve(Ad, d, 1e-2, xi, P=P, y0=y0, A_t=A_t, rtol=1e-9)
    y = y0.clone()
    nys.nys_pcg_solve_noalloc(Ad, d, 1e-2, xi, y, P=P, A_t=A_t, rtol=1e-9)
    assert torch.equal(y, y_ref)


def test_noalloc_refuses_sizes_beyond_its_scratch(nys):
    """m = 1.5e6 rows needs more than the 64 MiB scratch for the PCG vectors
    alone: NYS_EINVAL, nothing launched, y untouched."""
    m = 1_500_000
    A = torch.ones((m, 1), dtype=torch.float64, device=DEV)
    d = torch.ones(1, dtype=torch.float64, device=DEV)
    rhs = torch.ones(m, dtype=torch.float64, device=DEV)
    y = torch.full((m,), 7.0, dtype=torch.float64, device=DEV)
    with pytest.raises(nys.NysError) as e:
        nys.nys_pcg_solve_noalloc(A, d, 1.0, rhs, y)
    assert e.value.code == -1 and "scratch" in str(e.value)
    torch.cuda.synchronize()
    assert bool((y == 7.0).all())
