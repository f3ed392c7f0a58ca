"""Failure handling forced from the host: non-positive regularisation, an
iteration limit, an indefinite operator, an infeasible QP and a
rank-deficient A.  Each case ends with its documented status (include/
nysipm.h); where the oracle fixes values, the GPU result is compared with
them.  Every kernel still runs to its normal end: the conditions are in the
data, and the library's own checks turn them into status codes."""

import numpy as np
import pytest
import torch

from oracle import ippmm, nystrom, problem
from oracle import pcg as opcg

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


def _np(t):
    return t.detach().double().cpu().numpy()


def test_nonpositive_delta_is_rejected_with_the_preconditioner(nys):
    """eq. Nys_precond_inv needs delta > 0: NYS_EINVAL for 0, < 0 and NaN."""
    print("delta rejections", flush=True)
    rng = np.random.default_rng(1)
    m, n, ell = 50, 80, 5
    U, _ = np.linalg.qr(rng.standard_normal((m, ell)))
    P = nys.Precond(_t(U), _t(np.linspace(5.0, 1.0, ell)))
    r = _t(rng.standard_normal(m))
    for delta in (0.0, -1.0, float("nan")):
        with pytest.raises(nys.NysError) as e:
            nys.nys_precond_apply(P, delta, r)
        assert e.value.code == nys.nysipm.NYS_EINVAL
    A = _t(rng.standard_normal((m, n)))
    d = _t(rng.uniform(0.5, 1.5, n))
    with pytest.raises(nys.NysError) as e:
        nys.nys_pcg_solve(A, d, 0.0, r, P=P)
    assert e.value.code == nys.nysipm.NYS_EINVAL


def test_pcg_iteration_limit_returns_the_first_iterate(nys):
    """maxit = 1: NYS_MAXIT (a warning, no exception) and the first CG / PCG
    iterate, equal to the oracle's (the Nystrom factors come from the
    oracle)."""
    print("pcg maxit=1", flush=True)
    rng = np.random.default_rng(2)
    m, n, ell, delta = 300, 700, 10, 1e-2
    A = rng.standard_normal((m, n)) / np.sqrt(n)
    d = rng.uniform(0.1, 2.0, n)
    xi = rng.standard_normal(m)

    def M(v):
        return A @ (d * (A.T @ v)) + delta * v

    Om = nystrom.orthonormalize(rng.standard_normal((m, ell)))
    U, lam, _ = nystrom.nystrom(lambda V: A @ (d[:, None] * (A.T @ V)), Om)
    cases = ((None, None), (nys.Precond(_t(U), _t(lam)), lambda r: nystrom.precond_inv_apply(U, lam, delta, r)))
    for P, Pinv in cases:
        y, info = nys.nys_pcg_solve(_t(A), _t(d), delta, _t(xi), P=P, rtol=1e-14, maxit=1)
        assert info.status == nys.nysipm.NYS_MAXIT and info.iters == 1
        yo, it, tr, _ = opcg.pcg(M, xi, Pinv, tol=0.0, maxit=1)
        assert it == 1
        np.testing.assert_allclose(_np(y), yo, rtol=0, atol=1e-12 * np.linalg.norm(yo))
        assert abs(info.true_res - tr) <= 1e-10 * tr


def test_indefinite_operator_breaks_down(nys):
    """d < 0 makes A diag(d) A^T + delta I negative definite: PCG stops with
    NYS_EBREAKDOWN (p^T M p < 0 at the first step), and the sketch of
    N = A diag(d) A^T with NYS_ENOTPD (the shifted Gram matrix is never
    positive definite)."""
    print("indefinite operator", flush=True)
    rng = np.random.default_rng(3)
    m, n = 40, 90
    A = _t(rng.standard_normal((m, n)))
    d = _t(-np.ones(n))
    xi = _t(rng.standard_normal(m))
    with pytest.raises(nys.NysError) as e:
        nys.nys_pcg_solve(A, d, 1e-3, xi, rtol=1e-10, maxit=50)
    assert e.value.code == nys.nysipm.NYS_EBREAKDOWN
    with pytest.raises(nys.NysError) as e:
        nys.nys_sketch(A, d, 8, seed=1)
    assert e.value.code == nys.nysipm.NYS_ENOTPD


def test_infeasible_qp_stops_at_the_iteration_limit(nys):
    """Row 0 of A is positive and b_0 = -1, so no x >= 0 satisfies Ax = b:
    NYS_MAXIT (a warning) with the relative primal residual held far from
    zero (the oracle's run of the same iterations ends at 0.53)."""
    print("infeasible qp", flush=True)
    rng = np.random.default_rng(4)
    m, n = 3, 6
    A = rng.standard_normal((m, n))
    A[0] = rng.uniform(0.1, 1.0, n)
    b = rng.standard_normal(m)
    b[0] = -1.0
    c = rng.standard_normal(n)
    q = rng.uniform(0.5, 1.5, n)
    ref = ippmm.solve(A, b, c, q, tol=1e-8, max_iter=30)
    assert ref["status"] == 1 and ref["rp_rel"] > 0.5
    x, y, z, info = nys.ipm_solve(_t(A), _t(b), _t(c), _t(q), ell=2, tol=1e-8, max_iter=30)
    assert info.status == nys.nysipm.NYS_MAXIT
    assert info.rp_rel > 0.3
    assert np.all(_np(x) > 0) and np.all(_np(z) > 0)


def test_rank_deficient_constraints_still_converge(nys):
    """Two rows of A repeat others (rank m - 2): the regularisation keeps the
    normal equations definite, and the solve reaches the planted optimum
    (unique: Q > 0) with the KKT conditions met, measured on the CPU."""
    print("rank-deficient A", flush=True)
    rng = np.random.default_rng(3)
    m, n = 20, 60
    A = rng.standard_normal((m, n))
    A[1] = A[0]
    A[7] = 2.0 * A[3]
    xs = np.zeros(n)
    S = rng.choice(n, 25, replace=False)
    xs[S] = rng.uniform(0.1, 1.0, 25)
    ys = rng.standard_normal(m)
    zs = np.zeros(n)
    Sc = np.setdiff1d(np.arange(n), S)
    zs[Sc] = rng.uniform(0.1, 1.0, len(Sc))
    q = rng.uniform(0.5, 1.5, n)
    b = A @ xs
    c = A.T @ ys + zs - q * xs
    assert problem.kkt_measure(A, b, c, q, xs, ys, zs)["kkt"] < 1e-13
    tol = 1e-8
    x, y, z, info = nys.ipm_solve(_t(A), _t(b), _t(c), _t(q), ell=5, tol=tol)
    assert info.status == 0
    meas = problem.kkt_measure(A, b, c, q, _np(x), _np(y), _np(z))
    assert meas["kkt"] <= 1.01 * tol       # the same measure as the solver's stopping test
    assert np.linalg.norm(_np(x) - xs) <= 1e-6 * np.linalg.norm(xs)


def test_autograd_warns_when_a_solve_hits_its_iteration_limit(nys):
    """NysQP reports an unconverged forward solve and an unconverged adjoint
    PCG solve with NysConvergenceWarning instead of returning their last
    iterates silently.  The limits are forced from the host: two IP-PMM
    iterations, three PCG iterations per inner solve."""
    from instances import make_instance
    from paper_2404_14524_amd.autograd import NysConvergenceWarning, nys_qp
    print("autograd iteration-limit warnings", flush=True)
    inst = make_instance("gauss_200x500", seed=4)
    A, b, c, q = (_t(inst.A.double().numpy()), _t(inst.b.numpy()), _t(inst.c.numpy()), _t(inst.q.numpy()))
    c.requires_grad_(True)
    with pytest.warns(NysConvergenceWarning, match="forward"):
        x = nys_qp(A, b, c, q, ell=20, tol=1e-9, seed=0, max_iter=2, pcg_maxit=3)
    with pytest.warns(NysConvergenceWarning, match="backward"):
        (gc,) = torch.autograd.grad(0.5 * (x ** 2).sum(), (c,))
    assert torch.isfinite(gc).all()
