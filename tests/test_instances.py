"""CPU checks of the seeded input generators against the recipes they state
(planted optimum, low-rank-plus-noise spectrum, SVM and portfolio forms).
The generators hold none of the method's arithmetic; these tests pin the
structure both the oracle and the GPU path are fed with."""

import numpy as np
import pytest
import torch

from instances import CONFIGS, make_instance, portfolio_instance, svm_instance
from instances import planted


def test_planted_optimum_recipe():
    inst = make_instance("lowrank_5000x20000", seed=3, m=120, n=500, rank=20)
    n = inst.n
    x, z, S = inst.x_star.numpy(), inst.z_star.numpy(), inst.support.numpy()
    assert S.sum() == n // 2
    assert np.all((x[S] >= 0.1) & (x[S] <= 1.0)) and np.all(x[~S] == 0)
    assert np.all((z[~S] >= 0.1) & (z[~S] <= 1.0)) and np.all(z[S] == 0)
    q = inst.q.numpy()
    assert np.count_nonzero(q == 0) == (3 * n) // 10 and np.all((q >= 0) & (q <= 1))
    A = inst.A.double().numpy()
    np.testing.assert_allclose(inst.b.numpy(), A @ x, rtol=1e-13, atol=1e-13)
    np.testing.assert_allclose(inst.c.numpy(), A.T @ inst.y_star.numpy() + z - q * x, rtol=1e-13, atol=1e-13)


@pytest.mark.parametrize("name", ["lowrank_5000x20000", "lowrank_20000x100000"])
def test_lowrank_spectrum_without_noise(name, monkeypatch):
    """U diag(i^-p) V^T with U, V orthonormal: with the noise switched off the
    singular values are exactly i^-p for i <= rank, and zero beyond."""
    cfg = dict(CONFIGS[name], noise=0.0, a_dtype="f64")
    monkeypatch.setitem(planted.CONFIGS, name, cfg)
    r = 12
    inst = make_instance(name, seed=1, m=60, n=150, rank=r)
    s = np.linalg.svd(inst.A.numpy(), compute_uv=False)
    i = np.arange(1, r + 1)
    np.testing.assert_allclose(s[:r], i ** -float(cfg["sigma_pow"]), rtol=1e-12)
    assert np.all(s[r:] < 1e-12)


def test_lowrank_noise_is_entrywise(monkeypatch):
    """noise 1e-3 means 1e-3 N(0, 1) per entry: the same draws with the noise
    switched off differ from the instance by entries of mean 0 and standard
    deviation 1e-3."""
    name = "lowrank_5000x20000"
    A = make_instance(name, seed=2, m=200, n=800, rank=10).A.double().numpy()
    monkeypatch.setitem(planted.CONFIGS, name, dict(CONFIGS[name], noise=0.0))
    A0 = make_instance(name, seed=2, m=200, n=800, rank=10).A.double().numpy()
    E = (A - A0) / 1e-3
    assert abs(E.std() - 1.0) < 0.01 and abs(E.mean()) < 0.01


def test_svm_form_recipe():
    d, n, tau = 6, 40, 0.7
    f = svm_instance(d, n, seed=4, tau=tau)
    A, yl = f["A"].numpy(), f["labels"].numpy()
    assert A.shape == (d + 1, d + n)
    assert np.count_nonzero(yl == 1) == n // 2 and np.count_nonzero(yl == -1) == n - n // 2
    np.testing.assert_array_equal(A[:d, :d], np.eye(d))
    np.testing.assert_array_equal(A[d, :d], np.zeros(d))
    np.testing.assert_array_equal(A[d, d:], yl)
    np.testing.assert_array_equal(f["c"].numpy(), np.concatenate([np.zeros(d), -np.ones(n)]))
    np.testing.assert_array_equal(f["q"].numpy(), np.concatenate([np.ones(d), np.zeros(n)]))
    np.testing.assert_array_equal(f["u"].numpy()[d:], np.full(n, tau))
    np.testing.assert_array_equal(f["vtype"].numpy(), np.concatenate([np.ones(d), np.full(n, 2)]))
    assert np.all(f["b"].numpy() == 0)
    # the unit layout: same draws, variables ordered [p; v], identity on v as unit columns
    fu = svm_instance(d, n, seed=4, tau=tau, unit_columns=True)
    np.testing.assert_array_equal(fu["A"].numpy(), A[:, d:])
    rows, vals = (t.numpy() for t in fu["units"])
    np.testing.assert_array_equal(rows, np.arange(d))
    np.testing.assert_array_equal(vals, np.ones(d))


def test_portfolio_form_recipe():
    n, d, s = 400, 100, 10
    f = portfolio_instance(n=n, d=d, s=s, seed=5, with_parts=True)
    F, Dg, M, u_p = f["F"].numpy(), f["Dg"].numpy(), f["M"].numpy(), f["u_p"].numpy()
    A = f["A"].numpy()
    m = s + d + 1
    assert A.shape == (m, n + s + d)
    # F = G_s diag(sqrt(lam + 0.1)): orthogonal columns, Gram = lam_i + 0.1, lam_i ~ i^-2 at the top
    G = F.T @ F
    np.testing.assert_allclose(G - np.diag(np.diag(G)), 0.0, atol=1e-12 * np.abs(G).max())
    lam = np.diag(G) - 0.1
    np.testing.assert_allclose(lam[0] / lam[1:], np.arange(2, s + 1) ** 2.0, rtol=1e-10)
    # mean variance 1: trace(F F^T) + sum(Dg) = n, and Dg > 0
    np.testing.assert_allclose(np.trace(G) + Dg.sum(), n, rtol=1e-12)
    assert np.all(Dg > 0)
    assert np.all((u_p >= 0.05) & (u_p <= 1.0))
    np.testing.assert_array_equal(A[:s, n:n + s], -np.eye(s))
    np.testing.assert_array_equal(A[s:s + d, n + s:], np.eye(d))
    np.testing.assert_array_equal(A[s + d, :n], np.ones(n))
    np.testing.assert_array_equal(A[:s, :n], F.T)
    np.testing.assert_array_equal(A[s:s + d, :n], M)
    q = f["q"].numpy()
    np.testing.assert_array_equal(q, np.concatenate([2 * Dg, np.full(s, 2.0), np.zeros(d)]))
    np.testing.assert_array_equal(f["vtype"].numpy(), np.concatenate([np.zeros(n), np.ones(s), np.zeros(d)]))
    np.testing.assert_array_equal(f["b"].numpy(), np.concatenate([np.zeros(s), u_p, [1.0]]))
    np.testing.assert_array_equal(f["c"].numpy(), np.concatenate([-f["r"].numpy(), np.zeros(s + d)]))


def test_generators_are_seeded():
    a = make_instance("gauss_200x500", seed=7)
    b = make_instance("gauss_200x500", seed=7)
    c = make_instance("gauss_200x500", seed=8)
    assert torch.equal(a.A, b.A) and torch.equal(a.c, b.c)
    assert not torch.equal(a.A, c.A)


def test_fp32_workloads_are_defined_by_the_stored_matrix():
    """The FP32 workloads define the problem by the stored FP32 matrix promoted
    exactly to FP64: b = A32 x* and c = A32^T y* + z* - Q x* in FP64."""
    inst = make_instance("gauss_2000x8000", seed=6, m=90, n=300)
    assert inst.A.dtype == torch.float32
    A = inst.A.double().numpy()
    x, y, z, q = inst.x_star.numpy(), inst.y_star.numpy(), inst.z_star.numpy(), inst.q.numpy()
    np.testing.assert_allclose(inst.b.numpy(), A @ x, rtol=1e-13, atol=1e-14)
    np.testing.assert_allclose(inst.c.numpy(), A.T @ y + z - q * x, rtol=1e-13, atol=1e-14)
