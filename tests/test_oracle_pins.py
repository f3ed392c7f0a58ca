"""CPU pins of the FP64 oracle against facts that do not come from the oracle
itself: the unreduced Newton system solved by dense LU, closed forms of the
Nystrom preconditioner, Krylov finite termination, the planted optimum,
brute-force KKT enumeration, finite differences, torch's BF16 rounding and
published Philox known-answer vectors."""

import os

import numpy as np
import pytest
import scipy.linalg as sla
import torch

from instances import make_instance, random_feasible_instance
from oracle import adjoint, bruteforce, ippmm, lowprec, normal_eq, nystrom, pcg, philox, problem

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _np(inst):
    return (inst.A.double().numpy(), inst.b.numpy(), inst.c.numpy(), inst.q.numpy())


@pytest.fixture(scope="module")
def small():
    return make_instance("gauss_200x500", seed=1)


# ---------------------------------------------------------------- problem

def test_planted_point_is_kkt(small):
    A, b, c, q = _np(small)
    x, y, z = small.x_star.numpy(), small.y_star.numpy(), small.z_star.numpy()
    meas = problem.kkt_measure(A, b, c, q, x, y, z)
    assert meas["kkt"] < 1e-14
    # strong duality at the planted optimum: primal = dual objective
    assert abs(problem.primal_objective(x, c, q) - problem.dual_objective(x, y, b, q)) < 1e-10
    assert np.all(x * z == 0) and np.all(x + z > 0)


def test_kkt_measure_hand_computed():
    """The stopping measure (reading of the termination test the paper defers
    to the original IP-PMM: relative primal and dual infeasibility and mu) on
    a point worked by hand: A = 10 I, b = [5, 12], c = [3, 4], q = [1, 0],
    x = [0.2, 0.8], y = [0.1, -0.1], z = [2.2, 0]:
    r_p = [3, 4], ||b|| = 13 -> 5/14; r_d = c + Qx - A^T y - z = [0, 5],
    ||c|| = 5 -> 5/6; mu = x^T z / n = 0.44/2 = 0.22; KKT = max = 5/6."""
    A = 10.0 * np.eye(2)
    b, c, q = np.array([5.0, 12.0]), np.array([3.0, 4.0]), np.array([1.0, 0.0])
    x, y, z = np.array([0.2, 0.8]), np.array([0.1, -0.1]), np.array([2.2, 0.0])
    meas = problem.kkt_measure(A, b, c, q, x, y, z)
    np.testing.assert_allclose([meas["rp_rel"], meas["rd_rel"], meas["mu"], meas["kkt"]],
                               [5 / 14, 5 / 6, 0.22, 5 / 6], rtol=1e-14)


def test_box_kkt_measure_hand_computed():
    """The box form's measure on the same data with x_0 in [0, 1] (box) and
    x_1 >= 0, w = [0.5, 0], s = [1, 0], z = [3.2, 0]: r_u = 1 - 0.2 - 0.5 = 0.3,
    ||u_J|| = 1 -> 0.15; r_d = c + Qx - A^T y - z + s = [0, 5] -> 5/6;
    mu = (0.2*3.2 + 0.8*0 + 0.5*1) / (2 + 1) = 0.38; KKT = 5/6."""
    from oracle import boxqp
    A = 10.0 * np.eye(2)
    b, c, q = np.array([5.0, 12.0]), np.array([3.0, 4.0]), np.array([1.0, 0.0])
    vt = np.array([boxqp.BOX, boxqp.NONNEG])
    u = np.array([1.0, 0.0])
    x, y, z = np.array([0.2, 0.8]), np.array([0.1, -0.1]), np.array([3.2, 0.0])
    w, s_ = np.array([0.5, 0.0]), np.array([1.0, 0.0])
    meas = boxqp.kkt_measure(A, b, c, q, u, vt, x, y, z, w, s_)
    np.testing.assert_allclose([meas["rp_rel"], meas["rd_rel"], meas["ru_rel"], meas["mu"], meas["kkt"]],
                               [5 / 14, 5 / 6, 0.15, 0.38, 5 / 6], rtol=1e-14)


# ---------------------------------------------------------------- normal equations

def test_normal_apply_equals_sum_of_rank_one_terms():
    rng = np.random.default_rng(0)
    A = rng.standard_normal((7, 11))
    d = rng.uniform(0.1, 2, 11)
    v = rng.standard_normal(7)
    expect = 0.3 * v
    for j in range(11):                       # sum_j d_j a_j (a_j^T v), column by column
        expect = expect + d[j] * A[:, j] * float(A[:, j] @ v)
    np.testing.assert_allclose(normal_eq.normal_apply(A, d, 0.3, v), expect, rtol=1e-13, atol=1e-13)
    np.testing.assert_allclose(normal_eq.normal_matrix(A, d, 0.3) @ v, expect, rtol=1e-13, atol=1e-13)


def _random_state(m, n, seed):
    rng = np.random.default_rng(seed)
    A = rng.standard_normal((m, n))
    q = rng.uniform(0, 1, n)
    q[: n // 4] = 0.0
    x = rng.uniform(0.01, 2, n)
    z = rng.uniform(0.01, 2, n)
    rd, rp, rxz = rng.standard_normal(n), rng.standard_normal(m), rng.standard_normal(n)
    return A, q, x, z, rd, rp, rxz


@pytest.mark.parametrize("rho,delta", [(1.0, 1.0), (1e-3, 1e-6), (8.0, 8.0)])
def test_newton_elimination_matches_dense_lu(rho, delta):
    A, q, x, z, rd, rp, rxz = _random_state(9, 23, 3)
    D = normal_eq.scaling(x, z, q, rho)
    M = normal_eq.normal_matrix(A, D, delta)
    dx, dy, dz, _ = normal_eq.newton_step(A, x, z, D, delta, rd, rp, rxz, lambda xi: np.linalg.solve(M, xi))
    ex, ey, ez = normal_eq.newton_dense_lu(A, q, x, z, rho, delta, rd, rp, rxz)
    for a, e in ((dx, ex), (dy, ey), (dz, ez)):
        assert np.linalg.norm(a - e) <= 1e-10 * (1 + np.linalg.norm(e))


def _central_jacobian(R, v, h=1e-3):
    """Jacobian of R at v by central differences (exact up to rounding for
    maps that are at most quadratic, as the residual maps here are)."""
    return np.column_stack([(R(v + h * e) - R(v - h * e)) / (2 * h) for e in np.eye(v.size)])


def test_newton_matrix_is_the_jacobian_of_the_pmm_residuals():
    """eq. Newton is Newton's method on the residuals of the PMM subproblem
    of (P): r_d + rho (x - zeta), r_p - delta (y - lambda) and the products
    x_j z_j.  The unreduced matrix must equal minus the Jacobian of that map,
    here differentiated numerically from problem.residuals (pinned by the
    planted KKT point)."""
    rng = np.random.default_rng(31)
    m, n = 5, 11
    A = rng.standard_normal((m, n))
    b, c = rng.standard_normal(m), rng.standard_normal(n)
    q = rng.uniform(0.0, 2.0, n)
    rho, delta = 0.7, 0.3
    zeta, lam = rng.standard_normal(n), rng.standard_normal(m)

    def R(v):
        x, y, z = v[:n], v[n:n + m], v[n + m:]
        rp, rd, _ = problem.residuals(A, b, c, q, x, y, z)
        return np.concatenate([rd + rho * (x - zeta), rp - delta * (y - lam), -x * z])

    x, y, z = rng.uniform(0.5, 2.0, n), rng.standard_normal(m), rng.uniform(0.5, 2.0, n)
    K = normal_eq.newton_matrix(A, q, x, z, rho, delta)
    np.testing.assert_allclose(K, -_central_jacobian(R, np.concatenate([x, y, z])), rtol=0, atol=1e-9)


def test_box_newton_matrix_is_the_jacobian_of_the_pmm_residuals():
    """The same for eq. Newton-free-box: rows r_d, r_p, r_u (box indices),
    x_j z_j (non-free indices) and w_j s_j (box indices), from
    boxqp.residuals (pinned by planted optima and brute force)."""
    from oracle import boxqp
    rng = np.random.default_rng(32)
    m, n = 4, 12
    A = rng.standard_normal((m, n))
    vt = _box_types(n, rng)
    F, I, J = boxqp.kinds(vt)
    IJ = I | J
    iJ, iIJ = np.flatnonzero(J), np.flatnonzero(IJ)
    b, c = rng.standard_normal(m), rng.standard_normal(n)
    q = rng.uniform(0.0, 2.0, n)
    u = np.where(J, rng.uniform(1.0, 3.0, n), 0.0)
    rho, delta = 0.4, 0.2
    zeta, lam = rng.standard_normal(n), rng.standard_normal(m)
    x = np.where(F, rng.standard_normal(n), rng.uniform(0.5, 2.0, n))
    y = rng.standard_normal(m)
    z = np.where(IJ, rng.uniform(0.5, 2.0, n), 0.0)
    w = np.where(J, rng.uniform(0.5, 2.0, n), 0.0)
    s = np.where(J, rng.uniform(0.5, 2.0, n), 0.0)
    K, (ox, oy, ow, oz, os_), _ = boxqp.newton_matrix(A, q, vt, x, z, w, s, rho, delta)

    def unpack(v):
        xv, yv = v[ox:ox + n], v[oy:oy + m]
        wv, zv, sv = np.zeros(n), np.zeros(n), np.zeros(n)
        wv[iJ], zv[iIJ], sv[iJ] = v[ow:ow + len(iJ)], v[oz:oz + len(iIJ)], v[os_:os_ + len(iJ)]
        return xv, yv, zv, wv, sv

    def R(v):
        xv, yv, zv, wv, sv = unpack(v)
        rp, rd, ru, _ = boxqp.residuals(A, b, c, q, u, vt, xv, yv, zv, wv, sv)
        return np.concatenate([rd + rho * (xv - zeta), rp - delta * (yv - lam), ru[iJ],
                               -(xv * zv)[iIJ], -(wv * sv)[iJ]])

    v = np.concatenate([x, y, w[iJ], z[iIJ], s[iJ]])
    np.testing.assert_allclose(K, -_central_jacobian(R, v), rtol=0, atol=1e-9)


def test_combined_corrector_solve_is_the_sum_of_the_two_solves():
    """Algorithm 6 sums the predictor and corrector directions, both solutions
    of systems with one matrix: a single solve with the summed right-hand
    side (r_d, r_p, -XZ + mu~ - dXp dZp) gives the same direction, as the GPU
    path computes it.  Checked for the non-negative and the box forms."""
    from oracle import boxqp
    A, q, x, z, rd, rp, _ = _random_state(8, 21, 5)
    rho, delta, mu_t = 0.2, 0.1, 0.05
    D = normal_eq.scaling(x, z, q, rho)
    M = normal_eq.normal_matrix(A, D, delta)
    exact = lambda xi: np.linalg.solve(M, xi)
    m, n = A.shape
    dxp, dyp, dzp, _ = normal_eq.newton_step(A, x, z, D, delta, rd, rp, -x * z, exact)
    rc = mu_t - dxp * dzp
    dxc, dyc, dzc, _ = normal_eq.newton_step(A, x, z, D, delta, np.zeros(n), np.zeros(m), rc, exact)
    dx, dy, dz, _ = normal_eq.newton_step(A, x, z, D, delta, rd, rp, -x * z + rc, exact)
    for a, e in ((dx, dxp + dxc), (dy, dyp + dyc), (dz, dzp + dzc)):
        np.testing.assert_allclose(a, e, rtol=1e-10, atol=1e-12)
    rng = np.random.default_rng(6)
    vt = _box_types(n, rng)
    F, I, J = boxqp.kinds(vt)
    IJ = I | J
    xb = np.where(F, rng.standard_normal(n), x)
    zb = np.where(IJ, z, 0.0)
    w = np.where(J, rng.uniform(0.5, 2.0, n), 0.0)
    sb = np.where(J, rng.uniform(0.5, 2.0, n), 0.0)
    ru = np.where(J, rng.standard_normal(n), 0.0)
    Db = boxqp.scaling(vt, xb, zb, w, sb, q, rho)
    Mb = (A * Db) @ A.T + delta * np.eye(m)
    exb = lambda xi: np.linalg.solve(Mb, xi)
    rxz, rws = np.where(IJ, -xb * zb, 0.0), np.where(J, -w * sb, 0.0)
    p = boxqp.newton_step(A, vt, xb, zb, w, sb, Db, delta, rd, rp, ru, rxz, rws, exb)
    rcz = np.where(IJ, mu_t - p[0] * p[2], 0.0)
    rcs = np.where(J, mu_t - p[3] * p[4], 0.0)
    zn = np.zeros(n)
    c_ = boxqp.newton_step(A, vt, xb, zb, w, sb, Db, delta, zn, np.zeros(m), zn, rcz, rcs, exb)
    t = boxqp.newton_step(A, vt, xb, zb, w, sb, Db, delta, rd, rp, ru, rxz + rcz, rws + rcs, exb)
    for a, e1, e2 in zip(t, p, c_):
        np.testing.assert_allclose(a, e1 + e2, rtol=1e-10, atol=1e-12)


def test_inexact_newton_only_second_block_is_inexact():
    """Proposition 3.1: with an inexact normal-equation solve, blocks 1 and 3
    of the unreduced Newton residual vanish and block 2 equals the residual
    of the normal equations."""
    A, q, x, z, rd, rp, rxz = _random_state(12, 30, 4)
    rho, delta = 0.5, 0.25
    D = normal_eq.scaling(x, z, q, rho)
    Mop = lambda v: normal_eq.normal_apply(A, D, delta, v)

    def truncated(xi):
        return pcg.pcg(Mop, xi, None, tol=0.0, maxit=3)[0]

    dx, dy, dz, xi = normal_eq.newton_step(A, x, z, D, delta, rd, rp, rxz, truncated)
    K = normal_eq.newton_matrix(A, q, x, z, rho, delta)
    res = K @ np.concatenate([dx, dy, dz]) - np.concatenate([rd, rp, rxz])
    m, n = A.shape
    theta = Mop(dy) - xi
    assert np.linalg.norm(theta) > 1e-3                        # really inexact
    assert np.linalg.norm(res[:n]) < 1e-12 * (1 + np.linalg.norm(rd))
    assert np.linalg.norm(res[n + m:]) < 1e-12 * (1 + np.linalg.norm(rxz))
    np.testing.assert_allclose(res[n:n + m], theta, rtol=1e-10, atol=1e-12)


# ---------------------------------------------------------------- Nystrom

def _lowrank_psd(m, r, seed, decay=1.0):
    rng = np.random.default_rng(seed)
    U, _ = np.linalg.qr(rng.standard_normal((m, r)))
    lam = np.arange(1, r + 1) ** -decay
    return (U * lam) @ U.T


def test_nystrom_exact_when_sketch_exceeds_rank():
    m, r, ell = 120, 15, 25
    N = _lowrank_psd(m, r, 0)
    Om = nystrom.orthonormalize(np.random.default_rng(1).standard_normal((m, ell)))
    U, lam, nu = nystrom.nystrom(lambda V: N @ V, Om)
    Nh = (U * lam) @ U.T
    assert np.linalg.norm(N - Nh, 2) <= 1e-12 * np.linalg.norm(N, 2)
    assert np.all(lam >= 0) and np.all(np.diff(lam) <= 0)
    np.testing.assert_allclose(U.T @ U, np.eye(ell), atol=1e-12)
    assert np.count_nonzero(lam > 1e-10) == r


def test_nystrom_matches_formula_and_is_dominated():
    m, ell = 80, 12
    rng = np.random.default_rng(2)
    N = _lowrank_psd(m, m, 3, decay=2.0)
    Om = nystrom.orthonormalize(rng.standard_normal((m, ell)))
    Y = N @ Om
    U, lam, nu = nystrom.nystrom_from_sketch(Y, Om)
    Nh = (U * lam) @ U.T
    F = nystrom.nystrom_formula(Y, Om)
    assert np.linalg.norm(Nh - F, 2) <= 1e-8 * np.linalg.norm(N, 2)
    ev = np.linalg.eigvalsh(N - Nh)                  # 0 <= N_hat <= N up to O(nu)
    assert ev.min() >= -10 * nu * m
    assert np.linalg.eigvalsh(Nh).min() >= -10 * nu * m


def test_nystrom_invariant_under_rotation_of_test_matrix():
    m, ell = 60, 10
    rng = np.random.default_rng(4)
    N = _lowrank_psd(m, m, 5, decay=1.5)
    Om = rng.standard_normal((m, ell))
    R = rng.standard_normal((ell, ell))
    U1, l1, _ = nystrom.nystrom(lambda V: N @ V, nystrom.orthonormalize(Om))
    U2, l2, _ = nystrom.nystrom(lambda V: N @ V, nystrom.orthonormalize(Om @ R))
    np.testing.assert_allclose((U1 * l1) @ U1.T, (U2 * l2) @ U2.T, atol=1e-10)


def test_eps_at_matches_library_spacing():
    for v in (1.0, 3.7, 1e-5, 12345.678):
        assert nystrom.eps_at(v, "f64") == np.spacing(v)
        assert nystrom.eps_at(v, "f32") == float(np.spacing(np.float32(v)))
    assert nystrom.eps_at(1.0, "bf16") == torch.finfo(torch.bfloat16).eps


def test_preconditioner_closed_forms():
    m, ell, delta = 50, 8, 0.05
    rng = np.random.default_rng(6)
    U, _ = np.linalg.qr(rng.standard_normal((m, ell)))
    lam = np.sort(rng.uniform(0, 10, ell))[::-1]
    P = nystrom.precond_dense(U, lam, delta)
    Pinv = nystrom.precond_inv_dense(U, lam, delta)
    np.testing.assert_allclose(P @ Pinv, np.eye(m), atol=1e-12)
    np.testing.assert_allclose(Pinv, np.linalg.inv(P), atol=1e-10)
    R = rng.standard_normal((m, 3))
    np.testing.assert_allclose(nystrom.precond_inv_apply(U, lam, delta, R), np.linalg.solve(P, R), atol=1e-10)
    # Table 2: one apply costs 2 ell m + m + 5 ell flops; eigenvalues of P^{-1}
    # are 1 (on the complement) and (lam_l+delta)/(lam_i+delta) on range(U)
    ev = np.sort(np.linalg.eigvalsh(0.5 * (Pinv + Pinv.T)))
    expect = np.sort(np.concatenate([(lam.min() + delta) / (lam + delta), np.ones(m - ell)]))
    np.testing.assert_allclose(ev, expect, atol=1e-12)


@pytest.mark.parametrize("extra", [5, 0])
def test_pcg_finite_termination_with_exact_rank_preconditioner(extra):
    """N of exact rank r: with ell > r the preconditioned operator is delta*I
    (one iteration); with ell = r it has two eigenvalues (two iterations)."""
    m, r, delta = 100, 10, 1e-3
    N = _lowrank_psd(m, r, 7)
    Om = nystrom.orthonormalize(np.random.default_rng(8).standard_normal((m, r + extra)))
    U, lam, _ = nystrom.nystrom(lambda V: N @ V, Om)
    M = N + delta * np.eye(m)
    xi = np.random.default_rng(9).standard_normal(m)
    y, it, tr, _ = pcg.pcg(lambda v: M @ v, xi, lambda v: nystrom.precond_inv_apply(U, lam, delta, v),
                           tol=1e-9 * np.linalg.norm(xi), maxit=50)
    assert it == (1 if extra else 2)
    np.testing.assert_allclose(y, np.linalg.solve(M, xi), rtol=1e-7)


def test_pcg_matches_dense_solve():
    rng = np.random.default_rng(10)
    B = rng.standard_normal((40, 60))
    M = B @ B.T + 0.1 * np.eye(40)
    xi = rng.standard_normal(40)
    y, it, tr, _ = pcg.pcg(lambda v: M @ v, xi, None, tol=1e-12, maxit=400)
    np.testing.assert_allclose(y, sla.solve(M, xi, assume_a="pos"), rtol=1e-9)
    assert tr <= 1e-11


@pytest.mark.parametrize("precond", [False, True])
def test_pcg_iterate_is_the_krylov_galerkin_solution(precond):
    """After k steps from y = 0, (P)CG's iterate is the M-norm best
    approximation of M^{-1} xi in the Krylov space K_k(P^{-1} M, P^{-1} xi):
    y = V (V^T M V)^{-1} V^T xi for any basis V of that space.  A wrong sign
    or index in alpha, beta or the direction update leaves this space or this
    optimum at k >= 2."""
    rng = np.random.default_rng(21)
    m = 30
    B = rng.standard_normal((m, m))
    M = B @ B.T + 3.0 * np.eye(m)
    xi = rng.standard_normal(m)
    C = rng.standard_normal((m, m))
    G = C @ C.T / m + np.eye(m) if precond else np.eye(m)        # P^{-1}, SPD
    for k in (1, 2, 3, 6):
        y, it, _, _ = pcg.pcg(lambda v: M @ v, xi, (lambda r: G @ r) if precond else None, tol=0.0, maxit=k)
        assert it == k
        K = [G @ xi]
        for _ in range(k - 1):
            K.append(G @ (M @ K[-1]))
        V, _ = np.linalg.qr(np.array(K).T)
        yk = V @ np.linalg.solve(V.T @ M @ V, V.T @ xi)
        np.testing.assert_allclose(y, yk, rtol=0, atol=1e-10 * np.linalg.norm(yk))


# ---------------------------------------------------------------- IP-PMM

def test_step_length_fraction_to_boundary():
    rng = np.random.default_rng(11)
    v = rng.uniform(0.1, 1, 200)
    dv = rng.standard_normal(200)
    a = ippmm.step_length(v, dv)
    assert np.all(v + a * dv > 0)
    j = np.argmin(np.where(dv < 0, -v / np.where(dv < 0, dv, -1), np.inf))
    np.testing.assert_allclose(v[j] + a / 0.995 * dv[j], 0.0, atol=1e-12)
    assert ippmm.step_length(v, np.abs(dv)) == 0.995


def test_ippmm_reaches_planted_optimum(small):
    A, b, c, q = _np(small)
    r = ippmm.solve(A, b, c, q, tol=1e-10)
    assert r["status"] == 0 and r["kkt"] <= 1e-10
    xs = small.x_star.numpy()
    assert np.linalg.norm(r["x"] - xs) <= 1e-8 * np.linalg.norm(xs)
    np.testing.assert_allclose(r["y"], small.y_star.numpy(), atol=1e-7)
    xp, yp, zp, ok = ippmm.polish(A, b, c, q, r["x"], r["y"], r["z"])
    assert ok and np.linalg.norm(xp - xs) <= 1e-12 * np.linalg.norm(xs)
    assert np.all(r["x"] > 0) and np.all(r["z"] > 0)


def test_ippmm_lowrank_zero_curvature_instance():
    inst = make_instance("lowrank_5000x20000", seed=2, m=300, n=1200, rank=30)
    A, b, c, q = _np(inst)
    assert np.count_nonzero(q == 0) == 360
    r = ippmm.solve(A, b, c, q, tol=1e-9)
    xs = inst.x_star.numpy()
    assert r["status"] == 0
    assert np.linalg.norm(r["x"] - xs) <= 1e-6 * np.linalg.norm(xs)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_ippmm_matches_bruteforce(seed):
    d = {k: v.numpy() for k, v in random_feasible_instance(4, 10, seed).items()}
    best = bruteforce.optimum(d["A"], d["b"], d["c"], d["q"])
    r = ippmm.solve(d["A"], d["b"], d["c"], d["q"], tol=1e-11)
    assert r["status"] == 0
    obj = problem.primal_objective(r["x"], d["c"], d["q"])
    assert abs(obj - best["obj"]) <= 1e-8 * (1 + abs(best["obj"]))
    np.testing.assert_allclose(r["x"], best["x"], atol=1e-6)     # Q > 0: unique optimum


def test_initial_point_is_interior(small):
    A, b, c, q = _np(small)
    x0, y0, z0 = ippmm.initial_point(A, b, c, q)
    assert np.all(x0 > 0) and np.all(z0 > 0)
    m, n = A.shape
    # candidates as Tikhonov least-squares problems solved by a library lstsq:
    # x~ = argmin ||A x - b||^2 + 10 ||x||^2 (push-through identity), and
    # y~ = argmin ||A^T y - (c + Q x~)||^2 + 10 ||y||^2
    xt = np.linalg.lstsq(np.vstack([A, np.sqrt(10) * np.eye(n)]), np.concatenate([b, np.zeros(n)]),
                         rcond=None)[0]
    yt = np.linalg.lstsq(np.vstack([A.T, np.sqrt(10) * np.eye(m)]),
                         np.concatenate([c + q * xt, np.zeros(m)]), rcond=None)[0]
    np.testing.assert_allclose(y0, yt, atol=1e-10)
    zt = c - A.T @ yt + q * xt
    sx, sz = x0 - xt, z0 - zt            # the shifts are constant vectors
    assert np.ptp(sx) < 1e-10 and np.ptp(sz) < 1e-10
    dp = max(-1.5 * xt.min(), 0.0)
    dd = max(-1.5 * zt.min(), 0.0)
    gamma = (xt + dp) @ (zt + dd)
    np.testing.assert_allclose(sx[0], dp + 0.5 * gamma / np.sum(zt + dd), rtol=1e-9)
    np.testing.assert_allclose(sz[0], dd + 0.5 * gamma / np.sum(xt + dp), rtol=1e-9)


def _frac_vec(vals):
    from fractions import Fraction
    return np.array([float(Fraction(v)) for v in vals])


def _load_initial_point_cases():
    import json
    with open(os.path.join(GOLDEN, "initial_point_cases.json")) as f:
        return json.load(f)["cases"]


@pytest.mark.parametrize("case", _load_initial_point_cases(), ids=lambda c: c["name"])
def test_initial_point_hand_derived_cases(case):
    """The supplement's initial point on tiny problems whose every step was
    worked out by hand in exact rational arithmetic (tests/golden/
    initial_point_cases.json, with the derivation): x0, y0, z0 (and w0, s0 in
    the box form) equal the hand values, and the dual shift is the one of the
    (x~ + delta_p) reading, not of the printed (x~ + delta_d) form, which the
    fixture also records."""
    from oracle import boxqp
    A = np.array(case["A"], dtype=np.float64)
    b, c, q = (np.array(case[k], dtype=np.float64) for k in ("b", "c", "q"))
    if case["kind"] == "P":
        x0, y0, z0 = ippmm.initial_point(A, b, c, q)
        got = dict(x0=x0, y0=y0, z0=z0)
    else:
        kind = {"nonneg": boxqp.NONNEG, "free": boxqp.FREE, "box": boxqp.BOX}
        vt = np.array([kind[v] for v in case["vtype"]])
        u = np.array(case["u"], dtype=np.float64)
        x0, y0, z0, w0, s0 = boxqp.initial_point(A, b, c, q, u, vt)
        got = dict(x0=x0, y0=y0, z0=z0, w0=w0, s0=s0)
    for key, val in got.items():
        np.testing.assert_allclose(val, _frac_vec(case[key]), rtol=1e-14, atol=1e-15, err_msg=key)
    if "printed_z0" in case:
        assert np.max(np.abs(got["z0"] - _frac_vec(case["printed_z0"]))) > 1e-3


def _peu_check(hist):
    """The parameter update against what the paper fixes: rho_0 = delta_0 = 8
    (Algorithm 4); the published trajectories (the regularisation tables of
    the supplement) never increase and end at the floor 5e-10; the theory's
    choice rho_k = delta_k = mu_k (section 2.1.2, section 3) wherever mu_k lies
    between that floor and the previous value.  Returns which branches ran."""
    floor = 5e-10
    assert hist[0]["rho"] == 8.0 and hist[0]["delta"] == 8.0
    seen = set()
    for k in range(1, len(hist)):
        rho, delta, mu = hist[k]["rho"], hist[k]["delta"], hist[k]["mu"]
        prev = hist[k - 1]["rho"]
        assert rho == delta, k
        assert floor <= rho <= prev, k
        if floor <= mu <= prev:
            assert rho == mu, k
            seen.add("mu")
        elif mu < floor:
            assert rho == floor, k
            seen.add("floor")
        else:
            assert rho == prev, k
            seen.add("hold")
    return seen


def test_parameter_update_follows_the_paper():
    inst = make_instance("gauss_200x500", seed=5, m=40, n=100)
    A, b, c, q = _np(inst)
    hist = []
    r = ippmm.solve(A, b, c, q, tol=1e-12, max_iter=60, history=hist)
    assert r["status"] == 0
    seen = _peu_check(hist)
    assert {"mu", "floor", "hold"} <= seen, seen
    assert hist[-1]["rho"] == 5e-10


def test_box_parameter_update_follows_the_paper():
    from oracle import boxqp
    rng = np.random.default_rng(21)
    m, n = 12, 40
    A = rng.standard_normal((m, n)) / np.sqrt(n)
    vt = _box_types(n, rng)
    q = rng.uniform(0.5, 1.5, n)
    u = np.where(vt == 2, rng.uniform(0.5, 2.0, n), 0.0)
    b, c, *_ = boxqp.planted(A, q, vt, u, rng)
    hist = []
    # data scaled by 10 (the optimum scales with it): mu rises above rho at
    # some iterations, so all three branches of the rule run
    r = boxqp.solve(A, 10 * b, 10 * c, q, 10 * u, vt, tol=1e-12, max_iter=60, history=hist)
    assert r["status"] == 0
    seen = _peu_check(hist)
    assert {"mu", "floor", "hold"} <= seen, seen


# ---------------------------------------------------------------- adjoint

def test_adjoint_matches_finite_differences():
    inst = make_instance("gauss_2000x8000", seed=3, m=30, n=80)
    A, b, c, q = _np(inst)
    x, y, z = inst.x_star.numpy(), inst.y_star.numpy(), inst.z_star.numpy()
    S = x > 0
    x_tgt = x + 0.01 * np.random.default_rng(12).standard_normal(x.shape)
    g = x - x_tgt
    grad = adjoint.kkt_gradient(A, b, c, q, x, y, z, g)
    rng = np.random.default_rng(13)
    for block, size in (("c", 80), ("b", 30), ("q", 80), ("A", 30 * 80)):
        coords = rng.choice(size, 16, replace=False)
        fd = adjoint.fd_gradient(A, b, c, q, S, x_tgt, block, coords)
        an = grad[block].reshape(-1)[coords]
        assert np.linalg.norm(an - fd) <= 1e-7 * max(np.linalg.norm(fd), 1e-12), block


def test_fd_with_reused_factorisation_matches_full_resolves():
    inst = make_instance("gauss_2000x8000", seed=4, m=25, n=60)
    A, b, c, q = _np(inst)
    x = inst.x_star.numpy()
    S = x > 0
    x_tgt = x + 0.01 * np.random.default_rng(16).standard_normal(x.shape)
    for block, size in (("c", 60), ("b", 25)):
        coords = np.arange(size)
        full = adjoint.fd_gradient(A, b, c, q, S, x_tgt, block, coords)
        fast = adjoint.fd_gradient_rhs(A, b, c, q, S, x_tgt, block, coords)
        np.testing.assert_allclose(fast, full, rtol=1e-6, atol=1e-10)


@pytest.mark.parametrize("block", ["q", "A"])
def test_fd_through_low_rank_updates_matches_full_resolves(block):
    """Central differences for the matrix blocks (q, A) by Sherman-Morrison-
    Woodbury re-solves on one factorisation equal those by full re-solves,
    and both equal the dense reduced-KKT gradient."""
    inst = make_instance("gauss_2000x8000", seed=6, m=20, n=50)
    A, b, c, q = _np(inst)
    x, y, z = inst.x_star.numpy(), inst.y_star.numpy(), inst.z_star.numpy()
    S = x > 0
    x_tgt = x + 0.01 * np.random.default_rng(17).standard_normal(x.shape)
    size = 50 if block == "q" else 20 * 50
    coords = np.random.default_rng(18).choice(size, 24, replace=False)
    full = adjoint.fd_gradient(A, b, c, q, S, x_tgt, block, coords)
    fast = adjoint.fd_gradient_lowrank(A, b, c, q, S, x_tgt, block, coords)
    np.testing.assert_allclose(fast, full, rtol=1e-6, atol=1e-10)
    grad = adjoint.kkt_gradient(A, b, c, q, x, y, z, x - x_tgt)[block].reshape(-1)[coords]
    assert np.linalg.norm(fast - grad) <= 1e-7 * np.linalg.norm(grad)
    assert np.count_nonzero(fast) > 0
    # at a large step the re-solves still agree to rounding (they are exact,
    # not a linearisation), while the difference quotient moves by O(h^2)
    full = adjoint.fd_gradient(A, b, c, q, S, x_tgt, block, coords[:8], h_rel=1e-2)
    fast = adjoint.fd_gradient_lowrank(A, b, c, q, S, x_tgt, block, coords[:8], h_rel=1e-2)
    np.testing.assert_allclose(fast, full, rtol=1e-9, atol=1e-12)


# ---------------------------------------------------------------- low precision, RNG

def test_bf16_rounding_matches_torch_and_ties_to_even():
    rng = np.random.default_rng(14)
    v = rng.standard_normal(20000) * np.exp(rng.uniform(-20, 20, 20000))
    v32 = v.astype(np.float32)
    ref = torch.from_numpy(v32).to(torch.bfloat16).to(torch.float64).numpy()
    np.testing.assert_array_equal(lowprec.round_bf16(v32.astype(np.float64)), ref)
    assert lowprec.round_bf16(np.array([1.0 + 2.0 ** -8]))[0] == 1.0           # tie -> even
    assert lowprec.round_bf16(np.array([1.0 + 3 * 2.0 ** -8]))[0] == 1.0 + 2.0 ** -6
    assert lowprec.round_f32(np.array([1.0 + 2.0 ** -24]))[0] == 1.0


def test_bf16_sketch_rounding_points_hand_derived():
    """The three BF16 roundings of the mixed sketch (A, Omega and W, each round
    to nearest even through FP32) on a 4 x 3 case where each one changes the
    result.  Worked by hand (BF16 keeps 8 significant bits: spacing 2^-7 on
    [1, 2)):
      A[3,2] = 1 + 3*2^-9 -> 1 + 2^-7 (0x3F81);  Omega[0] = 1 + 3*2^-9 -> 1 + 2^-7;
      Omega = [1 + 2^-7, -1, 1, 1];  A^T Omega = [2^-7, 1, 1 + 2^-7];
      W = d .* A^T Omega = [2^-7, 1 + 2^-8 (a tie: to even, 1), 1 + 2^-7];
      Y = A W = [2^-7, 2^-7, 1, (1 + 2^-7)^2 = 1 + 2^-6 + 2^-14].
    Dropping the rounding of Omega gives Y[0] = 3*2^-9, of W gives
    Y[2] = 1 + 2^-8, of A gives Y[3] = (1 + 3*2^-9)(1 + 2^-7)."""
    e = 2.0 ** -9
    A32 = np.zeros((4, 3))
    A32[0, 0] = A32[1, 0] = A32[2, 1] = 1.0
    A32[3, 2] = 1.0 + 3 * e
    Om = np.array([[1.0 + 3 * e], [-1.0], [1.0], [1.0]])
    d = np.array([1.0, 1.0 + 2.0 ** -8, 1.0])
    assert [int(v) for v in lowprec.bf16_bits(np.array([1 + 3 * e, -1.0, 2.0 ** -7, 1 + 2.0 ** -8],
                                                         dtype=np.float32))] == [0x3F81, 0xBF80, 0x3C00, 0x3F80]
    Y = lowprec.sketch_bf16(A32, d, Om)
    np.testing.assert_array_equal(Y[:, 0], [2.0 ** -7, 2.0 ** -7, 1.0, 1.0 + 2.0 ** -6 + 2.0 ** -14])
    # each rounding matters: the same product without it differs
    Ab, Ob = lowprec.round_bf16(A32), lowprec.round_bf16(Om)
    no_om = Ab @ lowprec.round_bf16(d[:, None] * (Ab.T @ Om))
    no_w = Ab @ (d[:, None] * (Ab.T @ Ob))
    no_a = A32 @ lowprec.round_bf16(d[:, None] * (A32.T @ Ob))
    assert no_om[0, 0] == 3 * e and no_w[2, 0] == 1.0 + 2.0 ** -8
    assert no_a[3, 0] == (1.0 + 3 * e) * (1.0 + 2.0 ** -7)


def test_bf16_sketch_exact_on_representable_data():
    rng = np.random.default_rng(15)
    A = rng.integers(-8, 8, (20, 30)).astype(np.float64)
    Om = rng.integers(-4, 4, (20, 3)).astype(np.float64)
    d = np.full(30, 0.5)
    W = d[:, None] * (A.T @ Om)                  # small integers / 2: exact in BF16
    assert np.all(lowprec.round_bf16(W) == W)
    np.testing.assert_array_equal(lowprec.sketch_bf16(A, d, Om), A @ W)


def test_philox_known_answers():
    with open(os.path.join(GOLDEN, "philox4x32_10_kat.txt")) as f:
        rows = [ln.split() for ln in f if ln.strip() and not ln.startswith("#")]
    assert len(rows) == 3
    for row in rows:
        v = [int(t, 16) for t in row]
        out = philox.philox4x32_10(*v[:6])
        assert [int(o) for o in out] == v[6:]


def test_philox_gaussian_distribution():
    from scipy import stats
    G = philox.gaussian_matrix(400, 50, seed=123, counter=7)
    assert G.shape == (400, 50)
    assert abs(G.mean()) < 0.02 and abs(G.std() - 1) < 0.02
    assert stats.kstest(G.ravel(), "norm").pvalue > 1e-3
    G2 = philox.gaussian_matrix(400, 50, seed=123, counter=8)
    assert abs(np.corrcoef(G.ravel(), G2.ravel())[0, 1]) < 0.02
    np.testing.assert_array_equal(G, philox.gaussian_matrix(400, 50, seed=123, counter=7))


# ------------------------------------------------------------------ partial Cholesky (comparator)

def _pchol_case(m=40, n=90, seed=0):
    rng = np.random.default_rng(seed)
    A = rng.standard_normal((m, n)) * rng.uniform(0.2, 3.0, m)[:, None]   # uneven row scales
    d = rng.uniform(0.05, 4.0, n)
    return A, d, 1e-3


def test_pchol_inverse_formula_matches_dense_preconditioner():
    """eq. chol-precond-inv applied factor by factor equals a library solve
    with P_Chol assembled from eq. chol-precond."""
    from oracle import pchol
    A, d, delta = _pchol_case()
    P = pchol.build(A, d, delta, 12)
    Pd = pchol.precond_dense(P)
    r = np.random.default_rng(1).standard_normal(A.shape[0])
    np.testing.assert_allclose(pchol.precond_inv_apply(P, r), np.linalg.solve(Pd, r), rtol=1e-10, atol=1e-12)


def test_pchol_reproduces_pivot_block_and_diagonal():
    """P_Chol agrees with N + delta I exactly on the pivot rows and columns
    (L11, L21 are its exact Cholesky columns) and on the whole diagonal (diag S
    is exact); the pivots carry the ell largest diagonal entries."""
    from oracle import pchol
    A, d, delta = _pchol_case(seed=2)
    ell = 9
    P = pchol.build(A, d, delta, ell)
    Pd, Nd = pchol.precond_dense(P), P["Ndelta"]
    piv = P["piv"]
    np.testing.assert_allclose(Pd[:, piv], Nd[:, piv], rtol=1e-12, atol=1e-12 * np.abs(Nd).max())
    np.testing.assert_allclose(np.diag(Pd), np.diag(Nd), rtol=1e-12)
    np.testing.assert_allclose(pchol.normal_diag(A, d, delta), np.diag(Nd), rtol=1e-13)
    rest = P["rest"]
    assert np.diag(Nd)[piv].min() >= np.diag(Nd)[rest].max()
    assert len(piv) == ell and np.all(np.diff(piv) > 0)


def test_pchol_full_rank_is_exact():
    """ell = m: no Schur complement is left, P_Chol = N + delta I and the
    inverse formula is the exact inverse."""
    from oracle import pchol
    A, d, delta = _pchol_case(m=15, n=40, seed=3)
    P = pchol.build(A, d, delta, 15)
    np.testing.assert_allclose(pchol.precond_dense(P), P["Ndelta"], rtol=1e-12, atol=1e-12)
    r = np.random.default_rng(4).standard_normal(15)
    np.testing.assert_allclose(pchol.precond_inv_apply(P, r), np.linalg.solve(P["Ndelta"], r), rtol=1e-9)


def test_pchol_pivot_ties_go_to_smaller_index():
    from oracle import pchol
    piv = pchol.pivots(np.array([1.0, 3.0, 2.0, 3.0, 3.0, 0.5]), 2)
    np.testing.assert_array_equal(piv, [1, 3])


# ------------------------------------------------------------------ free and box-constrained variables

def _box_types(n, rng):
    return rng.choice([0, 1, 2], size=n, p=[0.4, 0.2, 0.4])


def test_box_newton_step_matches_unreduced_system():
    """Algorithm 5 (xi_au by index kind, normal equations, closed-form
    back-substitution) equals a dense solve of eq. Newton-free-box."""
    from oracle import boxqp
    rng = np.random.default_rng(0)
    m, n = 7, 19
    A = rng.standard_normal((m, n))
    vt = _box_types(n, rng)
    F, I, J = boxqp.kinds(vt)
    q = rng.uniform(0.0, 1.0, n)
    x = np.where(F, rng.standard_normal(n), rng.uniform(0.2, 2.0, n))
    z = np.where(F, 0.0, rng.uniform(0.2, 2.0, n))
    w = np.where(J, rng.uniform(0.2, 2.0, n), 0.0)
    s = np.where(J, rng.uniform(0.2, 2.0, n), 0.0)
    rho, delta = 0.3, 0.05
    rd, rp = rng.standard_normal(n), rng.standard_normal(m)
    ru = np.where(J, rng.standard_normal(n), 0.0)
    rxz = np.where(F, 0.0, rng.standard_normal(n))
    rws = np.where(J, rng.standard_normal(n), 0.0)
    D = boxqp.scaling(vt, x, z, w, s, q, rho)
    M = (A * D) @ A.T + delta * np.eye(m)
    dx, dy, dz, dw, ds = boxqp.newton_step(A, vt, x, z, w, s, D, delta, rd, rp, ru, rxz, rws,
                                           lambda xi: np.linalg.solve(M, xi))
    K, (ox, oy, ow, oz, os_), (iJ, iIJ) = boxqp.newton_matrix(A, q, vt, x, z, w, s, rho, delta)
    rhs = np.concatenate([rd, rp, ru[iJ], rxz[iIJ], rws[iJ]])
    sol = np.linalg.solve(K, rhs)
    np.testing.assert_allclose(dx, sol[ox:ox + n], rtol=1e-9, atol=1e-11)
    np.testing.assert_allclose(dy, sol[oy:oy + m], rtol=1e-9, atol=1e-11)
    np.testing.assert_allclose(dw[iJ], sol[ow:ow + len(iJ)], rtol=1e-9, atol=1e-11)
    np.testing.assert_allclose(dz[iIJ], sol[oz:oz + len(iIJ)], rtol=1e-9, atol=1e-11)
    np.testing.assert_allclose(ds[iJ], sol[os_:os_ + len(iJ)], rtol=1e-9, atol=1e-11)
    assert np.all(dz[F] == 0) and np.all(dw[~J] == 0) and np.all(ds[~J] == 0)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_box_solve_recovers_planted_optimum(seed):
    from oracle import boxqp
    rng = np.random.default_rng(10 + seed)
    m, n = 25, 70
    A = rng.standard_normal((m, n)) / np.sqrt(n)
    vt = _box_types(n, rng)
    q = rng.uniform(0.5, 1.5, n)                  # strictly convex: unique optimum
    u = np.where(vt == 2, rng.uniform(0.5, 2.0, n), 0.0)
    b, c, xs, ys, zs, ws, ss = boxqp.planted(A, q, vt, u, rng)
    assert boxqp.kkt_measure(A, b, c, q, u, vt, xs, ys, zs, ws, ss)["kkt"] <= 1e-13
    assert np.all(xs[vt == 2] <= u[vt == 2]) and np.any(xs[vt == 2] == u[vt == 2])
    res = boxqp.solve(A, b, c, q, u, vt, tol=1e-10)
    assert res["status"] == 0
    assert np.linalg.norm(res["x"] - xs) <= 1e-7 * np.linalg.norm(xs)
    assert np.linalg.norm(res["y"] - ys) <= 1e-6 * np.linalg.norm(ys)


@pytest.mark.parametrize("seed", range(4))
def test_box_solve_matches_bruteforce(seed):
    """Tiny non-planted instances: every free/zero/upper pattern enumerated."""
    from oracle import boxqp
    rng = np.random.default_rng(40 + seed)
    m, n = 2, 7
    A = rng.standard_normal((m, n))
    vt = _box_types(n, rng)
    q = rng.uniform(0.2, 1.0, n)
    u = np.where(vt == 2, rng.uniform(0.5, 1.5, n), 0.0)
    x0 = np.where(vt == 1, rng.standard_normal(n), np.where(vt == 2, 0.5 * u, rng.uniform(0.1, 1.0, n)))
    b = A @ x0                                      # feasible
    c = rng.standard_normal(n)
    xb, yb = boxqp.bruteforce(A, b, c, q, u, vt)
    res = boxqp.solve(A, b, c, q, u, vt, tol=1e-10)
    assert res["status"] == 0
    np.testing.assert_allclose(res["x"], xb, atol=1e-6 * (1 + np.abs(xb).max()))


def test_box_all_nonneg_reduces_to_the_pinned_oracle():
    """With every index NONNEG (u unused) the general algorithm takes the
    same steps as the non-negative oracle."""
    from oracle import boxqp
    rng = np.random.default_rng(5)
    m, n = 15, 40
    A = rng.standard_normal((m, n)) / np.sqrt(n)
    q = rng.uniform(0.0, 1.0, n)
    x0 = rng.uniform(0.1, 1.0, n)
    b, c = A @ x0, rng.standard_normal(n)
    vt = np.zeros(n, dtype=int)
    r1 = oipm_solve(A, b, c, q)
    r2 = boxqp.solve(A, b, c, q, np.zeros(n), vt, tol=1e-8)
    assert r1["iters"] == r2["iters"]
    np.testing.assert_allclose(r2["x"], r1["x"], rtol=1e-10, atol=1e-12)


def oipm_solve(A, b, c, q):
    from oracle import ippmm
    return ippmm.solve(A, b, c, q, tol=1e-8)


def test_box_oracle_solves_the_svm_form():
    """The dual SVM in form (P~) (v free, 0 <= p <= tau): at the oracle's
    solution v = X diag(y) p (first constraint block), y^T p = 0, and the
    classifier separates most of the training set."""
    from instances import svm_instance
    from oracle import boxqp
    S = svm_instance(8, 60, seed=3, sep=3.0)
    A, b, c, q, u, vt = (S[k].numpy() for k in ("A", "b", "c", "q", "u", "vtype"))
    res = boxqp.solve(A, b, c, q, u, vt.astype(int), tol=1e-9)
    assert res["status"] == 0
    d = 8
    v, p = res["x"][:d], res["x"][d:]
    yl = S["labels"].numpy()
    X = -A[:d, d:] * yl[None, :]
    np.testing.assert_allclose(v, X @ (yl * p), atol=1e-8)
    assert abs(yl @ p) <= 1e-8 and p.min() >= -1e-9 and p.max() <= 1.0 + 1e-9
    sv = (p > 1e-6) & (p < 1 - 1e-6)                  # margin support vectors fix the bias
    bias = float(np.median(yl[sv] - X[:, sv].T @ v)) if sv.any() else 0.0
    acc = float(np.mean(np.sign(X.T @ v + bias) == yl))
    assert acc >= 0.9, acc


# ---------------------------------------------------------------- sketch size and reuse

from oracle import adaptive  # noqa: E402


def test_deff_closed_forms_and_limits():
    """eq. effective-dim: c times a rank-r projector gives r c/(c+mu); mu -> 0
    counts the rank, mu -> inf gives tr(N)/mu."""
    m, r, cval = 50, 7, 3.5
    rng = np.random.default_rng(11)
    Q, _ = np.linalg.qr(rng.standard_normal((m, r)))
    N = cval * (Q @ Q.T)
    for mu in (1e-3, 0.7, 3.5, 40.0):
        # the m - r zero eigenvalues come out at about eps c and add eps c / mu each
        tol = 10 * m * np.finfo(float).eps * cval / mu
        assert abs(adaptive.d_eff_matrix(N, mu) - r * cval / (cval + mu)) <= tol
    N2 = _lowrank_psd(m, 12, 12, decay=1.0)
    # mu far below the smallest non-zero eigenvalue (1/12), far above eps |N|
    assert abs(adaptive.d_eff_matrix(N2, 1e-8) - 12) <= 1e-5
    big = 1e9
    assert abs(big * adaptive.d_eff_matrix(N2, big) - np.trace(N2)) <= 1e-6 * np.trace(N2)


@pytest.mark.parametrize("mu", [1e-4, 1e-2, 1.0])
def test_deff_estimate_is_a_lower_bound_and_exact_at_full_rank(mu):
    """N_hat <= N (Loewner), so the estimate from the Nystrom eigenvalues never
    exceeds d_eff(N, mu); it grows with nested test matrices and equals
    d_eff once the sketch covers the rank."""
    m, r = 90, 30
    N = _lowrank_psd(m, r, 13, decay=1.5)
    de = adaptive.d_eff_matrix(N, mu)
    Om = np.random.default_rng(14).standard_normal((m, 40))
    prev = -1.0
    for ell in (5, 10, 20, 29):
        U, lam, _ = nystrom.nystrom(lambda V: N @ V, nystrom.orthonormalize(Om[:, :ell]))
        dh = adaptive.d_eff_estimate(lam, mu)
        assert dh <= de + 1e-10
        assert dh >= prev - 1e-10
        prev = dh
    U, lam, _ = nystrom.nystrom(lambda V: N @ V, nystrom.orthonormalize(Om[:, :35]))
    assert abs(adaptive.d_eff_estimate(lam, mu) - de) <= 1e-8 * max(de, 1.0)


def test_theorem_sketch_size_values():
    """eq. main-thm-sketch-size at points evaluated by hand (natural log):
    d=0, k=0: 256 ln 32; d=100, k=0: 8 (10 + sqrt(32 ln 32))^2;
    d=0, k=3: 256 ln 80."""
    assert abs(adaptive.theorem_sketch_size(0.0, 0) - 887.2283911) < 1e-6
    assert abs(adaptive.theorem_sketch_size(100.0, 0) - 3372.2004537) < 1e-6
    assert abs(adaptive.theorem_sketch_size(0.0, 3) - 1121.7988185) < 1e-6
    assert adaptive.theorem_sketch_size(5.0, 4) > adaptive.theorem_sketch_size(5.0, 3)
    assert adaptive.theorem_sketch_size(6.0, 3) > adaptive.theorem_sketch_size(5.0, 3)


def test_sketch_size_rule_cases():
    F, D, T = adaptive.RULE_FIXED, adaptive.RULE_DEFF, adaptive.RULE_THEOREM
    rule = adaptive.sketch_size_rule
    # fixed: the previous size
    assert rule(F, 123.0, 5.0, 1.0, 3, 77, 8, 500, 2.0) == 77
    # ceil(2 * 10.2) = 21, sketch not saturated (lambda_hat_ell <= mu)
    assert rule(D, 10.2, 0.5, 1.0, 3, 40, 8, 500, 2.0) == 21
    # exact integer stays: 2 * 10 = 20
    assert rule(D, 10.0, 0.5, 1.0, 3, 40, 8, 500, 2.0) == 20
    # lower clamp
    assert rule(D, 1.0, 0.5, 1.0, 0, 40, 8, 500, 2.0) == 8
    # saturated: max(ceil(100), 2 * 60) = 120, then the upper clamp
    assert rule(D, 50.0, 2.0, 1.0, 3, 60, 8, 500, 2.0) == 120
    assert rule(D, 50.0, 2.0, 1.0, 3, 60, 8, 100, 2.0) == 100
    # lambda_hat_ell == mu is not saturated
    assert rule(D, 50.0, 1.0, 1.0, 3, 60, 8, 500, 2.0) == 100
    # theorem: ceil(887.228...) = 888, clamped or not
    assert rule(T, 0.0, 0.0, 1.0, 0, 60, 8, 2000, 2.0) == 888
    assert rule(T, 0.0, 0.0, 1.0, 0, 60, 8, 500, 2.0) == 500
    assert rule(T, 100.0, 0.0, 1.0, 0, 60, 8, 5000, 2.0) == 3373


def test_rebuild_due_cases():
    due = adaptive.rebuild_due
    assert due(0, -1, 0, 0, 3, 1.5)                  # nothing built yet
    assert due(5, 4, 100, 10, 0, 1.5)                # reuse off: every iteration
    assert not due(5, 4, 15, 10, 3, 1.5)             # age 1, 15 <= 1.5 * 10
    assert due(5, 4, 16, 10, 3, 1.5)                 # 16 > 15
    assert due(7, 4, 10, 10, 3, 1.5)                 # age 3 reaches the maximum
    assert not due(6, 4, 10, 10, 3, 1.5)


# ---------------------------------------------------------------- portfolio problem

from oracle import portfolio  # noqa: E402


def _np_parts(P):
    return {k: (v.numpy() if isinstance(v, torch.Tensor) else v) for k, v in P.items()}


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_portfolio_form_matches_bruteforce_of_the_original_problem(seed):
    """The (P~) form built by the instances (y = F^T x free, slack t >= 0),
    solved by the box-form IP-PMM oracle, gives the optimum of the original
    portfolio problem found by active-set enumeration (which never uses that
    form); y = F^T x and t = u - M x; the objectives agree after the 1/gamma
    scaling."""
    from oracle import boxqp
    n, d, s = 6, 3, 2
    P = _np_parts(_portfolio_tiny(n, d, s, seed))
    ref = portfolio.bruteforce(P["r"], P["F"], P["Dg"], P["M"], P["u_p"], P["gamma"])
    assert portfolio.kkt_residual(ref["x"], ref["eta"], ref["nu"], ref["zeta"], P["r"], P["F"], P["Dg"], P["M"],
                                  P["u_p"], P["gamma"]) <= 1e-9
    out = boxqp.solve(P["A"], P["b"], P["c"], P["q"], P["u"], P["vtype"], tol=1e-10)
    assert out["status"] == 0
    x = out["x"][:n]
    np.testing.assert_allclose(x, ref["x"], atol=1e-7)
    np.testing.assert_allclose(out["x"][n:n + s], P["F"].T @ x, atol=1e-7)
    np.testing.assert_allclose(out["x"][n + s:], P["u_p"] - P["M"] @ x, atol=1e-7)
    ob = 0.5 * out["x"] @ (P["q"] * out["x"]) + P["c"] @ out["x"]
    assert abs(ob * P["gamma"] - portfolio.objective(ref["x"], P["r"], P["F"], P["Dg"], P["gamma"])) <= 1e-7


def _portfolio_tiny(n, d, s, seed, gamma=2.0):
    from instances import portfolio_instance
    return portfolio_instance(n, d, s, seed=seed, gamma=gamma, with_parts=True)


def test_portfolio_bruteforce_matches_a_library_solver():
    """The enumeration against scipy's SLSQP on the original problem."""
    from scipy.optimize import minimize
    for seed in (0, 3):
        P = _np_parts(_portfolio_tiny(7, 4, 2, seed))
        ref = portfolio.bruteforce(P["r"], P["F"], P["Dg"], P["M"], P["u_p"], P["gamma"])
        n = len(P["r"])
        res = minimize(lambda x: portfolio.objective(x, P["r"], P["F"], P["Dg"], P["gamma"]), np.full(n, 1.0 / n),
                       method="SLSQP", bounds=[(0, None)] * n,
                       constraints=[dict(type="eq", fun=lambda x: x.sum() - 1.0),
                                    dict(type="ineq", fun=lambda x: P["u_p"] - P["M"] @ x)],
                       options=dict(ftol=1e-14, maxiter=500))
        assert res.success
        np.testing.assert_allclose(res.x, ref["x"], atol=1e-5)


# ---------------------------------------------------------------- instance layouts

def _dense_from_units(Ad, rows, vals):
    m, n = Ad.shape
    E = np.zeros((m, len(rows)))
    E[rows, np.arange(len(rows))] = vals
    return np.hstack([Ad, E])


def test_unit_column_layouts_match_the_dense_instances():
    """The generators' unit-column layouts describe the same problems as
    their dense layouts: the portfolio form column for column, the SVM form
    with the variables reordered from [v; p] to [p; v]."""
    from instances import portfolio_instance, svm_instance
    P = portfolio_instance(50, 20, 4, seed=3)
    U = portfolio_instance(50, 20, 4, seed=3, unit_columns=True)
    rows, vals = (t.numpy() for t in U["units"])
    assert np.all(np.diff(rows) > 0)
    np.testing.assert_array_equal(_dense_from_units(U["A"].numpy(), rows, vals), P["A"].numpy())
    for k in ("b", "c", "q", "u", "vtype"):
        np.testing.assert_array_equal(U[k].numpy(), P[k].numpy())
    d, n = 12, 40
    S = svm_instance(d, n, seed=6)
    V = svm_instance(d, n, seed=6, unit_columns=True)
    perm = np.concatenate([np.arange(d, d + n), np.arange(d)])
    rows, vals = (t.numpy() for t in V["units"])
    np.testing.assert_array_equal(_dense_from_units(V["A"].numpy(), rows, vals), S["A"].numpy()[:, perm])
    for k in ("c", "q", "u", "vtype"):
        np.testing.assert_array_equal(V[k].numpy(), S[k].numpy()[perm])
