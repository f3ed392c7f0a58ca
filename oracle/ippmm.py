"""IP-PMM for the separable QP with an exact inner solve: the oracle route to
the optimum of (P)/(D).

Steps, in the paper's order (Algorithm 4 -> Algorithm 6 -> Algorithm 5),
specialised to non-negative variables only (F = J = empty):

* initial point (supplement, "Construction for initial point"): candidate
  x~ = A^T (A A^T + 10 I)^{-1} b, y~ = (A A^T + 10 I)^{-1} A (c + Q x~),
  z~ = c - A^T y~ + Q x~, then the positivity shifts delta_p, delta_d and
  their centred versions;
* lambda = y0, zeta = x0, rho = delta = 8 (Algorithm 4);
* per iteration: stopping test; D = (Q + Z X^{-1} + rho I)^{-1}; one Cholesky
  factorisation of M = A D A^T + delta I shared by both Newton solves;
  Mehrotra predictor (sigma = 0), step lengths (eq. stepsize-p/-d, factor
  0.995), mu_aff (eq. mu-aff), mu~ = mu_aff^3 / mu^2, corrector, summed
  direction, new step lengths, update (Algorithm 6);
* parameter update.

Readings where the paper is silent or defers to another paper:
* initial point: the centring shift of the dual uses (x~ + delta_p)
  (Mehrotra's form) where the printed formula writes (x~ + delta_d); if the
  shifted point still has a non-positive entry (only possible when the
  product gamma is zero) that entry is set to 1.
* parameter update (deferred by the paper to the original IP-PMM): zeta <- x
  and lambda <- y every iteration; rho = delta = max(5e-10, min(rho, mu_new)).
  This is monotone like the published trajectories, ends at the published
  floor 5e-10 and follows the theory's choice rho = delta = mu.
* stopping test: max(||r_p||/(1+||b||), ||r_d||/(1+||c||), mu) <= tol.
These three readings shape the trajectory, not the optimum.  They are
pinned by CPU tests against values worked by hand (the initial point on tiny
problems, in exact rationals, which also tells the two dual-shift forms
apart; the stopping measure on a hand-computed point) and against what the
paper states for the update (rho_0 = delta_0 = 8, a non-increasing sequence
ending at the floor 5e-10, rho = delta = mu between the floor and the
previous value).  Agreement of iteration counts with the paper's own runs is
not claimed (their data are not available); the final point is pinned too
(planted optimum, brute force, active-set polish).

Test infrastructure (see the package docstring).
"""

import time

import numpy as np
import scipy.linalg as sla

from .normal_eq import newton_step, normal_matrix, scaling
from .problem import kkt_measure

STEP_FACTOR = 0.995
RHO0 = DELTA0 = 8.0
REG_FLOOR = 5e-10
INIT_REG = 10.0


def step_length(v, dv):
    """eq. stepsize-p / stepsize-d: 0.995 * min(1, min_{dv_i<0} -v_i/dv_i)."""
    neg = dv < 0
    a = 1.0
    if np.any(neg):
        a = min(1.0, float(np.min(-v[neg] / dv[neg])))
    return STEP_FACTOR * a


def initial_point(A, b, c, q, reg=INIT_REG):
    """Starting point for F = J = empty (u = 0)."""
    m = A.shape[0]
    K = A @ A.T
    K[np.diag_indices(m)] += reg
    cf = sla.cho_factor(K)
    xt = A.T @ sla.cho_solve(cf, b)
    yt = sla.cho_solve(cf, A @ (c + q * xt))
    zt = c - A.T @ yt + q * xt
    dp = max(-1.5 * float(np.min(xt)), 0.0)
    dd = max(-1.5 * float(np.min(zt)), 0.0)
    gamma = float((xt + dp) @ (zt + dd))
    dpt = dp + 0.5 * gamma / float(np.sum(zt + dd))
    ddt = dd + 0.5 * gamma / float(np.sum(xt + dp))
    x0 = xt + dpt
    z0 = zt + ddt
    x0[x0 <= 0] = 1.0
    z0[z0 <= 0] = 1.0
    return x0, yt.copy(), z0


def solve(A, b, c, q, tol=1e-8, max_iter=100, verbose=False, history=None, timings=None):
    """Returns dict(x, y, z, iters, status, kkt..., rho, delta).  status 0 =
    converged, 1 = iteration limit.  With a list `timings`, the wall-clock
    time (time.perf_counter) is appended after the initial point and after
    each iteration (instrumentation only)."""
    A = np.asarray(A, dtype=np.float64)
    m, n = A.shape
    x, y, z = initial_point(A, b, c, q)
    if timings is not None:
        timings.append(time.perf_counter())
    zeta, lam = x.copy(), y.copy()
    rho, delta = RHO0, DELTA0
    status = 1
    k = 0
    for k in range(max_iter + 1):
        meas = kkt_measure(A, b, c, q, x, y, z)
        if history is not None:
            history.append(dict(k=k, rho=rho, delta=delta, **meas))
        if verbose:
            print(f"[oracle] k={k} rp={meas['rp_rel']:.2e} rd={meas['rd_rel']:.2e} "
                  f"mu={meas['mu']:.2e} rho={rho:.2e}")
        if meas["kkt"] <= tol:
            status = 0
            break
        if k == max_iter:
            break
        mu = meas["mu"]
        D = scaling(x, z, q, rho)
        cf = sla.cho_factor(normal_matrix(A, D, delta))

        def exact(xi):
            return sla.cho_solve(cf, xi)

        # predictor
        rd = c + q * x - A.T @ y - z + rho * (x - zeta)
        rp = b - A @ x - delta * (y - lam)
        rxz = -x * z
        dxp, dyp, dzp, _ = newton_step(A, x, z, D, delta, rd, rp, rxz, exact)
        ap = step_length(x, dxp)
        ad = step_length(z, dzp)
        mu_aff = float((x + ap * dxp) @ (z + ad * dzp)) / n
        mu_t = mu_aff ** 3 / mu ** 2
        # corrector
        rxz_c = mu_t - dxp * dzp
        zero_n = np.zeros(n)
        zero_m = np.zeros(m)
        dxc, dyc, dzc, _ = newton_step(A, x, z, D, delta, zero_n, zero_m, rxz_c, exact)
        dx, dy, dz = dxp + dxc, dyp + dyc, dzp + dzc
        ap = step_length(x, dx)
        ad = step_length(z, dz)
        x = x + ap * dx
        y = y + ad * dy
        z = z + ad * dz
        mu_new = float(x @ z) / n
        # parameter update (reading, see module docstring)
        zeta, lam = x.copy(), y.copy()
        rho = delta = max(REG_FLOOR, min(rho, mu_new))
        if timings is not None:
            timings.append(time.perf_counter())
    meas = kkt_measure(A, b, c, q, x, y, z)
    return dict(x=x, y=y, z=z, iters=k, status=status, rho=rho, delta=delta, **meas)


def polish(A, b, c, q, x, y, z):
    """Active-set polish for parity: S = {x_j > z_j}; solve the equality QP
    KKT system [[diag(q_S), -A_S^T], [A_S, 0]] [x_S; y] = [-c_S; b] by dense
    LU; x_{S^c} = 0; z = Q x + c - A^T y.  Accepted only if x_S > 0,
    z_{S^c} > 0 and the KKT measure does not grow; else the input is returned."""
    m, n = A.shape
    S = x > z
    k = int(S.sum())
    AS = A[:, S]
    K = np.zeros((k + m, k + m))
    K[:k, :k] = np.diag(q[S])
    K[:k, k:] = -AS.T
    K[k:, :k] = AS
    rhs = np.concatenate([-c[S], b])
    try:
        sol = sla.lu_solve(sla.lu_factor(K), rhs)
    except (np.linalg.LinAlgError, ValueError):
        return x, y, z, False
    xp = np.zeros(n)
    xp[S] = sol[:k]
    yp = sol[k:]
    zp = q * xp + c - A.T @ yp
    zp[S] = 0.0
    ok = bool(np.all(xp[S] > 0) and np.all(zp[~S] > 0))
    if ok:
        before = kkt_measure(A, b, c, q, x, y, z)["kkt"]
        after = kkt_measure(A, b, c, q, xp, yp, zp)["kkt"]
        ok = after <= max(before, 1e-14)
    if not ok:
        return x, y, z, False
    return xp, yp, zp, True
