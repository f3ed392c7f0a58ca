"""IP-PMM for QPs with free, non-negative and box-constrained variables
(section "Free and box-constrained variables"): the primal-dual pair

  (P~): min 1/2 x^T Q x + c^T x  s.t. A x = b, x_F free, x_I >= 0, 0 <= x_J <= u_J
  (D~): max -1/2 x^T Q x + b^T y - u^T s  s.t. -Q x + A^T y + z - s = c,
        z_I, z_J >= 0, s_J >= 0,

with slack w_J = u_J - x_J.  Variable kinds are given per index by vtype:
FREE, NONNEG or BOX; u holds the upper bounds of BOX indices (ignored
elsewhere).  Conventions of the paper kept: z, w, s have length n with
z_F = 0, w_{IF} = 0, s_{IF} = 0.

Steps, in the paper's order: the initial point of the supplement
("Construction for initial point"); Algorithm 4's start (lambda = y0,
zeta = x0, rho = delta = 8); per iteration the Newton direction of
Algorithm 5 (xi_au by index kind, eq. normal-eq-free-box solved exactly by a
dense Cholesky, eq. delta-x/-w/-z/-s-free-box), Mehrotra predictor and
corrector (Algorithm 6) and the step lengths of the supplement
("Stepsizes").

Readings (in addition to those of ``ippmm``):
* eq. delta-z-free-box / delta-s-free-box: X^{-1} and W^{-1} multiply both
  terms, dz = X^{-1}(r_xz - Z dx), ds = W^{-1}(r_ws - S dw) -- the last two
  block rows of eq. Newton-free-box; the printed formulas drop the inverse
  from the second term.
* mu = (x_{IJ}^T z_{IJ} + w_J^T s_J) / (|IJ| + |J|); the corrector target
  replaces -X Z and -W S by mu~ - dx dz and mu~ - dw ds; r_u = u - x - w.
* initial point: as in the non-negative case, the dual centring shift uses
  the primal quantities shifted by delta_p (x~ + delta_p, w~ + delta_p)
  where the printed formula writes delta_d; entries of x_{IJ}, w_J, z_{IJ},
  s_J still <= 0 after the shifts are set to 1.
* stopping test: max(rp_rel, rd_rel, ||r_u|| / (1 + ||u||), mu) <= tol.
These readings shape the trajectory only.  As for ``ippmm`` they are pinned
by hand-worked cases (initial points with box, non-negative and free
variables; the stopping measure) and by the update rule's stated properties;
the final point is pinned too (planted optima, brute force).

Test infrastructure (see the package docstring).
"""

import itertools

import numpy as np
import scipy.linalg as sla

from .ippmm import DELTA0, INIT_REG, REG_FLOOR, RHO0, STEP_FACTOR

NONNEG, FREE, BOX = 0, 1, 2


def kinds(vtype):
    vtype = np.asarray(vtype)
    F = vtype == FREE
    J = vtype == BOX
    I = vtype == NONNEG
    return F, I, J


def residuals(A, b, c, q, u, vtype, x, y, z, w, s):
    """r_p = b - A x, r_d = c + Q x - A^T y - z + s, r_u = (u - x - w) on J
    (zero elsewhere), mu."""
    F, I, J = kinds(vtype)
    IJ = I | J
    rp = b - A @ x
    rd = c + q * x - A.T @ y - z + s
    ru = np.where(J, u - x - w, 0.0)
    cnt = int(IJ.sum()) + int(J.sum())
    mu = (float(x[IJ] @ z[IJ]) + float(w[J] @ s[J])) / cnt if cnt else 0.0
    return rp, rd, ru, mu


def kkt_measure(A, b, c, q, u, vtype, x, y, z, w, s):
    rp, rd, ru, mu = residuals(A, b, c, q, u, vtype, x, y, z, w, s)
    _, _, J = kinds(vtype)
    unorm = float(np.linalg.norm(np.where(J, u, 0.0)))
    rp_rel = float(np.linalg.norm(rp)) / (1.0 + float(np.linalg.norm(b)))
    rd_rel = float(np.linalg.norm(rd)) / (1.0 + float(np.linalg.norm(c)))
    ru_rel = float(np.linalg.norm(ru)) / (1.0 + unorm)
    return dict(rp_rel=rp_rel, rd_rel=rd_rel, ru_rel=ru_rel, mu=mu, kkt=max(rp_rel, rd_rel, ru_rel, mu))


def scaling(vtype, x, z, w, s, q, rho):
    """D = (Q + Theta^{-1} + rho I)^{-1}, Theta^{-1}_jj = z_j/x_j (I),
    z_j/x_j + s_j/w_j (J), 0 (F)."""
    F, I, J = kinds(vtype)
    th = np.zeros_like(x)
    th[I | J] = z[I | J] / x[I | J]
    th[J] += s[J] / w[J]
    return 1.0 / (q + th + rho)


def newton_step(A, vtype, x, z, w, s, D, delta, rd, rp, ru, rxz, rws, solve):
    """Algorithm 5: returns dx, dy, dz, dw, ds.  ``solve`` maps xi to dy."""
    F, I, J = kinds(vtype)
    IJ = I | J
    xi_au = np.zeros_like(x)
    xi_au[IJ] = -rxz[IJ] / x[IJ]
    xi_au[J] += rws[J] / w[J] - s[J] / w[J] * ru[J]
    xi = rp + A @ (D * (rd + xi_au))
    dy = solve(xi)
    dx = D * (A.T @ dy - rd - xi_au)
    dw = np.where(J, ru - dx, 0.0)
    dz = np.zeros_like(x)
    dz[IJ] = (rxz[IJ] - z[IJ] * dx[IJ]) / x[IJ]
    ds = np.zeros_like(x)
    ds[J] = (rws[J] - s[J] * dw[J]) / w[J]
    return dx, dy, dz, dw, ds


def newton_matrix(A, q, vtype, x, z, w, s, rho, delta):
    """The unreduced Newton matrix of eq. Newton-free-box in the unknowns
    (dx, dy, dw_J, dz_IJ, ds_J), rows (r_d, r_p, r_u_J, r_xz_IJ, r_ws_J)."""
    m, n = A.shape
    F, I, J = kinds(vtype)
    IJ = I | J
    iJ, iIJ = np.flatnonzero(J), np.flatnonzero(IJ)
    nJ, nIJ = len(iJ), len(iIJ)
    N = n + m + nJ + nIJ + nJ
    K = np.zeros((N, N))
    ox, oy, ow, oz, os_ = 0, n, n + m, n + m + nJ, n + m + nJ + nIJ
    K[:n, ox:ox + n] = -np.diag(q + rho)
    K[:n, oy:oy + m] = A.T
    K[iIJ, oz + np.arange(nIJ)] = 1.0
    K[iJ, os_ + np.arange(nJ)] = -1.0
    K[oy:oy + m, ox:ox + n] = A
    K[oy:oy + m, oy:oy + m] = delta * np.eye(m)
    r = ow
    for k, j in enumerate(iJ):
        K[r + k, ox + j] = 1.0
        K[r + k, ow + k] = 1.0
    r = oz
    for k, j in enumerate(iIJ):
        K[r + k, ox + j] = z[j]
        K[r + k, oz + k] = x[j]
    r = os_
    for k, j in enumerate(iJ):
        K[r + k, ow + k] = s[j]
        K[r + k, os_ + k] = w[j]
    return K, (ox, oy, ow, oz, os_), (iJ, iIJ)


def step_length(v, dv, mask):
    """0.995 * min(1, min over masked dv_i < 0 of -v_i / dv_i) (eq. stepsize-p/-d)."""
    neg = mask & (dv < 0)
    a = 1.0
    if np.any(neg):
        a = min(1.0, float(np.min(-v[neg] / dv[neg])))
    return a


def initial_point(A, b, c, q, u, vtype, reg=INIT_REG):
    F, I, J = kinds(vtype)
    IJ = I | J
    m, n = A.shape
    uu = np.where(J, u, 0.0)
    K = A @ A.T
    K[np.diag_indices(m)] += reg
    cf = sla.cho_factor(K)
    xt = 0.5 * uu + A.T @ sla.cho_solve(cf, b - 0.5 * (A @ uu))
    yt = sla.cho_solve(cf, A @ (c + q * xt))
    g = c - A.T @ yt + q * xt
    zt = np.where(J, 0.5 * g, g)
    st = np.where(J, -zt, 0.0)
    wt = np.where(J, uu - xt, 0.0)
    cand_p = [-1.5 * float(np.min(xt[IJ]))] if IJ.any() else []
    cand_p += [-1.5 * float(np.min(wt[J]))] if J.any() else []
    cand_d = [-1.5 * float(np.min(zt[IJ]))] if IJ.any() else []
    cand_d += [-1.5 * float(np.min(st[J]))] if J.any() else []
    dp = max(cand_p + [0.0])
    dd = max(cand_d + [0.0])
    gxz = float((xt[IJ] + dp) @ (zt[IJ] + dd))
    gws = float((wt[J] + dp) @ (st[J] + dd))
    den_p = float(np.sum(zt[IJ] + dd)) + float(np.sum(st[J] + dd))
    den_d = float(np.sum(xt[IJ] + dp)) + float(np.sum(wt[J] + dp))
    dpt = dp + (0.5 * (gxz + gws) / den_p if den_p > 0 else 0.0)
    ddt = dd + (0.5 * (gxz + gws) / den_d if den_d > 0 else 0.0)
    x0 = xt.copy()
    x0[IJ] += dpt
    w0 = np.where(J, wt + dpt, 0.0)
    z0 = np.where(IJ, zt + ddt, 0.0)
    s0 = np.where(J, st + ddt, 0.0)
    for v, mask in ((x0, IJ), (w0, J), (z0, IJ), (s0, J)):
        v[mask & (v <= 0)] = 1.0
    return x0, yt.copy(), z0, w0, s0


def solve(A, b, c, q, u, vtype, tol=1e-8, max_iter=100, history=None):
    """Returns dict(x, y, z, w, s, iters, status, rho, delta, kkt...)."""
    A = np.asarray(A, dtype=np.float64)
    m, n = A.shape
    F, I, J = kinds(vtype)
    IJ = I | J
    u = np.where(J, u, 0.0)
    cnt = int(IJ.sum()) + int(J.sum())
    x, y, z, w, s = initial_point(A, b, c, q, u, vtype)
    zeta, lam = x.copy(), y.copy()
    rho, delta = RHO0, DELTA0
    status, k = 1, 0
    for k in range(max_iter + 1):
        meas = kkt_measure(A, b, c, q, u, vtype, x, y, z, w, s)
        if history is not None:
            history.append(dict(k=k, rho=rho, delta=delta, **meas))
        if meas["kkt"] <= tol:
            status = 0
            break
        if k == max_iter:
            break
        mu = meas["mu"]
        D = scaling(vtype, x, z, w, s, q, rho)
        M = (A * D) @ A.T
        M = 0.5 * (M + M.T) + delta * np.eye(m)
        cf = sla.cho_factor(M)

        def exact(xi):
            return sla.cho_solve(cf, xi)

        rd = c + q * x - A.T @ y - z + s + rho * (x - zeta)
        rp = b - A @ x - delta * (y - lam)
        ru = np.where(J, u - x - w, 0.0)
        rxz = np.where(IJ, -x * z, 0.0)
        rws = np.where(J, -w * s, 0.0)
        dxp, dyp, dzp, dwp, dsp = newton_step(A, vtype, x, z, w, s, D, delta, rd, rp, ru, rxz, rws, exact)
        ap = STEP_FACTOR * min(step_length(x, dxp, IJ), step_length(w, dwp, J))
        ad = STEP_FACTOR * min(step_length(z, dzp, IJ), step_length(s, dsp, J))
        mu_aff = 0.0
        if cnt:
            mu_aff = (float((x[IJ] + ap * dxp[IJ]) @ (z[IJ] + ad * dzp[IJ]))
                      + float((w[J] + ap * dwp[J]) @ (s[J] + ad * dsp[J]))) / cnt
        mu_t = mu_aff ** 3 / mu ** 2 if mu > 0 else 0.0
        zn, zm = np.zeros(n), np.zeros(m)
        rxz_c = np.where(IJ, mu_t - dxp * dzp, 0.0)
        rws_c = np.where(J, mu_t - dwp * dsp, 0.0)
        dxc, dyc, dzc, dwc, dsc = newton_step(A, vtype, x, z, w, s, D, delta, zn, zm, zn, rxz_c, rws_c, exact)
        dx, dy, dz, dw, ds = dxp + dxc, dyp + dyc, dzp + dzc, dwp + dwc, dsp + dsc
        ap = STEP_FACTOR * min(step_length(x, dx, IJ), step_length(w, dw, J))
        ad = STEP_FACTOR * min(step_length(z, dz, IJ), step_length(s, ds, J))
        x = x + ap * dx
        w = w + ap * dw
        y = y + ad * dy
        z = z + ad * dz
        s = s + ad * ds
        _, _, _, mu_new = residuals(A, b, c, q, u, vtype, x, y, z, w, s)
        zeta, lam = x.copy(), y.copy()
        rho = delta = max(REG_FLOOR, min(rho, mu_new))
    meas = kkt_measure(A, b, c, q, u, vtype, x, y, z, w, s)
    return dict(x=x, y=y, z=z, w=w, s=s, iters=k, status=status, rho=rho, delta=delta, **meas)


def planted(A, q, vtype, u, rng):
    """Planted KKT point: FREE ~ N(0,1); NONNEG half at 0 (z > 0), half in
    U[0.1, 1]; BOX a third at 0 (z > 0), a third at u (s > 0), a third
    inside; y ~ N(0,1).  Returns (b, c, x, y, z, w, s)."""
    m, n = A.shape
    F, I, J = kinds(vtype)
    x, z, s = np.zeros(n), np.zeros(n), np.zeros(n)
    for j in range(n):
        r = rng.integers(3)
        if F[j]:
            x[j] = rng.standard_normal()
        elif I[j]:
            if r == 0:
                z[j] = rng.uniform(0.1, 1.0)
            else:
                x[j] = rng.uniform(0.1, 1.0)
        else:
            if r == 0:
                z[j] = rng.uniform(0.1, 1.0)
            elif r == 1:
                x[j] = u[j]
                s[j] = rng.uniform(0.1, 1.0)
            else:
                x[j] = rng.uniform(0.1, 0.9) * u[j]
    y = rng.standard_normal(m)
    w = np.where(J, u - x, 0.0)
    b = A @ x
    c = A.T @ y + z - s - q * x
    return b, c, x, y, z, w, s


def bruteforce(A, b, c, q, u, vtype, feas_tol=1e-9):
    """Optimum of a tiny (P~) by enumerating, for every NONNEG index, x_j = 0
    or free, and for every BOX index, x_j = 0, x_j = u_j or free; each case is
    the equality-constrained QP on the free indices, kept when x and the
    multipliers have the right signs (n <= 8)."""
    m, n = A.shape
    F, I, J = kinds(vtype)
    opts = [("f",) if F[j] else ("0", "f") if I[j] else ("0", "u", "f") for j in range(n)]
    best = None
    for case in itertools.product(*opts):
        S = [j for j in range(n) if case[j] == "f"]
        xfix = np.array([u[j] if case[j] == "u" else 0.0 for j in range(n)])
        k = len(S)
        AS = A[:, S]
        K = np.zeros((k + m, k + m))
        K[:k, :k] = np.diag(q[S])
        K[:k, k:] = -AS.T
        K[k:, :k] = AS
        rhs = np.concatenate([-c[S], b - A @ xfix])
        sol, *_ = np.linalg.lstsq(K, rhs, rcond=None)
        if np.linalg.norm(K @ sol - rhs) > feas_tol * (1 + np.linalg.norm(rhs)):
            continue
        x = xfix.copy()
        x[S] = sol[:k]
        y = sol[k:]
        g = c + q * x - A.T @ y          # = z - s
        ok = True
        for j in range(n):
            if case[j] == "f":
                ok &= (not I[j] or x[j] >= -feas_tol) and (not J[j] or -feas_tol <= x[j] <= u[j] + feas_tol)
            elif case[j] == "0":
                ok &= g[j] >= -feas_tol
            else:
                ok &= g[j] <= feas_tol
        if ok:
            obj = 0.5 * float(x @ (q * x)) + float(c @ x)
            if best is None or obj < best[0]:
                best = (obj, x, y)
    if best is None:
        raise ValueError("no KKT point")
    return best[1], best[2]
