"""The factor-model portfolio problem in its original form (section
"Large-scale portfolio optimization problem", eq. portfolio; the supplement's
"QP formulation for portfolio optimization", eq. portfolio-risk):

    min  -r^T x + gamma x^T (F F^T + diag(Dg)) x
    s.t. M x <= u,  1^T x = 1,  x >= 0.

Used to pin the (P~) form that the instances build (variables x, y = F^T x
free, slack t = u - M x >= 0, objective divided by gamma) and the IP-PMM
oracle with free variables: the brute-force optimum below never goes through
that form.

KKT conditions of the original problem (multipliers eta >= 0 for M x <= u,
nu for 1^T x = 1, zeta >= 0 for x >= 0):
    2 gamma Sigma x - r + M^T eta + nu 1 - zeta = 0,
    eta o (u - M x) = 0,  zeta o x = 0.
For gamma > 0 and Dg > 0 the objective is strictly convex, so x is unique.

Test infrastructure (see the package docstring).
"""

import itertools

import numpy as np


def objective(x, r, F, Dg, gamma):
    Fx = F.T @ x
    return float(-r @ x + gamma * (Fx @ Fx + x @ (Dg * x)))


def sigma(F, Dg):
    return F @ F.T + np.diag(Dg)


def kkt_residual(x, eta, nu, zeta, r, F, Dg, M, u, gamma):
    """Largest violation of the KKT conditions above (stationarity, primal
    and dual feasibility, complementarity)."""
    g = 2.0 * gamma * sigma(F, Dg) @ x - r + M.T @ eta + nu - zeta
    slack = u - M @ x
    viol = [np.abs(g).max(), abs(x.sum() - 1.0), max(0.0, -x.min()), max(0.0, -slack.min()),
            max(0.0, -eta.min()) if eta.size else 0.0, max(0.0, -zeta.min()),
            np.abs(eta * slack).max() if eta.size else 0.0, np.abs(zeta * x).max()]
    return float(max(viol))


def bruteforce(r, F, Dg, M, u, gamma, tol=1e-10):
    """Enumerate every pair (Z, B): x_Z = 0 and M_B x = u_B.  For each, solve
    the equality-constrained QP's KKT system; keep the point that is feasible
    with non-negative multipliers.  Returns dict(x, eta, nu, zeta).  Only for
    tiny n and d (2^(n + d) linear solves)."""
    n, d = len(r), len(u)
    S2 = 2.0 * gamma * sigma(F, Dg)
    best = None
    for zmask in itertools.product([False, True], repeat=n):
        Z = np.flatnonzero(zmask)
        P = np.flatnonzero(~np.asarray(zmask))
        if len(P) == 0:
            continue
        for bmask in itertools.product([False, True], repeat=d):
            B = np.flatnonzero(bmask)
            k = len(P) + len(B) + 1
            K = np.zeros((k, k))
            rhs = np.zeros(k)
            p = len(P)
            K[:p, :p] = S2[np.ix_(P, P)]
            K[:p, p:p + len(B)] = M[np.ix_(B, P)].T
            K[:p, -1] = 1.0
            K[p:p + len(B), :p] = M[np.ix_(B, P)]
            K[-1, :p] = 1.0
            rhs[:p] = r[P]
            rhs[p:p + len(B)] = u[B]
            rhs[-1] = 1.0
            try:
                sol = np.linalg.solve(K, rhs)
            except np.linalg.LinAlgError:
                continue
            if not np.allclose(K @ sol, rhs, atol=1e-9):
                continue
            x = np.zeros(n)
            x[P] = sol[:p]
            eta = np.zeros(d)
            eta[B] = sol[p:p + len(B)]
            nu = sol[-1]
            zeta = S2 @ x - r + M.T @ eta + nu
            zeta[P] = 0.0
            if (x.min() >= -tol and (u - M @ x).min() >= -tol and eta.min() >= -tol
                    and (zeta[Z].min() if len(Z) else 0.0) >= -tol):
                cand = dict(x=x, eta=eta, nu=nu, zeta=zeta)
                if best is None or objective(x, r, F, Dg, gamma) < objective(best["x"], r, F, Dg, gamma):
                    best = cand
    if best is None:
        raise RuntimeError("no KKT point found (degenerate instance)")
    return best
