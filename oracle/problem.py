"""Definitions of the primal-dual pair (P)/(D) (paper, section 1).

(P): min 1/2 x^T Q x + c^T x   s.t. A x = b, x >= 0,  Q = diag(q) PSD
(D): max b^T y - 1/2 x^T Q x   s.t. A^T y + z = Q x + c, z >= 0

Test infrastructure (see the package docstring).
"""

import numpy as np


def primal_objective(x, c, q):
    return 0.5 * float(x @ (q * x)) + float(c @ x)


def dual_objective(x, y, b, q):
    return float(b @ y) - 0.5 * float(x @ (q * x))


def residuals(A, b, c, q, x, y, z):
    """r_p = b - A x and r_d = c + Q x - A^T y - z (the infeasibilities that
    the inexact IP-PMM algorithm of section 3 tracks) and mu = x^T z / n."""
    rp = b - A @ x
    rd = c + q * x - A.T @ y - z
    mu = float(x @ z) / x.shape[0]
    return rp, rd, mu


def kkt_measure(A, b, c, q, x, y, z):
    """Relative KKT measure used as the stopping test.

    The paper delegates the exact test to the termination routine of the
    original IP-PMM and only states that relative primal/dual infeasibility
    and the duality measure mu are driven below the tolerance (section 5.1).
    Reading: rp_rel = ||r_p|| / (1 + ||b||), rd_rel = ||r_d|| / (1 + ||c||),
    KKT = max(rp_rel, rd_rel, mu)."""
    rp, rd, mu = residuals(A, b, c, q, x, y, z)
    rp_rel = float(np.linalg.norm(rp)) / (1.0 + float(np.linalg.norm(b)))
    rd_rel = float(np.linalg.norm(rd)) / (1.0 + float(np.linalg.norm(c)))
    return dict(rp_rel=rp_rel, rd_rel=rd_rel, mu=mu, kkt=max(rp_rel, rd_rel, mu))
