"""Brute-force solution of tiny instances of (P) by enumerating the KKT
conditions over every candidate support.

For a support S, the KKT conditions of (P)/(D) with x_{S^c} = 0 and z_S = 0
reduce to the equality-constrained system
    q_S * x_S + c_S - A_S^T y = 0,   A_S x_S = b,
and a KKT point additionally needs x_S >= 0 and z = Q x + c - A^T y >= 0.
Every KKT point of a convex QP is optimal, so the minimum objective over the
enumerated points is the optimal value (n <= 12: at most 4096 supports).

Test infrastructure (see the package docstring).
"""

import itertools

import numpy as np

from .problem import primal_objective


def kkt_points(A, b, c, q, feas_tol=1e-9):
    m, n = A.shape
    out = []
    for k in range(0, n + 1):
        for S in itertools.combinations(range(n), k):
            S = list(S)
            AS = A[:, S]
            K = np.zeros((k + m, k + m))
            K[:k, :k] = np.diag(q[S])
            K[:k, k:] = -AS.T
            K[k:, :k] = AS
            rhs = np.concatenate([-c[S], b])
            sol, _, rank, _ = np.linalg.lstsq(K, rhs, rcond=None)
            if np.linalg.norm(K @ sol - rhs) > feas_tol * (1 + np.linalg.norm(rhs)):
                continue                       # inconsistent on this support
            x = np.zeros(n)
            x[S] = sol[:k]
            y = sol[k:]
            z = q * x + c - A.T @ y
            z[S] = 0.0
            if np.all(x >= -feas_tol) and np.all(z >= -feas_tol):
                out.append(dict(S=tuple(S), x=x, y=y, z=z, obj=primal_objective(x, c, q),
                                unique=(rank == k + m)))
    return out


def optimum(A, b, c, q):
    pts = kkt_points(A, b, c, q)
    if not pts:
        raise ValueError("no KKT point: infeasible or unbounded instance")
    return min(pts, key=lambda p: p["obj"])
