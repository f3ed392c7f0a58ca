"""Textbook preconditioned conjugate gradients (paper section 2.2; the method
of Golub and Van Loan, Matrix Computations, section 11.5), on M y = xi with
M SPD given by a matvec and P^{-1} given by an apply.

Stopping rule used by the solver (the paper gives none; its theory asks for a
normal-equation residual of order mu_k): stop as soon as the recursively
updated residual satisfies ||r|| <= tol, then report the true residual.

Test infrastructure (see the package docstring).
"""

import numpy as np


def pcg(M_apply, xi, Pinv_apply=None, tol=1e-10, maxit=1000, y0=None):
    """Returns (y, iterations, true residual norm, history of ||r||)."""
    y = np.zeros_like(xi) if y0 is None else y0.copy()
    r = xi - M_apply(y) if y0 is not None else xi.copy()
    s = r.copy() if Pinv_apply is None else Pinv_apply(r)
    p = s.copy()
    rs = float(r @ s)
    hist = [float(np.linalg.norm(r))]
    it = 0
    while hist[-1] > tol and it < maxit:
        q = M_apply(p)
        alpha = rs / float(p @ q)
        y += alpha * p
        r -= alpha * q
        s = r.copy() if Pinv_apply is None else Pinv_apply(r)
        rs_new = float(r @ s)
        beta = rs_new / rs
        rs = rs_new
        p = s + beta * p
        it += 1
        hist.append(float(np.linalg.norm(r)))
    true_res = float(np.linalg.norm(xi - M_apply(y)))
    return y, it, true_res, hist
