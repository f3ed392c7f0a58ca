"""Partial Cholesky preconditioner of N + delta I (section "Partial Cholesky
preconditioners"; eq. partialCholeskyfact, eq. chol-precond and
eq. chol-precond-inv) -- the preconditioner of the Chol-IP-PMM comparator.

Definition followed: E permutes the ell largest diagonal entries of
N_delta = N + delta I to the front; L11 L11^T = N_delta,11 (Cholesky, lower),
L21 = N_delta,21 L11^{-T}; the Schur complement S = N_delta,22 - L21 L21^T is
replaced by its diagonal, diag(S)_i = (N_delta)_ii - ||L21[i, :]||^2.

Readings of the paper used here:
* Pivots: the ell largest diagonal entries of N_delta, chosen once from the
  diagonal (the paper's leading block holds the largest diagonal entries);
  ties go to the smaller index.  Only the set matters: any order of the
  pivots inside the leading block gives the same P_Chol.
* The paper's experiments form the diagonal with entrywise access to A,
  (N_delta)_ii = sum_j A_ij^2 d_j + delta; so does this oracle.

Test infrastructure (see the package docstring).
"""

import numpy as np
import scipy.linalg as sla


def pivots(diag, ell):
    """Indices of the ell largest entries of diag (ties: smaller index first),
    returned in ascending index order."""
    diag = np.asarray(diag, dtype=np.float64)
    order = sorted(range(len(diag)), key=lambda i: (-diag[i], i))
    return np.sort(np.array(order[:ell], dtype=np.int64))


def normal_diag(A, d, delta):
    """(N + delta I)_ii = sum_j A_ij^2 d_j + delta, N = A diag(d) A^T."""
    A = np.asarray(A, dtype=np.float64)
    return (A * A) @ d + delta


def build(A, d, delta, ell):
    """Partial Cholesky data of N_delta = A diag(d) A^T + delta I.
    Returns dict(piv, rest, L11, L21, diagS, Ndelta) (Ndelta dense, for tests)."""
    A = np.asarray(A, dtype=np.float64)
    m = A.shape[0]
    Nd = A @ (d[:, None] * A.T) + delta * np.eye(m)
    piv = pivots(normal_diag(A, d, delta), ell)
    rest = np.setdiff1d(np.arange(m), piv)
    N11 = Nd[np.ix_(piv, piv)]
    N21 = Nd[np.ix_(rest, piv)]
    L11 = np.linalg.cholesky(0.5 * (N11 + N11.T))
    L21 = sla.solve_triangular(L11, N21.T, lower=True).T      # N21 L11^{-T}
    diagS = np.diag(Nd)[rest] - np.sum(L21 * L21, axis=1)
    return dict(piv=piv, rest=rest, L11=L11, L21=L21, diagS=diagS, Ndelta=Nd)


def permutation(P):
    """E as an index array: (E v) = v[perm]."""
    return np.concatenate([P["piv"], P["rest"]])


def precond_dense(P):
    """P_Chol of eq. chol-precond, assembled densely."""
    perm = permutation(P)
    ell, mr = len(P["piv"]), len(P["rest"])
    m = ell + mr
    Lb = np.zeros((m, m))
    Lb[:ell, :ell] = P["L11"]
    Lb[ell:, :ell] = P["L21"]
    Lb[ell:, ell:] = np.eye(mr)
    mid = np.diag(np.concatenate([np.ones(ell), P["diagS"]]))
    inner = Lb @ mid @ Lb.T                  # E P E^T
    out = np.zeros((m, m))
    out[np.ix_(perm, perm)] = inner
    return out


def precond_inv_apply(P, r):
    """P_Chol^{-1} r by eq. chol-precond-inv, factor by factor."""
    perm = permutation(P)
    ell = len(P["piv"])
    rp = np.asarray(r, dtype=np.float64)[perm]
    r1, r2 = rp[:ell], rp[ell:]
    # [L11^{-1} 0; -L21 L11^{-1} I]
    t1 = sla.solve_triangular(P["L11"], r1, lower=True)
    t2 = r2 - P["L21"] @ t1
    # [I 0; 0 diag(S)^{-1}]
    u1, u2 = t1, t2 / P["diagS"]
    # [L11^{-T}  -L11^{-T} L21^T; 0 I]
    o1 = sla.solve_triangular(P["L11"].T, u1 - P["L21"].T @ u2, lower=False)
    out = np.empty_like(rp)
    out[perm] = np.concatenate([o1, u2])
    return out
