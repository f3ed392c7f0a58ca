"""Randomized Nystrom approximation (Algorithm 1, eq. Nystrom-approx) and the
Nystrom preconditioner (Algorithm 2, eq. Nys_precond and Nys_precond_inv).

Readings of the paper used here:
* The matrix that is sketched is the PSD N = A D A^T, without delta: Alg. 2
  takes N_k, and delta enters only through eq. Nys_precond_inv.
* nu = eps(||Y||_F) is the spacing of floating-point numbers at ||Y||_F in
  the working precision of the sketch: 2^(floor(log2 ||Y||_F) - (p - 1)) with
  p = 53 significant bits for FP64 (numpy.spacing) and p = 8 for BF16,
  multiplied by a stated constant c_nu (1 unless given).
* The Gaussian test matrix is orthonormalised (thin QR) before use; the
  approximation N_hat = Y (Omega^T Y)^+ Y^T depends on range(Omega) only.
* chol gives the upper factor C with C^T C = Omega^T Y_nu; the Gram matrix is
  symmetrised first.  On a failed factorisation nu is multiplied by 10 and
  the factorisation retried (at most 6 times).
* svd(B) is taken as a library thin SVD here.

Test infrastructure (see the package docstring).
"""

import math

import numpy as np
import scipy.linalg as sla

SIGNIFICAND_BITS = {"f64": 53, "f32": 24, "bf16": 8}


def eps_at(x, precision="f64"):
    """Spacing of floating-point numbers of the given precision at x > 0."""
    p = SIGNIFICAND_BITS[precision]
    return math.ldexp(1.0, math.floor(math.log2(x)) - (p - 1))


def orthonormalize(Omega):
    """Thin QR of the test matrix: Q factor, m x ell."""
    Q, _ = np.linalg.qr(Omega, mode="reduced")
    return Q


def nystrom_from_sketch(Y, Omega, precision="f64", c_nu=1.0, max_retry=6):
    """Algorithm 1 from the sketch Y = N Omega onwards.

    nu = eps(||Y||_F); Y_nu = Y + nu Omega; C = chol(Omega^T Y_nu);
    B = Y_nu C^{-1}; [U, Sigma] = svd(B); Lambda = max(0, Sigma^2 - nu).
    Returns (U_hat, lam_hat descending, nu)."""
    nrm = float(np.linalg.norm(Y, "fro"))
    nu = c_nu * eps_at(nrm, precision) if nrm > 0 else c_nu * np.finfo(float).tiny
    for _ in range(max_retry + 1):
        Ynu = Y + nu * Omega
        G = Omega.T @ Ynu
        G = 0.5 * (G + G.T)
        try:
            C = sla.cholesky(G, lower=False)
        except np.linalg.LinAlgError:
            nu *= 10.0
            continue
        # B = Y_nu C^{-1}  <=>  C^T B^T = Y_nu^T
        B = sla.solve_triangular(C, Ynu.T, trans="T", lower=False).T
        U, S, _ = np.linalg.svd(B, full_matrices=False)
        lam = np.maximum(0.0, S * S - nu)
        order = np.argsort(-lam, kind="stable")
        return U[:, order], lam[order], nu
    raise np.linalg.LinAlgError("Nystrom: Cholesky of Omega^T Y_nu failed after retries")


def nystrom(N_apply, Omega, precision="f64", c_nu=1.0):
    """Algorithm 1 with the sketch formed by the matvec oracle: Y = N Omega."""
    Y = N_apply(Omega)
    return nystrom_from_sketch(Y, Omega, precision=precision, c_nu=c_nu)


def nystrom_formula(Y, Omega):
    """eq. Nystrom-approx: N_hat = Y (Omega^T Y)^+ Y^T (the unstable closed form)."""
    G = Omega.T @ Y
    G = 0.5 * (G + G.T)
    return Y @ np.linalg.pinv(G, hermitian=True) @ Y.T


def precond_inv_apply(U, lam, delta, r):
    """eq. Nys_precond_inv applied to r:
    P^{-1} r = (lam_l + delta) U (Lambda + delta I)^{-1} U^T r + (I - U U^T) r,
    with lam_l the smallest retained eigenvalue."""
    lam_l = float(np.min(lam))
    t = U.T @ r
    inv = 1.0 / (lam + delta)
    if t.ndim == 2:
        inv = inv[:, None]
    return (lam_l + delta) * (U @ (inv * t)) + r - U @ t


def precond_dense(U, lam, delta):
    """eq. Nys_precond as a dense m x m matrix."""
    m = U.shape[0]
    lam_l = float(np.min(lam))
    return (U * ((lam + delta) / (lam_l + delta))) @ U.T + np.eye(m) - U @ U.T


def precond_inv_dense(U, lam, delta):
    """eq. Nys_precond_inv as a dense m x m matrix."""
    m = U.shape[0]
    lam_l = float(np.min(lam))
    return (U * ((lam_l + delta) / (lam + delta))) @ U.T + np.eye(m) - U @ U.T
