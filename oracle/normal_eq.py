"""The regularised normal equations and the Newton step (paper section 2.1.2,
eq. normal-eq / delta_x / delta_z; Algorithm 5 with only non-negative
variables, i.e. F = J = empty).

Test infrastructure (see the package docstring).
"""

import numpy as np
import scipy.linalg as sla


def scaling(x, z, q, rho):
    """D = (Q + Theta^{-1} + rho I)^{-1} with Theta^{-1} = Z X^{-1}
    (definition under eq. normal-eq; Theta = X Z^{-1})."""
    return 1.0 / (q + z / x + rho)


def normal_apply(A, d, delta, v):
    """(A diag(d) A^T + delta I) v, written out as the two products."""
    return A @ (d * (A.T @ v)) + delta * v


def normal_matrix(A, d, delta=0.0):
    """Dense N = A diag(d) A^T (+ delta I)."""
    N = (A * d) @ A.T
    N = 0.5 * (N + N.T)
    if delta:
        N[np.diag_indices_from(N)] += delta
    return N


def newton_rhs_aux(x, rxz):
    """xi_au = -X^{-1} r_xz (Algorithm 5, case j in I)."""
    return -rxz / x


def newton_step(A, x, z, D, delta, rd, rp, rxz, solve):
    """Algorithm 5 restricted to non-negative variables.

    xi_au = -X^{-1} r_xz;  xi = r_p + A D (r_d + xi_au);  solve M dy = xi with
    M = A D A^T + delta I;  dx = D (A^T dy - r_d - xi_au);
    dz = X^{-1}(r_xz - Z dx)  (eq. delta_z; X^{-1} multiplies both terms).
    ``solve`` maps xi to dy (an exact or an inexact solve)."""
    xi_au = newton_rhs_aux(x, rxz)
    xi = rp + A @ (D * (rd + xi_au))
    dy = solve(xi)
    dx = D * (A.T @ dy - rd - xi_au)
    dz = (rxz - z * dx) / x
    return dx, dy, dz, xi


def newton_matrix(A, q, x, z, rho, delta):
    """The unreduced 3x3 block Newton matrix of eq. Newton:
    [[-(Q + rho I), A^T, I], [A, delta I, 0], [Z, 0, X]]."""
    m, n = A.shape
    K = np.zeros((2 * n + m, 2 * n + m))
    K[:n, :n] = -np.diag(q + rho)
    K[:n, n:n + m] = A.T
    K[:n, n + m:] = np.eye(n)
    K[n:n + m, :n] = A
    K[n:n + m, n:n + m] = delta * np.eye(m)
    K[n + m:, :n] = np.diag(z)
    K[n + m:, n + m:] = np.diag(x)
    return K


def newton_dense_lu(A, q, x, z, rho, delta, rd, rp, rxz):
    """Solve the unreduced Newton system by a dense LU (textbook route)."""
    m, n = A.shape
    K = newton_matrix(A, q, x, z, rho, delta)
    sol = sla.lu_solve(sla.lu_factor(K), np.concatenate([rd, rp, rxz]))
    return sol[:n], sol[n:n + m], sol[n + m:]
