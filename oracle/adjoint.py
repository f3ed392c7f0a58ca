"""Gradient of a loss of the QP solution with respect to the data (c, b, diag Q, A).

The paper has no adjoint; this is derived from the KKT conditions of (P)/(D).
At a strictly complementary optimum with support S (x_S > 0, z_{S^c} > 0) the
solution is locally the solution of the equality-constrained system
    F(x_S, y) = [q_S * x_S + c_S - A_S^T y ;  A_S x_S - b] = 0,
with x_{S^c} = 0.  For L(x) with g = dL/dx, solve the adjoint system
    [[diag(q_S), A_S^T], [A_S, 0]] [u1_S; u2] = [g_S; 0],   u1_{S^c} = 0,
then dL/dc = -u1, dL/db = u2, dL/dq = -u1 * x, dL/dA = y u1^T - u2 x^T.

The finite-difference reference re-solves the equality system on the same
support for perturbed data and checks that the support is unchanged.

Test infrastructure (see the package docstring).
"""

import numpy as np
import scipy.linalg as sla


def active_set(x, z):
    return x > z


def kkt_gradient(A, b, c, q, x, y, z, g, S=None):
    """Dense reduced-KKT gradient.  Returns dict(c, b, q, A)."""
    m, n = A.shape
    if S is None:
        S = active_set(x, z)
    k = int(S.sum())
    AS = A[:, S]
    K = np.zeros((k + m, k + m))
    K[:k, :k] = np.diag(q[S])
    K[:k, k:] = AS.T
    K[k:, :k] = AS
    sol = sla.lu_solve(sla.lu_factor(K), np.concatenate([g[S], np.zeros(m)]))
    u1 = np.zeros(n)
    u1[S] = sol[:k]
    u2 = sol[k:]
    return dict(c=-u1, b=u2.copy(), q=-u1 * x, A=np.outer(y, u1) - np.outer(u2, x),
                u1=u1, u2=u2)


def resolve_on_support(A, b, c, q, S):
    """x*(data) on a fixed support S (equality-constrained KKT, dense LU).
    Returns (x, y, z, support_ok)."""
    m, n = A.shape
    k = int(S.sum())
    AS = A[:, S]
    K = np.zeros((k + m, k + m))
    K[:k, :k] = np.diag(q[S])
    K[:k, k:] = -AS.T
    K[k:, :k] = AS
    sol = sla.lu_solve(sla.lu_factor(K), np.concatenate([-c[S], b]))
    x = np.zeros(n)
    x[S] = sol[:k]
    y = sol[k:]
    z = q * x + c - A.T @ y
    z[S] = 0.0
    ok = bool(np.all(x[S] > 0) and np.all(z[~S] > 0))
    return x, y, z, ok


def loss(x, x_tgt):
    """L = 1/2 ||x - x_tgt||^2; dL/dx = x - x_tgt."""
    d = x - x_tgt
    return 0.5 * float(d @ d), d


def fd_gradient_rhs(A, b, c, q, S, x_tgt, block, coords, h_rel=1e-6):
    """Central differences for the blocks that enter only the right-hand side
    of the equality-constrained system on S ('c' or 'b'): the same central
    differences as fd_gradient, with one LU factorisation reused for every
    perturbed right-hand side (exact re-solves, affordable at m, n in the
    thousands).  A perturbed c_j with j outside S leaves x unchanged."""
    m, n = A.shape
    k = int(S.sum())
    AS = A[:, S]
    K = np.zeros((k + m, k + m))
    K[:k, :k] = np.diag(q[S])
    K[:k, k:] = -AS.T
    K[k:, :k] = AS
    lu = sla.lu_factor(K)
    base = np.concatenate([-c[S], b])
    pos = np.full(n, -1)
    pos[np.flatnonzero(S)] = np.arange(k)

    def loss_of(rhs):
        sol = sla.lu_solve(lu, rhs)
        x = np.zeros(n)
        x[S] = sol[:k]
        return loss(x, x_tgt)[0]

    out = np.zeros(len(coords))
    for t, idx in enumerate(coords):
        theta = float((c if block == "c" else b)[idx])
        h = h_rel * max(1.0, abs(theta))
        if block == "c":
            if pos[idx] < 0:
                continue
            e = np.zeros(k + m)
            e[pos[idx]] = -1.0            # rhs entry is -c_j
        else:
            e = np.zeros(k + m)
            e[k + idx] = 1.0
        out[t] = (loss_of(base + h * e) - loss_of(base - h * e)) / (2 * h)
    return out


def _support_system(A, q, S):
    """K = [[diag(q_S), -A_S^T], [A_S, 0]] of the equality-constrained system
    on S, and the position of each column of S among the unknowns."""
    m, n = A.shape
    k = int(S.sum())
    AS = A[:, S]
    K = np.zeros((k + m, k + m))
    K[:k, :k] = np.diag(q[S])
    K[:k, k:] = -AS.T
    K[k:, :k] = AS
    pos = np.full(n, -1)
    pos[np.flatnonzero(S)] = np.arange(k)
    return K, pos, k


def fd_gradient_lowrank(A, b, c, q, S, x_tgt, block, coords, h_rel=1e-6):
    """Central differences for the blocks that enter the MATRIX of the
    equality-constrained system on S ('q' or 'A'; coords are flat indices):
    the same differences as fd_gradient, with exact re-solves of every
    perturbed system.  A perturbed q_j (j in S) changes K by a rank-one term,
    a perturbed A_ij (j in S) by a rank-two term; each perturbed solve is
    K^{-1} r minus the Sherman-Morrison-Woodbury correction
    Z (I + V^T Z)^{-1} V^T K^{-1} r with Z = K^{-1} U, all on one LU
    factorisation of K (Golub & Van Loan, 'Matrix Computations', sec. 2.1.4).
    Coordinates outside S leave x unchanged (difference 0).  The support is
    checked unchanged (x_S > 0, z off S > 0) for every perturbed solve."""
    m, n = A.shape
    K, pos, k = _support_system(A, q, S)
    lu = sla.lu_factor(K)
    x0 = sla.lu_solve(lu, np.concatenate([-c[S], b]))
    Sc = ~S
    A_off = np.ascontiguousarray(A[:, Sc])
    c_off = c[Sc]
    coords = np.asarray(coords)
    # the unit vectors every coordinate needs, solved together
    need = []
    for idx in coords:
        if block == "q":
            j = int(idx)
            if pos[j] >= 0:
                need.append(pos[j])
        else:
            i, j = divmod(int(idx), n)
            if pos[j] >= 0:
                need += [pos[j], k + i]
    need = sorted(set(need))
    col = {e: t for t, e in enumerate(need)}
    E = np.zeros((k + m, max(len(need), 1)))
    for e, t in col.items():
        E[e, t] = 1.0
    Z_all = sla.lu_solve(lu, E)

    def loss_of(sol):
        x = np.zeros(n)
        x[S] = sol[:k]
        z_off = c_off - A_off.T @ sol[k:]
        if not (np.all(sol[:k] > 0) and np.all(z_off > 0)):
            raise ValueError("support changed under the finite-difference step")
        return loss(x, x_tgt)[0]

    out = np.zeros(len(coords))
    for t, idx in enumerate(coords):
        if block == "q":
            j = int(idx)
            theta = float(q[j])
        else:
            i, j = divmod(int(idx), n)
            theta = float(A[i, j])
        if pos[j] < 0:
            continue
        p = pos[j]
        h = h_rel * max(1.0, abs(theta))
        vals = []
        for s in (+1.0, -1.0):
            dlt = s * h
            if block == "q":
                # K' = K + dlt e_p e_p^T
                Z = Z_all[:, [col[p]]]
                VtZ = np.array([[dlt * Z[p, 0]]])
                Vtx = np.array([dlt * x0[p]])
            else:
                # K'[p, k+i] = -(A_ij + dlt), K'[k+i, p] = A_ij + dlt:
                # K' = K + U V^T, U = [e_p, e_{k+i}], V = [-dlt e_{k+i}, dlt e_p]
                r = k + i
                Z = Z_all[:, [col[p], col[r]]]
                VtZ = np.array([[-dlt * Z[r, 0], -dlt * Z[r, 1]],
                                [dlt * Z[p, 0], dlt * Z[p, 1]]])
                Vtx = np.array([-dlt * x0[r], dlt * x0[p]])
            corr = np.linalg.solve(np.eye(len(Vtx)) + VtZ, Vtx)
            vals.append(loss_of(x0 - Z @ corr))
        out[t] = (vals[0] - vals[1]) / (2 * h)
    return out


def fd_gradient(A, b, c, q, S, x_tgt, block, coords, h_rel=1e-6):
    """Central differences of L(x*(data)) in the given coordinates of one data
    block ('c', 'b', 'q' or 'A'; coords are flat indices).  Step
    h = h_rel * max(1, |theta|)."""
    data = dict(A=A.copy(), b=b.copy(), c=c.copy(), q=q.copy())
    out = np.zeros(len(coords))
    for t, idx in enumerate(coords):
        arr = data[block].reshape(-1)
        theta = float(arr[idx])
        h = h_rel * max(1.0, abs(theta))
        vals = []
        for s in (+1.0, -1.0):
            arr[idx] = theta + s * h
            x, _, _, ok = resolve_on_support(data["A"], data["b"], data["c"], data["q"], S)
            if not ok:
                raise ValueError("support changed under the finite-difference step")
            vals.append(loss(x, x_tgt)[0])
        arr[idx] = theta
        out[t] = (vals[0] - vals[1]) / (2 * h)
    return out
