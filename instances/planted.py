"""Planted-optimum instances of min 1/2 x^T Q x + c^T x  s.t. Ax = b, x >= 0.

Recipe (the five workloads are named by what they are, with their sizes):

* ``gauss_200x500``      m=200,   n=500,    A_ij ~ N(0, 1/n), FP64, q ~ U[0,1], sketch 20
* ``lowrank_5000x20000`` m=5000,  n=20000,  A = U diag(i^-1) V^T (rank 200) + 1e-3 N(0,1),
                         FP64, q ~ U[0,1] with floor(0.3 n) exact zeros, sketch 100
* ``lowrank_20000x100000`` m=20000, n=100000, rank 400, sigma_i = i^-1.5, noise 1e-3,
                         A defined in FP32 (a BF16 copy is derived from it), q as above, sketch 200
* ``gauss_2000x8000``    m=2000,  n=8000,   A_ij ~ N(0, 1/n) defined in FP32, q ~ U[0,1], sketch 50
* ``lowrank_50000x200000`` m=50000, n=200000, rank 800, sigma_i = i^-1, noise 1e-3, FP32,
                         q ~ U[0,2], sketch 400

Planted optimum: exactly floor(n/2) indices (a seeded permutation) form the
support S; x*_S ~ U[0.1,1], x*_{S^c} = 0; z*_{S^c} ~ U[0.1,1], z*_S = 0
(strict complementarity); y* ~ N(0,1).  Then b = A x* and
c = A^T y* + z* - Q x*, so (x*, y*, z*) satisfies the KKT conditions of
(P)/(D) exactly (up to the FP64 rounding of b and c).

Where A is "defined in FP32", the FP32 array *is* the problem matrix: it is
promoted exactly to FP64 to form b and c, so the planted point is optimal for
every consumer regardless of the precision it reads A in.

U and V are orthonormalised Gaussian matrices (two passes of Cholesky-QR on
a Gaussian r-column block, which is well conditioned for n >> r).  Large
matrices are produced in row panels so that the FP64 temporaries stay small.

All draws come from one ``torch.Generator`` seeded with ``seed`` on the
requested device, in a fixed order.  CPU and GPU generators produce different
streams, so an instance is identified by (workload, seed, device).
"""

from __future__ import annotations

from dataclasses import dataclass, field
from typing import Optional

import torch

CONFIGS = {
    "gauss_200x500": dict(m=200, n=500, kind="gauss", q="U01", ell=20, a_dtype="f64"),
    "lowrank_5000x20000": dict(m=5000, n=20000, kind="lowrank", rank=200, sigma_pow=1.0,
                               noise=1e-3, q="U01z30", ell=100, a_dtype="f64"),
    "lowrank_20000x100000": dict(m=20000, n=100000, kind="lowrank", rank=400, sigma_pow=1.5,
                                 noise=1e-3, q="U01z30", ell=200, a_dtype="f32"),
    "gauss_2000x8000": dict(m=2000, n=8000, kind="gauss", q="U01", ell=50, a_dtype="f32"),
    "lowrank_50000x200000": dict(m=50000, n=200000, kind="lowrank", rank=800, sigma_pow=1.0,
                                 noise=1e-3, q="U02", ell=400, a_dtype="f32"),
}


@dataclass
class Instance:
    name: str
    A: torch.Tensor          # defining matrix, m x n row-major, FP64 or FP32
    q: torch.Tensor          # diag(Q), FP64, >= 0
    b: torch.Tensor          # FP64 (m)
    c: torch.Tensor          # FP64 (n)
    x_star: torch.Tensor     # planted primal optimum, FP64
    y_star: torch.Tensor     # planted multipliers, FP64
    z_star: torch.Tensor     # planted dual slacks, FP64
    support: torch.Tensor    # bool (n): x*_j > 0
    ell: int
    seed: int
    meta: dict = field(default_factory=dict)

    @property
    def m(self) -> int:
        return self.A.shape[0]

    @property
    def n(self) -> int:
        return self.A.shape[1]


def _orthonormal_columns(G: torch.Tensor) -> torch.Tensor:
    """Two passes of Cholesky-QR (r x r factorisations on the CPU)."""
    for _ in range(2):
        S = (G.T @ G).cpu()
        L = torch.linalg.cholesky(S)
        Linv_t = torch.linalg.inv(L).T.contiguous().to(G.device)
        G = G @ Linv_t
    return G


def _panel_rows(m: int, n: int, budget_elems: int = 1 << 27) -> int:
    return max(1, min(m, budget_elems // max(n, 1)))


def make_instance(name: str, seed: int = 0, device: str | torch.device = "cpu",
                  m: Optional[int] = None, n: Optional[int] = None,
                  rank: Optional[int] = None, ell: Optional[int] = None) -> Instance:
    """Draw the named workload.  ``m``/``n``/``rank``/``ell`` override the sizes
    (used for scaled-down cases with the same structure)."""
    cfg = dict(CONFIGS[name])
    m = int(m if m is not None else cfg["m"])
    n = int(n if n is not None else cfg["n"])
    ell = int(ell if ell is not None else cfg["ell"])
    device = torch.device(device)
    f64 = torch.float64
    g = torch.Generator(device=device)
    g.manual_seed(int(seed))

    def uni(k, lo, hi):
        return lo + (hi - lo) * torch.rand(k, generator=g, device=device, dtype=f64)

    # planted optimum
    perm_s = torch.randperm(n, generator=g, device=device)
    support = torch.zeros(n, dtype=torch.bool, device=device)
    support[perm_s[: n // 2]] = True
    x_star = torch.where(support, uni(n, 0.1, 1.0), torch.zeros((), dtype=f64, device=device))
    z_star = torch.where(~support, uni(n, 0.1, 1.0), torch.zeros((), dtype=f64, device=device))
    y_star = torch.randn(m, generator=g, device=device, dtype=f64)

    # diagonal of Q
    if cfg["q"] == "U01":
        q = uni(n, 0.0, 1.0)
    elif cfg["q"] == "U02":
        q = uni(n, 0.0, 2.0)
    elif cfg["q"] == "U01z30":
        q = uni(n, 0.0, 1.0)
        perm_q = torch.randperm(n, generator=g, device=device)
        q[perm_q[: (3 * n) // 10]] = 0.0
    else:
        raise ValueError(cfg["q"])

    a_dtype = torch.float32 if cfg["a_dtype"] == "f32" else f64
    A = torch.empty((m, n), dtype=a_dtype, device=device)
    b = torch.zeros(m, dtype=f64, device=device)
    aty = torch.zeros(n, dtype=f64, device=device)
    rows = _panel_rows(m, n)
    if cfg["kind"] == "gauss":
        sd = 1.0 / (n ** 0.5)
        for i0 in range(0, m, rows):
            i1 = min(m, i0 + rows)
            P = sd * torch.randn((i1 - i0, n), generator=g, device=device, dtype=f64)
            A[i0:i1] = P.to(a_dtype)
    elif cfg["kind"] == "lowrank":
        r = int(rank if rank is not None else cfg["rank"])
        r = min(r, m, n)
        U = _orthonormal_columns(torch.randn((m, r), generator=g, device=device, dtype=f64))
        V = _orthonormal_columns(torch.randn((n, r), generator=g, device=device, dtype=f64))
        sig = torch.arange(1, r + 1, device=device, dtype=f64) ** (-float(cfg["sigma_pow"]))
        Vt = (V * sig).T.contiguous()             # r x n, sigma folded in
        for i0 in range(0, m, rows):
            i1 = min(m, i0 + rows)
            P = U[i0:i1] @ Vt
            P += cfg["noise"] * torch.randn((i1 - i0, n), generator=g, device=device, dtype=f64)
            A[i0:i1] = P.to(a_dtype)
        del U, V, Vt
    else:
        raise ValueError(cfg["kind"])

    # b = A x*, c = A^T y* + z* - Q x*, from the defining (exactly promoted) A
    for i0 in range(0, m, rows):
        i1 = min(m, i0 + rows)
        P = A[i0:i1].to(f64)
        b[i0:i1] = P @ x_star
        aty += P.T @ y_star[i0:i1]
    c = aty + z_star - q * x_star
    return Instance(name=name, A=A, q=q, b=b, c=c, x_star=x_star, y_star=y_star,
                    z_star=z_star, support=support, ell=ell, seed=int(seed),
                    meta=dict(cfg, m=m, n=n, ell=ell, device=str(device)))


def random_feasible_instance(m: int, n: int, seed: int, q_lo: float = 0.1,
                             q_hi: float = 1.0) -> dict:
    """A small non-planted instance: A ~ N(0,1), q ~ U[q_lo,q_hi] (Q positive
    definite, so the optimum is unique), b = A x0 for some x0 >= 0 (feasible),
    c ~ N(0,1).  CPU, FP64 torch tensors."""
    g = torch.Generator()
    g.manual_seed(int(seed))
    f64 = torch.float64
    A = torch.randn((m, n), generator=g, dtype=f64)
    x0 = torch.rand(n, generator=g, dtype=f64)
    b = A @ x0
    c = torch.randn(n, generator=g, dtype=f64)
    q = q_lo + (q_hi - q_lo) * torch.rand(n, generator=g, dtype=f64)
    return dict(A=A, b=b, c=c, q=q)


def svm_instance(d: int, n: int, seed: int = 0, tau: float = 1.0, sep: float = 2.0, decay: float = 1.5,
                 device: str | torch.device = "cpu", dtype=torch.float64, unit_columns: bool = False) -> dict:
    """Dual linear SVM in the box-constrained form (P~) (the paper's SVM
    formulation): x = [v; p], Q = diag(1_d, 0_n), A = [[I_d, -X diag(y)],
    [0, y^T]], b = 0, c = [0_d; -1_n] (the objective 1/2 v^T v - sum p), v
    free, 0 <= p <= tau.  Synthetic dense features standing in for the paper's
    datasets: latent coordinate i has variance i^-decay (a power-law covariance
    spectrum, as in image or expression data) and the class label shifts the
    first min(10, d) latent coordinates by +-sep/sqrt(min(10, d)); the features
    are a dense random mixing M (d x d, N(0, 1/d) entries) of the latent
    coordinates, so the dominant directions are not aligned with the feature
    axes; labels +-1 in equal numbers (a seeded permutation).  Returns A
    (dtype), b, c, q, u (float64), vtype (int8), labels.  With unit_columns
    the variables are ordered [p; v]: A holds only the dense block
    [-X diag(y); y^T] and units = (rows 0..d-1 int32, values 1.0) describes
    the identity on v (same draws, so x_unit = [p; v] for x_dense = [v; p])."""
    g = torch.Generator(device=device)
    g.manual_seed(int(seed))
    f64 = torch.float64
    yl = torch.ones(n, dtype=f64, device=device)
    yl[torch.randperm(n, generator=g, device=device)[: n // 2]] = -1.0
    sd = torch.arange(1, d + 1, dtype=f64, device=device) ** (-0.5 * decay)
    L = torch.randn((d, n), generator=g, dtype=f64, device=device) * sd[:, None]
    k = min(10, d)
    L[:k] += (sep / k ** 0.5) * yl[None, :]
    M = torch.randn((d, d), generator=g, dtype=f64, device=device) / d ** 0.5
    X = M @ L
    del L, M
    if unit_columns:
        Ad = torch.empty((d + 1, n), dtype=f64, device=device)
        Ad[:d] = -X * yl[None, :]
        Ad[d] = yl
        units = (torch.arange(d, dtype=torch.int32, device=device), torch.ones(d, dtype=f64, device=device))
        b = torch.zeros(d + 1, dtype=f64, device=device)
        c = torch.cat([-torch.ones(n, dtype=f64, device=device), torch.zeros(d, dtype=f64, device=device)])
        q = torch.cat([torch.zeros(n, dtype=f64, device=device), torch.ones(d, dtype=f64, device=device)])
        u = torch.cat([torch.full((n,), tau, dtype=f64, device=device), torch.zeros(d, dtype=f64, device=device)])
        vtype = torch.cat([torch.full((n,), 2, dtype=torch.int8, device=device),
                           torch.full((d,), 1, dtype=torch.int8, device=device)])
        return dict(A=Ad.to(dtype), units=units, b=b, c=c, q=q, u=u, vtype=vtype, labels=yl)
    A = torch.zeros((d + 1, d + n), dtype=f64, device=device)
    A[:d, :d] = torch.eye(d, dtype=f64, device=device)
    A[:d, d:] = -X * yl[None, :]
    A[d, d:] = yl
    A = A.to(dtype)
    b = torch.zeros(d + 1, dtype=f64, device=device)
    c = torch.cat([torch.zeros(d, dtype=f64, device=device), -torch.ones(n, dtype=f64, device=device)])
    q = torch.cat([torch.ones(d, dtype=f64, device=device), torch.zeros(n, dtype=f64, device=device)])
    u = torch.cat([torch.zeros(d, dtype=f64, device=device), torch.full((n,), tau, dtype=f64, device=device)])
    vtype = torch.cat([torch.full((d,), 1, dtype=torch.int8, device=device),
                       torch.full((n,), 2, dtype=torch.int8, device=device)])
    return dict(A=A, b=b, c=c, q=q, u=u, vtype=vtype, labels=yl)


def portfolio_instance(n: int = 80000, d: int = 50000, s: int = 100, seed: int = 0, gamma: float = 1.0,
                       components: Optional[int] = None, device: str | torch.device = "cpu",
                       dtype=torch.float64, with_parts: bool = False, unit_columns: bool = False) -> dict:
    """The factor-model portfolio problem (the paper's portfolio experiment)
    min -r^T x + gamma x^T (F F^T + diag(Dg)) x  s.t.  M x <= u_p, 1^T x = 1,
    x >= 0, in the form (P~) of its reformulation with y = F^T x free and a
    slack t = u_p - M x >= 0, the objective divided by gamma:
      variables [x (n, >= 0); y (s, free); t (d, >= 0)],
      A = [[F^T, -I_s, 0], [M, 0, I_d], [1^T, 0, 0]]  ((s + d + 1) x (n + s + d)),
      b = [0_s; u_p; 1], c = [-r / gamma; 0; 0], Q = diag(2 Dg, 2 I_s, 0_d).
    Data: a true covariance Sigma = G diag(lam) G^T + sig2 I with G (n x R)
    orthonormal, lam_i = i^-2 for i <= R/10 then decaying as i^-1/2 (rapid,
    then slow decay), scaled so that the mean variance is 1 (sig2 = 0.1);
    F = G_s diag(sqrt(lam_{1..s} + sig2)), the exact rank-s truncation of
    Sigma, and Dg = diag(Sigma - F F^T) >= sig2 (1 - |G_{j,1..s}|^2); rows of M
    ~ N(0, I); r ~ N(0, 1); u_p ~ U[0.05, 1] (x = 1/n is strictly feasible once the largest
    (M 1/n)_i, about 4.5/sqrt(n), is below 0.05, as at the paper's size).
    A holds the stored values (dtype); F and M of the returned parts are those
    values promoted to FP64.  Returns A, b, c, q, u, vtype and, with
    with_parts, F, Dg, M, u_p, r, gamma.  With unit_columns A holds only the
    dense columns [F^T; M; 1^T] (m x n) and units = (rows int32, values)
    describes the -I_s and I_d blocks (same variable order and draws)."""
    g = torch.Generator(device=device)
    g.manual_seed(int(seed))
    f64 = torch.float64
    R = components if components is not None else min(1000, max(s + 1, n // 2))
    k0 = max(1, R // 10)
    i = torch.arange(1, R + 1, dtype=f64, device=device)
    lam = torch.where(i <= k0, i ** -2.0, (k0 ** -2.0) * (i / k0) ** -0.5)
    sig2 = 0.1
    lam = lam * (0.9 * n / lam.sum())
    G = _orthonormal_columns(torch.randn((n, R), generator=g, dtype=f64, device=device))
    F = G[:, :s] * torch.sqrt(lam[:s] + sig2)[None, :]
    Dg = (G[:, s:] ** 2) @ lam[s:] + sig2 * (1.0 - (G[:, :s] ** 2).sum(dim=1))
    del G
    r = torch.randn(n, generator=g, dtype=f64, device=device)
    u_p = 0.05 + 0.95 * torch.rand(d, generator=g, dtype=f64, device=device)
    m, N = s + d + 1, n + s + d
    A = torch.zeros((m, n if unit_columns else N), dtype=dtype, device=device)
    A[:s, :n] = F.T.to(dtype)
    step = _panel_rows(d, n)
    for r0 in range(0, d, step):                    # M in row panels, drawn in the storage type
        r1 = min(d, r0 + step)
        A[s + r0:s + r1, :n] = torch.randn((r1 - r0, n), generator=g, dtype=f64 if dtype == f64 else torch.float32,
                                           device=device).to(dtype)
    A[s + d, :n] = 1.0
    units = None
    if unit_columns:
        units = (torch.arange(s + d, dtype=torch.int32, device=device),
                 torch.cat([torch.full((s,), -1.0, dtype=f64, device=device), torch.ones(d, dtype=f64, device=device)]))
    else:
        A[:s, n:n + s] = -torch.eye(s, dtype=dtype, device=device)
        A[s:s + d, n + s:] = torch.eye(d, dtype=dtype, device=device)
    b = torch.cat([torch.zeros(s, dtype=f64, device=device), u_p, torch.ones(1, dtype=f64, device=device)])
    c = torch.cat([-r / gamma, torch.zeros(s + d, dtype=f64, device=device)])
    q = torch.cat([2.0 * Dg, torch.full((s,), 2.0, dtype=f64, device=device), torch.zeros(d, dtype=f64, device=device)])
    vtype = torch.cat([torch.zeros(n, dtype=torch.int8, device=device), torch.ones(s, dtype=torch.int8, device=device),
                       torch.zeros(d, dtype=torch.int8, device=device)])
    out = dict(A=A, b=b, c=c, q=q, u=torch.zeros(N, dtype=f64, device=device), vtype=vtype)
    if unit_columns:
        out["units"] = units
    if with_parts:
        out.update(F=A[:s, :n].T.to(f64), Dg=Dg, M=A[s:s + d, :n].to(f64), u_p=u_p, r=r, gamma=gamma)
    return out
