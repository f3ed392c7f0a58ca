"""GPU parity of the unit columns of A = [A_d | E] (nys_matrix.n_unit: one
entry val_t in row row_t per column, stored as two short arrays instead of
dense columns) against the FP64 oracle run on the same matrix written out
densely.  The unit columns are applied exactly in FP64, so every tolerance
is the one the dense tests derive for the dense block."""

import numpy as np
import pytest
import torch

from oracle import lowprec, normal_eq

pytestmark = pytest.mark.gpu

DEV = "cuda"


@pytest.fixture(scope="module")
def nys():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2404_14524_amd as pkg
    return pkg


def _t(a, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device=DEV)


def _np(t):
    return t.detach().double().cpu().numpy()


def _case(m, n, k, seed):
    """Dense block, k unit columns in sorted random rows with values of either
    sign, d over all n + k columns, v."""
    rng = np.random.default_rng(seed)
    A = rng.standard_normal((m, n)) / np.sqrt(max(n, 1))
    rows = np.sort(rng.choice(m, size=k, replace=False)).astype(np.int32)
    vals = rng.choice([-1.0, 1.0], size=k) * rng.uniform(0.5, 2.0, k)
    d = rng.uniform(0.0, 2.0, n + k)
    v = rng.standard_normal(m)
    return A, rows, vals, d, v


def _full(A, rows, vals):
    m, n = A.shape
    E = np.zeros((m, len(rows)))
    E[rows, np.arange(len(rows))] = vals
    return np.hstack([A, E])


def _units(rows, vals):
    return (_t(rows, torch.int32), _t(vals))


SHAPES = [(300, 700, 300), (257, 1031, 100), (1000, 3 * 1024 + 37, 999), (50, 0, 30), (7, 5, 1)]


@pytest.mark.parametrize("layout", ["rows", "transposed"])
@pytest.mark.parametrize("dtype", [torch.float64, torch.float32, torch.bfloat16])
@pytest.mark.parametrize("m,n,k", SHAPES)
def test_normal_apply_with_units(nys, m, n, k, dtype, layout):
    print(f"normal_apply units {dtype} {m}x{n}+{k} {layout}", flush=True)
    A, rows, vals, d, v = _case(m, n, k, seed=m + n + k)
    At = _t(A).to(dtype)
    Aq = _np(At)
    A_t = nys.nys_transpose(At) if layout == "transposed" and n > 0 else None
    out = nys.nys_normal_apply(At, _t(d), 0.37, _t(v), A_t=A_t, units=_units(rows, vals))
    F = _full(Aq, rows, vals)
    ref = normal_eq.normal_apply(F, d, 0.37, v)
    bound = np.abs(F) @ (np.abs(d) * (np.abs(F).T @ np.abs(v))) + 0.37 * np.abs(v)
    assert np.all(np.abs(_np(out) - ref) <= 1e-12 * bound + 1e-300)


@pytest.mark.parametrize("m,n,k,ell", [(400, 900, 250, 40), (129, 300, 129, 64)])
def test_sketch_product_with_units(nys, m, n, k, ell):
    print(f"sketch units {m}x{n}+{k} ell={ell}", flush=True)
    A, rows, vals, d, _ = _case(m, n, k, seed=ell)
    Om = np.random.default_rng(5).standard_normal((m, ell))
    un = _units(rows, vals)
    F = _full(A, rows, vals)
    Y = _np(nys.nys_sketch_product(_t(A), _t(d), _t(Om), "f64", units=un))
    ref = F @ (d[:, None] * (F.T @ Om))
    bound = np.abs(F) @ (d[:, None] * (np.abs(F).T @ np.abs(Om)))
    assert np.all(np.abs(Y - ref) <= 1e-12 * bound + 1e-300)
    # BF16 matrix cores for the dense block (emulated by the oracle), the unit
    # columns' exact FP64 terms added
    A32 = A.astype(np.float32).astype(np.float64)
    Abf = _t(A32, torch.float32).to(torch.bfloat16)
    E = _full(np.zeros((m, 0)), rows, vals)
    refb = lowprec.sketch_bf16(A32, d[:n], Om) + E @ (d[n:, None] * (E.T @ Om))
    Ab = lowprec.round_bf16(A32)
    boundb = np.abs(Ab) @ (d[:n, None] * (np.abs(Ab).T @ np.abs(lowprec.round_bf16(Om))))
    for A_t in (None, nys.nys_transpose(Abf)):
        Yb = _np(nys.nys_sketch_product(Abf, _t(d), _t(Om), "bf16", A_t=A_t, units=un))
        err = np.abs(Yb - refb)
        assert np.all(err <= (2.0 ** -8 + 2.0 ** -24 * (m + n)) * boundb + 1e-12 * np.abs(refb) + 1e-300)


def test_sketch_exact_at_rank_with_units(nys):
    """N = A_d D A_d^T + E D_E E^T has rank at most rank(A_d) + k (16 here):
    a sketch of size 30 reproduces it."""
    m, n, r, k = 200, 300, 6, 10
    rng = np.random.default_rng(4)
    A = rng.standard_normal((m, r)) @ rng.standard_normal((r, n)) / n
    rows = np.sort(rng.choice(m, size=k, replace=False)).astype(np.int32)
    vals = rng.uniform(0.5, 1.5, k)
    d = rng.uniform(0.5, 2.0, n + k)
    P = nys.nys_sketch(_t(A), _t(d), 30, seed=1, counter=2, units=_units(rows, vals))
    N = normal_eq.normal_matrix(_full(A, rows, vals), d)
    Nh = _np(P.U) @ np.diag(_np(P.lam)) @ _np(P.U).T
    assert np.linalg.norm(N - Nh, 2) <= 1e-10 * np.linalg.norm(N, 2)


def test_pcg_with_units_matches_dense_solve(nys):
    m, n, k = 300, 500, 200
    A, rows, vals, d, _ = _case(m, n, k, seed=11)
    delta = 1e-3
    xi = np.random.default_rng(3).standard_normal(m)
    un = _units(rows, vals)
    P = nys.nys_sketch(_t(A), _t(d), 30, seed=2, units=un)
    y, info = nys.nys_pcg_solve(_t(A), _t(d), delta, _t(xi), P=P, units=un, rtol=1e-11, maxit=3000, poll_every=1)
    assert info.status == 0
    M = normal_eq.normal_matrix(_full(A, rows, vals), d, delta)
    assert np.linalg.norm(xi - M @ _np(y)) <= 1.01e-11 * np.linalg.norm(xi) + 1e-14


def test_pchol_with_units(nys):
    """Pivots, factor, diag(S) and the apply of the partial Cholesky
    preconditioner against the oracle on the dense matrix; unit rows with
    large entries make sure some of them are pivots."""
    from oracle import pchol as opc
    m, n, k, ell = 150, 400, 60, 25
    A, rows, vals, d, _ = _case(m, n, k, seed=12)
    vals = vals * 3.0
    un = _units(rows, vals)
    delta = 1e-3
    P = nys.nys_pchol_build(_t(A), _t(d), delta, ell, units=un)
    F = _full(A, rows, vals)
    ref = opc.build(F, d, delta, ell)
    assert len(set(ref["piv"]) & set(rows)) > 0
    np.testing.assert_array_equal(P.piv.cpu().numpy(), ref["piv"])
    Lo = np.empty((m, ell))
    Lo[ref["piv"]] = ref["L11"]
    Lo[ref["rest"]] = ref["L21"]
    np.testing.assert_allclose(_np(P.L), Lo, rtol=0, atol=1e-10 * np.abs(Lo).max())
    np.testing.assert_allclose(_np(P.diagS)[ref["rest"]], ref["diagS"], rtol=1e-8)
    r = np.random.default_rng(1).standard_normal(m)
    ro = opc.precond_inv_apply(ref, r)
    np.testing.assert_allclose(_np(nys.nys_pchol_apply(P, _t(r))), ro, rtol=0, atol=1e-9 * np.abs(ro).max())


def test_newton_step_with_units(nys):
    m, n, k = 120, 300, 80
    A, rows, vals, _, _ = _case(m, n, k, seed=13)
    F = _full(A, rows, vals)
    N = n + k
    rng = np.random.default_rng(2)
    x, z = rng.uniform(0.01, 2, N), rng.uniform(0.01, 2, N)
    q = rng.uniform(0, 1, N)
    rho, delta = 0.1, 0.05
    rd, rp, rxz = rng.standard_normal(N), rng.standard_normal(m), rng.standard_normal(N)
    D = normal_eq.scaling(x, z, q, rho)
    M = normal_eq.normal_matrix(F, D, delta)
    ex, ey, ez, _ = normal_eq.newton_step(F, x, z, D, delta, rd, rp, rxz, lambda xi: np.linalg.solve(M, xi))
    dx, dy, dz, info = nys.nys_newton_solve(_t(A), _t(q), _t(x), _t(z), rho, delta, _t(rd), _t(rp), _t(rxz),
                                            units=_units(rows, vals), rtol=1e-13, maxit=2000)
    for g, e in ((dx, ex), (dy, ey), (dz, ez)):
        assert np.linalg.norm(_np(g) - e) <= 1e-9 * (1 + np.linalg.norm(e))


def test_ipm_solve_with_slack_units(nys):
    """(P) with a slack per row in half of the rows (A = [A_d | I_S]): the
    planted optimum, as with the dense matrix."""
    from oracle import ippmm as oipm
    from oracle import problem
    m, n = 150, 400
    rng = np.random.default_rng(21)
    A = rng.standard_normal((m, n)) / np.sqrt(n)
    rows = np.sort(rng.choice(m, size=m // 2, replace=False)).astype(np.int32)
    vals = np.ones(len(rows))
    F = _full(A, rows, vals)
    N = F.shape[1]
    q = rng.uniform(0.2, 1.0, N)
    xs = np.where(rng.random(N) < 0.5, rng.uniform(0.1, 1.0, N), 0.0)
    zs = np.where(xs > 0, 0.0, rng.uniform(0.1, 1.0, N))
    ys = rng.standard_normal(m)
    b, c = F @ xs, F.T @ ys + zs - q * xs
    x, y, z, info = nys.ipm_solve(_t(A), _t(b), _t(c), _t(q), ell=20, tol=1e-8, seed=1, units=_units(rows, vals))
    assert info.status == 0, info.kkt_rel
    assert problem.kkt_measure(F, b, c, q, _np(x), _np(y), _np(z))["kkt"] <= 1e-8
    assert np.linalg.norm(_np(x) - xs) <= 1e-6 * np.linalg.norm(xs)
    ref = oipm.solve(F, b, c, q, tol=1e-10)
    assert np.linalg.norm(ref["x"] - xs) <= 1e-7 * np.linalg.norm(xs)


@pytest.mark.parametrize("precond", ["nystrom", "pchol", "none"])
def test_ipm_solve_box_svm_units_match_dense_layout(nys, precond):
    """The SVM form with the identity on v as unit columns ([p; v] order)
    against the same instance stored densely ([v; p]) and the oracle."""
    from instances import svm_instance
    from oracle import boxqp
    print(f"svm units {precond}", flush=True)
    d_, n_ = 40, 400
    S = svm_instance(d_, n_, seed=7)
    U = svm_instance(d_, n_, seed=7, unit_columns=True)
    npd = {k: v.numpy() for k, v in S.items()}
    ref = boxqp.solve(npd["A"], npd["b"], npd["c"], npd["q"], npd["u"], npd["vtype"], tol=1e-10)
    x, y, z, w, s, info = nys.ipm_solve_box(U["A"].to(DEV), *(U[k].to(DEV) for k in ("b", "c", "q", "vtype", "u")),
                                            ell=20, tol=1e-8, seed=2, precond=precond,
                                            units=tuple(t.to(DEV) for t in U["units"]))
    assert info.status == 0, (info.kkt_rel, info.iters)
    xg = _np(x)
    v_ref = ref["x"][:d_]
    np.testing.assert_allclose(xg[n_:], v_ref, atol=1e-6 * (1 + np.abs(v_ref).max()))
    obj = lambda xx, q, c: 0.5 * xx @ (q * xx) + c @ xx
    assert abs(obj(xg, U["q"].numpy(), U["c"].numpy()) - obj(ref["x"], npd["q"], npd["c"])) <= 1e-6 * (
        1 + abs(obj(ref["x"], npd["q"], npd["c"])))


@pytest.mark.parametrize("storage", ["f64", "f32"])
def test_ipm_solve_box_portfolio_units(nys, storage):
    """The portfolio form with -I_s and I_d as unit columns against the oracle
    on the dense form of the same instance (FP32 storage: the FP32 draws)."""
    from instances import portfolio_instance
    from oracle import boxqp
    print(f"portfolio units {storage}", flush=True)
    dt = torch.float64 if storage == "f64" else torch.float32
    P = portfolio_instance(600, 300, 12, seed=1, dtype=dt)
    U = portfolio_instance(600, 300, 12, seed=1, dtype=dt, unit_columns=True)
    npd = {k: v.double().numpy() if k == "A" else v.numpy() for k, v in P.items()}
    ref = boxqp.solve(npd["A"], npd["b"], npd["c"], npd["q"], npd["u"], npd["vtype"], tol=1e-11)
    A = U["A"].to(DEV)
    x, y, z, w, s, info = nys.ipm_solve_box(A, *(U[k].to(DEV) for k in ("b", "c", "q", "vtype", "u")), ell=20,
                                            tol=1e-8, seed=3, units=tuple(t.to(DEV) for t in U["units"]),
                                            sketch_dtype="bf16" if storage == "f32" else "f64",
                                            A_lo=A.to(torch.bfloat16) if storage == "f32" else None)
    assert info.status == 0, (info.kkt_rel, info.iters)
    assert np.linalg.norm(_np(x) - ref["x"]) <= 1e-6 * np.linalg.norm(ref["x"])


def test_units_rejected_when_malformed(nys):
    A, rows, vals, d, v = _case(20, 30, 5, seed=1)
    bad = [(rows[::-1].copy(), vals), (np.array([0, 3, 3, 7, 9], np.int32), vals),
           (np.array([0, 3, 5, 7, 20], np.int32), vals), (np.array([-1, 3, 5, 7, 9], np.int32), vals),
           (rows, np.array([1.0, np.nan, 1.0, 1.0, 1.0]))]
    for r, vv in bad:
        with pytest.raises(nys.NysError):
            nys.nys_normal_apply(_t(A), _t(d), 1.0, _t(v), units=_units(r, vv))
    with pytest.raises(ValueError):
        nys.nys_normal_apply(_t(A), _t(d), 1.0, _t(v), units=(_t(rows, torch.int64), _t(vals)))
    with pytest.raises(ValueError):            # d must cover the unit columns too
        nys.nys_normal_apply(_t(A), _t(d[:30]), 1.0, _t(v), units=_units(rows, vals))


def test_ipm_solve_box_units_with_rules_reuse_and_trace(nys):
    """Unit columns together with the sketch-size rule, reuse and the trace
    on the (P~) solver: the oracle's optimum, decisions that follow the rules,
    and per-iteration residuals recorded."""
    from instances import portfolio_instance
    from oracle import boxqp
    P = portfolio_instance(600, 300, 12, seed=4)
    U = portfolio_instance(600, 300, 12, seed=4, unit_columns=True)
    npd = {k: v.numpy() for k, v in P.items()}
    ref = boxqp.solve(npd["A"], npd["b"], npd["c"], npd["q"], npd["u"], npd["vtype"], tol=1e-11)
    tr = np.full((100, len(nys.TRACE_FIELDS)), np.nan)
    x, y, z, w, s, info = nys.ipm_solve_box(U["A"].to(DEV), *(U[k].to(DEV) for k in ("b", "c", "q", "vtype", "u")),
                                            ell=20, tol=1e-8, seed=3, units=tuple(t.to(DEV) for t in U["units"]),
                                            ell_rule="deff", ell_min=8, ell_max=80, reuse_max_age=2, trace=tr)
    assert info.status == 0, (info.kkt_rel, info.iters)
    assert np.linalg.norm(_np(x) - ref["x"]) <= 1e-6 * np.linalg.norm(ref["x"])
    K = info.iters
    f = {k: i for i, k in enumerate(nys.TRACE_FIELDS)}
    assert np.all(np.isfinite(tr[:K, f["rp_rel"]])) and np.all(np.diff(tr[:K, f["time_ms"]]) > 0)
    ells = tr[:K, f["ell"]].astype(int)
    assert np.all((ells >= 8) & (ells <= 80))
    built = tr[:K, f["built"]] == 1.0
    assert built[0] and int(built.sum()) == info.builds
    gaps = np.diff(np.flatnonzero(np.append(built, True)))
    assert np.all(gaps <= 2)                         # never older than the maximal age


def test_units_with_caller_bf16_copy(nys):
    """A caller-supplied BF16 copy of the dense block is combined with A's
    unit columns for the sketch (the copy itself carries none)."""
    from instances import svm_instance
    U = svm_instance(30, 300, seed=5, unit_columns=True, dtype=torch.float32)
    A = U["A"].to(DEV)
    args = [U[k].to(DEV) for k in ("b", "c", "q", "vtype", "u")]
    un = tuple(t.to(DEV) for t in U["units"])
    x1, *_, i1 = nys.ipm_solve_box(A, *args, ell=10, tol=1e-7, seed=1, sketch_dtype="bf16", units=un)
    x2, *_, i2 = nys.ipm_solve_box(A, *args, ell=10, tol=1e-7, seed=1, sketch_dtype="bf16", units=un,
                                   A_lo=A.to(torch.bfloat16))
    assert i1.status == 0 and i2.status == 0
    assert torch.equal(x1, x2) and i1.pcg_iters_total == i2.pcg_iters_total


def test_adjoint_rejects_units(nys):
    A, rows, vals, d, v = _case(20, 30, 5, seed=2)
    n = 35
    vec = torch.ones(n, dtype=torch.float64, device=DEV)
    with pytest.raises(nys.NysError):
        nys.ipm_adjoint(_t(A), torch.ones(20, dtype=torch.float64, device=DEV), vec, vec, vec, torch.zeros(
            20, dtype=torch.float64, device=DEV), vec, 1e-6, 1e-6, vec, ell=5, units=_units(rows, vals))
