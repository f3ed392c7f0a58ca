"""GPU parity of every entry point of the C ABI against the FP64 CPU oracle,
on the same seeded inputs.

Tolerances are derived from the arithmetic (see the design notes):
* products with A accumulate in FP64 in a different order than numpy, so an
  entry may differ by a few units of 2^-53 times the matching entry of the
  absolute-value product |A| (|d| (|A|^T |v|)); the tests use 1e-12 times
  that bound;
* quantities produced by an iterative method (PCG, IP-PMM) are compared at
  the method's own stopping tolerance.
"""

import numpy as np
import pytest
import torch

from instances import make_instance
from oracle import adjoint as oadj
from oracle import ippmm as oipm
from oracle import lowprec, normal_eq, nystrom, philox, problem

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


def _case(m, n, seed, scale=1.0):
    rng = np.random.default_rng(seed)
    A = rng.standard_normal((m, n)) * scale
    d = rng.uniform(0.0, 2.0, n)
    v = rng.standard_normal(m)
    return A, d, v


# ------------------------------------------------------------------ normal apply

SHAPES = [(1, 1), (7, 5), (200, 500), (257, 1031), (1000, 3 * 1024 + 37), (3000, 2048), (5, 20000)]


@pytest.mark.parametrize("layout", ["rows", "transposed"])
@pytest.mark.parametrize("dtype", [torch.float64, torch.float32, torch.bfloat16])
@pytest.mark.parametrize("m,n", SHAPES)
def test_normal_apply_parity(nys, dtype, m, n, layout):
    print(f"normal_apply {dtype} {m}x{n} {layout}", flush=True)
    A, d, v = _case(m, n, seed=m * 7 + n)
    At = _t(A).to(dtype)
    Aq = _np(At)          # the values the GPU sees (exact FP64 promotion)
    if dtype == torch.bfloat16:
        np.testing.assert_array_equal(Aq, lowprec.round_bf16(A.astype(np.float32).astype(np.float64)))
    delta = 0.37
    A_t = None
    if layout == "transposed":
        A_t = nys.nys_transpose(At)
        np.testing.assert_array_equal(_np(A_t), Aq.T)     # a transpose moves values only
    out = nys.nys_normal_apply(At, _t(d), delta, _t(v), A_t=A_t)
    ref = normal_eq.normal_apply(Aq, d, delta, v)
    bound = np.abs(Aq) @ (np.abs(d) * (np.abs(Aq).T @ np.abs(v))) + delta * np.abs(v)
    err = np.abs(_np(out) - ref)
    assert np.all(err <= 1e-12 * bound + 1e-300), (err / bound).max()


def test_normal_apply_strided_and_empty(nys):
    A, d, v = _case(300, 777, seed=3)
    big = _t(np.hstack([A, np.zeros((300, 5))]))      # ld = 782: 16-byte rows broken
    At = big[:, :777]
    out = nys.nys_normal_apply(At, _t(d), 0.0, _t(v))
    ref = normal_eq.normal_apply(A, d, 0.0, v)
    np.testing.assert_allclose(_np(out), ref, rtol=1e-11, atol=1e-11 * np.abs(ref).max())
    A32 = _t(np.hstack([A, np.zeros((300, 3))]), torch.float32)[:, :777]
    out = nys.nys_normal_apply(A32, _t(d), 0.5, _t(v))
    ref = normal_eq.normal_apply(_np(A32), d, 0.5, v)
    np.testing.assert_allclose(_np(out), ref, rtol=1e-11, atol=1e-11 * np.abs(ref).max())
    # transposed copies with a padded leading dimension (16-byte rows broken
    # for FP64/BF16: the scalar path)
    for dt, pad in ((torch.float64, 1), (torch.float32, 4), (torch.bfloat16, 3)):
        Aw = _t(A).to(dt)
        wide = torch.zeros((777, 300 + pad), dtype=dt, device=DEV)
        wide[:, :300] = nys.nys_transpose(Aw)
        out = nys.nys_normal_apply(Aw, _t(d), 0.25, _t(v), A_t=wide[:, :300])
        ref = normal_eq.normal_apply(_np(Aw), d, 0.25, v)
        np.testing.assert_allclose(_np(out), ref, rtol=1e-11, atol=1e-11 * np.abs(ref).max())
    # n = 0: out = delta v
    out = nys.nys_normal_apply(torch.zeros((4, 0), dtype=torch.float64, device=DEV),
                               torch.zeros(0, dtype=torch.float64, device=DEV), 2.0, _t(np.arange(4.0)))
    np.testing.assert_array_equal(_np(out), 2.0 * np.arange(4.0))


def test_normal_apply_rejects_bad_arguments(nys):
    A, d, v = _case(10, 12, seed=4)
    with pytest.raises(nys.NysError):
        nys.nys_normal_apply(_t(A), _t(d), float("nan"), _t(v))
    with pytest.raises(ValueError):      # A_t of the wrong shape never reaches the library
        nys.nys_normal_apply(_t(A), _t(d), 1.0, _t(v), A_t=_t(A))


# ------------------------------------------------------------------ test matrix (Philox)

def test_test_matrix_matches_oracle_philox(nys):
    G = nys.nys_test_matrix(1001, 37, seed=12345, counter=9)
    ref = philox.gaussian_matrix(1001, 37, 12345, 9)
    np.testing.assert_allclose(_np(G), ref, rtol=1e-13, atol=1e-13)


# ------------------------------------------------------------------ preconditioner

def test_precond_apply_parity(nys):
    rng = np.random.default_rng(5)
    m, ell = 3001, 45
    U, _ = np.linalg.qr(rng.standard_normal((m, ell)))
    lam = np.sort(rng.uniform(0, 100, ell))[::-1].copy()
    lam[-1] = 0.0
    r = rng.standard_normal(m)
    P = nys.Precond(_t(U), _t(lam))
    for delta in (1e-8, 0.3, 50.0):
        out = nys.nys_precond_apply(P, delta, _t(r))
        ref = nystrom.precond_inv_apply(U, lam, delta, r)
        np.testing.assert_allclose(_np(out), ref, rtol=1e-12, atol=1e-12 * np.abs(r).max())
    with pytest.raises(nys.NysError):
        nys.nys_precond_apply(P, 0.0, _t(r))


# ------------------------------------------------------------------ sketch

def _nhat(U, lam):
    return (U * lam) @ U.T


@pytest.mark.parametrize("m,n,ell", [(120, 300, 10), (700, 2000, 64), (1500, 4000, 100), (1200, 3000, 300),
                                     (1300, 3000, 1100), (1800, 3600, 1600), (2000, 4000, 1800),
                                     (2200, 4400, 2100), (1100, 2500, 999), (1500, 3000, 1280),
                                     (900, 2000, 600), (1000, 2500, 800), (1600, 3200, 1400),
                                     (700, 1500, 301), (1300, 2600, 1151)])
def test_sketch_fp64_parity(nys, m, n, ell):
    """Algorithm 1 in FP64 against the oracle; the larger sizes take the
    multi-workgroup Cholesky (ell >= 128), the blocked triangular inverse, and
    the Jacobi SVD's wide groups of 8 columns for even 256 < ell <= 2048 with
    each register-group size (300; 600 and 800; 1100 and 1280; 1400; 1600;
    1800); the block variant's 8-wave groups with each register-chunk size
    (10 to 100; the odd 301, 999 and 1151), and its smaller groups with the
    pairs in LDS at 2100."""
    print(f"sketch {m}x{n} ell={ell}", flush=True)
    inst = make_instance("lowrank_5000x20000", seed=11, m=m, n=n, rank=max(ell // 2, 4))
    A = inst.A.double().numpy()
    rng = np.random.default_rng(ell)
    d = rng.uniform(0.01, 10.0, n)
    Om = rng.standard_normal((m, ell))
    P = nys.nys_sketch(_t(A), _t(d), ell, omega=_t(Om))
    Omq = nystrom.orthonormalize(Om)
    Uo, lo, nuo = nystrom.nystrom(lambda V: A @ (d[:, None] * (A.T @ V)), Omq)
    Ug, lg = _np(P.U), _np(P.lam)
    # orthogonality of Cholesky-QR-based bases: a few ell eps
    np.testing.assert_allclose(Ug.T @ Ug, np.eye(ell), atol=max(1e-12, 10 * ell * np.finfo(float).eps))
    assert np.all(np.diff(lg) <= 0) and np.all(lg >= 0)
    scale = lo[0]
    np.testing.assert_allclose(lg, lo, rtol=1e-8, atol=1e-10 * scale)
    Nh_g, Nh_o = _nhat(Ug, lg), _nhat(Uo, lo)
    assert np.linalg.norm(Nh_g - Nh_o, 2) <= 1e-8 * scale
    assert abs(P.nu - nuo) <= 1e-12 * max(nuo, 1e-300) or P.nu == nuo


@pytest.mark.parametrize("m,n,ell", [(1, 9, 1), (130, 257, 7), (1000, 3000, 100), (2000, 8000, 50),
                                     (777, 5001, 200), (300, 1000, 257), (515, 2049, 400), (600, 1500, 1000),
                                     (300, 70000, 16), (200, 40000, 300)])
def test_sketch_product_parity(nys, m, n, ell):
    """Y = A diag(d) A^T Omega in FP64 and on BF16 matrix cores, with the
    operands as A alone, with a transposed copy, and as sketch tiles (made
    from the BF16 copy and from the FP32 matrix: the same BF16 values).  The
    last two shapes give the W product more row tiles than one round of
    blocks with the last round under half full (274 of 256 rows, 313 of 128
    rows): that round runs split over K."""
    print(f"sketch_product {m}x{n} ell={ell}", flush=True)
    rng = np.random.default_rng(m + n + ell)
    A = rng.standard_normal((m, n)) / np.sqrt(n)
    d = rng.uniform(0.0, 3.0, n)
    Om = rng.standard_normal((m, ell))
    # FP64 arithmetic on FP64 storage
    Y = nys.nys_sketch_product(_t(A), _t(d), _t(Om), "f64")
    ref = A @ (d[:, None] * (A.T @ Om))
    bound = np.abs(A) @ (d[:, None] * (np.abs(A).T @ np.abs(Om)))
    assert np.all(np.abs(_np(Y) - ref) <= 1e-12 * bound + 1e-300)
    # BF16 matrix cores, FP32 accumulation, against the emulated-BF16 oracle
    A32 = A.astype(np.float32)
    Abf = _t(A32, torch.float32).to(torch.bfloat16)
    refb = lowprec.sketch_bf16(A32.astype(np.float64), d, Om)
    Ab = lowprec.round_bf16(A32.astype(np.float64))
    boundb = np.abs(Ab) @ (d[:, None] * (np.abs(Ab).T @ np.abs(lowprec.round_bf16(Om))))
    tiles = (nys.nys_sketch_tiles(Abf), nys.nys_sketch_tiles(Abf, transposed=True))
    tiles32 = (nys.nys_sketch_tiles(_t(A32, torch.float32)), nys.nys_sketch_tiles(_t(A32, torch.float32), True))
    for A_t, T in ((None, None), (nys.nys_transpose(Abf), None), (None, tiles), (None, tiles32)):
        Yb = _np(nys.nys_sketch_product(Abf, _t(d), _t(Om), "bf16", A_t=A_t, tiles=T))
        # Worst case per entry: FP32 accumulation errors (m + n terms) plus a BF16
        # rounding of W that lands on the other side of a tie, at most 2^-8 |W|.
        err = np.abs(Yb - refb)
        assert np.all(err <= (2.0 ** -8 + 2.0 ** -24 * (m + n)) * boundb + 1e-300)
        # typical: the flips are rare and the FP32 errors average out
        assert np.linalg.norm(Yb - refb) <= 1e-4 * np.linalg.norm(refb)


@pytest.mark.parametrize("m,n,ell", [(600, 2000, 40), (1500, 6000, 120)])
def test_sketch_bf16_parity(nys, m, n, ell):
    """Nystrom approximation from the BF16 matrix-core sketch vs the oracle's
    Algorithm 1 run on the emulated-BF16 sketch (same Omega, BF16 shift)."""
    inst = make_instance("lowrank_20000x100000", seed=21, m=m, n=n, rank=max(ell, 8))
    A32 = inst.A.numpy()
    rng = np.random.default_rng(ell)
    d = rng.uniform(0.01, 10.0, n)
    Om = rng.standard_normal((m, ell))
    Abf = inst.A.to(DEV).to(torch.bfloat16)
    P = nys.nys_sketch(Abf, _t(d), ell, omega=_t(Om), sketch_dtype="bf16", A_t=nys.nys_transpose(Abf))
    Omq = nystrom.orthonormalize(Om)
    Y = lowprec.sketch_bf16(A32.astype(np.float64), d, Omq)
    Uo, lo, nuo = nystrom.nystrom_from_sketch(Y, Omq, precision="bf16")
    assert P.nu == nuo
    Ug, lg = _np(P.U), _np(P.lam)
    np.testing.assert_allclose(Ug.T @ Ug, np.eye(ell), atol=1e-12)
    assert np.linalg.norm(_nhat(Ug, lg) - _nhat(Uo, lo), 2) <= 1e-4 * lo[0]


@pytest.mark.parametrize("layout", ["A", "At", "tiles"])
def test_sketch_bf16_rounding_points_hand_derived(nys, layout):
    """The BF16 sketch product on the 4 x 3 case worked by hand (the CPU pin
    of the emulation): A[3,2] = 1 + 3*2^-9 and Omega[0] = 1 + 3*2^-9 round up
    to 1 + 2^-7, W[1] = 1 + 2^-8 is a tie rounded to even (1), so
    Y = [2^-7, 2^-7, 1, 1 + 2^-6 + 2^-14] exactly (every FP32 accumulation on
    these values is exact), in both operand layouts."""
    print(f"bf16 rounding points {layout}", flush=True)
    e = 2.0 ** -9
    A32 = torch.zeros((4, 3), dtype=torch.float32)
    A32[0, 0] = A32[1, 0] = A32[2, 1] = 1.0
    A32[3, 2] = 1.0 + 3 * e
    Abf = A32.to(torch.bfloat16).to(DEV)
    Om = _t(np.array([[1.0 + 3 * e], [-1.0], [1.0], [1.0]]))
    d = _t(np.array([1.0, 1.0 + 2.0 ** -8, 1.0]))
    A_t = nys.nys_transpose(Abf) if layout == "At" else None
    T = (nys.nys_sketch_tiles(Abf), nys.nys_sketch_tiles(Abf, True)) if layout == "tiles" else None
    Y = nys.nys_sketch_product(Abf, d, Om, "bf16", A_t=A_t, tiles=T)
    np.testing.assert_array_equal(_np(Y)[:, 0], [2.0 ** -7, 2.0 ** -7, 1.0, 1.0 + 2.0 ** -6 + 2.0 ** -14])


def _tiles_reference(Xb, transposed):
    """The sketch-tile layout written out from its definition: stage kb of
    row r is 64 bytes at (kb * Rp + r) * 64, Rp = rows rounded up to 256, its
    8-element chunk c at position c ^ (((r >> 1) & 3) ^ ((r >> 3) & 1)) of
    r % 16; zero past the matrix.  Xb: BF16 bit patterns (uint16), m x n."""
    X = Xb.T if transposed else Xb
    R, K = X.shape
    Rp, nkb = -(-R // 256) * 256, -(-K // 32)
    T = np.zeros((nkb, Rp, 4, 8), dtype=np.uint16)
    P = np.zeros((Rp, nkb * 32), dtype=np.uint16)
    P[:R, :K] = X
    for r in range(Rp):
        f = ((r % 16 >> 1) & 3) ^ ((r % 16 >> 3) & 1)
        for c in range(4):
            T[:, r, c ^ f, :] = P[r].reshape(nkb, 4, 8)[:, c, :]
    return T.reshape(-1).view(np.uint8)


@pytest.mark.parametrize("m,n", [(1, 1), (37, 70), (300, 517), (16, 64)])
def test_sketch_tiles_layout(nys, m, n):
    """nys_sketch_tiles against the layout's definition, byte for byte, from
    BF16 storage and from FP32 (rounded to nearest even), both orientations."""
    print(f"sketch tiles {m}x{n}", flush=True)
    rng = np.random.default_rng(m * 7 + n)
    A32 = rng.standard_normal((m, n)).astype(np.float32)
    Xb = lowprec.bf16_bits(A32)
    for tr in (False, True):
        ref = _tiles_reference(Xb, tr)
        assert nys.nys_sketch_tiles_bytes(m, n, int(tr)) == ref.size
        for src in (_t(A32, torch.float32).to(torch.bfloat16), _t(A32, torch.float32)):
            got = nys.nys_sketch_tiles(src, transposed=tr).cpu().numpy()
            np.testing.assert_array_equal(got, ref)


def test_sketch_exact_at_rank(nys):
    # N of exact rank r < ell: the approximation reproduces N
    m, n, r, ell = 600, 900, 12, 20
    rng = np.random.default_rng(8)
    A = rng.standard_normal((m, r)) @ rng.standard_normal((r, n)) / n
    d = rng.uniform(0.5, 2.0, n)
    P = nys.nys_sketch(_t(A), _t(d), ell, seed=3, counter=1)
    N = normal_eq.normal_matrix(A, d)
    Nh = _nhat(_np(P.U), _np(P.lam))
    assert np.linalg.norm(N - Nh, 2) <= 1e-10 * np.linalg.norm(N, 2)


def test_sketch_rejects_bad_sizes(nys):
    A, d, v = _case(10, 12, seed=4)
    with pytest.raises(nys.NysError):
        nys.nys_sketch(_t(A), _t(d), 11)


# ------------------------------------------------------------------ PCG

@pytest.mark.parametrize("layout", ["rows", "transposed"])
@pytest.mark.parametrize("use_p", [False, True])
def test_pcg_parity_with_dense_solve(nys, use_p, layout):
    inst = make_instance("lowrank_5000x20000", seed=12, m=800, n=3000, rank=40)
    A = inst.A.double().numpy()
    rng = np.random.default_rng(1)
    d = rng.uniform(0.01, 5.0, 3000)
    delta = 1e-3
    xi = rng.standard_normal(800)
    P = nys.nys_sketch(_t(A), _t(d), 60, seed=1) if use_p else None
    A_t = _t(A.T) if layout == "transposed" else None
    y, info = nys.nys_pcg_solve(_t(A), _t(d), delta, _t(xi), P=P, rtol=1e-11, maxit=3000, A_t=A_t)
    M = normal_eq.normal_matrix(A, d, delta)
    ref = np.linalg.solve(M, xi)
    assert info.status == 0
    assert np.linalg.norm(xi - M @ _np(y)) <= 1.01e-11 * np.linalg.norm(xi) + 1e-14
    np.testing.assert_allclose(_np(y), ref, rtol=0, atol=1e-6 * np.abs(ref).max())


def test_pcg_one_iteration_with_exact_rank_preconditioner(nys):
    m, n, r = 500, 700, 10
    rng = np.random.default_rng(9)
    A = rng.standard_normal((m, r)) @ rng.standard_normal((r, n)) / np.sqrt(n)
    d = np.ones(n)
    P = nys.nys_sketch(_t(A), _t(d), r + 6, seed=5)
    xi = rng.standard_normal(m)
    y, info = nys.nys_pcg_solve(_t(A), _t(d), 1e-2, _t(xi), P=P, rtol=1e-9, poll_every=1)
    assert info.iters == 1 and info.status == 0


# ------------------------------------------------------------------ Newton step

def test_newton_step_parity(nys):
    inst = make_instance("gauss_200x500", seed=4)
    A = inst.A.double().numpy()
    m, n = A.shape
    rng = np.random.default_rng(2)
    x = rng.uniform(0.01, 2, n)
    z = rng.uniform(0.01, 2, n)
    q = inst.q.numpy()
    rho, delta = 0.1, 0.05
    rd, rp, rxz = rng.standard_normal(n), rng.standard_normal(m), rng.standard_normal(n)
    D = normal_eq.scaling(x, z, q, rho)
    M = normal_eq.normal_matrix(A, D, delta)
    ex, ey, ez, _ = normal_eq.newton_step(A, x, z, D, delta, rd, rp, rxz, lambda xi: np.linalg.solve(M, xi))
    dx, dy, dz, info = nys.nys_newton_solve(_t(A), _t(q), _t(x), _t(z), rho, delta, _t(rd), _t(rp), _t(rxz),
                                            rtol=1e-13, maxit=2000)
    for g, e in ((dx, ex), (dy, ey), (dz, ez)):
        assert np.linalg.norm(_np(g) - e) <= 1e-9 * (1 + np.linalg.norm(e))


# ------------------------------------------------------------------ IP-PMM

def test_ipm_solve_gauss_small(nys):
    inst = make_instance("gauss_200x500", seed=1)
    A, b, c, q = (inst.A.double().numpy(), inst.b.numpy(), inst.c.numpy(), inst.q.numpy())
    ref = oipm.solve(A, b, c, q, tol=1e-10)
    x, y, z, info = nys.ipm_solve(_t(A), _t(b), _t(c), _t(q), ell=20, tol=1e-6, seed=0)
    assert info.status == 0, info.kkt_rel
    meas = problem.kkt_measure(A, b, c, q, _np(x), _np(y), _np(z))
    assert meas["kkt"] <= 1e-6
    assert np.linalg.norm(_np(x) - ref["x"]) <= 1e-5 * np.linalg.norm(ref["x"])
    assert np.all(_np(x) > 0) and np.all(_np(z) > 0)


@pytest.mark.parametrize("sk,tcopy", [("f64", True), ("bf16", True), ("bf16", False)])
def test_ipm_solve_mixed_precision_fp32_matrix(nys, sk, tcopy):
    """FP32-defined matrix, FP64-accumulated products, FP64 or BF16 sketch,
    with and without the library's transposed copy of A: KKT <= 1e-6 and x
    within 1e-5 of the oracle's (polished) optimum."""
    inst = make_instance("gauss_2000x8000", seed=5, m=400, n=1600)
    A = inst.A.double().numpy()
    b, c, q = inst.b.numpy(), inst.c.numpy(), inst.q.numpy()
    At = inst.A.to(DEV)
    x, y, z, info = nys.ipm_solve(At, _t(b), _t(c), _t(q), ell=50, tol=1e-6, seed=1, sketch_dtype=sk,
                                  A_lo=At.to(torch.bfloat16) if sk == "bf16" else None,
                                  transposed_copy=tcopy)
    assert info.status == 0, (info.kkt_rel, info.iters)
    meas = problem.kkt_measure(A, b, c, q, _np(x), _np(y), _np(z))
    assert meas["kkt"] <= 1e-6
    xs = inst.x_star.numpy()                 # planted optimum = oracle optimum (pinned)
    assert np.linalg.norm(_np(x) - xs) <= 1e-5 * np.linalg.norm(xs)


def test_ipm_solve_rejects_bad_data(nys):
    inst = make_instance("gauss_200x500", seed=2)
    A, b, c, q = (_t(inst.A.double().numpy()), _t(inst.b.numpy()), _t(inst.c.numpy()), _t(inst.q.numpy()))
    qb = q.clone()
    qb[3] = -1.0
    with pytest.raises(nys.NysError) as e:
        nys.ipm_solve(A, b, c, qb, ell=20)
    assert e.value.code == -1
    Ab = A.clone()
    Ab[5, 7] = float("nan")
    with pytest.raises(nys.NysError) as e:
        nys.ipm_solve(Ab, b, c, q, ell=20)
    assert e.value.code == -1
    with pytest.raises(nys.NysError):
        nys.ipm_solve(A, b, c, q, ell=0)


def _planted(m, n, nsupp, q, seed):
    """Planted KKT point (x*, y*, z*) with |support| = nsupp and b, c from it."""
    rng = np.random.default_rng(seed)
    A = rng.standard_normal((m, n)) / np.sqrt(n)
    S = rng.permutation(n)[:nsupp]
    xs = np.zeros(n)
    xs[S] = rng.uniform(0.1, 1.0, nsupp)
    zs = rng.uniform(0.1, 1.0, n)
    zs[S] = 0.0
    ys = rng.standard_normal(m)
    return A, A @ xs, A.T @ ys + zs - q * xs, xs, ys, zs


def test_ipm_solve_lp_planted_vertex(nys):
    """Q = 0 (a linear program): the planted optimum is a vertex with m basic
    variables, unique because A_S is square and nonsingular."""
    m, n = 30, 80
    q = np.zeros(n)
    A, b, c, xs, ys, zs = _planted(m, n, m, q, seed=3)
    ref = oipm.solve(A, b, c, q, tol=1e-10)
    xo, _, _, polished = oipm.polish(A, b, c, q, ref["x"], ref["y"], ref["z"])
    assert polished and np.linalg.norm(xo - xs) <= 1e-10 * np.linalg.norm(xs)
    x, y, z, info = nys.ipm_solve(_t(A), _t(b), _t(c), _t(q), ell=10, tol=1e-8, seed=0)
    assert info.status == 0
    assert problem.kkt_measure(A, b, c, q, _np(x), _np(y), _np(z))["kkt"] <= 1e-8
    assert np.linalg.norm(_np(x) - xs) <= 1e-5 * np.linalg.norm(xs)


def test_ipm_solve_single_constraint(nys):
    """m = 1 (ell = 1): the smallest problem the method defines."""
    n = 7
    q = np.random.default_rng(4).uniform(0.5, 1.0, n)
    A, b, c, xs, ys, zs = _planted(1, n, 3, q, seed=4)
    x, y, z, info = nys.ipm_solve(_t(A), _t(b), _t(c), _t(q), ell=1, tol=1e-8, seed=0)
    assert info.status == 0
    assert problem.kkt_measure(A, b, c, q, _np(x), _np(y), _np(z))["kkt"] <= 1e-8
    assert np.linalg.norm(_np(x) - xs) <= 1e-6 * np.linalg.norm(xs)


def test_pcg_zero_rhs_and_full_rank_sketch(nys):
    """rhs = 0 returns y = 0 without iterating; with ell = m the Nystrom
    approximation is N itself, so P^{-1} M is a multiple of I and PCG takes
    one iteration."""
    m, n = 64, 300
    rng = np.random.default_rng(6)
    A = rng.standard_normal((m, n)) / np.sqrt(n)
    d = rng.uniform(0.1, 2.0, n)
    y, info = nys.nys_pcg_solve(_t(A), _t(d), 1e-2, _t(np.zeros(m)))
    assert info.iters == 0 and info.status == 0 and not bool(y.any())
    P = nys.nys_sketch(_t(A), _t(d), m, seed=2)
    xi = rng.standard_normal(m)
    y, info = nys.nys_pcg_solve(_t(A), _t(d), 1e-2, _t(xi), P=P, rtol=1e-9, poll_every=1)
    assert info.status == 0 and info.iters <= 2, info.iters
    M = normal_eq.normal_matrix(A, d, 1e-2)
    np.testing.assert_allclose(_np(y), np.linalg.solve(M, xi), rtol=1e-7, atol=1e-9)


def test_ipm_adjoint_parity(nys):
    inst = make_instance("gauss_2000x8000", seed=3, m=150, n=400)
    A32 = inst.A
    A = A32.double().numpy()
    b, c, q = inst.b.numpy(), inst.c.numpy(), inst.q.numpy()
    x, y, z, info = nys.ipm_solve(_t(A32, torch.float32), _t(b), _t(c), _t(q), ell=30, tol=1e-9)
    assert info.status == 0
    xs, ys, zs = inst.x_star.numpy(), inst.y_star.numpy(), inst.z_star.numpy()
    x_tgt = xs + 0.01 * np.random.default_rng(0).standard_normal(xs.shape)
    g = _np(x) - x_tgt
    ref = oadj.kkt_gradient(A, b, c, q, xs, ys, zs, xs - x_tgt)
    grads, pinfo = nys.ipm_adjoint(_t(A32, torch.float32), _t(b), _t(c), _t(q), x, y, z, info.rho,
                                   info.delta, _t(g), ell=30)
    for k in ("c", "b", "q", "A"):
        e = ref[k]
        gk = _np(grads[k])
        assert np.linalg.norm(gk - e) <= 1e-4 * np.linalg.norm(e), k


# ------------------------------------------------------------------ comparators (partial Cholesky, plain CG)

def _pchol_case(m, n, seed):
    rng = np.random.default_rng(seed)
    A = rng.standard_normal((m, n)) * rng.uniform(0.2, 3.0, m)[:, None] / np.sqrt(n)
    d = rng.uniform(0.05, 4.0, n)
    return A, d


@pytest.mark.parametrize("m,n,ell", [(300, 900, 20), (1000, 2500, 64), (77, 200, 77)])
def test_pchol_build_and_apply_parity(nys, m, n, ell):
    from oracle import pchol as opc
    print(f"pchol {m}x{n} ell={ell}", flush=True)
    A, d = _pchol_case(m, n, seed=m + ell)
    delta = 1e-3
    P = nys.nys_pchol_build(_t(A), _t(d), delta, ell)
    ref = opc.build(A, d, delta, ell)
    np.testing.assert_array_equal(P.piv.cpu().numpy(), ref["piv"])
    pos = P.pos.cpu().numpy()
    assert np.all(pos[ref["piv"]] == np.arange(ell)) and np.all(pos[ref["rest"]] == -1)
    Lo = np.empty((m, ell))
    Lo[ref["piv"]] = ref["L11"]
    Lo[ref["rest"]] = ref["L21"]
    scale = np.abs(Lo).max()
    np.testing.assert_allclose(_np(P.L), Lo, rtol=0, atol=1e-10 * scale)
    np.testing.assert_allclose(_np(P.diagS)[ref["rest"]], ref["diagS"], rtol=1e-8)
    r = np.random.default_rng(1).standard_normal(m)
    out = _np(nys.nys_pchol_apply(P, _t(r)))
    ro = opc.precond_inv_apply(ref, r)
    np.testing.assert_allclose(out, ro, rtol=0, atol=1e-9 * np.abs(ro).max())


def test_pchol_pivot_ties(nys):
    """Equal diagonal entries: the smaller index is taken first."""
    from oracle import pchol as opc
    A, d = _pchol_case(50, 120, seed=9)
    A[7] = A[3] = 10.0 * A[3]          # two equal, largest rows
    for ell in (1, 2, 3):
        P = nys.nys_pchol_build(_t(A), _t(d), 1e-3, ell)
        ref = opc.build(A, d, 1e-3, ell)
        np.testing.assert_array_equal(P.piv.cpu().numpy(), ref["piv"])
        assert 3 in ref["piv"]


@pytest.mark.parametrize("ell", [30, 120])
def test_pcg_pchol_parity_with_dense_solve(nys, ell):
    m, n = 120, 400
    A, d = _pchol_case(m, n, seed=ell)
    delta = 1e-4
    P = nys.nys_pchol_build(_t(A), _t(d), delta, ell)
    xi = np.random.default_rng(2).standard_normal(m)
    y, info = nys.nys_pcg_solve(_t(A), _t(d), delta, _t(xi), P=P, rtol=1e-11, maxit=2000, poll_every=1)
    M = normal_eq.normal_matrix(A, d, delta)
    assert info.status == 0
    if ell == m:                       # P_Chol = N + delta I exactly
        assert info.iters <= 2, info.iters
    assert np.linalg.norm(xi - M @ _np(y)) <= 1.01e-11 * np.linalg.norm(xi) + 1e-14


@pytest.mark.parametrize("precond", ["pchol", "none"])
def test_ipm_solve_comparators(nys, precond):
    """Chol-IP-PMM and CG-IP-PMM reach the same optimum as Nys-IP-PMM."""
    inst = make_instance("gauss_200x500", seed=1)
    A, b, c, q = (inst.A.double().numpy(), inst.b.numpy(), inst.c.numpy(), inst.q.numpy())
    x, y, z, info = nys.ipm_solve(_t(A), _t(b), _t(c), _t(q), ell=20, tol=1e-6, seed=0, precond=precond)
    assert info.status == 0, info.kkt_rel
    assert problem.kkt_measure(A, b, c, q, _np(x), _np(y), _np(z))["kkt"] <= 1e-6
    xs = inst.x_star.numpy()
    assert np.linalg.norm(_np(x) - xs) <= 1e-5 * np.linalg.norm(xs)


# ------------------------------------------------------------------ free and box-constrained variables

def _box_case(m, n, seed, q_lo=0.5):
    from oracle import boxqp
    rng = np.random.default_rng(seed)
    A = rng.standard_normal((m, n)) / np.sqrt(n)
    vt = rng.choice([0, 1, 2], size=n, p=[0.4, 0.2, 0.4]).astype(np.int8)
    q = rng.uniform(q_lo, 1.5, n)
    u = np.where(vt == 2, rng.uniform(0.5, 2.0, n), 0.0)
    b, c, xs, ys, zs, ws, ss = boxqp.planted(A, q, vt, u, rng)
    return A, b, c, q, u, vt, xs, ys


@pytest.mark.parametrize("m,n,precond", [(40, 120, "nystrom"), (300, 1000, "nystrom"), (300, 1000, "pchol")])
def test_ipm_solve_box_planted(nys, m, n, precond):
    """Free, non-negative and box-constrained variables: the planted optimum
    (some x at 0, some at u, some inside, some free), and the oracle's."""
    from oracle import boxqp
    print(f"ipm_solve_box {m}x{n} {precond}", flush=True)
    A, b, c, q, u, vt, xs, ys = _box_case(m, n, seed=m + n)
    x, y, z, w, s, info = nys.ipm_solve_box(_t(A), _t(b), _t(c), _t(q),
                                            torch.as_tensor(vt, device=DEV), _t(u), ell=20, tol=1e-8,
                                            precond=precond)
    assert info.status == 0, (info.kkt_rel, info.iters)
    xg, yg, zg, wg, sg = (_np(t) for t in (x, y, z, w, s))
    meas = boxqp.kkt_measure(A, b, c, q, u, vt.astype(int), xg, yg, zg, wg, sg)
    assert meas["kkt"] <= 1e-8, meas
    assert np.all(xg[vt == 2] >= 0) and np.all(xg[vt == 2] <= u[vt == 2]) and np.all(xg[vt == 0] >= 0)
    assert np.all(zg[vt == 1] == 0) and np.all(wg[vt != 2] == 0) and np.all(sg[vt != 2] == 0)
    assert np.linalg.norm(xg - xs) <= 1e-6 * np.linalg.norm(xs)
    ref = boxqp.solve(A, b, c, q, u, vt.astype(int), tol=1e-10)
    assert np.linalg.norm(xg - ref["x"]) <= 1e-6 * np.linalg.norm(ref["x"])


def test_ipm_solve_box_all_nonneg_matches_ipm_solve(nys):
    """vtype all NONNEG: the box form takes the same steps as ipm_solve."""
    inst = make_instance("gauss_200x500", seed=1)
    A, b, c, q = (_t(inst.A.double().numpy()), _t(inst.b.numpy()), _t(inst.c.numpy()), _t(inst.q.numpy()))
    n = A.shape[1]
    x1, y1, z1, i1 = nys.ipm_solve(A, b, c, q, ell=20, tol=1e-8, seed=0)
    vt = torch.zeros(n, dtype=torch.int8, device=DEV)
    x2, y2, z2, w2, s2, i2 = nys.ipm_solve_box(A, b, c, q, vt, torch.zeros(n, dtype=torch.float64, device=DEV),
                                               ell=20, tol=1e-8, seed=0)
    assert i1.iters == i2.iters
    assert float((x1 - x2).abs().max()) <= 1e-12 * float(x1.abs().max())
    assert not bool(w2.any()) and not bool(s2.any())


def test_ipm_solve_box_svm_form(nys):
    """The dual linear SVM in form (P~): v free with Q = I, 0 <= p <= tau,
    A = [I, -X diag(y); 0, y^T] -- against the oracle (v and the objective
    are unique; p need not be)."""
    from instances import svm_instance
    from oracle import boxqp
    S = svm_instance(40, 400, seed=7, sep=2.0)
    A, b, c, q, u, vt = (S[k].numpy() for k in ("A", "b", "c", "q", "u", "vtype"))
    x, y, z, w, s, info = nys.ipm_solve_box(_t(A), _t(b), _t(c), _t(q), torch.as_tensor(vt, device=DEV), _t(u),
                                            ell=20, tol=1e-8)
    assert info.status == 0, info.kkt_rel
    xg = _np(x)
    assert boxqp.kkt_measure(A, b, c, q, u, vt.astype(int), xg, _np(y), _np(z), _np(w), _np(s))["kkt"] <= 1e-8
    ref = boxqp.solve(A, b, c, q, u, vt.astype(int), tol=1e-10)
    obj = lambda v: 0.5 * float(v @ (q * v)) + float(c @ v)
    assert abs(obj(xg) - obj(ref["x"])) <= 1e-6 * (1 + abs(obj(ref["x"])))
    np.testing.assert_allclose(xg[:40], ref["x"][:40], atol=1e-5 * (1 + np.abs(ref["x"][:40]).max()))


def test_ipm_solve_box_rejects_bad_kinds(nys):
    A, b, c, q, u, vt, xs, ys = _box_case(20, 50, seed=3)
    bad = vt.copy()
    bad[4] = 7
    with pytest.raises(nys.NysError):
        nys.ipm_solve_box(_t(A), _t(b), _t(c), _t(q), torch.as_tensor(bad, device=DEV), _t(u), ell=5)
    j = int(np.flatnonzero(vt == 2)[0])
    ub = u.copy()
    ub[j] = 0.0
    with pytest.raises(nys.NysError):
        nys.ipm_solve_box(_t(A), _t(b), _t(c), _t(q), torch.as_tensor(vt, device=DEV), _t(ub), ell=5)


# ------------------------------------------------------------------ sketch size from d_eff; reuse

@pytest.mark.parametrize("ell", [1, 7, 200, 1000])
def test_deff_estimate_parity(nys, ell):
    """nys_deff_estimate against the oracle's estimate (eq. effective-dim over
    the Nystrom eigenvalues), zero eigenvalues included."""
    from oracle import adaptive
    print(f"deff_estimate ell={ell}", flush=True)
    rng = np.random.default_rng(ell)
    lam = np.sort(np.exp(rng.uniform(-12, 6, ell)))[::-1].copy()
    if ell > 3:
        lam[-2:] = 0.0
    for mu in (1e-9, 1e-3, 1.0, 1e4):
        got = nys.nys_deff_estimate(_t(lam), mu)
        ref = adaptive.d_eff_estimate(lam, mu)
        assert abs(got - ref) <= 1e-13 * max(ref, 1.0), (mu, got, ref)


def _check_trace(nys, tr, info, rule, ell0, ell_min, ell_max, c_ell, max_age, growth, nystrom=True):
    """The driver's decisions follow its (CPU-pinned) rules on what it observed:
    a build exactly when the reuse rule says so, the size the sketch-size rule
    gives for the recorded inputs, the size kept between builds, and
    0 <= d_hat <= ell."""
    K = info.iters
    tr = tr[:K]
    assert np.array_equal(tr[:, 0], np.arange(K))
    built = tr[:, 4] == 1.0
    ells = tr[:, 3].astype(int)
    assert built[0] and int(built.sum()) == info.builds and ells[-1] == info.ell_last
    k_build, pcg_ref, pcg_prev, ell_prev = -1, 0, 0, ell0
    for k in range(K):
        assert nys.nys_precond_rebuild_due(k, k_build, pcg_prev, pcg_ref, max_age, growth) == built[k], k
        if built[k]:
            if rule == "fixed":
                assert ells[k] == ell0
            else:
                exp = nys.nys_sketch_size_rule(rule, tr[k, 8], tr[k, 9], tr[k, 1], k, ell_prev, ell_min, ell_max,
                                               c_ell)
                assert ells[k] == exp, (k, ells[k], exp)
            k_build, pcg_ref = k, int(tr[k, 7])
        else:
            assert ells[k] == ell_prev and np.isnan(tr[k, 8])
        if nystrom:
            assert 0.0 <= tr[k, 5] <= ells[k] + 1e-9
        pcg_prev, ell_prev = int(tr[k, 7]), ells[k]
    assert int(tr[:, 7].sum()) <= info.pcg_iters_total


@pytest.mark.parametrize("rule,max_age,growth", [("deff", 0, 1.5), ("deff", 3, 1.5), ("theorem", 0, 1.5),
                                                  ("fixed", 2, 1.5), ("fixed", 50, 1e9)])
def test_ipm_solve_sketch_size_rule_and_reuse(nys, rule, max_age, growth):
    """Sketch size from the d_eff estimate (and the main theorem's bound), and
    reuse of the preconditioner: the planted optimum (the oracle's, pinned)
    at KKT <= 1e-6, with decisions that follow the rules."""
    print(f"ipm rule={rule} reuse={max_age}", flush=True)
    inst = make_instance("lowrank_5000x20000", seed=3, m=500, n=2000, rank=40)
    A, b, c, q = (inst.A.double().numpy(), inst.b.numpy(), inst.c.numpy(), inst.q.numpy())
    ell0, ell_min, ell_max, c_ell = 20, 8, 160, 2.0
    tr = np.full((100, len(nys.TRACE_FIELDS)), -1.0)
    x, y, z, info = nys.ipm_solve(_t(A), _t(b), _t(c), _t(q), ell=ell0, tol=1e-6, seed=2, ell_rule=rule,
                                  ell_min=ell_min, ell_max=ell_max, c_ell=c_ell, reuse_max_age=max_age,
                                  reuse_growth=growth, trace=tr)
    assert info.status == 0, (info.kkt_rel, info.iters)
    assert problem.kkt_measure(A, b, c, q, _np(x), _np(y), _np(z))["kkt"] <= 1e-6
    xs = inst.x_star.numpy()
    assert np.linalg.norm(_np(x) - xs) <= 1e-5 * np.linalg.norm(xs)
    _check_trace(nys, tr, info, rule, ell0, ell_min, ell_max, c_ell, max_age, growth)
    if max_age == 0:
        assert info.builds == info.iters
    if max_age == 50:                                  # one preconditioner for the whole solve
        assert info.builds == 1
    assert np.all(tr[info.iters:] == -1.0)           # nothing written past the last Newton solve


def test_ipm_solve_reuse_with_partial_cholesky(nys):
    print("ipm pchol reuse", flush=True)
    inst = make_instance("gauss_200x500", seed=1)
    A, b, c, q = (inst.A.double().numpy(), inst.b.numpy(), inst.c.numpy(), inst.q.numpy())
    tr = np.zeros((100, len(nys.TRACE_FIELDS)))
    x, y, z, info = nys.ipm_solve(_t(A), _t(b), _t(c), _t(q), ell=20, tol=1e-6, seed=0, precond="pchol",
                                  reuse_max_age=3, trace=tr)
    assert info.status == 0
    xs = inst.x_star.numpy()
    assert np.linalg.norm(_np(x) - xs) <= 1e-5 * np.linalg.norm(xs)
    _check_trace(nys, tr, info, "fixed", 20, 1, 20, 2.0, 3, 1.5, nystrom=False)
    assert np.all(np.isnan(tr[:info.iters, 5]))       # no Nystrom estimate for this preconditioner


def test_ipm_solve_defaults_unchanged_by_trace(nys):
    """Fixed size, no reuse: the same iterates with and without a trace, one
    build per iteration."""
    inst = make_instance("gauss_200x500", seed=1)
    A, b, c, q = (_t(inst.A.double().numpy()), _t(inst.b.numpy()), _t(inst.c.numpy()), _t(inst.q.numpy()))
    x1, y1, z1, i1 = nys.ipm_solve(A, b, c, q, ell=20, tol=1e-6, seed=0)
    tr = np.zeros((100, len(nys.TRACE_FIELDS)))
    x2, y2, z2, i2 = nys.ipm_solve(A, b, c, q, ell=20, tol=1e-6, seed=0, trace=tr)
    assert torch.equal(x1, x2) and torch.equal(y1, y2) and i1.pcg_iters_total == i2.pcg_iters_total
    assert i2.builds == i2.iters and np.all(tr[:i2.iters, 3] == 20) and np.all(np.isnan(tr[:i2.iters, 8]))


def test_ipm_solve_rejects_bad_rule_options(nys):
    inst = make_instance("gauss_200x500", seed=1)
    A, b, c, q = (_t(inst.A.double().numpy()), _t(inst.b.numpy()), _t(inst.c.numpy()), _t(inst.q.numpy()))
    for kw in (dict(ell_rule="deff", precond="pchol"), dict(ell_rule="deff", ell_max=201),
               dict(ell_rule="deff", ell_min=30, ell_max=25), dict(ell_rule="deff", ell_max=10),
               dict(reuse_max_age=-1)):
        with pytest.raises(nys.NysError):
            nys.ipm_solve(A, b, c, q, ell=20, tol=1e-6, **kw)
    with pytest.raises(ValueError):
        nys.ipm_solve(A, b, c, q, ell=20, tol=1e-6, trace=np.zeros((10, 3)))


# ------------------------------------------------------------------ portfolio problem

@pytest.mark.parametrize("precond,storage", [("nystrom", "f64"), ("nystrom", "f32"), ("pchol", "f64"),
                                             ("none", "f64")])
def test_ipm_solve_box_portfolio(nys, precond, storage):
    """The factor-model portfolio problem in form (P~) (x >= 0, y = F^T x
    free, slacks >= 0) at tolerance 1e-8: the oracle's optimum (unique: the
    objective is strictly convex in x and y, and t = u - M x)."""
    from instances import portfolio_instance
    from oracle import boxqp
    print(f"portfolio precond={precond} storage={storage}", flush=True)
    dt = torch.float64 if storage == "f64" else torch.float32
    P = portfolio_instance(600, 300, 12, seed=1, dtype=dt)
    npd = {k: v.double().numpy() if k == "A" else v.numpy() for k, v in P.items()}
    ref = boxqp.solve(npd["A"], npd["b"], npd["c"], npd["q"], npd["u"], npd["vtype"], tol=1e-11)
    assert ref["status"] == 0
    A = P["A"].to(DEV)
    x, y, z, w, s, info = nys.ipm_solve_box(A, _t(npd["b"]), _t(npd["c"]), _t(npd["q"]),
                                            _t(npd["vtype"], torch.int8), _t(npd["u"]), ell=20, tol=1e-8, seed=3,
                                            precond=precond, sketch_dtype="bf16" if storage == "f32" else "f64",
                                            A_lo=A.to(torch.bfloat16) if storage == "f32" else None)
    assert info.status == 0, (info.kkt_rel, info.iters)
    meas = boxqp.kkt_measure(npd["A"], npd["b"], npd["c"], npd["q"], npd["u"], npd["vtype"], _np(x), _np(y), _np(z),
                             _np(w), _np(s))
    assert meas["kkt"] <= 1e-8
    assert np.linalg.norm(_np(x) - ref["x"]) <= 1e-6 * np.linalg.norm(ref["x"])
    # the budget row is one entry of r_p, whose norm the tolerance bounds by
    # tol (1 + ||b||)
    assert abs(_np(x)[:600].sum() - 1.0) <= 1e-8 * (1.0 + np.linalg.norm(npd["b"]))


# ------------------------------------------------------------------ predictor-corrector forms

@pytest.mark.parametrize("box", [False, True])
def test_ipm_solve_combined_and_separate_corrector(nys, box):
    """Algorithm 6's direction computed as predictor + corrector (two solves)
    and as one solve with the summed right-hand side (the default, with a
    loose predictor): both reach the oracle's optimum at KKT <= 1e-8."""
    print(f"corrector forms box={box}", flush=True)
    if box:
        from oracle import boxqp
        A, b, c, q, u, vt, xs, ys = _box_case(300, 1000, seed=8)
        ref = boxqp.solve(A, b, c, q, u, vt, tol=1e-11)["x"]
        args = (_t(A), _t(b), _t(c), _t(q), _t(vt, torch.int8), _t(u))
        run = lambda **kw: nys.ipm_solve_box(*args, ell=20, tol=1e-8, seed=1, **kw)
    else:
        inst = make_instance("lowrank_5000x20000", seed=5, m=400, n=1600, rank=30)
        A, b, c, q = (inst.A.double().numpy(), inst.b.numpy(), inst.c.numpy(), inst.q.numpy())
        ref = inst.x_star.numpy()
        run = lambda **kw: nys.ipm_solve(_t(A), _t(b), _t(c), _t(q), ell=20, tol=1e-8, seed=1, **kw)
    for kw in (dict(separate_corrector=True), dict(), dict(predictor_rtol=1e-4)):
        out = run(**kw)
        x, info = out[0], out[-1]
        assert info.status == 0, (kw, info.kkt_rel)
        assert np.linalg.norm(_np(x) - ref) <= 1e-6 * np.linalg.norm(ref), kw


# ------------------------------------------------------------------ initial point

@pytest.mark.parametrize("case", ["gauss", "lowrank", "box", "box_units"])
def test_initial_point_measures_match_the_oracle(nys, case):
    """The supplement's initial point (reading 9; the regularised A A^T + 10 I
    systems): the GPU's mu, rp_rel and rd_rel at k = 0 (from the trace) equal
    the oracle's for the point it constructs, to the initial solves' accuracy."""
    from oracle import boxqp
    print(f"initial point {case}", flush=True)
    tr = np.full((100, len(nys.TRACE_FIELDS)), np.nan)
    f = {k: i for i, k in enumerate(nys.TRACE_FIELDS)}
    if case in ("gauss", "lowrank"):
        inst = (make_instance("gauss_200x500", seed=2) if case == "gauss"
                else make_instance("lowrank_5000x20000", seed=2, m=300, n=1200, rank=20))
        A, b, c, q = (inst.A.double().numpy(), inst.b.numpy(), inst.c.numpy(), inst.q.numpy())
        x0, y0, z0 = oipm.initial_point(A, b, c, q)
        ref = problem.kkt_measure(A, b, c, q, x0, y0, z0)
        nys.ipm_solve(_t(A), _t(b), _t(c), _t(q), ell=20, tol=1e-6, seed=0, trace=tr)
    else:
        A, b, c, q, u, vt, xs, ys = _box_case(120, 400, seed=6)
        x0, y0, z0, w0, s0 = boxqp.initial_point(A, b, c, q, u, vt)
        ref = boxqp.kkt_measure(A, b, c, q, u, vt, x0, y0, z0, w0, s0)
        args = (_t(b), _t(c), _t(q), _t(vt, torch.int8), _t(u))
        if case == "box":
            nys.ipm_solve_box(_t(A), *args, ell=20, tol=1e-6, seed=0, trace=tr)
        else:
            # A with 40 slack columns on its last rows: unit columns on the GPU,
            # written out densely for the oracle
            m, n = A.shape
            rows = np.arange(m - 40, m, dtype=np.int32)
            F = np.hstack([A, np.zeros((m, 40))])
            F[rows, n + np.arange(40)] = 1.0
            vt2 = np.concatenate([vt, np.zeros(40, np.int8)])
            q2, u2 = np.concatenate([q, np.full(40, 0.5)]), np.concatenate([u, np.zeros(40)])
            c2 = np.concatenate([c, np.ones(40)])
            x0, y0, z0, w0, s0 = boxqp.initial_point(F, b, c2, q2, u2, vt2)
            ref = boxqp.kkt_measure(F, b, c2, q2, u2, vt2, x0, y0, z0, w0, s0)
            nys.ipm_solve_box(_t(A), _t(b), _t(c2), _t(q2), _t(vt2, torch.int8), _t(u2), ell=20, tol=1e-6, seed=0,
                              trace=tr, units=(_t(rows, torch.int32), _t(np.ones(40))))
    for key in ("mu", "rp_rel", "rd_rel"):
        got = tr[0, f[key]]
        assert abs(got - ref[key]) <= 1e-7 * abs(ref[key]) + 1e-14, (key, got, ref[key])


@pytest.mark.parametrize("corrector", ["separate", "combined"])
@pytest.mark.parametrize("case", ["qp", "box"])
def test_first_iterations_follow_the_oracle(nys, case, corrector):
    """With near-exact inner solves, the GPU driver's first IP-PMM iterations
    (step lengths, mu_aff, the corrector, the parameter update) reproduce the
    oracle's Algorithm 6, which solves the predictor and the corrector
    separately: mu, rp_rel and rd_rel at k = 0..4 agree to 1e-6 relative.
    'separate' runs the two solves as printed; 'combined' runs the library's
    default direction path (one solve of the summed right-hand side, warm-
    started from the predictor's dy) with the predictor tolerance tightened
    to the inner one, so both paths are pinned step by step."""
    from oracle import boxqp
    print(f"first iterations {case} {corrector}", flush=True)
    tr = np.full((100, len(nys.TRACE_FIELDS)), np.nan)
    f = {k: i for i, k in enumerate(nys.TRACE_FIELDS)}
    hist = []
    tight = dict(separate_corrector=corrector == "separate", predictor_rtol=1e-13, inner_factor=1e-9,
                 pcg_rtol=1e-13, pcg_maxit=5000, tol=1e-9, seed=0, trace=tr)
    if case == "qp":
        inst = make_instance("gauss_200x500", seed=3)
        A, b, c, q = (inst.A.double().numpy(), inst.b.numpy(), inst.c.numpy(), inst.q.numpy())
        oipm.solve(A, b, c, q, tol=1e-9, history=hist)
        nys.ipm_solve(_t(A), _t(b), _t(c), _t(q), ell=20, **tight)
    else:
        A, b, c, q, u, vt, xs, ys = _box_case(120, 400, seed=7)
        boxqp.solve(A, b, c, q, u, vt, tol=1e-9, history=hist)
        nys.ipm_solve_box(_t(A), _t(b), _t(c), _t(q), _t(vt, torch.int8), _t(u), ell=20, **tight)
    for k in range(5):
        for key in ("mu", "rp_rel", "rd_rel"):
            got, ref = tr[k, f[key]], hist[k][key]
            assert abs(got - ref) <= 1e-6 * abs(ref) + 1e-13, (k, key, got, ref)


# ------------------------------------------------------------------ autograd wrapper

def test_autograd_wrapper_matches_the_adjoint(nys):
    """x*(A, b, c, q) through torch.autograd: the gradients of
    L = 1/2 ||x* - x_tgt||^2 with respect to b and c equal ipm_adjoint's for
    g = x* - x_tgt, and A, q get none when not requested."""
    from paper_2404_14524_amd.autograd import nys_qp
    inst = make_instance("gauss_200x500", seed=4)
    A, b, c, q = (_t(inst.A.double().numpy()), _t(inst.b.numpy()), _t(inst.c.numpy()), _t(inst.q.numpy()))
    b.requires_grad_(True)
    c.requires_grad_(True)
    x = nys_qp(A, b, c, q, ell=20, tol=1e-9, seed=0)
    tgt = x.detach() + 0.01 * torch.randn(x.shape, generator=torch.Generator(device=DEV).manual_seed(1),
                                          dtype=torch.float64, device=DEV)
    L = 0.5 * ((x - tgt) ** 2).sum()
    gb, gc = torch.autograd.grad(L, (b, c))
    x2, y2, z2, info = nys.ipm_solve(A, b.detach(), c.detach(), q, ell=20, tol=1e-9, seed=0)
    assert torch.equal(x2, x.detach())
    ref, _ = nys.ipm_adjoint(A, b.detach(), c.detach(), q, x2, y2, z2, info.rho, info.delta,
                             (x2 - tgt).contiguous(), ell=20, seed=0, want=("b", "c"))
    np.testing.assert_allclose(_np(gb), _np(ref["b"]), rtol=0, atol=1e-12 * (1 + np.abs(_np(ref["b"])).max()))
    np.testing.assert_allclose(_np(gc), _np(ref["c"]), rtol=0, atol=1e-12 * (1 + np.abs(_np(ref["c"])).max()))
    assert A.grad is None and q.grad is None
