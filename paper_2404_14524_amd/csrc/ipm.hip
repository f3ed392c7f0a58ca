// Nys-IP-PMM for (P) with non-negative variables (Algorithm 4 with the
// Mehrotra predictor-corrector of Algorithm 6 and the Newton solve of
// Algorithm 5), and the adjoint of the converged KKT system.
//
// Readings where the paper is silent or defers to the original IP-PMM:
// * initial point: the supplement's construction with F = J = empty; the
//   regularised systems (A A^T + 10 I) are solved by Nystrom-PCG; the dual
//   centring shift uses (x~ + delta_p); non-positive entries left after the
//   shifts (possible only when the product gamma is zero) are set to 1.
// * parameter update: zeta <- x, lambda <- y every iteration and
//   rho = delta = max(5e-10, min(rho, mu)).
// * stopping test: max(||r_p||/(1+||b||), ||r_d||/(1+||c||), mu) <= tol.
// * inner tolerance: ||xi - M dy|| <= max(1e-12 ||xi||, min(1e-2 ||xi||, tau)) with
//   tau = f max(mu, tol (1 + ||b||)), f = 0.9 by default, judged on the true residual (the
//   theory asks for a residual of order mu; the floor keeps solves from being
//   asked for accuracy that the primal-feasibility target cannot use).
// * a fresh test matrix per iteration (Philox key = seed, counter = k), shared
//   by predictor and corrector.

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>

#include "common.hpp"
#include "kernels.hpp"
#include "mapreduce.hpp"

namespace nys {
int ipm_pcg(nys_handle h, const nys_matrix* A, const double* d, double delta, const double* U,
            const double* lam, int ell, const nys_pchol* pch, const double* rhs, double* y,
            const nys_pcg_opts* o, nys_pcg_info* info);
int ipm_sketch(nys_handle h, const nys_matrix* A, const double* d, int ell, uint64_t seed,
               uint64_t counter, nys_dtype mode, double c_nu, double* U, double* lam, double* nu);
int ipm_newton(nys_handle h, const nys_matrix* A, const double* x, const double* z, const double* D,
               double delta, const double* U, const double* lam, int ell, const nys_pchol* pch,
               const double* rd, const double* rp, const double* rxz, const nys_pcg_opts* o,
               double mu_abs, double* dx, double* dy, double* dz, nys_pcg_info* info,
               const BoxNewton& bx, double loose_rel = 0.0, const double* dy_guess = nullptr);
int grad_A_rank2(nys_handle h, int64_t m, int64_t n, const double* y, const double* u1,
                 const double* u2, const double* x, double* G);

namespace {

constexpr double STEP = 0.995;
constexpr double REG0 = 8.0;
constexpr double REG_FLOOR = 5e-10;
constexpr double INIT_REG = 10.0;
constexpr uint64_t CTR_INIT = 0xFFFFFFFFFFFFFFFFull;
constexpr uint64_t CTR_ADJ = 0xFFFFFFFFFFFFFFFEull;

using clk = std::chrono::steady_clock;
double ms_since(clk::time_point t0) {
  return std::chrono::duration<double, std::milli>(clk::now() - t0).count();
}

// ---------------------------------------------------------------- element-wise steps
// vt (index kinds) NULL: every variable non-negative and the box arrays
// (w, s and their right-hand sides and directions) are not used.
__device__ __forceinline__ int kind_of(const int8_t* vt, int64_t j) { return vt ? (int)vt[j] : NYS_VAR_NONNEG; }

struct ResidD {       // r_d = c + Q x - A^T y - z + s; ||r_d||^2, mu numerator, #non-finite, ||r_u||^2
  double* rd;
  const double *c, *q, *x, *aty, *z;
  const int8_t* vt;
  const double *u, *w, *s;
  __device__ void operator()(int64_t j, double* a, double*) const {
    const int k = kind_of(vt, j);
    double v = c[j] + q[j] * x[j] - aty[j] - z[j];
    if (k == NYS_VAR_BOX) v += s[j];
    rd[j] = v;
    a[0] = fma(v, v, a[0]);
    if (k != NYS_VAR_FREE) a[1] = fma(x[j], z[j], a[1]);
    bool bad = !isfinite(x[j]) || !isfinite(z[j]);
    if (k == NYS_VAR_BOX) {
      a[1] = fma(w[j], s[j], a[1]);
      const double ru = u[j] - x[j] - w[j];
      a[3] = fma(ru, ru, a[3]);
      bad = bad || !isfinite(w[j]) || !isfinite(s[j]);
    }
    if (bad) a[2] += 1.0;
  }
};
struct Scaling {      // D = (Q + Theta^{-1} + rho I)^{-1}: z/x (I), z/x + s/w (J), 0 (F)
  double* D;
  const double *q, *x, *z;
  double rho;
  const int8_t* vt;
  const double *w, *s;
  __device__ void operator()(int64_t j, double*, double*) const {
    const int k = kind_of(vt, j);
    double th = k == NYS_VAR_FREE ? 0.0 : z[j] / x[j];
    if (k == NYS_VAR_BOX) th += s[j] / w[j];
    D[j] = 1.0 / (q[j] + th + rho);
  }
};
struct PredN {        // R_d = r_d + rho (x - zeta), R_xz = -X Z, R_ws = -W S, R_u = u - x - w
  double *Rd, *Rxz;
  const double *rd, *x, *zeta, *z;
  double rho;
  const int8_t* vt;
  double *Rws, *Ru;
  const double *u, *w, *s;
  __device__ void operator()(int64_t j, double*, double*) const {
    const int k = kind_of(vt, j);
    Rd[j] = rd[j] + rho * (x[j] - zeta[j]);
    Rxz[j] = k == NYS_VAR_FREE ? 0.0 : -x[j] * z[j];
    if (Rws) {
      Rws[j] = k == NYS_VAR_BOX ? -w[j] * s[j] : 0.0;
      Ru[j] = k == NYS_VAR_BOX ? u[j] - x[j] - w[j] : 0.0;
    }
  }
};
struct PredM {        // R_p = r_p - delta (y - lambda)
  double* Rp;
  const double *rp, *y, *lam;
  double delta;
  __device__ void operator()(int64_t j, double*, double*) const { Rp[j] = rp[j] - delta * (y[j] - lam[j]); }
};
struct Ratio {        // primal: min -x/dx (I, J) and -w/dw (J); dual: min -z/dz (I, J) and -s/ds (J)
  const double *x, *dx, *z, *dz;
  const int8_t* vt;
  const double *w, *dw, *s, *ds;
  __device__ void operator()(int64_t j, double*, double* mn) const {
    const int k = kind_of(vt, j);
    if (k != NYS_VAR_FREE) {
      if (dx[j] < 0.0) mn[0] = fmin(mn[0], -x[j] / dx[j]);
      if (dz[j] < 0.0) mn[1] = fmin(mn[1], -z[j] / dz[j]);
    }
    if (k == NYS_VAR_BOX) {
      if (dw[j] < 0.0) mn[0] = fmin(mn[0], -w[j] / dw[j]);
      if (ds[j] < 0.0) mn[1] = fmin(mn[1], -s[j] / ds[j]);
    }
  }
};
struct MuAff {        // (x + ap dx)^T (z + ad dz) over I, J plus (w + ap dw)^T (s + ad ds) over J
  const double *x, *dx, *z, *dz;
  double ap, ad;
  const int8_t* vt;
  const double *w, *dw, *s, *ds;
  __device__ void operator()(int64_t j, double* a, double*) const {
    const int k = kind_of(vt, j);
    if (k != NYS_VAR_FREE) a[0] = fma(fma(ap, dx[j], x[j]), fma(ad, dz[j], z[j]), a[0]);
    if (k == NYS_VAR_BOX) a[0] = fma(fma(ap, dw[j], w[j]), fma(ad, ds[j], s[j]), a[0]);
  }
};
struct CorrRxz {      // R_xz = mu~ - dxp .* dzp (I, J); R_ws = mu~ - dwp .* dsp (J); with add: +=
  double* R;
  const double *dxp, *dzp;
  double mut;
  const int8_t* vt;
  double* Rws;
  const double *dwp, *dsp;
  bool add;
  __device__ void operator()(int64_t j, double*, double*) const {
    const int k = kind_of(vt, j);
    const double r = k == NYS_VAR_FREE ? 0.0 : mut - dxp[j] * dzp[j];
    R[j] = add ? R[j] + r : r;
    if (Rws) {
      const double rw = k == NYS_VAR_BOX ? mut - dwp[j] * dsp[j] : 0.0;
      Rws[j] = add ? Rws[j] + rw : rw;
    }
  }
};
struct AddTo {        // a += b
  double* a;
  const double* b;
  __device__ void operator()(int64_t j, double*, double*) const { a[j] += b[j]; }
};
struct UpdXZ {        // x, w += ap (dx, dw); z, s += ad (dz, ds); zeta = x; mu numerator, #non-finite
  double *x, *z, *zeta;
  const double *dx, *dz;
  double ap, ad;
  const int8_t* vt;
  double *w, *s;
  const double *dw, *ds;
  __device__ void operator()(int64_t j, double* a, double*) const {
    const int k = kind_of(vt, j);
    const double xn = fma(ap, dx[j], x[j]), zn = fma(ad, dz[j], z[j]);
    x[j] = xn;
    z[j] = zn;
    zeta[j] = xn;
    if (k != NYS_VAR_FREE) a[0] = fma(xn, zn, a[0]);
    bool bad = !isfinite(xn) || !isfinite(zn);
    if (k == NYS_VAR_BOX) {
      const double wn = fma(ap, dw[j], w[j]), sn = fma(ad, ds[j], s[j]);
      w[j] = wn;
      s[j] = sn;
      a[0] = fma(wn, sn, a[0]);
      bad = bad || !isfinite(wn) || !isfinite(sn);
    }
    if (bad) a[1] += 1.0;
  }
};
struct UpdY {         // y += ad dy, lambda = y ; #non-finite
  double *y, *lam;
  const double* dy;
  double ad;
  __device__ void operator()(int64_t j, double* s, double*) const {
    const double yn = fma(ad, dy[j], y[j]);
    y[j] = yn;
    lam[j] = yn;
    if (!isfinite(yn)) s[0] += 1.0;
  }
};
struct CPlusQX {      // t = c + Q x
  double* t;
  const double *c, *q, *x;
  __device__ void operator()(int64_t j, double*, double*) const { t[j] = c[j] + q[j] * x[j]; }
};
struct HalfU {        // t = u/2 on J, 0 elsewhere (centre of the initial primal candidate)
  double* t;
  const int8_t* vt;
  const double* u;
  __device__ void operator()(int64_t j, double*, double*) const {
    t[j] = kind_of(vt, j) == NYS_VAR_BOX ? 0.5 * u[j] : 0.0;
  }
};
struct InitZ {        // from g = c + Q x~ - A^T y~ (in z): z~_J = g/2, s~_J = -g/2, w~_J = u - x~
  double *z, *w, *s;
  const double *x, *u;
  const int8_t* vt;
  __device__ void operator()(int64_t j, double*, double*) const {
    if (kind_of(vt, j) == NYS_VAR_BOX) {
      const double g = z[j];
      z[j] = 0.5 * g;
      s[j] = -0.5 * g;
      w[j] = u[j] - x[j];
    } else {
      w[j] = 0.0;
      s[j] = 0.0;
    }
  }
};
struct MinXZ {        // min of (x~_IJ, w~_J) and of (z~_IJ, s~_J)
  const double *x, *z;
  const int8_t* vt;
  const double *w, *s;
  __device__ void operator()(int64_t j, double*, double* mn) const {
    const int k = kind_of(vt, j);
    if (k != NYS_VAR_FREE) {
      mn[0] = fmin(mn[0], x[j]);
      mn[1] = fmin(mn[1], z[j]);
    }
    if (k == NYS_VAR_BOX) {
      mn[0] = fmin(mn[0], w[j]);
      mn[1] = fmin(mn[1], s[j]);
    }
  }
};
struct InitSums {     // gamma_xz + gamma_ws, sum of dual and of primal shifted entries
  const double *x, *z;
  double dp, dd;
  const int8_t* vt;
  const double *w, *s;
  __device__ void operator()(int64_t j, double* a, double*) const {
    const int k = kind_of(vt, j);
    if (k != NYS_VAR_FREE) {
      const double xa = x[j] + dp, zb = z[j] + dd;
      a[0] = fma(xa, zb, a[0]);
      a[1] += zb;
      a[2] += xa;
    }
    if (k == NYS_VAR_BOX) {
      const double wa = w[j] + dp, sb = s[j] + dd;
      a[0] = fma(wa, sb, a[0]);
      a[1] += sb;
      a[2] += wa;
    }
  }
};
struct InitShift {    // x_IJ, w_J += sp; z_IJ, s_J += sd (entries still <= 0 set to 1); z_F = 0
  double *x, *z, *zeta;
  double sp, sd;
  const int8_t* vt;
  double *w, *s;
  __device__ void operator()(int64_t j, double*, double*) const {
    const int k = kind_of(vt, j);
    if (k != NYS_VAR_FREE) {
      double xn = x[j] + sp, zn = z[j] + sd;
      if (!(xn > 0.0)) xn = 1.0;
      if (!(zn > 0.0)) zn = 1.0;
      x[j] = xn;
      z[j] = zn;
    } else {
      z[j] = 0.0;
    }
    if (k == NYS_VAR_BOX) {
      double wn = w[j] + sp, sn = s[j] + sd;
      if (!(wn > 0.0)) wn = 1.0;
      if (!(sn > 0.0)) sn = 1.0;
      w[j] = wn;
      s[j] = sn;
    }
    zeta[j] = x[j];
  }
};
struct KindStats {    // #free, #box, #bad kind or bound, ||u_J||^2
  const int8_t* vt;
  const double* u;
  __device__ void operator()(int64_t j, double* a, double*) const {
    const int k = vt[j];
    if (k == NYS_VAR_FREE) a[0] += 1.0;
    if (k == NYS_VAR_BOX) {
      a[1] += 1.0;
      if (!(u[j] > 0.0) || !isfinite(u[j])) a[2] += 1.0;
      else a[3] = fma(u[j], u[j], a[3]);
    }
    if (k != NYS_VAR_NONNEG && k != NYS_VAR_FREE && k != NYS_VAR_BOX) a[2] += 1.0;
  }
};
struct AdjD {         // D_adj = 0 where x <= z, else max(q, rho)^{-1}; tn = D g
  double *D, *tn;
  const double *q, *x, *z, *g;
  double rho;
  __device__ void operator()(int64_t j, double*, double*) const {
    // The adjoint of the converged KKT system needs Q_S^{-1} exactly: the
    // iterate's barrier term z/x (zero at the optimum) is left out, and only
    // curvature below rho (zero-curvature columns included) is floored at rho.
    const double d = x[j] > z[j] ? 1.0 / fmax(q[j], rho) : 0.0;
    D[j] = d;
    tn[j] = d * g[j];
  }
};
struct AdjOut {       // grad_c = -u1, grad_q = -u1 x
  double *gc, *gq;
  const double *u1, *x;
  __device__ void operator()(int64_t j, double*, double*) const {
    if (gc) gc[j] = -u1[j];
    if (gq) gq[j] = -u1[j] * x[j];
  }
};

int check_qp(nys_handle h, const nys_qp* qp, const char* who) {
  if (!qp || !qp->A || !qp->b || !qp->c || !qp->q) return set_error(h, NYS_EINVAL, "%s: NULL problem data", who);
  const nys_matrix* A = qp->A;
  if (A->m < 1 || A->n < 1 || A->ld < A->n || !A->data)
    return set_error(h, NYS_EINVAL, "%s: bad A (m=%lld n=%lld)", who, (long long)A->m, (long long)A->n);
  if (A->dtype != NYS_F64 && A->dtype != NYS_F32)
    return set_error(h, NYS_EINVAL, "%s: A must be FP64 or FP32 storage", who);
  if (A->data_t && A->ld_t < A->m)
    return set_error(h, NYS_EINVAL, "%s: ld_t=%lld < m=%lld", who, (long long)A->ld_t, (long long)A->m);
  if (qp->A_lo) {
    const nys_matrix* L = qp->A_lo;
    if (L->m != A->m || L->n != A->n || L->ld < L->n || L->dtype != NYS_BF16 || !L->data)
      return set_error(h, NYS_EINVAL, "%s: A_lo must be a BF16 matrix of A's shape", who);
  }
  return check_units(h, A, who);
}

// BF16 storage for the matrix-core sketch: the caller's copy, or one made here.
int lo_matrix(nys_handle h, const nys_qp* qp, nys_matrix* out) {
  // the unit columns are A's (applied exactly, whatever the storage of A_d)
  auto with_units = [&](nys_matrix* L) {
    L->n_unit = qp->A->n_unit;
    L->unit_row = qp->A->unit_row;
    L->unit_val = qp->A->unit_val;
  };
  if (qp->A_lo) {
    *out = *qp->A_lo;
    with_units(out);
    return NYS_OK;
  }
  const nys_matrix* A = qp->A;
  uint16_t* lo;
  NYS_CHECK(ws(h, WS_ALO, (size_t)A->m * A->n, &lo));
  if (A->dtype == NYS_F32) {
    NYS_CHECK(f32_to_bf16(h, (const float*)A->data, A->m, A->n, A->ld, lo));
  } else {
    for (int64_t i = 0; i < A->m; ++i)
      NYS_CHECK(to_bf16(h, (const double*)A->data + i * A->ld, lo + i * A->n, A->n));
  }
  *out = nys_matrix{A->m, A->n, A->n, NYS_BF16, lo};
  with_units(out);
  return NYS_OK;
}

struct Opts {
  double tol = 1e-6;
  int max_iter = 100;
  int ell = 0;
  uint64_t seed = 0;
  nys_dtype sk = NYS_F64;
  double c_nu = 1.0;
  nys_pcg_opts pcg{};
  int verbose = 0;
  bool transpose = true;
  int precond = NYS_PRECOND_NYSTROM;
  int ell_rule = NYS_ELL_FIXED;
  int ell_min = 0, ell_max = 0;
  double c_ell = 2.0;
  int reuse_age = 0;
  double reuse_growth = 1.5;
  double* trace = nullptr;
  int trace_len = 0;
  bool separate_corrector = false;
  double predictor_rtol = 2e-3;
  double inner_factor = 0.9;
};

// Transposed copies only where the transpose kernel's grid (65535 tiles of 64
// rows) covers A's m rows; beyond that the passes read A as it is.
inline bool copy_allowed(const Opts& o, const nys_matrix* A) {
  return o.transpose && (A->m + 63) / 64 <= 65535;
}

// The matrix the BF16 sketch reads: sketch tiles of A and of A^T in the
// workspace, made from the caller's BF16 copy or, without one, from A itself
// (rounded to BF16 on the way).  Without memory for them, or with transposed
// copies switched off, the BF16 copy (the caller's or one made here) as it is,
// with a transposed copy where allowed.
int sketch_matrix(nys_handle h, const nys_qp* qp, const Opts& o, nys_matrix* out) {
  const nys_matrix* src = qp->A_lo ? qp->A_lo : qp->A;
  const int64_t m = src->m, n = src->n;
  if (o.transpose && m > 0 && n > 0 && n <= 16776960LL) {
    void *t = nullptr, *tt = nullptr;
    int rc = ws_get(h, WS_ALO, (size_t)sketch_tiles_bytes(m, n), &t);
    if (rc == NYS_OK) rc = ws_get(h, WS_ALOT, (size_t)sketch_tiles_bytes(n, m), &tt);
    if (rc == NYS_OK) {
      NYS_CHECK(sketch_tiles(h, src, false, t));
      NYS_CHECK(sketch_tiles(h, src, true, tt));
      *out = *src;
      out->data_t = nullptr;
      out->ld_t = 0;
      out->tiles = t;
      out->tiles_t = tt;
      out->n_unit = qp->A->n_unit;      // the unit columns are A's
      out->unit_row = qp->A->unit_row;
      out->unit_val = qp->A->unit_val;
      return NYS_OK;
    }
    if (rc != NYS_ENOMEM) return rc;
    h->err.clear();
  }
  nys_matrix lo{};
  NYS_CHECK(lo_matrix(h, qp, &lo));
  return with_transpose(h, &lo, copy_allowed(o, &lo), WS_ALOT, out);
}

// Workspace-backed partial Cholesky preconditioner for the comparator runs.
int pchol_storage(nys_handle h, int64_t m, int ell, nys_pchol* P) {
  const size_t nd = (size_t)m * ell + (size_t)ell * ell + m + ((size_t)ell + m + 1) / 2 + 4;
  double* base;
  NYS_CHECK(ws(h, WS_PCHB, nd, &base));
  P->m = m;
  P->ell = ell;
  P->L = base;
  P->Cinv = base + (size_t)m * ell;
  P->diagS = P->Cinv + (size_t)ell * ell;
  P->piv = reinterpret_cast<int32_t*>(P->diagS + m);
  P->pos = P->piv + ell;
  return NYS_OK;
}

Opts read_opts(const nys_ipm_opts* o) {
  Opts r;
  if (!o) return r;
  if (o->tol > 0) r.tol = o->tol;
  if (o->max_iter > 0) r.max_iter = o->max_iter;
  r.ell = o->ell;
  r.seed = o->seed;
  r.sk = o->sketch_dtype;
  if (o->c_nu > 0) r.c_nu = o->c_nu;
  r.pcg = o->pcg;
  r.verbose = o->verbose;
  r.transpose = o->no_transposed_copy == 0;
  r.precond = o->precond;
  r.ell_rule = o->ell_rule;
  r.ell_min = o->ell_min;
  r.ell_max = o->ell_max;
  if (o->c_ell > 0) r.c_ell = o->c_ell;
  r.reuse_age = o->reuse_max_age;
  if (o->reuse_growth > 0) r.reuse_growth = o->reuse_growth;
  r.trace = o->trace;
  r.trace_len = o->trace_len;
  r.separate_corrector = o->separate_corrector != 0;
  if (o->predictor_rtol > 0) r.predictor_rtol = o->predictor_rtol;
  if (o->inner_factor > 0 && o->inner_factor < 1) r.inner_factor = o->inner_factor;
  return r;
}

struct DeffSum {      // sum_i lambda_i / (lambda_i + mu), and lambda[last]
  const double* lam;
  double mu;
  int64_t last;
  __device__ void operator()(int64_t j, double* a, double*) const {
    const double l = fmax(lam[j], 0.0);
    a[0] += l / (l + mu);
    if (j == last) a[1] += lam[j];
  }
};

// d_hat of eq. effective-dim from the Nystrom eigenvalues, and the smallest one
int deff_pair(nys_handle h, const double* lam, int ell, double mu, double* dhat, double* lam_last) {
  double* sc = h->dscal;
  NYS_CHECK((map_reduce<2, 0>(h, ell, DeffSum{lam, mu, (int64_t)ell - 1}, sc + SC_RED0)));
  NYS_CHECK(read_scalars(h, SC_RED0, 2));
  *dhat = h->hscal[SC_RED0];
  if (lam_last) *lam_last = h->hscal[SC_RED0 + 1];
  return NYS_OK;
}


}  // namespace
}  // namespace nys

using namespace nys;

static int ipm_core(nys_handle h, const nys_qp* qp, const nys_ipm_opts* opts_in, double* x, double* y,
                    double* z, double* w_out, double* s_out, nys_ipm_info* info) {
  if (!h) return NYS_EINVAL;
  NYS_CHECK(check_qp(h, qp, "ipm_solve"));
  if (!x || !y || !z) return set_error(h, NYS_EINVAL, "ipm_solve: NULL output");
  Opts o = read_opts(opts_in);
  const nys_matrix* A = qp->A;
  const int64_t m = A->m, n = ncols(A);
  if (o.ell < 1 || o.ell > m) return set_error(h, NYS_EINVAL, "ipm_solve: ell must be in [1, m]");
  if (o.sk != NYS_F64 && o.sk != NYS_BF16) return set_error(h, NYS_EINVAL, "ipm_solve: bad sketch dtype");
  if (o.precond < NYS_PRECOND_NYSTROM || o.precond > NYS_PRECOND_PCHOL)
    return set_error(h, NYS_EINVAL, "ipm_solve: bad preconditioner kind %d", o.precond);
  if (o.sk == NYS_F64 && A->dtype != NYS_F64 && A->dtype != NYS_F32) return set_error(h, NYS_EINVAL, "ipm_solve: bad A");
  if (o.ell_rule < NYS_ELL_FIXED || o.ell_rule > NYS_ELL_THEOREM)
    return set_error(h, NYS_EINVAL, "ipm_solve: bad ell_rule %d", o.ell_rule);
  if (o.ell_rule != NYS_ELL_FIXED && o.precond != NYS_PRECOND_NYSTROM)
    return set_error(h, NYS_EINVAL, "ipm_solve: a sketch-size rule needs the Nystrom preconditioner");
  if (o.reuse_age < 0) return set_error(h, NYS_EINVAL, "ipm_solve: reuse_max_age < 0");
  if (o.trace_len < 0 || (o.trace_len > 0 && !o.trace)) return set_error(h, NYS_EINVAL, "ipm_solve: bad trace buffer");
  if (!o.trace) o.trace_len = 0;
  // sizes the basis may take: ell alone, or [ell_min, ell_max] under a rule
  int ell_cap = o.ell;
  if (o.ell_rule != NYS_ELL_FIXED) {
    if (o.ell_min <= 0) o.ell_min = std::min(8, o.ell);
    if (o.ell_max <= 0) o.ell_max = (int)std::min<int64_t>(m, 4 * (int64_t)o.ell);
    if (o.ell_min > o.ell_max || o.ell_max > m || o.ell > o.ell_max)
      return set_error(h, NYS_EINVAL, "ipm_solve: need 1 <= ell_min <= ell_max <= m and ell <= ell_max");
    ell_cap = o.ell_max;
  }
  if (o.precond == NYS_PRECOND_PCHOL && o.ell > 65535)
    return set_error(h, NYS_EINVAL, "ipm_solve: the partial Cholesky preconditioner takes ell <= 65535");
  NYS_HIP(h, hipSetDevice(h->device));
  const auto t_start = clk::now();
  h->t_sketch = h->t_pcg = h->t_other = 0.0;
  double* sc = h->dscal;

  // ---- data validation: NaN/Inf anywhere, q < 0
  NYS_CHECK(count_nonfinite_matrix(h, A, sc + SC_RED0));
  NYS_CHECK(count_bad(h, qp->b, m, sc + SC_RED0 + 1));
  NYS_CHECK(count_bad(h, qp->c, n, sc + SC_RED0 + 3));
  NYS_CHECK(count_bad(h, qp->q, n, sc + SC_RED0 + 5));
  NYS_CHECK(read_scalars(h, SC_RED0, 7));
  {
    const double* hs = h->hscal + SC_RED0;
    if (hs[0] + hs[1] + hs[3] + hs[5] > 0) return set_error(h, NYS_EINVAL, "ipm_solve: non-finite problem data");
    if (hs[6] > 0) return set_error(h, NYS_EINVAL, "ipm_solve: q has negative entries");
  }
  // ---- variable kinds: counts for mu, ||u_J||, validation
  const int8_t* vt = qp->vtype;
  double cnt = (double)n, unorm = 0.0;
  if (vt) {
    if (!qp->u) return set_error(h, NYS_EINVAL, "ipm_solve: vtype given without u");
    NYS_CHECK((map_reduce<4, 0>(h, n, KindStats{vt, qp->u}, sc + SC_RED0)));
    NYS_CHECK(read_scalars(h, SC_RED0, 4));
    const double* hs = h->hscal + SC_RED0;
    if (hs[2] > 0) return set_error(h, NYS_EINVAL, "ipm_solve: bad variable kind or upper bound (need 0 < u < inf)");
    cnt = (double)n - hs[0] + hs[1];
    unorm = std::sqrt(hs[3]);
  }
  const bool box = vt != nullptr;
  nys_matrix At{};
  NYS_CHECK(with_transpose(h, A, copy_allowed(o, A), WS_AT, &At));
  A = &At;

  // ---- workspace
  double* base;
  NYS_CHECK(ws(h, WS_IPM, (size_t)12 * n + 8 * m + 64 + (box ? (size_t)8 * n : 0), &base));
  double* D = base;
  double* zeta = base + n;
  double* aty = base + 2 * n;
  double* rd = base + 3 * n;
  double* Rd = base + 4 * n;
  double* Rxz = base + 5 * n;
  double* dxp = base + 6 * n;
  double* dzp = base + 7 * n;
  double* dxc = base + 8 * n;
  double* dzc = base + 9 * n;
  double* tn = base + 10 * n;
  double* ones = base + 11 * n;
  double* mb = base + 12 * n;
  double* lam = mb;
  double* rp = mb + m;
  double* Rp = mb + 2 * m;
  double* dyp = mb + 3 * m;
  double* dyc = mb + 4 * m;
  double* rhs = mb + 5 * m;
  double* tm = mb + 6 * m;
  // box arrays: slack w and its dual s (the caller's when given), the r_ws
  // and r_u right-hand sides, and the w, s directions of both solves
  double *w = nullptr, *s = nullptr, *Rws = nullptr, *Ru = nullptr;
  double *dwp = nullptr, *dsp = nullptr, *dwc = nullptr, *dsc = nullptr;
  if (box) {
    double* bb = base + 12 * n + 8 * m + 64;
    w = w_out ? w_out : bb;
    s = s_out ? s_out : bb + n;
    Rws = bb + 2 * n;
    Ru = bb + 3 * n;
    dwp = bb + 4 * n;
    dsp = bb + 5 * n;
    dwc = bb + 6 * n;
    dsc = bb + 7 * n;
  }
  double *U, *lamh;
  NYS_CHECK(ws(h, WS_PCU, (size_t)m * ell_cap, &U));
  NYS_CHECK(ws(h, WS_PCL, (size_t)ell_cap + 8, &lamh));
  const nys_matrix* Ask = A;
  nys_matrix Alsk{};
  if (o.sk == NYS_BF16 && o.precond == NYS_PRECOND_NYSTROM) {
    NYS_CHECK(sketch_matrix(h, qp, o, &Alsk));
    Ask = &Alsk;
  }
  nys_pchol pch{};
  if (o.precond == NYS_PRECOND_PCHOL) NYS_CHECK(pchol_storage(h, m, o.ell, &pch));
  const double* Un = o.precond == NYS_PRECOND_NYSTROM ? U : nullptr;
  const nys_pchol* pchp = o.precond == NYS_PRECOND_PCHOL ? &pch : nullptr;
  int pcg_total = 0;

  // preconditioner construction for the current D and delta (Nystrom sketch,
  // partial Cholesky, or nothing for plain CG)
  auto timed_sketch = [&](const double* d, uint64_t ctr, double dlt, int ell) -> int {
    const auto t0 = clk::now();
    double nu = 0;
    if (o.precond == NYS_PRECOND_NYSTROM)
      NYS_CHECK(ipm_sketch(h, Ask, d, ell, o.seed, ctr, o.sk, o.c_nu, U, lamh, &nu));
    else if (o.precond == NYS_PRECOND_PCHOL)
      NYS_CHECK(pchol_build(h, A, d, dlt, &pch));
    NYS_CHECK(sync(h));
    h->t_sketch += ms_since(t0);
    return NYS_OK;
  };

  // ---- norms of b, c
  NYS_CHECK(dot(h, qp->b, qp->b, m, sc + SC_RED0));
  NYS_CHECK(dot(h, qp->c, qp->c, n, sc + SC_RED0 + 1));
  NYS_CHECK(read_scalars(h, SC_RED0, 2));
  const double bnorm = std::sqrt(h->hscal[SC_RED0]), cnorm = std::sqrt(h->hscal[SC_RED0 + 1]);

  // ---- initial point
  {
    NYS_CHECK(fill(h, ones, n, 1.0));
    NYS_CHECK(timed_sketch(ones, CTR_INIT, INIT_REG, o.ell));
    nys_pcg_opts ip = o.pcg;
    ip.rtol = 1e-10;
    ip.atol = 0.0;
    nys_pcg_info pi{};
    // x~ = u/2 + A^T (A A^T + 10 I)^{-1} (b - A u/2)  (u/2 on J only; 0 without box variables)
    const double* r0 = qp->b;
    if (box) {
      NYS_CHECK(map_reduce<0, 0>(h, n, HalfU{tn, vt, qp->u}, nullptr));
      GemvN gu;
      gu.A = A;
      gu.w = tn;
      gu.sA = -1.0;
      gu.x0 = qp->b;
      gu.out = rhs;
      NYS_CHECK(gemv_n(h, gu));
      r0 = rhs;
    }
    auto t0 = clk::now();
    int rc = ipm_pcg(h, A, ones, INIT_REG, Un, lamh, o.ell, pchp, r0, tm, &ip, &pi);
    h->t_pcg += ms_since(t0);
    if (rc < 0) return rc;
    pcg_total += pi.iters;
    GemvT g1;
    g1.A = A;
    g1.v = tm;
    g1.x0 = box ? tn : nullptr;
    g1.w = x;
    NYS_CHECK(gemv_t(h, g1));                                          // x~
    NYS_CHECK(map_reduce<0, 0>(h, n, CPlusQX{tn, qp->c, qp->q, x}, nullptr));
    GemvN g2;
    g2.A = A;
    g2.w = tn;
    g2.out = rhs;
    NYS_CHECK(gemv_n(h, g2));                                          // A (c + Q x~)
    t0 = clk::now();
    rc = ipm_pcg(h, A, ones, INIT_REG, Un, lamh, o.ell, pchp, rhs, y, &ip, &pi);
    h->t_pcg += ms_since(t0);
    if (rc < 0) return rc;
    pcg_total += pi.iters;
    GemvT g3;
    g3.A = A;
    g3.v = y;
    g3.sA = -1.0;
    g3.x0 = tn;
    g3.w = z;
    NYS_CHECK(gemv_t(h, g3));                                          // z~ = c + Q x~ - A^T y~
    if (box) NYS_CHECK(map_reduce<0, 0>(h, n, InitZ{z, w, s, x, qp->u, vt}, nullptr));
    NYS_CHECK((map_reduce<0, 2>(h, n, MinXZ{x, z, vt, w, s}, sc + SC_RED0)));
    NYS_CHECK(read_scalars(h, SC_RED0, 2));
    const double dp = std::max(-1.5 * h->hscal[SC_RED0], 0.0);
    const double dd = std::max(-1.5 * h->hscal[SC_RED0 + 1], 0.0);
    NYS_CHECK((map_reduce<3, 0>(h, n, InitSums{x, z, dp, dd, vt, w, s}, sc + SC_RED0)));
    NYS_CHECK(read_scalars(h, SC_RED0, 3));
    const double gamma = h->hscal[SC_RED0];
    const double sz = h->hscal[SC_RED0 + 1], sx = h->hscal[SC_RED0 + 2];
    const double sp = dp + (sz != 0 ? 0.5 * gamma / sz : 0.0);
    const double sd = dd + (sx != 0 ? 0.5 * gamma / sx : 0.0);
    NYS_CHECK(map_reduce<0, 0>(h, n, InitShift{x, z, zeta, sp, sd, vt, w, s}, nullptr));
    NYS_CHECK(copy(h, lam, y, m));
  }

  double rho = REG0, delta = REG0;
  nys_ipm_info inf{};
  int status = NYS_MAXIT;
  // preconditioner in use: its size, build iteration, the PCG iterations of
  // that iteration and of the previous one, and its d_hat and smallest
  // eigenvalue at the current mu (Nystrom only)
  const bool nys_pc = o.precond == NYS_PRECOND_NYSTROM;
  int ell_cur = o.ell, k_build = -1, pcg_ref = 0, pcg_prev = 0, builds = 0;
  double dhat = NAN, lam_last = NAN, deff_last = NAN;
  int k = 0;
  for (k = 0;; ++k) {
    // residuals and stopping test
    GemvT ga;
    ga.A = A;
    ga.v = y;
    ga.w = aty;
    NYS_CHECK(gemv_t(h, ga));
    GemvN gp;
    gp.A = A;
    gp.w = x;
    gp.sA = -1.0;
    gp.x0 = qp->b;
    gp.out = rp;
    NYS_CHECK(gemv_n(h, gp));                                          // r_p = b - A x
    NYS_CHECK((map_reduce<4, 0>(h, n, ResidD{rd, qp->c, qp->q, x, aty, z, vt, qp->u, w, s}, sc + SC_RED0)));
    NYS_CHECK(dot(h, rp, rp, m, sc + SC_RED0 + 4));
    NYS_CHECK(read_scalars(h, SC_RED0, 5));
    const double* hs = h->hscal + SC_RED0;
    if (hs[2] > 0) {
      status = set_error(h, NYS_ENUMERIC, "ipm_solve: non-finite iterate at iteration %d", k);
      break;
    }
    const double mu = cnt > 0 ? hs[1] / cnt : 0.0;
    const double rp_rel = std::sqrt(hs[4]) / (1.0 + bnorm);
    const double rd_rel = std::sqrt(hs[0]) / (1.0 + cnorm);
    const double ru_rel = std::sqrt(hs[3]) / (1.0 + unorm);
    const double kkt = std::max(std::max(rp_rel, rd_rel), std::max(ru_rel, mu));
    inf.kkt_rel = kkt;
    inf.rp_rel = rp_rel;
    inf.rd_rel = rd_rel;
    inf.ru_rel = ru_rel;
    inf.mu = mu;
    const double t_test = ms_since(t_start);
    if (o.verbose)
      std::fprintf(stderr, "[nysipm] k=%d rp=%.2e rd=%.2e mu=%.2e rho=%.2e pcg_total=%d t=%.1fms ell=%d\n", k,
                   rp_rel, rd_rel, mu, rho, pcg_total, ms_since(t_start), ell_cur);
    if (kkt <= o.tol) {
      status = NYS_OK;
      break;
    }
    if (k >= o.max_iter) break;

    NYS_CHECK(map_reduce<0, 0>(h, n, Scaling{D, qp->q, x, z, rho, vt, w, s}, nullptr));
    const int built = nys_precond_rebuild_due(k, k_build, pcg_prev, pcg_ref, o.reuse_age, o.reuse_growth);
    double rule_dhat = NAN, rule_lam = NAN;
    if (built) {
      // the size from the most recent Nystrom eigenvalues (the initial point's
      // sketch at k = 0) taken at the current mu
      if (o.ell_rule != NYS_ELL_FIXED) {
        NYS_CHECK(deff_pair(h, lamh, ell_cur, mu, &rule_dhat, &rule_lam));
        ell_cur = nys_sketch_size_rule(o.ell_rule, rule_dhat, rule_lam, mu, k, ell_cur, o.ell_min, o.ell_max,
                                       o.c_ell);
        if (ell_cur < 1) return set_error(h, NYS_EINVAL, "ipm_solve: sketch-size rule failed");
      }
      NYS_CHECK(timed_sketch(D, (uint64_t)k, delta, ell_cur));
      k_build = k;
      if (o.precond != NYS_PRECOND_NONE) ++builds;
    }
    if (nys_pc && (built || o.trace_len > k)) {
      NYS_CHECK(deff_pair(h, lamh, ell_cur, mu, &dhat, &lam_last));
      if (built) deff_last = dhat;
    }
    const int pcg_before = pcg_total;

    // predictor
    NYS_CHECK(map_reduce<0, 0>(h, n, PredN{Rd, Rxz, rd, x, zeta, z, rho, vt, Rws, Ru, qp->u, w, s}, nullptr));
    NYS_CHECK(map_reduce<0, 0>(h, m, PredM{Rp, rp, y, lam, delta}, nullptr));
    // inner tolerance: max(1e-12 ||xi||, min(cap ||xi||, tau)), cap = pcg.rtol or 1e-2,
    // tau = f max(mu, tol (1 + ||b||)), f = inner_factor (0.9): the normal-equation
    // residual enters only the primal block of the Newton system (Proposition 3.1),
    // so no solve is asked for a residual below a fraction f of the
    // primal-feasibility target.
    const double tau = std::max(o.inner_factor * mu, o.inner_factor * o.tol * (1.0 + bnorm));
    nys_pcg_info pi{};
    auto t0 = clk::now();
    const BoxNewton bxp = box ? BoxNewton{vt, w, s, Ru, Rws, dwp, dsp} : BoxNewton{};
    // combined mode: the predictor only sets the step lengths and mu_aff, so a
    // relative residual of predictor_rtol suffices; the direction itself comes
    // from the one solve with the summed right-hand side below
    const bool comb = !o.separate_corrector;
    int rc = ipm_newton(h, A, x, z, D, delta, Un, lamh, ell_cur, pchp, Rd, Rp, Rxz, &o.pcg, tau, dxp, dyp, dzp,
                        &pi, bxp, comb ? o.predictor_rtol : 0.0);
    h->t_pcg += ms_since(t0);
    if (rc < 0) {
      status = rc;
      break;
    }
    pcg_total += pi.iters;
    if (o.verbose)
      std::fprintf(stderr, "[nysipm]   predictor pcg: iters=%d status=%d |res|=%.2e tau=%.2e\n", pi.iters,
                   pi.status, pi.true_res, tau);
    NYS_CHECK((map_reduce<0, 2>(h, n, Ratio{x, dxp, z, dzp, vt, w, dwp, s, dsp}, sc + SC_RED0)));
    NYS_CHECK(read_scalars(h, SC_RED0, 2));
    double ap = STEP * std::min(1.0, h->hscal[SC_RED0]);
    double ad = STEP * std::min(1.0, h->hscal[SC_RED0 + 1]);
    NYS_CHECK((map_reduce<1, 0>(h, n, MuAff{x, dxp, z, dzp, ap, ad, vt, w, dwp, s, dsp}, sc + SC_RED0)));
    NYS_CHECK(read_scalars(h, SC_RED0, 1));
    const double mu_aff = cnt > 0 ? h->hscal[SC_RED0] / cnt : 0.0;
    const double mut = mu > 0 ? mu_aff * mu_aff * mu_aff / (mu * mu) : 0.0;

    // corrector.  Separate (the scheme as printed): solve with r_d = r_p = r_u = 0
    // and R_xz = mu~ - dxp dzp, then add the two directions.  Combined: by
    // linearity the sum is the solution of the system with the summed
    // right-hand side (r_d, r_p, r_u of the predictor, R_xz = -XZ + mu~ -
    // dxp dzp), solved once to the inner tolerance from the predictor's dy.
    NYS_CHECK(map_reduce<0, 0>(h, n, CorrRxz{Rxz, dxp, dzp, mut, vt, Rws, dwp, dsp, comb}, nullptr));
    t0 = clk::now();
    const BoxNewton bxc = box ? BoxNewton{vt, w, s, comb ? Ru : nullptr, Rws, dwc, dsc} : BoxNewton{};
    rc = comb ? ipm_newton(h, A, x, z, D, delta, Un, lamh, ell_cur, pchp, Rd, Rp, Rxz, &o.pcg, tau, dxc, dyc, dzc, &pi,
                           bxc, 0.0, dyp)
              : ipm_newton(h, A, x, z, D, delta, Un, lamh, ell_cur, pchp, nullptr, nullptr, Rxz, &o.pcg, tau, dxc,
                           dyc, dzc, &pi, bxc);
    h->t_pcg += ms_since(t0);
    if (rc < 0) {
      status = rc;
      break;
    }
    pcg_total += pi.iters;
    if (o.verbose)
      std::fprintf(stderr, "[nysipm]   corrector pcg: iters=%d status=%d |res|=%.2e alpha=(%.3f,%.3f) mu_aff=%.2e\n",
                   pi.iters, pi.status, pi.true_res, ap, ad, mu_aff);
    // the direction: the combined solve's, or predictor + corrector
    double *fdx = dxc, *fdy = dyc, *fdz = dzc, *fdw = dwc, *fds = dsc;
    if (!comb) {
      NYS_CHECK(map_reduce<0, 0>(h, n, AddTo{dxp, dxc}, nullptr));
      NYS_CHECK(map_reduce<0, 0>(h, n, AddTo{dzp, dzc}, nullptr));
      NYS_CHECK(map_reduce<0, 0>(h, m, AddTo{dyp, dyc}, nullptr));
      if (box) {
        NYS_CHECK(map_reduce<0, 0>(h, n, AddTo{dwp, dwc}, nullptr));
        NYS_CHECK(map_reduce<0, 0>(h, n, AddTo{dsp, dsc}, nullptr));
      }
      fdx = dxp, fdy = dyp, fdz = dzp, fdw = dwp, fds = dsp;
    }
    NYS_CHECK((map_reduce<0, 2>(h, n, Ratio{x, fdx, z, fdz, vt, w, fdw, s, fds}, sc + SC_RED0)));
    NYS_CHECK(read_scalars(h, SC_RED0, 2));
    ap = STEP * std::min(1.0, h->hscal[SC_RED0]);
    ad = STEP * std::min(1.0, h->hscal[SC_RED0 + 1]);
    NYS_CHECK((map_reduce<2, 0>(h, n, UpdXZ{x, z, zeta, fdx, fdz, ap, ad, vt, w, s, fdw, fds}, sc + SC_RED0)));
    NYS_CHECK((map_reduce<1, 0>(h, m, UpdY{y, lam, fdy, ad}, sc + SC_RED0 + 2)));
    NYS_CHECK(read_scalars(h, SC_RED0, 3));
    if (h->hscal[SC_RED0 + 1] + h->hscal[SC_RED0 + 2] > 0) {
      status = set_error(h, NYS_ENUMERIC, "ipm_solve: non-finite iterate at iteration %d", k);
      break;
    }
    const double mu_new = cnt > 0 ? h->hscal[SC_RED0] / cnt : 0.0;
    const int pcg_k = pcg_total - pcg_before;
    if (k < o.trace_len) {
      double* t = o.trace + (size_t)k * NYS_TRACE_FIELDS;
      t[NYS_TR_K] = k;
      t[NYS_TR_MU] = mu;
      t[NYS_TR_DELTA] = delta;
      t[NYS_TR_ELL] = o.precond == NYS_PRECOND_NONE ? 0 : ell_cur;
      t[NYS_TR_BUILT] = built && o.precond != NYS_PRECOND_NONE ? 1 : 0;
      t[NYS_TR_DHAT] = nys_pc ? dhat : NAN;
      t[NYS_TR_LAMLAST] = nys_pc ? lam_last : NAN;
      t[NYS_TR_PCG] = pcg_k;
      t[NYS_TR_RULE_DHAT] = rule_dhat;
      t[NYS_TR_RULE_LAMLAST] = rule_lam;
      t[NYS_TR_RP] = rp_rel;
      t[NYS_TR_RD] = rd_rel;
      t[NYS_TR_TIME_MS] = t_test;
    }
    if (k == k_build) pcg_ref = pcg_k;
    pcg_prev = pcg_k;
    rho = delta = std::max(REG_FLOOR, std::min(rho, mu_new));
  }
  NYS_CHECK(sync(h));
  const double total = ms_since(t_start);
  h->t_other = std::max(0.0, total - h->t_sketch - h->t_pcg);
  inf.iters = k;
  inf.pcg_iters_total = pcg_total;
  inf.status = status;
  inf.rho = rho;
  inf.delta = delta;
  inf.t_sketch_ms = h->t_sketch;
  inf.t_pcg_ms = h->t_pcg;
  inf.t_other_ms = h->t_other;
  inf.deff_last = deff_last;
  inf.builds = builds;
  inf.ell_last = o.precond == NYS_PRECOND_NONE ? 0 : ell_cur;
  if (info) *info = inf;
  if (status == NYS_MAXIT)
    set_error(h, NYS_MAXIT, "ipm_solve: %d iterations without reaching tol (KKT %.3e)", k, inf.kkt_rel);
  return status;
}

extern "C" int ipm_solve(nys_handle h, const nys_qp* qp, const nys_ipm_opts* opts, double* x, double* y,
                         double* z, nys_ipm_info* info) {
  return ipm_core(h, qp, opts, x, y, z, nullptr, nullptr, info);
}

extern "C" int ipm_solve_box(nys_handle h, const nys_qp* qp, const nys_ipm_opts* opts, double* x, double* y,
                             double* z, double* w, double* s, nys_ipm_info* info) {
  if (h && qp && !qp->vtype) return set_error(h, NYS_EINVAL, "ipm_solve_box: vtype is NULL (use ipm_solve)");
  return ipm_core(h, qp, opts, x, y, z, w, s, info);
}

extern "C" int ipm_adjoint(nys_handle h, const nys_qp* qp, const nys_ipm_opts* opts_in, const double* x,
                           const double* y, const double* z, double rho, double delta, const double* g,
                           double* grad_c, double* grad_b, double* grad_q, double* grad_A,
                           nys_pcg_info* info) {
  if (!h) return NYS_EINVAL;
  NYS_CHECK(check_qp(h, qp, "ipm_adjoint"));
  if (!x || !y || !z || !g) return set_error(h, NYS_EINVAL, "ipm_adjoint: NULL input");
  if (qp->vtype) return set_error(h, NYS_EINVAL, "ipm_adjoint: free or box-constrained variables are not supported");
  if (qp->A->n_unit != 0) return set_error(h, NYS_EINVAL, "ipm_adjoint: unit columns are not supported");
  if (!(delta > 0) || !std::isfinite(delta) || !(rho >= 0) || !std::isfinite(rho))
    return set_error(h, NYS_EINVAL, "ipm_adjoint: need delta > 0 and rho >= 0");
  Opts o = read_opts(opts_in);
  const nys_matrix* A = qp->A;
  const int64_t m = A->m, n = A->n;
  if (o.ell < 1 || o.ell > m) return set_error(h, NYS_EINVAL, "ipm_adjoint: ell must be in [1, m]");
  if (o.precond < NYS_PRECOND_NYSTROM || o.precond > NYS_PRECOND_PCHOL)
    return set_error(h, NYS_EINVAL, "ipm_adjoint: bad preconditioner kind %d", o.precond);
  if (o.precond == NYS_PRECOND_NYSTROM) {
    if (o.sk != NYS_F64 && o.sk != NYS_BF16) return set_error(h, NYS_EINVAL, "ipm_adjoint: bad sketch dtype");
  }
  if (o.precond == NYS_PRECOND_PCHOL && o.ell > 65535)
    return set_error(h, NYS_EINVAL, "ipm_adjoint: the partial Cholesky preconditioner takes ell <= 65535");
  NYS_HIP(h, hipSetDevice(h->device));
  const auto t_start = clk::now();
  h->t_sketch = h->t_pcg = h->t_other = 0.0;
  nys_matrix At{};
  NYS_CHECK(with_transpose(h, A, copy_allowed(o, A), WS_AT, &At));
  A = &At;
  double* base;
  NYS_CHECK(ws(h, WS_IPM, (size_t)12 * n + 8 * m + 64, &base));
  double* D = base;
  double* tn = base + n;
  double* u1 = base + 2 * n;
  double* rhs = base + 12 * n;
  double* u2 = rhs + m;
  double *U, *lamh;
  NYS_CHECK(ws(h, WS_PCU, (size_t)m * o.ell, &U));
  NYS_CHECK(ws(h, WS_PCL, (size_t)o.ell + 8, &lamh));
  const nys_matrix* Ask = A;
  nys_matrix Alsk{};
  if (o.sk == NYS_BF16 && o.precond == NYS_PRECOND_NYSTROM) {
    NYS_CHECK(sketch_matrix(h, qp, o, &Alsk));
    Ask = &Alsk;
  }
  nys_pchol pch{};
  if (o.precond == NYS_PRECOND_PCHOL) NYS_CHECK(pchol_storage(h, m, o.ell, &pch));
  const double* Un = o.precond == NYS_PRECOND_NYSTROM ? U : nullptr;
  const nys_pchol* pchp = o.precond == NYS_PRECOND_PCHOL ? &pch : nullptr;
  NYS_CHECK(map_reduce<0, 0>(h, n, AdjD{D, tn, qp->q, x, z, g, rho}, nullptr));
  GemvN g2;
  g2.A = A;
  g2.w = tn;
  g2.out = rhs;
  NYS_CHECK(gemv_n(h, g2));                                            // A D g
  auto t0 = clk::now();
  double nu = 0;
  if (o.precond == NYS_PRECOND_NYSTROM)
    NYS_CHECK(ipm_sketch(h, Ask, D, o.ell, o.seed, CTR_ADJ, o.sk, o.c_nu, U, lamh, &nu));
  else if (o.precond == NYS_PRECOND_PCHOL)
    NYS_CHECK(pchol_build(h, A, D, delta, &pch));
  NYS_CHECK(sync(h));
  h->t_sketch += ms_since(t0);
  nys_pcg_opts po = o.pcg;
  if (!(po.rtol > 0)) po.rtol = 1e-10;
  if (po.maxit <= 0) po.maxit = (int)std::max<int64_t>(m, 20000);
  t0 = clk::now();
  int rc = ipm_pcg(h, A, D, delta, Un, lamh, o.ell, pchp, rhs, u2, &po, info);
  h->t_pcg += ms_since(t0);
  if (rc < 0) return rc;
  GemvT g1;
  g1.A = A;
  g1.v = u2;
  g1.sA = -1.0;
  g1.x0 = g;
  g1.d = D;
  g1.w = u1;
  NYS_CHECK(gemv_t(h, g1));                                            // u1 = D (g - A^T u2)
  if (grad_c || grad_q) NYS_CHECK(map_reduce<0, 0>(h, n, AdjOut{grad_c, grad_q, u1, x}, nullptr));
  if (grad_b) NYS_CHECK(copy(h, grad_b, u2, m));
  if (grad_A) NYS_CHECK(grad_A_rank2(h, m, n, y, u1, u2, x, grad_A));
  NYS_CHECK(sync(h));
  h->t_other = std::max(0.0, ms_since(t_start) - h->t_sketch - h->t_pcg);
  return rc;
}

extern "C" int nys_deff_estimate(nys_handle h, const double* lambda, int32_t ell, double mu, double* out_host) {
  if (!h) return NYS_EINVAL;
  if (!lambda || !out_host || ell < 1 || !(mu > 0) || !std::isfinite(mu))
    return set_error(h, NYS_EINVAL, "nys_deff_estimate: need lambda, out_host, ell >= 1 and finite mu > 0");
  NYS_HIP(h, hipSetDevice(h->device));
  return deff_pair(h, lambda, ell, mu, out_host, nullptr);
}

extern "C" int nys_sketch_size_rule(int32_t rule, double d_hat, double lam_last, double mu, int32_t k,
                                    int32_t ell_prev, int32_t ell_min, int32_t ell_max, double c_ell) {
  if (ell_min < 1 || ell_min > ell_max) return NYS_EINVAL;
  double target;
  switch (rule) {
    case NYS_ELL_FIXED:
      return ell_prev;
    case NYS_ELL_DEFF:
      if (!(c_ell > 0)) return NYS_EINVAL;
      target = std::ceil(c_ell * d_hat);
      if (lam_last > mu) target = std::max(target, 2.0 * (double)ell_prev);
      break;
    case NYS_ELL_THEOREM: {
      const double r = std::sqrt(d_hat) + std::sqrt(32.0 * std::log(16.0 * (double)(k + 2)));
      target = std::ceil(8.0 * r * r);
      break;
    }
    default:
      return NYS_EINVAL;
  }
  if (!std::isfinite(target)) return ell_max;
  return (int32_t)std::min((double)ell_max, std::max((double)ell_min, target));
}

extern "C" int nys_precond_rebuild_due(int32_t k, int32_t k_build, int32_t pcg_prev, int32_t pcg_ref,
                                       int32_t max_age, double growth) {
  if (k_build < 0 || max_age <= 0) return 1;
  if (k - k_build >= max_age) return 1;
  return (double)pcg_prev > growth * (double)pcg_ref ? 1 : 0;
}
