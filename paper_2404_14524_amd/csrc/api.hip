// C ABI of libnysipm: handle and workspace, argument validation, and the host
// drivers of the Nystrom sketch (Algorithms 1-2), PCG, the Newton step
// (Algorithm 5), Nys-IP-PMM (Algorithms 4 and 6) and the KKT adjoint.
// Every arithmetic step runs in the kernels of this library; the host only
// sequences launches and takes the scalar decisions of the algorithms.

#include <algorithm>
#include <chrono>
#include <cmath>
#include <vector>
#include <cstring>
#include <mutex>

#include "common.hpp"
#include "kernels.hpp"
#include "mapreduce.hpp"

namespace nys {

int set_error(nys_handle h, int code, const char* fmt, ...) {
  if (!h) return code;
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  h->err = buf;
  return code;
}

int ws_get(nys_handle h, int slot, size_t bytes, void** out) {
  if (bytes == 0) bytes = 8;
  if (h->arena) {
    // allocation-free call: the slot's piece of the fixed scratch, never a new buffer
    if (bytes > h->arena->len[slot])
      return set_error(h, NYS_EINVAL, "allocation-free call: workspace slot %d needs %zu bytes, planned %zu", slot,
                       bytes, h->arena->len[slot]);
    *out = h->arena->base + h->arena->off[slot];
    return NYS_OK;
  }
  if (h->slot_bytes[slot] < bytes) {
    if (h->slot_ptr[slot]) {
      // a kernel still queued may use the old buffer
      NYS_HIP(h, hipStreamSynchronize(h->stream));
      NYS_HIP(h, hipFree(h->slot_ptr[slot]));
      h->slot_ptr[slot] = nullptr;
      h->slot_bytes[slot] = 0;
    }
    const size_t rounded = (bytes + (1u << 20) - 1) & ~(size_t)((1u << 20) - 1);
    void* p = nullptr;
    if (hipMalloc(&p, rounded) != hipSuccess || !p) {
      (void)hipGetLastError();
      return set_error(h, NYS_ENOMEM, "workspace allocation of %zu bytes failed", rounded);
    }
    h->slot_ptr[slot] = p;
    h->slot_bytes[slot] = rounded;
  }
  *out = h->slot_ptr[slot];
  return NYS_OK;
}

int read_scalars(nys_handle h, int first, int count) {
  NYS_HIP(h, hipMemcpyAsync(h->hscal + first, h->dscal + first, sizeof(double) * count,
                            hipMemcpyDeviceToHost, h->stream));
  NYS_HIP(h, hipStreamSynchronize(h->stream));
  return NYS_OK;
}

int sync(nys_handle h) {
  NYS_HIP(h, hipStreamSynchronize(h->stream));
  return NYS_OK;
}

int prof_drain(nys_handle h) {
  nys_prof& p = h->prof;
  if (p.used == 0) return NYS_OK;
  NYS_HIP(h, hipEventSynchronize(p.stop[p.used - 1]));
  for (int i = 0; i < p.used; ++i) {
    float ms = 0.f;
    NYS_HIP(h, hipEventElapsedTime(&ms, p.start[i], p.stop[i]));
    p.total_ms[p.cls[i]] += ms;
    p.count[p.cls[i]] += 1;
  }
  p.used = 0;
  return NYS_OK;
}

int prof_begin(nys_handle h, int kclass) {
  nys_prof& p = h->prof;
  if (!p.on) return -1;
  if (p.used == (int)p.start.size() && prof_drain(h) < 0) return -1;
  const int s = p.used++;
  p.cls[s] = kclass;
  if (hipEventRecord(p.start[s], h->stream) != hipSuccess) return -1;
  return s;
}

void prof_end(nys_handle h, int slot) {
  if (slot >= 0) (void)hipEventRecord(h->prof.stop[slot], h->stream);
}

namespace {

// ---------------------------------------------------------------- small kernels
__global__ void k_set_scalars(double* s, int n, int i0, double v0, int i1, double v1, int i2,
                              double v2, int i3, double v3) {
  if (threadIdx.x != 0) return;
  if (n > 0) s[i0] = v0;
  if (n > 1) s[i1] = v1;
  if (n > 2) s[i2] = v2;
  if (n > 3) s[i3] = v3;
}

int set_scalars(nys_handle h, int n, int i0, double v0, int i1 = 0, double v1 = 0, int i2 = 0,
                double v2 = 0, int i3 = 0, double v3 = 0) {
  hipLaunchKernelGGL(k_set_scalars, dim3(1), dim3(64), 0, h->stream, h->dscal, n, i0, v0, i1, v1,
                     i2, v2, i3, v3);
  NYS_LAUNCH_CHECK(h);
  return NYS_OK;
}

// lambda_hat = max(0, sig2 - nu)
struct LamF {
  const double* sig2;
  double* lam;
  double nu;
  __device__ void operator()(int64_t j, double*, double*) const { lam[j] = fmax(0.0, sig2[j] - nu); }
};
// out[j] = G[j][j] (the diagonal of an ell x ell row-major matrix, gathered
// for one contiguous copy to the host)
struct DiagF {
  const double* G;
  double* out;
  int64_t ell;
  __device__ void operator()(int64_t j, double*, double*) const { out[j] = G[j * (ell + 1)]; }
};
// Y_nu = Y + nu Omega
struct ShiftF {
  double* out;
  const double* Y;
  const double* O;
  double nu;
  __device__ void operator()(int64_t j, double*, double*) const { out[j] = fma(nu, O[j], Y[j]); }
};
// r = rhs - Mv (FP64) and ||r||^2
struct ResF {
  double* r;
  const double* rhs;
  const double* mv;
  __device__ void operator()(int64_t j, double* s, double*) const {
    const double v = rhs[j] - mv[j];
    r[j] = v;
    s[0] = fma(v, v, s[0]);
  }
};

// rank-2 update grad_A = y u1^T - u2 x^T (m x n, ld n)
__global__ __launch_bounds__(NYS_BLOCK) void k_grad_A(int64_t m, int64_t n, const double* y,
                                                      const double* u1, const double* u2,
                                                      const double* x, double* G) {
  const int64_t total = m * n;
  for (int64_t idx = (int64_t)blockIdx.x * NYS_BLOCK + threadIdx.x; idx < total;
       idx += (int64_t)gridDim.x * NYS_BLOCK) {
    const int64_t i = idx / n, j = idx % n;
    G[idx] = y[i] * u1[j] - u2[i] * x[j];
  }
}

// ---------------------------------------------------------------- validation
bool is_fin(double v) { return std::isfinite(v); }

int check_matrix(nys_handle h, const nys_matrix* A, const char* who) {
  if (!A) return set_error(h, NYS_EINVAL, "%s: matrix is NULL", who);
  if (A->m < 0 || A->n < 0 || A->ld < A->n || A->ld < 1)
    return set_error(h, NYS_EINVAL, "%s: bad shape m=%lld n=%lld ld=%lld", who, (long long)A->m,
                     (long long)A->n, (long long)A->ld);
  if (A->dtype != NYS_F64 && A->dtype != NYS_F32 && A->dtype != NYS_BF16)
    return set_error(h, NYS_EINVAL, "%s: bad dtype %d", who, (int)A->dtype);
  if (A->m > 0 && A->n > 0 && !A->data) return set_error(h, NYS_EINVAL, "%s: data is NULL", who);
  if (A->data_t && A->ld_t < std::max<int64_t>(A->m, 1))
    return set_error(h, NYS_EINVAL, "%s: ld_t=%lld < m=%lld", who, (long long)A->ld_t, (long long)A->m);
  if ((A->tiles == nullptr) != (A->tiles_t == nullptr))
    return set_error(h, NYS_EINVAL, "%s: give both sketch tiles (of A and of A^T) or neither", who);
  return check_units(h, A, who);
}

int check_precond(nys_handle h, const nys_precond* P, int64_t m, const char* who) {
  if (!P) return NYS_OK;
  if (P->m != m || P->ell < 1 || P->ell > m || !P->U || !P->lambda)
    return set_error(h, NYS_EINVAL, "%s: bad preconditioner (m=%lld ell=%d)", who, (long long)P->m,
                     P->ell);
  return NYS_OK;
}

struct PcgCfg {
  double rtol = 1e-10, atol = 0.0;
  int maxit = 0, replace_every = 100, poll_every = 8;
  // mu rule of the interior-point inner solves (mu_abs >= 0):
  // tol = max(floor_rel ||rhs||, min(rtol ||rhs||, mu_abs)), then at least loose_rel ||rhs||
  double mu_abs = -1.0, floor_rel = 1e-12, loose_rel = 0.0;
};

PcgCfg pcg_cfg(const nys_pcg_opts* o, int64_t m) {
  PcgCfg c;
  if (o) {
    c.rtol = o->rtol;
    c.atol = o->atol;
    c.maxit = o->maxit;
    c.replace_every = o->replace_every;
    c.poll_every = o->poll_every;
  }
  // default cap: the dimension (CG's exact-arithmetic bound), at least 2000;
  // late interior-point systems need thousands of iterations, and a capped,
  // unconverged direction costs more outer iterations than it saves
  if (c.maxit <= 0) c.maxit = (int)std::min<int64_t>(std::max<int64_t>(m, 2000), 1 << 30);
  if (c.replace_every <= 0) c.replace_every = 100;
  if (c.poll_every <= 0) c.poll_every = 8;
  if (!(c.rtol >= 0)) c.rtol = 0;
  if (!(c.atol >= 0)) c.atol = 0;
  return c;
}

// ---------------------------------------------------------------- PCG driver
// Nystrom data (U, lam, ell) or a partial Cholesky preconditioner (pc); none: plain CG.
struct Precond {
  const double* U = nullptr;
  const double* lam = nullptr;
  int ell = 0;
  const nys_pchol* pc = nullptr;
};

// Solves (A diag(d) A^T + delta I) y = rhs.  y_zero: y is taken as 0 (and set).
int pcg_run(nys_handle h, const nys_matrix* A, const double* d, double delta, const Precond& P,
            const double* rhs, double* y, bool y_zero, const PcgCfg& cfg, nys_pcg_info* info) {
  const int64_t m = A->m;
  const bool pre = P.U != nullptr;
  const bool pch = P.pc != nullptr;
  double* base;
  NYS_CHECK(ws(h, WS_PCG, (size_t)6 * m + P.ell + 8, &base));
  double* r = base;
  double* s = base + m;
  double* pa = base + 2 * m;
  double* pb = base + 3 * m;
  double* q = base + 4 * m;
  double* tmp = base + 5 * m;
  double* t = base + 6 * m;
  double* sc = h->dscal;
  nys_pcg_info out{0, NYS_OK, 0.0, 0.0};

  NYS_CHECK(dot(h, rhs, rhs, m, sc + SC_RED0));
  NYS_CHECK(read_scalars(h, SC_RED0, 1));
  const double bnorm = std::sqrt(h->hscal[SC_RED0]);
  const double tol = std::max(cfg.loose_rel * bnorm,
                              cfg.mu_abs >= 0 ? std::max(cfg.floor_rel * bnorm, std::min(cfg.rtol * bnorm, cfg.mu_abs))
                                              : std::max(cfg.rtol * bnorm, cfg.atol));

  // true residual r = rhs - M y into `dst`, ||.||^2 -> sc[SC_RED0 + 1]
  auto true_residual = [&](double* dst) -> int {
    NYS_CHECK(normal_apply(h, A, d, delta, y, q, nullptr));
    return map_reduce<1, 0>(h, m, ResF{dst, rhs, q}, sc + SC_RED0 + 1);
  };
  // s = P^{-1} r and rs = r^T s (or rs = ||r||^2 without a preconditioner)
  auto refresh_s = [&]() -> int {
    if (pre) {
      NYS_CHECK(precond_reduce(h, P.U, P.lam, m, P.ell, delta, r, t));
      return precond_expand(h, P.U, m, P.ell, r, t, s, sc + SC_RS);
    }
    if (pch) return pchol_apply(h, P.pc, r, s, true, nullptr);
    return dot(h, r, r, m, sc + SC_RS);
  };

  if (y_zero) NYS_CHECK(fill(h, y, m, 0.0));
  if (bnorm == 0.0 && y_zero) {
    if (info) *info = out;
    return NYS_OK;
  }
  double r0norm = bnorm;
  if (y_zero) {
    NYS_CHECK(copy(h, r, rhs, m));
  } else {
    NYS_CHECK(true_residual(r));
    NYS_CHECK(read_scalars(h, SC_RED0 + 1, 1));
    r0norm = std::sqrt(h->hscal[SC_RED0 + 1]);
  }
  if (r0norm <= tol) {
    // the starting point already meets the tolerance (a zero right-hand side
    // with a zero guess included): no iteration, and none could proceed, since
    // r = 0 gives p = 0 and p^T M p = 0
    out.true_res = r0norm;
    out.rel_res = bnorm > 0 ? r0norm / bnorm : r0norm;
    if (info) *info = out;
    return NYS_OK;
  }
  NYS_CHECK(set_scalars(h, 4, SC_DONE, 0.0, SC_BREAK, 0.0, SC_ITERS, 0.0, SC_BETA, 0.0));
  NYS_CHECK(set_scalars(h, 1, SC_TOL2, tol * tol));
  NYS_CHECK(fill(h, pa, m, 0.0));
  NYS_CHECK(refresh_s());
  // refresh_s leaves beta = (r^T s) / (the previous solve's r^T s); the first
  // direction is p = s, and beta * 0 would be NaN if that old value were 0
  NYS_CHECK(set_scalars(h, 1, SC_BETA, 0.0));
  const double* sdir = (pre || pch) ? s : r;

  int status = NYS_MAXIT;
  bool final_res_known = false;
  double final_res = 0.0;
  int it = 0;
  while (it < cfg.maxit) {
    double* pold = (it % 2 == 0) ? pa : pb;
    double* pnew = (it % 2 == 0) ? pb : pa;
    GemvT g1;
    g1.A = A;
    g1.skip = sc + SC_DONE;
    g1.s = sdir;
    g1.pold = pold;
    g1.pnew = pnew;
    g1.beta = sc + SC_BETA;
    g1.d = d;
    double* w;
    NYS_CHECK(ws(h, WS_W, (size_t)std::max<int64_t>(ncols(A), 1), &w));
    g1.w = w;
    NYS_CHECK(gemv_t(h, g1));
    GemvN g2;
    g2.A = A;
    g2.skip = sc + SC_DONE;
    g2.w = w;
    g2.v = pnew;
    g2.sV = delta;
    g2.out = q;
    g2.dot_out = sc + SC_PQ;
    NYS_CHECK(gemv_n(h, g2));
    NYS_CHECK(pcg_update(h, m, y, r, pnew, q, P.U, P.lam, P.ell, delta, t, pch));
    if (pre) NYS_CHECK(pcg_expand(h, m, P.U, P.ell, r, t, s));
    if (pch) NYS_CHECK(pchol_apply(h, P.pc, r, s, true, nullptr));
    ++it;
    const bool poll = (it % cfg.poll_every == 0) || it == cfg.maxit;
    if (poll) {
      NYS_CHECK(read_scalars(h, 0, SC_RED0));
      if (h->hscal[SC_BREAK] != 0.0) {
        status = NYS_EBREAKDOWN;
        break;
      }
      if (h->hscal[SC_DONE] != 0.0) {
        NYS_CHECK(true_residual(tmp));
        NYS_CHECK(read_scalars(h, SC_RED0 + 1, 1));
        const double tr = std::sqrt(h->hscal[SC_RED0 + 1]);
        if (tr <= tol) {
          status = NYS_OK;
          final_res_known = true;
          final_res = tr;
          break;
        }
        // the recursion drifted: restart from the true residual
        NYS_CHECK(copy(h, r, tmp, m));
        NYS_CHECK(refresh_s());
        NYS_CHECK(set_scalars(h, 2, SC_DONE, 0.0, SC_BETA, 0.0));
        continue;
      }
    }
    if (it % cfg.replace_every == 0 && it < cfg.maxit) {
      NYS_CHECK(true_residual(r));
      NYS_CHECK(refresh_s());
    }
  }
  NYS_CHECK(read_scalars(h, 0, SC_RED0));
  out.iters = (int)h->hscal[SC_ITERS];
  if (h->prof.on && it > out.iters) {
    // launches after convergence returned at once: not reads of A
    NYS_CHECK(prof_drain(h));
    h->prof.count[NYS_K_NORMAL_PASS1] -= it - out.iters;
    h->prof.count[NYS_K_NORMAL_PASS2] -= it - out.iters;
  }
  if (!final_res_known) {
    NYS_CHECK(true_residual(tmp));
    NYS_CHECK(read_scalars(h, SC_RED0 + 1, 1));
    final_res = std::sqrt(h->hscal[SC_RED0 + 1]);
    if (status == NYS_MAXIT && final_res <= tol) status = NYS_OK;
  }
  out.status = status;
  out.true_res = final_res;
  out.rel_res = bnorm > 0 ? final_res / bnorm : final_res;
  if (info) *info = out;
  if (status == NYS_EBREAKDOWN)
    return set_error(h, NYS_EBREAKDOWN, "PCG breakdown after %d iterations (p^T M p <= 0)", out.iters);
  return status;
}

// ---------------------------------------------------------------- Nystrom sketch
struct SketchOut {
  double* U;
  double* lam;
  double nu;
};

int sketch_run(nys_handle h, const nys_matrix* A, const double* d, int ell, uint64_t seed,
               uint64_t counter, nys_dtype mode, double c_nu, const double* omega,
               SketchOut* outp) {
  const int64_t m = A->m;
  double *Om, *Y, *B, *Q1, *small;
  NYS_CHECK(ws(h, WS_OMEGA, (size_t)m * ell, &Om));
  NYS_CHECK(ws(h, WS_Y, (size_t)m * ell, &Y));
  NYS_CHECK(ws(h, WS_B, (size_t)m * ell, &B));
  NYS_CHECK(ws(h, WS_Q1, (size_t)m * ell, &Q1));
  const int64_t l2 = (int64_t)ell * ell;
  NYS_CHECK(ws(h, WS_SMALL, (size_t)8 * l2 + 2 * ell + 16, &small));
  double* G = small;
  double* Cinv = small + l2;
  double* R1 = small + 2 * l2;
  double* R2 = small + 3 * l2;
  double* T = small + 4 * l2;
  double* jw = small + 5 * l2;          // Jacobi work: l2 + ell + 2 words
  double* sig2 = small + 7 * l2;
  double* fail = h->dscal + SC_FAIL;

  // test matrix and its thin QR by Cholesky-QR: two passes for a caller's
  // Omega or a nearly square one; one for the library's Gaussian with
  // m >= 4 ell, whose condition number is then below 3 (about
  // (1 + sqrt(ell/m)) / (1 - sqrt(ell/m))), so that one pass leaves
  // Q^T Q - I at a few units of rounding
  if (omega) NYS_CHECK(copy(h, Om, omega, m * ell));
  else NYS_CHECK(philox_gaussian(h, m, ell, seed, counter, Om));
  const bool one_pass = !omega && m >= 4 * (int64_t)ell;
  // One Cholesky-QR pass on X (m x ell): R = chol(X^T X + shift) in G (and
  // Rout), R^{-1} in Cinv; with Xout, Xout = X R^{-1}.
  auto cholqr_pass = [&](double* X, double* Xout, double shift_rel, double* Rout) -> int {
    NYS_CHECK(gemm_f64(h, true, false, ell, ell, m, X, NYS_F64, ell, X, ell, G, ell, nullptr));
    NYS_CHECK(chol_upper(h, G, ell, 0.0, shift_rel, fail));
    NYS_CHECK(read_scalars(h, SC_FAIL, 1));
    if (h->hscal[SC_FAIL] != 0.0) return set_error(h, NYS_ENOTPD, "Cholesky-QR: Gram matrix not positive definite");
    NYS_CHECK(tri_inv_upper(h, G, Cinv, ell, jw));
    if (Xout) NYS_CHECK(gemm_f64(h, false, false, m, ell, ell, X, NYS_F64, ell, Cinv, ell, Xout, ell, nullptr, true));
    if (Rout) NYS_CHECK(copy(h, Rout, G, l2));
    return NYS_OK;
  };
  NYS_CHECK(cholqr_pass(Om, Q1, 0.0, nullptr));
  if (one_pass) NYS_CHECK(copy(h, Om, Q1, m * ell));
  else NYS_CHECK(cholqr_pass(Q1, Om, 0.0, nullptr));

  // Y = N Omega
  NYS_CHECK(sketch_product(h, A, d, Om, ell, mode, Y));
  NYS_CHECK(sumsq(h, Y, m * ell, h->dscal + SC_RED0));
  NYS_CHECK(read_scalars(h, SC_RED0, 1));
  const double ynorm = std::sqrt(h->hscal[SC_RED0]);
  if (!std::isfinite(ynorm)) return set_error(h, NYS_ENUMERIC, "sketch: non-finite Y");
  const int pbits = (mode == NYS_BF16) ? 8 : 53;
  double nu = ynorm > 0 ? c_nu * std::ldexp(1.0, std::ilogb(ynorm) - (pbits - 1)) : c_nu * 1e-300;

  // C = chol(Omega^T Y_nu) with retries; B = Y_nu C^{-1}
  bool ok = false;
  for (int attempt = 0; attempt <= 6; ++attempt) {
    NYS_CHECK(map_reduce<0, 0>(h, m * ell, ShiftF{B, Y, Om, nu}, nullptr));
    NYS_CHECK(gemm_f64(h, true, false, ell, ell, m, Om, NYS_F64, ell, B, ell, G, ell, nullptr));
    NYS_CHECK(chol_upper(h, G, ell, 0.0, 0.0, fail));
    NYS_CHECK(read_scalars(h, SC_FAIL, 1));
    if (h->hscal[SC_FAIL] == 0.0) {
      ok = true;
      break;
    }
    nu *= 10.0;
  }
  if (!ok) return set_error(h, NYS_ENOTPD, "sketch: chol(Omega^T Y_nu) failed after 6 shift increases (nu=%g)", nu);
  NYS_CHECK(tri_inv_upper(h, G, Cinv, ell, jw));
  NYS_CHECK(gemm_f64(h, false, false, m, ell, ell, B, NYS_F64, ell, Cinv, ell, Q1, ell, nullptr, true));
  // thin QR of B (now in Q1).  B B^T is the Nystrom approximation of N + nu I,
  // so the singular values of B lie in [sqrt(nu), sqrt(lambda_max + nu)]:
  // with the BF16 shift B is well conditioned, with the FP64 one it need not be.
  // First an unshifted Cholesky-QR pass; if it succeeds and the spread of the
  // factor's diagonal (a lower bound on cond(B)) is at most 1 / sqrt(10 s),
  // s = 11 (m ell + ell(ell+1)) u, one more plain pass leaves Q^T Q - I at
  // rounding level (Cholesky-QR2).  Otherwise shifted Cholesky-QR3 from B:
  // R1 = chol(B^T B + s ||B||_F^2 I), then two plain passes.
  const double u = 1.1102230246251565e-16;
  const double srel = 11.0 * ((double)m * ell + (double)ell * (ell + 1)) * u;
  // The last pass forms no Q: with Q = P R_last^{-1} (P the previous pass's
  // output, R_last^{-1} in Cinv), U_hat = Q U_R = P (R_last^{-1} U_R), one
  // ell x ell x ell product in place of an m x ell x ell one.
  double* P = B;
  double* Rf = R2;
  bool two_pass = false;
  NYS_CHECK(gemm_f64(h, true, false, ell, ell, m, Q1, NYS_F64, ell, Q1, ell, G, ell, nullptr));
  NYS_CHECK(chol_upper(h, G, ell, 0.0, 0.0, fail));
  NYS_CHECK(read_scalars(h, SC_FAIL, 1));
  if (h->hscal[SC_FAIL] == 0.0) {
    // the diagonal goes through the Jacobi work area and one contiguous copy
    // (a strided 2D copy to the host read zeros under a kernel tracer)
    std::vector<double> dg((size_t)ell);
    NYS_CHECK(map_reduce<0, 0>(h, ell, DiagF{G, jw, ell}, nullptr));
    NYS_HIP(h, hipMemcpyAsync(dg.data(), jw, (size_t)ell * sizeof(double), hipMemcpyDeviceToHost, h->stream));
    NYS_HIP(h, hipStreamSynchronize(h->stream));
    double dmin = INFINITY, dmax = 0.0;
    for (double v : dg) {
      dmin = std::min(dmin, std::fabs(v));
      dmax = std::max(dmax, std::fabs(v));
    }
    two_pass = dmin > 0.0 && std::isfinite(dmax) && dmax <= dmin / std::sqrt(10.0 * srel);
  }
  if (two_pass) {
    NYS_CHECK(tri_inv_upper(h, G, Cinv, ell, jw));
    NYS_CHECK(gemm_f64(h, false, false, m, ell, ell, Q1, NYS_F64, ell, Cinv, ell, B, ell, nullptr, true));
    NYS_CHECK(copy(h, R1, G, l2));
    NYS_CHECK(cholqr_pass(B, nullptr, 0.0, R2));
    NYS_CHECK(small_mm(h, R2, R1, T, ell));         // R = R2 R1 in T, Q = B R2^{-1}
    P = B;
    Rf = T;
  } else {
    NYS_CHECK(cholqr_pass(Q1, B, srel, R1));
    NYS_CHECK(cholqr_pass(B, Q1, 0.0, R2));
    NYS_CHECK(small_mm(h, R2, R1, T, ell));         // T = R2 R1
    NYS_CHECK(cholqr_pass(Q1, nullptr, 0.0, R1));   // R3 in R1, Q = Q1 R3^{-1}
    NYS_CHECK(small_mm(h, R1, T, R2, ell));         // R = R3 R2 R1 in R2
    P = Q1;
  }
  // SVD of the triangular factor: left singular vectors U_R, Sigma^2
  NYS_CHECK(jacobi_svd(h, Rf, ell, sig2, jw));
  // U_hat = Q U_R = P (R_last^{-1} U_R) ; Lambda_hat = max(0, Sigma^2 - nu)
  NYS_CHECK(gemm_f64(h, false, false, ell, ell, ell, Cinv, NYS_F64, ell, Rf, ell, R1, ell, nullptr));
  NYS_CHECK(gemm_f64(h, false, false, m, ell, ell, P, NYS_F64, ell, R1, ell, outp->U, ell, nullptr));
  NYS_CHECK(map_reduce<0, 0>(h, ell, LamF{sig2, outp->lam, nu}, nullptr));
  outp->nu = nu;
  return NYS_OK;
}

// ---------------------------------------------------------------- Newton step (Alg. 5)
struct NewtonPre {
  // tn = D (r_d + xi_au), x0n = -(r_d + xi_au), with xi_au by index kind:
  // free 0; non-negative -r_xz/x; box -r_xz/x + r_ws/w - (s/w) r_u
  double* tn;
  double* x0n;
  const double* D;
  const double* rd;   // may be NULL (zero)
  const double* rxz;
  const double* x;
  BoxNewton bx;
  __device__ void operator()(int64_t j, double*, double*) const {
    const int k = bx.vt ? bx.vt[j] : NYS_VAR_NONNEG;
    double xa = 0.0;
    if (k != NYS_VAR_FREE) xa = -rxz[j] / x[j];
    if (k == NYS_VAR_BOX) {
      const double ru = bx.ru ? bx.ru[j] : 0.0;
      xa += (bx.rws[j] - bx.s[j] * ru) / bx.w[j];
    }
    const double a = (rd ? rd[j] : 0.0) + xa;
    tn[j] = D[j] * a;
    x0n[j] = -a;
  }
};
struct NewtonDz {     // eq. delta-z/-w/-s-free-box (X^{-1}, W^{-1} on both terms)
  double* dz;
  const double* rxz;
  const double* z;
  const double* dx;
  const double* x;
  BoxNewton bx;
  __device__ void operator()(int64_t j, double*, double*) const {
    const int k = bx.vt ? bx.vt[j] : NYS_VAR_NONNEG;
    dz[j] = k == NYS_VAR_FREE ? 0.0 : (rxz[j] - z[j] * dx[j]) / x[j];
    if (bx.dw) {
      double dw = 0.0, ds = 0.0;
      if (k == NYS_VAR_BOX) {
        dw = (bx.ru ? bx.ru[j] : 0.0) - dx[j];
        ds = (bx.rws[j] - bx.s[j] * dw) / bx.w[j];
      }
      bx.dw[j] = dw;
      bx.ds[j] = ds;
    }
  }
};
struct ScalingF {
  double* D;
  const double* q;
  const double* x;
  const double* z;
  double rho;
  __device__ void operator()(int64_t j, double*, double*) const { D[j] = 1.0 / (q[j] + z[j] / x[j] + rho); }
};

int newton_run(nys_handle h, const nys_matrix* A, const double* x, const double* z, const double* D,
               double delta, const Precond& P, const double* rd, const double* rp, const double* rxz,
               const PcgCfg& cfg, double* dx, double* dy, double* dz, nys_pcg_info* info,
               const BoxNewton& bx = BoxNewton{}, const double* dy_guess = nullptr) {
  const int64_t m = A->m, n = ncols(A);
  double* base;
  NYS_CHECK(ws(h, WS_NEWTON, (size_t)2 * n + m + 8, &base));
  double* tn = base;
  double* x0n = base + n;
  double* xi = base + 2 * n;
  NYS_CHECK(map_reduce<0, 0>(h, n, NewtonPre{tn, x0n, D, rd, rxz, x, bx}, nullptr));
  GemvN g2;
  g2.A = A;
  g2.w = tn;
  g2.x0 = rp;
  g2.out = xi;
  if (!rp) {
    // xi = A tn
    g2.x0 = nullptr;
  }
  NYS_CHECK(gemv_n(h, g2));
  // a warm start (the predictor's dy for the combined corrector solve)
  if (dy_guess) NYS_CHECK(copy(h, dy, dy_guess, m));
  int rc = pcg_run(h, A, D, delta, P, xi, dy, dy_guess == nullptr, cfg, info);
  if (rc < 0) return rc;
  GemvT g1;
  g1.A = A;
  g1.v = dy;
  g1.x0 = x0n;
  g1.d = D;
  g1.w = dx;
  NYS_CHECK(gemv_t(h, g1));
  NYS_CHECK(map_reduce<0, 0>(h, n, NewtonDz{dz, rxz, z, dx, x, bx}, nullptr));
  return rc;
}

}  // namespace
}  // namespace nys

// ---------------------------------------------------------------- fixed scratch
// Device scratch of the allocation-free PCG entry point
// (nys_pcg_solve_noalloc): every GPU the library runs on holds one copy of
// this array until the process ends.  On the host, `scratch` names only a
// stand-in for the device symbol, never device memory: host code uses the
// address that nys_create looks up per device (nys_scratch_attach) wherever
// the array's memory is meant.
#define NYS_SCRATCH_BYTES NYS_NOALLOC_SCRATCH_BYTES
static __device__ __align__(256) char scratch[NYS_SCRATCH_BYTES];

namespace nys {
namespace {

constexpr int kMaxScratchDevices = 64;
std::mutex g_scratch_mu;
char* g_scratch_dev[kMaxScratchDevices] = {};   // per-device address of `scratch`

// With `device` current: look up that device's copy of the scratch array (once per device).
int nys_scratch_attach(nys_handle h, int device) {
  if (device < 0 || device >= kMaxScratchDevices) return NYS_OK;   // the allocation-free call refuses it
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (g_scratch_dev[device]) return NYS_OK;
  void* p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !p) {
    (void)hipGetLastError();
    return set_error(h, NYS_EHIP, "hipGetSymbolAddress(scratch) failed on device %d: %s", device,
                     hipGetErrorString(e));
  }
  g_scratch_dev[device] = (char*)p;
  return NYS_OK;
}

char* scratch_of(int device) {
  if (device < 0 || device >= kMaxScratchDevices) return nullptr;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  return g_scratch_dev[device];
}

// The workspace one pcg_run call requests, slot by slot, carved out of the
// scratch at 256-byte aligned offsets; *total = bytes used.  Slots pcg_run
// does not request get no piece (a request for one is refused by ws_get).
void pcg_scratch_plan(const nys_matrix* A, int ell, nys_arena* ar, size_t* total) {
  const int64_t m = A->m, n = ncols(A);
  size_t need[WS_NSLOTS] = {};
  need[WS_PCG] = ((size_t)6 * m + ell + 8) * sizeof(double);
  need[WS_W] = (size_t)std::max<int64_t>(n, 1) * sizeof(double);
  need[WS_PART] = std::max(gemv_t_part_doubles(A), update_part_doubles(m, ell, ell > 0)) * sizeof(double);
  size_t p2 = std::max(gemv_n_part_doubles(m), expand_part_doubles(m));
  p2 = std::max<size_t>(p2, map_reduce_blocks(m));                  // dot products, true residuals
  p2 = std::max<size_t>(p2, map_reduce_blocks(A->n_unit));          // the unit-column check
  need[WS_PART2] = p2 * sizeof(double);
  if (A->n_unit > 0) need[WS_UNIT] = (size_t)std::max<int64_t>(m, 1) * sizeof(double);
  size_t off = 0;
  for (int s = 0; s < WS_NSLOTS; ++s) {
    ar->off[s] = off;
    ar->len[s] = 0;
    if (!need[s]) continue;
    ar->len[s] = (need[s] + 255) / 256 * 256;
    off += ar->len[s];
  }
  *total = off;
}

}  // namespace
}  // namespace nys

using namespace nys;

// ================================================================== C ABI

extern "C" int nys_create(nys_handle* out, int device, void* stream) {
  if (!out) return NYS_EINVAL;
  *out = nullptr;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) return NYS_EINVAL;
  auto* h = new (std::nothrow) nys_handle_s();
  if (!h) return NYS_ENOMEM;
  h->device = device;
  h->stream = (hipStream_t)stream;
  if (hipSetDevice(device) != hipSuccess) {
    delete h;
    return NYS_EHIP;
  }
  if (hipMalloc(&h->dscal, SC_NSCAL * sizeof(double)) != hipSuccess ||
      hipMemset(h->dscal, 0, SC_NSCAL * sizeof(double)) != hipSuccess ||
      hipHostMalloc(&h->hscal, SC_NSCAL * sizeof(double), hipHostMallocDefault) != hipSuccess ||
      hipDeviceSynchronize() != hipSuccess) {
    (void)hipGetLastError();
    nys_destroy(h);
    return NYS_EHIP;
  }
  if (nys_scratch_attach(h, device) < 0) {
    nys_destroy(h);
    return NYS_EHIP;
  }
  *out = h;
  return NYS_OK;
}

extern "C" int nys_profile_enable(nys_handle h, int enable) {
  if (!h) return NYS_EINVAL;
  NYS_HIP(h, hipSetDevice(h->device));
  nys_prof& p = h->prof;
  if (enable && p.start.empty()) {
    const int cap = 2048;
    p.start.resize(cap);
    p.stop.resize(cap);
    p.cls.resize(cap);
    for (int i = 0; i < cap; ++i) {
      NYS_HIP(h, hipEventCreate(&p.start[i]));
      NYS_HIP(h, hipEventCreate(&p.stop[i]));
    }
  }
  NYS_CHECK(prof_drain(h));
  for (int k = 0; k < NYS_K_NCLASSES; ++k) {
    p.total_ms[k] = 0.0;
    p.count[k] = 0;
  }
  p.on = enable != 0;
  return NYS_OK;
}

extern "C" int nys_profile_read(nys_handle h, int kclass, int64_t* launches, double* total_ms) {
  if (!h || kclass < 0 || kclass >= NYS_K_NCLASSES) return NYS_EINVAL;
  NYS_HIP(h, hipSetDevice(h->device));
  NYS_CHECK(prof_drain(h));
  if (launches) *launches = h->prof.count[kclass];
  if (total_ms) *total_ms = h->prof.total_ms[kclass];
  return NYS_OK;
}

extern "C" int nys_stream_read(nys_handle h, const void* data, int64_t bytes, double* ms) {
  if (!h) return NYS_EINVAL;
  if (!data || bytes <= 0 || bytes % 16 != 0 || (uintptr_t)data % 16 != 0 || !ms)
    return set_error(h, NYS_EINVAL, "nys_stream_read: need 16-byte aligned data and a size multiple of 16");
  NYS_HIP(h, hipSetDevice(h->device));
  int nbmax = 0;
  for (int sh = 0; sh < stream_read_shapes(); ++sh) nbmax = std::max(nbmax, stream_read_blocks(bytes, sh));
  unsigned* part;
  NYS_CHECK(ws_get(h, WS_PART2, (size_t)nbmax * 4 * sizeof(unsigned), (void**)&part));
  hipEvent_t e0, e1;
  NYS_HIP(h, hipEventCreate(&e0));
  NYS_HIP(h, hipEventCreate(&e1));
  // the fastest of the shapes
  float best = INFINITY;
  int rc = NYS_OK;
  for (int sh = 0; sh < stream_read_shapes() && rc == NYS_OK; ++sh) {
    NYS_HIP(h, hipEventRecord(e0, h->stream));
    rc = stream_read(h, data, bytes, part, sh);
    NYS_HIP(h, hipEventRecord(e1, h->stream));
    NYS_HIP(h, hipEventSynchronize(e1));
    float t = 0.f;
    NYS_HIP(h, hipEventElapsedTime(&t, e0, e1));
    best = std::min(best, t);
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  *ms = best;
  return rc;
}

extern "C" int nys_destroy(nys_handle h) {
  if (!h) return NYS_OK;
  (void)hipSetDevice(h->device);
  (void)hipStreamSynchronize(h->stream);
  for (size_t i = 0; i < h->prof.start.size(); ++i) {
    (void)hipEventDestroy(h->prof.start[i]);
    (void)hipEventDestroy(h->prof.stop[i]);
  }
  for (int s = 0; s < WS_NSLOTS; ++s)
    if (h->slot_ptr[s]) (void)hipFree(h->slot_ptr[s]);
  if (h->dscal) (void)hipFree(h->dscal);
  if (h->hscal) (void)hipHostFree(h->hscal);
  delete h;
  return NYS_OK;
}

extern "C" int nys_set_stream(nys_handle h, void* stream) {
  if (!h) return NYS_EINVAL;
  (void)hipStreamSynchronize(h->stream);
  h->stream = (hipStream_t)stream;
  return NYS_OK;
}

extern "C" const char* nys_last_error(nys_handle h) { return h ? h->err.c_str() : "null handle"; }

extern "C" int nys_last_timing(nys_handle h, double* ts, double* tp, double* to) {
  if (!h) return NYS_EINVAL;
  if (ts) *ts = h->t_sketch;
  if (tp) *tp = h->t_pcg;
  if (to) *to = h->t_other;
  return NYS_OK;
}

extern "C" int nys_normal_apply(nys_handle h, const nys_matrix* A, const double* d, double delta,
                                const double* v, double* out) {
  if (!h) return NYS_EINVAL;
  NYS_CHECK(check_matrix(h, A, "nys_normal_apply"));
  if (!is_fin(delta)) return set_error(h, NYS_EINVAL, "nys_normal_apply: non-finite delta");
  if (A->m > 0 && (!v || !out)) return set_error(h, NYS_EINVAL, "nys_normal_apply: NULL vector");
  if (ncols(A) > 0 && A->m > 0 && !d) return set_error(h, NYS_EINVAL, "nys_normal_apply: NULL d");
  if (v == out && A->m > 0) return set_error(h, NYS_EINVAL, "nys_normal_apply: out aliases v");
  NYS_HIP(h, hipSetDevice(h->device));
  if (A->m == 0) return NYS_OK;
  return normal_apply(h, A, d, delta, v, out, nullptr);
}

extern "C" int nys_transpose(nys_handle h, const nys_matrix* A, void* out, int64_t ld_out) {
  if (!h) return NYS_EINVAL;
  NYS_CHECK(check_matrix(h, A, "nys_transpose"));
  if (A->m > 0 && A->n > 0 && (!out || ld_out < A->m))
    return set_error(h, NYS_EINVAL, "nys_transpose: need out != NULL and ld_out >= m");
  if (out == A->data && A->m * A->n > 0) return set_error(h, NYS_EINVAL, "nys_transpose: out aliases A");
  NYS_HIP(h, hipSetDevice(h->device));
  return transpose(h, A, out, ld_out);
}

extern "C" int nys_test_matrix(nys_handle h, int64_t m, int32_t ell, uint64_t seed, uint64_t counter,
                               double* out) {
  if (!h) return NYS_EINVAL;
  if (m < 0 || ell < 0 || (m * ell > 0 && !out)) return set_error(h, NYS_EINVAL, "nys_test_matrix: bad arguments");
  NYS_HIP(h, hipSetDevice(h->device));
  if (m * ell == 0) return NYS_OK;
  return philox_gaussian(h, m, ell, seed, counter, out);
}

extern "C" int nys_sketch_product(nys_handle h, const nys_matrix* A, const double* d,
                                  const double* omega, int32_t ell, nys_dtype sketch_dtype, double* Y) {
  if (!h) return NYS_EINVAL;
  NYS_CHECK(check_matrix(h, A, "nys_sketch_product"));
  if (ell < 1 || !d || !omega || !Y) return set_error(h, NYS_EINVAL, "nys_sketch_product: bad arguments");
  if (sketch_dtype == NYS_BF16 && A->dtype != NYS_BF16 && !A->tiles)
    return set_error(h, NYS_EINVAL, "nys_sketch_product: a BF16 sketch needs BF16 storage of A or its sketch tiles");
  if (sketch_dtype == NYS_F64 && A->dtype == NYS_BF16)
    return set_error(h, NYS_EINVAL, "nys_sketch_product: an FP64 sketch needs FP64 or FP32 storage");
  if (sketch_dtype != NYS_BF16 && sketch_dtype != NYS_F64)
    return set_error(h, NYS_EINVAL, "nys_sketch_product: sketch dtype must be NYS_F64 or NYS_BF16");
  NYS_HIP(h, hipSetDevice(h->device));
  if (A->m == 0) return NYS_OK;
  return sketch_product(h, A, d, omega, ell, sketch_dtype, Y);
}

extern "C" int nys_sketch_tiles_bytes(int64_t m, int64_t n, int transposed, int64_t* bytes) {
  if (m < 0 || n < 0 || !bytes || (transposed != 0 && transposed != 1)) return NYS_EINVAL;
  *bytes = transposed ? sketch_tiles_bytes(n, m) : sketch_tiles_bytes(m, n);
  return NYS_OK;
}

extern "C" int nys_sketch_tiles(nys_handle h, const nys_matrix* A, int transposed, void* out) {
  if (!h) return NYS_EINVAL;
  NYS_CHECK(check_matrix(h, A, "nys_sketch_tiles"));
  if (transposed != 0 && transposed != 1) return set_error(h, NYS_EINVAL, "nys_sketch_tiles: transposed must be 0 or 1");
  if (A->m > 0 && A->n > 0 && (!out || (uintptr_t)out % 16 != 0))
    return set_error(h, NYS_EINVAL, "nys_sketch_tiles: need a 16-byte aligned output buffer");
  if (A->n > 16776960LL) return set_error(h, NYS_EINVAL, "nys_sketch_tiles: n=%lld above 16776960", (long long)A->n);
  NYS_HIP(h, hipSetDevice(h->device));
  return sketch_tiles(h, A, transposed != 0, out);
}

extern "C" int nys_sketch(nys_handle h, const nys_matrix* A, const double* d, int32_t ell,
                          uint64_t seed, uint64_t counter, nys_dtype sketch_dtype,
                          const double* omega, nys_precond* P, double* nu_out) {
  if (!h) return NYS_EINVAL;
  NYS_CHECK(check_matrix(h, A, "nys_sketch"));
  if (!P || !P->U || !P->lambda) return set_error(h, NYS_EINVAL, "nys_sketch: NULL output");
  if (P->m != A->m || ell != P->ell || ell < 1 || ell > A->m)
    return set_error(h, NYS_EINVAL, "nys_sketch: need 1 <= ell <= m and P sized m x ell");
  if (!d) return set_error(h, NYS_EINVAL, "nys_sketch: NULL d");
  if (sketch_dtype == NYS_BF16 && A->dtype != NYS_BF16 && !A->tiles)
    return set_error(h, NYS_EINVAL, "nys_sketch: a BF16 sketch needs BF16 storage of A or its sketch tiles");
  if (sketch_dtype != NYS_BF16 && sketch_dtype != NYS_F64)
    return set_error(h, NYS_EINVAL, "nys_sketch: sketch dtype must be NYS_F64 or NYS_BF16");
  NYS_HIP(h, hipSetDevice(h->device));
  SketchOut so{P->U, P->lambda, 0.0};
  int rc = sketch_run(h, A, d, ell, seed, counter, sketch_dtype, 1.0, omega, &so);
  if (rc < 0) return rc;
  NYS_CHECK(sync(h));
  if (nu_out) *nu_out = so.nu;
  return NYS_OK;
}

extern "C" int nys_precond_apply(nys_handle h, const nys_precond* P, double delta, const double* r,
                                 double* out) {
  if (!h) return NYS_EINVAL;
  if (!P || !r || !out) return set_error(h, NYS_EINVAL, "nys_precond_apply: NULL argument");
  NYS_CHECK(check_precond(h, P, P->m, "nys_precond_apply"));
  if (!(delta > 0) || !is_fin(delta)) return set_error(h, NYS_EINVAL, "nys_precond_apply: delta must be > 0");
  if (r == out) return set_error(h, NYS_EINVAL, "nys_precond_apply: out aliases r");
  NYS_HIP(h, hipSetDevice(h->device));
  double* base;
  NYS_CHECK(ws(h, WS_PCG, (size_t)6 * P->m + P->ell + 8, &base));
  double* t = base + 6 * P->m;
  NYS_CHECK(precond_reduce(h, P->U, P->lambda, P->m, P->ell, delta, r, t));
  return precond_expand(h, P->U, P->m, P->ell, r, t, out, nullptr);
}

extern "C" int nys_pcg_solve(nys_handle h, const nys_matrix* A, const double* d, double delta,
                             const nys_precond* P, const double* rhs, double* y,
                             const nys_pcg_opts* opts, nys_pcg_info* info) {
  if (!h) return NYS_EINVAL;
  NYS_CHECK(check_matrix(h, A, "nys_pcg_solve"));
  NYS_CHECK(check_precond(h, P, A->m, "nys_pcg_solve"));
  if (!(delta >= 0) || !is_fin(delta)) return set_error(h, NYS_EINVAL, "nys_pcg_solve: delta must be finite and >= 0");
  if (P && !(delta > 0)) return set_error(h, NYS_EINVAL, "nys_pcg_solve: the Nystrom preconditioner needs delta > 0");
  if (A->m > 0 && (!rhs || !y || !d)) return set_error(h, NYS_EINVAL, "nys_pcg_solve: NULL vector");
  NYS_HIP(h, hipSetDevice(h->device));
  if (A->m == 0) {
    if (info) *info = nys_pcg_info{0, NYS_OK, 0.0, 0.0};
    return NYS_OK;
  }
  Precond pc;
  if (P) pc = Precond{P->U, P->lambda, P->ell};
  return pcg_run(h, A, d, delta, pc, rhs, y, false, pcg_cfg(opts, A->m), info);
}

extern "C" int nys_pcg_solve_noalloc(nys_handle h, const nys_matrix* A, const double* d, double delta,
                                     const nys_precond* P, const double* rhs, double* y,
                                     const nys_pcg_opts* opts, nys_pcg_info* info) {
  static const char* who = "nys_pcg_solve_noalloc";
  if (!h) return NYS_EINVAL;
  if (!A) return set_error(h, NYS_EINVAL, "%s: matrix is NULL", who);
  if (A->m < 0 || A->n < 0 || A->n_unit < 0)
    return set_error(h, NYS_EINVAL, "%s: bad shape m=%lld n=%lld n_unit=%lld", who, (long long)A->m,
                     (long long)A->n, (long long)A->n_unit);
  NYS_CHECK(check_precond(h, P, A->m, who));
  if (!(delta >= 0) || !is_fin(delta)) return set_error(h, NYS_EINVAL, "%s: delta must be finite and >= 0", who);
  if (P && !(delta > 0)) return set_error(h, NYS_EINVAL, "%s: the Nystrom preconditioner needs delta > 0", who);
  if (A->m > 0 && (!rhs || !y || !d)) return set_error(h, NYS_EINVAL, "%s: NULL vector", who);
  nys_arena ar;
  size_t total = 0;
  pcg_scratch_plan(A, P ? P->ell : 0, &ar, &total);
  if (total > NYS_SCRATCH_BYTES)
    return set_error(h, NYS_EINVAL, "%s: m=%lld, %lld columns, ell=%d need %zu bytes of scratch, above its fixed %zu",
                     who, (long long)A->m, (long long)ncols(A), P ? P->ell : 0, total, NYS_SCRATCH_BYTES);
  ar.base = scratch_of(h->device);
  if (!ar.base) return set_error(h, NYS_EHIP, "%s: no scratch array for device %d", who, h->device);
  NYS_HIP(h, hipSetDevice(h->device));
  // from here every workspace request is a piece of the scratch (ws_get), so
  // the unit-column check in check_matrix allocates nothing either
  h->arena = &ar;
  int rc = check_matrix(h, A, who);
  if (rc >= 0) {
    if (A->m == 0) {
      if (info) *info = nys_pcg_info{0, NYS_OK, 0.0, 0.0};
      rc = NYS_OK;
    } else {
      Precond pc;
      if (P) pc = Precond{P->U, P->lambda, P->ell};
      rc = pcg_run(h, A, d, delta, pc, rhs, y, false, pcg_cfg(opts, A->m), info);
    }
  }
  h->arena = nullptr;
  return rc;
}

int check_pchol(nys_handle h, const nys_pchol* P, int64_t m, const char* who) {
  if (!P || P->m != m || P->ell < 1 || P->ell > m || !P->piv || !P->pos || !P->L || !P->Cinv || !P->diagS)
    return set_error(h, NYS_EINVAL, "%s: bad partial Cholesky preconditioner", who);
  return NYS_OK;
}

extern "C" int nys_pchol_build(nys_handle h, const nys_matrix* A, const double* d, double delta, nys_pchol* P) {
  if (!h) return NYS_EINVAL;
  NYS_CHECK(check_matrix(h, A, "nys_pchol_build"));
  if (A->m < 1) return set_error(h, NYS_EINVAL, "nys_pchol_build: m must be >= 1");
  NYS_CHECK(check_pchol(h, P, A->m, "nys_pchol_build"));
  if (!(delta > 0) || !is_fin(delta)) return set_error(h, NYS_EINVAL, "nys_pchol_build: delta must be finite and > 0");
  if (ncols(A) > 0 && !d) return set_error(h, NYS_EINVAL, "nys_pchol_build: NULL d");
  NYS_HIP(h, hipSetDevice(h->device));
  return pchol_build(h, A, d, delta, P);
}

extern "C" int nys_pchol_apply(nys_handle h, const nys_pchol* P, const double* r, double* out) {
  if (!h) return NYS_EINVAL;
  NYS_CHECK(check_pchol(h, P, P ? P->m : 0, "nys_pchol_apply"));
  if (!r || !out || r == out) return set_error(h, NYS_EINVAL, "nys_pchol_apply: bad vectors");
  NYS_HIP(h, hipSetDevice(h->device));
  return pchol_apply(h, P, r, out, false, nullptr);
}

extern "C" int nys_pcg_solve_pchol(nys_handle h, const nys_matrix* A, const double* d, double delta,
                                   const nys_pchol* P, const double* rhs, double* y,
                                   const nys_pcg_opts* opts, nys_pcg_info* info) {
  if (!h) return NYS_EINVAL;
  NYS_CHECK(check_matrix(h, A, "nys_pcg_solve_pchol"));
  if (A->m < 1) return set_error(h, NYS_EINVAL, "nys_pcg_solve_pchol: m must be >= 1");
  NYS_CHECK(check_pchol(h, P, A->m, "nys_pcg_solve_pchol"));
  if (!(delta > 0) || !is_fin(delta)) return set_error(h, NYS_EINVAL, "nys_pcg_solve_pchol: delta must be finite and > 0");
  if (!rhs || !y || (ncols(A) > 0 && !d)) return set_error(h, NYS_EINVAL, "nys_pcg_solve_pchol: NULL vector");
  NYS_HIP(h, hipSetDevice(h->device));
  Precond pc;
  pc.pc = P;
  return pcg_run(h, A, d, delta, pc, rhs, y, false, pcg_cfg(opts, A->m), info);
}

extern "C" int nys_newton_solve(nys_handle h, const nys_matrix* A, const double* q, const double* x,
                                const double* z, double rho, double delta, const nys_precond* P,
                                const double* r_d, const double* r_p, const double* r_xz,
                                const nys_pcg_opts* opts, double* dx, double* dy, double* dz,
                                nys_pcg_info* info) {
  if (!h) return NYS_EINVAL;
  NYS_CHECK(check_matrix(h, A, "nys_newton_solve"));
  NYS_CHECK(check_precond(h, P, A->m, "nys_newton_solve"));
  if (!(delta > 0) || !is_fin(delta) || !(rho >= 0) || !is_fin(rho))
    return set_error(h, NYS_EINVAL, "nys_newton_solve: need delta > 0, rho >= 0");
  if (!q || !x || !z || !r_d || !r_p || !r_xz || !dx || !dy || !dz)
    return set_error(h, NYS_EINVAL, "nys_newton_solve: NULL vector");
  NYS_HIP(h, hipSetDevice(h->device));
  double* D;
  NYS_CHECK(ws(h, WS_IPM, (size_t)ncols(A) + 8, &D));
  NYS_CHECK(map_reduce<0, 0>(h, ncols(A), ScalingF{D, q, x, z, rho}, nullptr));
  Precond pc;
  if (P) pc = Precond{P->U, P->lambda, P->ell};
  int rc = newton_run(h, A, x, z, D, delta, pc, r_d, r_p, r_xz, pcg_cfg(opts, A->m), dx, dy, dz, info);
  if (rc < 0) return rc;
  NYS_CHECK(sync(h));
  return rc;
}

// ipm_solve and ipm_adjoint live in ipm.hip; they reuse the drivers above
// through these internal entry points.
namespace nys {
int ipm_pcg(nys_handle h, const nys_matrix* A, const double* d, double delta, const double* U,
            const double* lam, int ell, const nys_pchol* pch, const double* rhs, double* y,
            const nys_pcg_opts* o, nys_pcg_info* info) {
  Precond pc{U, lam, U ? ell : 0, pch};
  return pcg_run(h, A, d, delta, pc, rhs, y, true, pcg_cfg(o, A->m), info);
}
int ipm_sketch(nys_handle h, const nys_matrix* A, const double* d, int ell, uint64_t seed,
               uint64_t counter, nys_dtype mode, double c_nu, double* U, double* lam, double* nu) {
  SketchOut so{U, lam, 0.0};
  NYS_CHECK(sketch_run(h, A, d, ell, seed, counter, mode, c_nu, nullptr, &so));
  if (nu) *nu = so.nu;
  return NYS_OK;
}
int ipm_newton(nys_handle h, const nys_matrix* A, const double* x, const double* z, const double* D,
               double delta, const double* U, const double* lam, int ell, const nys_pchol* pch,
               const double* rd, const double* rp, const double* rxz, const nys_pcg_opts* o,
               double mu_abs, double* dx, double* dy, double* dz, nys_pcg_info* info,
               const BoxNewton& bx, double loose_rel, const double* dy_guess) {
  Precond pc{U, lam, U ? ell : 0, pch};
  PcgCfg cfg = pcg_cfg(o, A->m);
  cfg.rtol = (o && o->rtol > 0) ? o->rtol : 1e-2;
  cfg.atol = 0.0;
  cfg.mu_abs = mu_abs;
  cfg.loose_rel = loose_rel;
  return newton_run(h, A, x, z, D, delta, pc, rd, rp, rxz, cfg, dx, dy, dz, info, bx, dy_guess);
}
int grad_A_rank2(nys_handle h, int64_t m, int64_t n, const double* y, const double* u1,
                 const double* u2, const double* x, double* G) {
  int64_t nb = std::min<int64_t>(std::max<int64_t>((m * n + NYS_BLOCK - 1) / NYS_BLOCK, 1), 16384);
  hipLaunchKernelGGL(k_grad_A, dim3((unsigned)nb), dim3(NYS_BLOCK), 0, h->stream, m, n, y, u1, u2, x, G);
  NYS_LAUNCH_CHECK(h);
  return NYS_OK;
}
}  // namespace nys
