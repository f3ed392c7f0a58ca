// Partial Cholesky preconditioner of N + delta I (section "Partial Cholesky
// preconditioners", eq. partialCholeskyfact, eq. chol-precond,
// eq. chol-precond-inv): the preconditioner of the paper's Chol-IP-PMM
// comparator.
//
// Build (once per interior-point iteration):
//   diag(N + delta I) by the squared form of pass 2 (one read of A);
//   the ell largest entries by a one-block radix select on their bit patterns
//   (positive doubles order like their unsigned 64-bit patterns), pivots kept
//   in ascending index order (only the set matters for P_Chol);
//   Y = (N + delta I)[:, piv] = A (d .* A[piv, :]^T) + delta E_piv: the
//   gathered, scaled pivot rows of A and one FP64 tile product;
//   C = chol(Y[piv, :]) (upper, C^T C = N11, so L11 = C^T), Cinv = C^{-1};
//   L = Y Cinv (rows piv give L11, the others L21);
//   diag(S)_i = (N + delta I)_ii - ||L[i, :]||^2 off the pivots.
// Apply (eq. chol-precond-inv): t1 = L11^{-1} r[piv] = Cinv^T r[piv];
//   u_i = (r_i - L[i, :] t1) / diag(S)_i off the pivots (the second block);
//   out[piv] = L11^{-T} (t1 - L21^T u) = Cinv (t1 - sum_i L[i, :] u_i);
//   out_i = u_i off the pivots.

#include "common.hpp"
#include "kernels.hpp"

namespace nys {
namespace {

constexpr int SB = 1024;     // threads of the one-block select
constexpr int RBP = 64;      // rows per block of the apply's row pass

__device__ __forceinline__ int block_sum_int(int v, int* sm) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, NYS_WAVE);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) sm[wid] = v;
  __syncthreads();
  int s = 0;
  for (int w = 0; w < (int)(blockDim.x >> 6); ++w) s += sm[w];
  return s;
}

// Exclusive prefix sum over the block's threads (Hillis-Steele in LDS).
__device__ __forceinline__ int block_exscan_int(int v, int* buf) {
  const int t = threadIdx.x;
  __syncthreads();
  buf[t] = v;
  __syncthreads();
  for (int off = 1; off < (int)blockDim.x; off <<= 1) {
    const int add = t >= off ? buf[t - off] : 0;
    __syncthreads();
    buf[t] += add;
    __syncthreads();
  }
  return buf[t] - v;
}

// piv = the ell largest entries of diag (> 0), ties to the smaller index,
// ascending; pos[i] = k for i = piv[k], else -1.
__global__ __launch_bounds__(SB) void k_pchol_select(const double* diag, int64_t m, int ell, int* piv,
                                                     int* pos) {
  __shared__ int sm[SB / NYS_WAVE];
  __shared__ int buf[SB];
  const int64_t chunk = (m + SB - 1) / SB;
  const int64_t i0 = min(m, (int64_t)threadIdx.x * chunk), i1 = min(m, i0 + chunk);
  auto key = [&](int64_t i) { return (unsigned long long)__double_as_longlong(diag[i]); };
  // T = the ell-th largest key, built bit by bit from the top
  unsigned long long T = 0;
  for (int bit = 63; bit >= 0; --bit) {
    const unsigned long long cand = T | (1ull << bit);
    int c = 0;
    for (int64_t i = i0; i < i1; ++i) c += key(i) >= cand ? 1 : 0;
    if (block_sum_int(c, sm) >= ell) T = cand;
  }
  int gt = 0, eq = 0;
  for (int64_t i = i0; i < i1; ++i) {
    const unsigned long long k = key(i);
    gt += k > T ? 1 : 0;
    eq += k == T ? 1 : 0;
  }
  const int need = ell - block_sum_int(gt, sm);      // ties taken, smallest indices first
  int tie = block_exscan_int(eq, buf);
  int sel = 0;
  for (int64_t i = i0; i < i1; ++i) {
    const unsigned long long k = key(i);
    if (k > T) ++sel;
    else if (k == T && tie++ < need) ++sel;
  }
  int off = block_exscan_int(sel, buf);
  tie = block_exscan_int(eq, buf);
  for (int64_t i = i0; i < i1; ++i) {
    const unsigned long long k = key(i);
    bool s = k > T;
    if (k == T) s = tie++ < need;
    if (s) {
      piv[off] = (int)i;
      pos[i] = off++;
    } else {
      pos[i] = -1;
    }
  }
}

// Wt[k][j] = d[j] * A[piv[k]][j]  (ell x n, FP64)
template <class T>
__global__ __launch_bounds__(NYS_BLOCK) void k_pchol_gather(const char* A, int64_t row_bytes, int64_t n,
                                                            const int* piv, const double* d, double* Wt) {
  using raw = typename T::raw;
  const int k = blockIdx.y;
  const raw* row = (const raw*)(A + (int64_t)piv[k] * row_bytes);
  for (int64_t j = (int64_t)blockIdx.x * NYS_BLOCK + threadIdx.x; j < n; j += (int64_t)gridDim.x * NYS_BLOCK)
    Wt[(int64_t)k * n + j] = d[j] * to_f64(row[j]);
}

// Y[piv[k]][k] += delta; G[k][k'] = Y[piv[k]][k'] (the pivot block N11)
__global__ __launch_bounds__(NYS_BLOCK) void k_pchol_n11(double* Y, int ell, const int* piv, double delta,
                                                         double* G) {
  const int k = blockIdx.x;
  double* yr = Y + (int64_t)piv[k] * ell;
  if (threadIdx.x == 0) yr[k] += delta;
  __syncthreads();
  for (int c = threadIdx.x; c < ell; c += NYS_BLOCK) G[(int64_t)k * ell + c] = yr[c];
}

// diagS_i = diag_i - ||L[i, :]||^2 off the pivots (at least delta: S is a
// Schur complement of a matrix >= delta I), 1 on pivots.  One wave per row.
__global__ __launch_bounds__(NYS_BLOCK) void k_pchol_diags(const double* L, int64_t m, int ell, const int* pos,
                                                           const double* diag, double delta, double* diagS) {
  const int lane = threadIdx.x & 63;
  const int64_t i = (int64_t)blockIdx.x * (NYS_BLOCK / NYS_WAVE) + (threadIdx.x >> 6);
  if (i >= m) return;
  double s = 0.0;
  for (int k = lane; k < ell; k += NYS_WAVE) s = fma(L[i * ell + k], L[i * ell + k], s);
  s = wave_sum(s);
  if (lane == 0) diagS[i] = pos[i] >= 0 ? 1.0 : fmax(diag[i] - s, delta);
}

struct ApArgs {
  const double* skip;
  int64_t m;
  int ell;
  const int* piv;
  const int* pos;
  const double* L;
  const double* Cinv;
  const double* diagS;
  const double* r;
  double* out;
  double* t1;          // ell
  double* sv;          // ell + 1 (sum_i L[i, :] u_i, then the rows' part of r^T out)
  double* part;        // nb x (ell + 1)
  double* scal;        // PCG scalars (or NULL)
  double* dot_out;     // standalone r^T out (or NULL)
};

// t1[k] = sum_{k' <= k} Cinv[k'][k] r[piv[k']]   (one block)
__global__ __launch_bounds__(NYS_BLOCK) void k_pchol_t1(ApArgs a) {
  if (a.skip && *a.skip != 0.0) return;
  for (int k = threadIdx.x; k < a.ell; k += NYS_BLOCK) {
    double s = 0.0;
    for (int kp = 0; kp <= k; ++kp) s = fma(a.Cinv[(int64_t)kp * a.ell + k], a.r[a.piv[kp]], s);
    a.t1[k] = s;
  }
}

// u_i for RBP rows (one wave per row), out_i = u_i off the pivots; partial
// sums of L[i, :] u_i over the block's rows and of r_i u_i.
__global__ __launch_bounds__(NYS_BLOCK) void k_pchol_rows(ApArgs a) {
  extern __shared__ double tl[];           // t1 (ell)
  __shared__ double ul[RBP];
  __shared__ double smem[NYS_BLOCK / NYS_WAVE];
  if (a.skip && *a.skip != 0.0) return;
  for (int k = threadIdx.x; k < a.ell; k += NYS_BLOCK) tl[k] = a.t1[k];
  __syncthreads();
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int64_t i0 = (int64_t)blockIdx.x * RBP;
  const int nr = (int)min((int64_t)RBP, a.m - i0);
  double rs[1] = {0.0};
  for (int rr = wid; rr < nr; rr += NYS_BLOCK / NYS_WAVE) {
    const int64_t i = i0 + rr;
    double s = 0.0;
    for (int k = lane; k < a.ell; k += NYS_WAVE) s = fma(a.L[i * a.ell + k], tl[k], s);
    s = wave_sum(s);
    if (lane == 0) {
      double u = 0.0;
      if (a.pos[i] < 0) {
        u = (a.r[i] - s) / a.diagS[i];
        a.out[i] = u;
        rs[0] = fma(a.r[i], u, rs[0]);
      }
      ul[rr] = u;
    }
  }
  __syncthreads();
  double* mypart = a.part + (int64_t)blockIdx.x * (a.ell + 1);
  for (int k = threadIdx.x; k < a.ell; k += NYS_BLOCK) {
    double acc = 0.0;
    for (int rr = 0; rr < nr; ++rr) acc = fma(a.L[(i0 + rr) * a.ell + k], ul[rr], acc);
    mypart[k] = acc;
  }
  block_sum<1>(rs, smem);
  if (threadIdx.x == 0) mypart[a.ell] = rs[0];
}

// sv[k] = sum over blocks of the partials (ell + 1 blocks, fixed order)
__global__ __launch_bounds__(NYS_BLOCK) void k_pchol_fin1(ApArgs a, int nb) {
  __shared__ double smem[NYS_BLOCK / NYS_WAVE];
  if (a.skip && *a.skip != 0.0) return;
  const int col = blockIdx.x;
  double s[1] = {0.0};
  for (int b = threadIdx.x; b < nb; b += NYS_BLOCK) s[0] += a.part[(int64_t)b * (a.ell + 1) + col];
  block_sum<1>(s, smem);
  if (threadIdx.x == 0) a.sv[col] = s[0];
}

// out[piv[k]] = (Cinv (t1 - sv))_k; r^T out; PCG: beta = rs_new / rs, rs = rs_new.
__global__ __launch_bounds__(NYS_BLOCK) void k_pchol_fin2(ApArgs a) {
  __shared__ double smem[NYS_BLOCK / NYS_WAVE];
  if (a.skip && *a.skip != 0.0) return;
  double dotp[1] = {0.0};
  for (int k = threadIdx.x; k < a.ell; k += NYS_BLOCK) {
    double s = 0.0;
    for (int kp = k; kp < a.ell; ++kp) s = fma(a.Cinv[(int64_t)k * a.ell + kp], a.t1[kp] - a.sv[kp], s);
    const int i = a.piv[k];
    a.out[i] = s;
    dotp[0] = fma(a.r[i], s, dotp[0]);
  }
  block_sum<1>(dotp, smem);
  if (threadIdx.x == 0) {
    const double rs = a.sv[a.ell] + dotp[0];
    if (a.dot_out) *a.dot_out = rs;
    if (a.scal) {
      const bool dn = a.scal[SC_DONE] != 0.0;
      a.scal[SC_BETA] = dn ? 0.0 : rs / a.scal[SC_RS];
      a.scal[SC_RS] = rs;
    }
  }
}

int elem_bytes(nys_dtype dt) { return dt == NYS_F64 ? 8 : dt == NYS_F32 ? 4 : 2; }

// Y[piv[k], k] += e[piv[k]]: the unit columns' part of N[:, piv] (diagonal only,
// since no two unit columns share a row)
__global__ __launch_bounds__(NYS_BLOCK) void k_pchol_unit(double* Y, int ell, const int* piv, const double* e) {
  for (int k = blockIdx.x * NYS_BLOCK + threadIdx.x; k < ell; k += gridDim.x * NYS_BLOCK)
    Y[(int64_t)piv[k] * ell + k] += e[piv[k]];
}

}  // namespace

int pchol_build(nys_handle h, const nys_matrix* A, const double* d, double delta, nys_pchol* P) {
  const int64_t m = A->m, n = A->n;
  const int ell = P->ell;
  // the gather's grid has one y index per pivot and stops at 65535
  if (ell > 65535) return set_error(h, NYS_EINVAL, "partial Cholesky: ell=%d above 65535 pivots", ell);
  double *Y, *Wt, *G, *diag;
  NYS_CHECK(ws(h, WS_Y, (size_t)m * ell, &Y));
  NYS_CHECK(ws(h, WS_SK_W, (size_t)ell * std::max<int64_t>(n, 1), &Wt));
  NYS_CHECK(ws(h, WS_SMALL, (size_t)ell * ell + (size_t)ell * ell / 4 + 16, &G));   // G, then the inverse's work
  NYS_CHECK(ws(h, WS_B, (size_t)m, &diag));
  // diag(N + delta I) = (A .* A) d + delta
  GemvN gd;
  gd.A = A;
  gd.w = d;
  gd.square = true;
  gd.shift = delta;
  gd.out = diag;
  NYS_CHECK(gemv_n(h, gd));
  hipLaunchKernelGGL(k_pchol_select, dim3(1), dim3(SB), 0, h->stream, (const double*)diag, m, ell, P->piv, P->pos);
  NYS_LAUNCH_CHECK(h);
  // Y = A Wt^T with Wt = (d .* A[piv, :]^T)^T, then + delta on the pivot entries
  if (n > 0) {
    const int es = elem_bytes(A->dtype);
    dim3 g((unsigned)std::min<int64_t>((n + NYS_BLOCK - 1) / NYS_BLOCK, 64), (unsigned)ell);
    switch (A->dtype) {
      case NYS_F64: hipLaunchKernelGGL(k_pchol_gather<F64>, g, dim3(NYS_BLOCK), 0, h->stream, (const char*)A->data, A->ld * es, n, (const int*)P->piv, d, Wt); break;
      case NYS_F32: hipLaunchKernelGGL(k_pchol_gather<F32>, g, dim3(NYS_BLOCK), 0, h->stream, (const char*)A->data, A->ld * es, n, (const int*)P->piv, d, Wt); break;
      default: hipLaunchKernelGGL(k_pchol_gather<BF16>, g, dim3(NYS_BLOCK), 0, h->stream, (const char*)A->data, A->ld * es, n, (const int*)P->piv, d, Wt); break;
    }
    NYS_LAUNCH_CHECK(h);
    NYS_CHECK(gemm_f64(h, false, true, m, ell, n, A->data, A->dtype, A->ld, Wt, n, Y, ell, nullptr));
  } else {
    NYS_CHECK(fill(h, Y, m * ell, 0.0));
  }
  if (A->n_unit > 0) {
    double* e;
    NYS_CHECK(ws(h, WS_UNIT, (size_t)m, &e));
    NYS_CHECK(unit_diag(h, A, d, e));
    hipLaunchKernelGGL(k_pchol_unit, dim3((unsigned)((ell + NYS_BLOCK - 1) / NYS_BLOCK)), dim3(NYS_BLOCK), 0,
                       h->stream, Y, ell, (const int*)P->piv, (const double*)e);
    NYS_LAUNCH_CHECK(h);
  }
  hipLaunchKernelGGL(k_pchol_n11, dim3((unsigned)ell), dim3(NYS_BLOCK), 0, h->stream, Y, ell, (const int*)P->piv,
                     delta, G);
  NYS_LAUNCH_CHECK(h);
  double* fail = h->dscal + SC_FAIL;
  NYS_CHECK(chol_upper(h, G, ell, 0.0, 0.0, fail));
  NYS_CHECK(read_scalars(h, SC_FAIL, 1));
  if (h->hscal[SC_FAIL] != 0.0)
    return set_error(h, NYS_ENOTPD, "partial Cholesky: the pivot block is not positive definite");
  NYS_CHECK(tri_inv_upper(h, G, P->Cinv, ell, G + (size_t)ell * ell + 8));
  NYS_CHECK(gemm_f64(h, false, false, m, ell, ell, Y, NYS_F64, ell, P->Cinv, ell, P->L, ell, nullptr, true));
  hipLaunchKernelGGL(k_pchol_diags, dim3((unsigned)((m + 3) / 4)), dim3(NYS_BLOCK), 0, h->stream,
                     (const double*)P->L, m, ell, (const int*)P->pos, (const double*)diag, delta, P->diagS);
  NYS_LAUNCH_CHECK(h);
  return NYS_OK;
}

int pchol_apply(nys_handle h, const nys_pchol* P, const double* r, double* out, bool pcg, double* dot_out) {
  const int64_t m = P->m;
  const int ell = P->ell;
  const int nb = (int)((m + RBP - 1) / RBP);
  double *vecs, *part;
  NYS_CHECK(ws(h, WS_PCH, (size_t)2 * ell + 8, &vecs));
  NYS_CHECK(ws(h, WS_PART, (size_t)nb * (ell + 1), &part));
  ApArgs a{};
  a.skip = pcg ? h->dscal + SC_DONE : nullptr;
  a.m = m;
  a.ell = ell;
  a.piv = P->piv;
  a.pos = P->pos;
  a.L = P->L;
  a.Cinv = P->Cinv;
  a.diagS = P->diagS;
  a.r = r;
  a.out = out;
  a.t1 = vecs;
  a.sv = vecs + ell;
  a.part = part;
  a.scal = pcg ? h->dscal : nullptr;
  a.dot_out = dot_out;
  hipLaunchKernelGGL(k_pchol_t1, dim3(1), dim3(NYS_BLOCK), 0, h->stream, a);
  hipLaunchKernelGGL(k_pchol_rows, dim3((unsigned)nb), dim3(NYS_BLOCK), (size_t)ell * sizeof(double), h->stream, a);
  hipLaunchKernelGGL(k_pchol_fin1, dim3((unsigned)(ell + 1)), dim3(NYS_BLOCK), 0, h->stream, a, nb);
  hipLaunchKernelGGL(k_pchol_fin2, dim3(1), dim3(NYS_BLOCK), 0, h->stream, a);
  NYS_LAUNCH_CHECK(h);
  return NYS_OK;
}

}  // namespace nys
