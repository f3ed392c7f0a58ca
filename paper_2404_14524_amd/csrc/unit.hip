// Unit columns of A = [A_d | E] (nys_matrix.n_unit): column t of E has the
// single entry val_t in row row_t, rows strictly increasing.  They are the
// identity and slack blocks of the forms (P~) of the SVM and portfolio
// problems (the identity on the free v of the SVM dual; -I on the factor
// returns y and +I on the correlation slacks of the portfolio problem).
// Stored densely they would be streamed by every pass of the normal-equation
// operator although each holds one non-zero; here they cost O(n_unit) FP64
// work per pass:
//   pass 1:  w[n + t] = d[n + t] (sA val_t v[row_t] + x0[n + t]),
//   pass 2:  out[row_t] += sA val_t w[n + t]   (val_t^2 for the diagonal),
// the second folded into the x0 term of the dense pass 2 (a per-row vector it
// already adds), so its fused p^T (M p) dot product includes them.  Rows
// outside [0, m) are skipped by every kernel; the entry points reject them
// beforehand (check_units).

#include <cmath>

#include "common.hpp"
#include "kernels.hpp"
#include "mapreduce.hpp"

namespace nys {
namespace {

inline unsigned unit_blocks(int64_t k) {
  return (unsigned)std::max<int64_t>(1, std::min<int64_t>((k + NYS_BLOCK - 1) / NYS_BLOCK, 1024));
}

// w[t] = d[t] (sA val[t] v[row[t]] + x0[t]); d, x0, w already offset by n
__global__ __launch_bounds__(NYS_BLOCK) void k_unit_t(const double* skip, int64_t k, int64_t m,
                                                       const int32_t* row, const double* val, const double* v,
                                                       const double* d, const double* x0, double sA, double* w) {
  if (skip && *skip != 0.0) return;
  const int64_t stride = (int64_t)gridDim.x * NYS_BLOCK;
  for (int64_t t = (int64_t)blockIdx.x * NYS_BLOCK + threadIdx.x; t < k; t += stride) {
    const int32_t r = row[t];
    double s = (r >= 0 && r < m) ? sA * val[t] * v[r] : 0.0;
    if (x0) s += x0[t];
    w[t] = d ? d[t] * s : s;
  }
}

// base[i] = x0[i], or 0 without x0
__global__ __launch_bounds__(NYS_BLOCK) void k_unit_base(const double* skip, int64_t m, const double* x0,
                                                          double* base) {
  if (skip && *skip != 0.0) return;
  const int64_t stride = (int64_t)gridDim.x * NYS_BLOCK;
  for (int64_t i = (int64_t)blockIdx.x * NYS_BLOCK + threadIdx.x; i < m; i += stride) base[i] = x0 ? x0[i] : 0.0;
}

// base[row[t]] += sA val[t] w[t]  (val[t]^2 with square); w offset by n.
// Rows are distinct, so no two threads add to one entry.
__global__ __launch_bounds__(NYS_BLOCK) void k_unit_scatter(const double* skip, int64_t k, int64_t m,
                                                             const int32_t* row, const double* val,
                                                             const double* w, double sA, int square, double* base) {
  if (skip && *skip != 0.0) return;
  const int64_t stride = (int64_t)gridDim.x * NYS_BLOCK;
  for (int64_t t = (int64_t)blockIdx.x * NYS_BLOCK + threadIdx.x; t < k; t += stride) {
    const int32_t r = row[t];
    if (r < 0 || r >= m) continue;
    const double a = square ? val[t] * val[t] : val[t];
    base[r] += sA * a * w[t];
  }
}

// Y[row_t, c] += val_t^2 d[t] Omega[row_t, c]; d offset by n
__global__ __launch_bounds__(NYS_BLOCK) void k_unit_sketch(int64_t k, int64_t m, int ell, const int32_t* row,
                                                            const double* val, const double* d, const double* Om,
                                                            double* Y) {
  const int64_t total = k * (int64_t)ell;
  const int64_t stride = (int64_t)gridDim.x * NYS_BLOCK;
  for (int64_t e = (int64_t)blockIdx.x * NYS_BLOCK + threadIdx.x; e < total; e += stride) {
    const int64_t t = e / ell;
    const int c = (int)(e - t * ell);
    const int32_t r = row[t];
    if (r < 0 || r >= m) continue;
    const int64_t at = (int64_t)r * ell + c;
    Y[at] += val[t] * val[t] * d[t] * Om[at];
  }
}

struct UnitCheck {   // violations of: 0 <= row < m, strictly increasing, finite value
  const int32_t* row;
  const double* val;
  int64_t m;
  __device__ void operator()(int64_t t, double* a, double*) const {
    const int32_t r = row[t];
    const bool bad = r < 0 || r >= m || (t > 0 && row[t - 1] >= r) || !isfinite(val[t]);
    if (bad) a[0] += 1.0;
  }
};

}  // namespace

int unit_pass1(nys_handle h, const GemvT& a, const double* v) {
  const nys_matrix* A = a.A;
  const int64_t k = A->n_unit, n = A->n;
  if (k <= 0) return NYS_OK;
  hipLaunchKernelGGL(k_unit_t, dim3(unit_blocks(k)), dim3(NYS_BLOCK), 0, h->stream, a.skip, k, A->m, A->unit_row,
                     A->unit_val, v, a.d ? a.d + n : nullptr, a.x0 ? a.x0 + n : nullptr, a.sA, a.w + n);
  NYS_LAUNCH_CHECK(h);
  return NYS_OK;
}

int unit_pass2_base(nys_handle h, const GemvN& a, const double** x0_eff) {
  const nys_matrix* A = a.A;
  const int64_t k = A->n_unit, n = A->n, m = A->m;
  *x0_eff = a.x0;
  if (k <= 0) return NYS_OK;
  double* base;
  NYS_CHECK(ws(h, WS_UNIT, (size_t)std::max<int64_t>(m, 1), &base));
  hipLaunchKernelGGL(k_unit_base, dim3(unit_blocks(m)), dim3(NYS_BLOCK), 0, h->stream, a.skip, m, a.x0, base);
  hipLaunchKernelGGL(k_unit_scatter, dim3(unit_blocks(k)), dim3(NYS_BLOCK), 0, h->stream, a.skip, k, m,
                     A->unit_row, A->unit_val, a.w + n, a.sA, a.square ? 1 : 0, base);
  NYS_LAUNCH_CHECK(h);
  *x0_eff = base;
  return NYS_OK;
}

int unit_diag(nys_handle h, const nys_matrix* A, const double* d, double* e) {
  const int64_t k = A->n_unit, m = A->m;
  hipLaunchKernelGGL(k_unit_base, dim3(unit_blocks(m)), dim3(NYS_BLOCK), 0, h->stream, nullptr, m, nullptr, e);
  if (k > 0)
    hipLaunchKernelGGL(k_unit_scatter, dim3(unit_blocks(k)), dim3(NYS_BLOCK), 0, h->stream, nullptr, k, m,
                       A->unit_row, A->unit_val, d + A->n, 1.0, 1, e);
  NYS_LAUNCH_CHECK(h);
  return NYS_OK;
}

int unit_sketch(nys_handle h, const nys_matrix* A, const double* d, const double* Omega, int ell, double* Y) {
  const int64_t k = A->n_unit;
  if (k <= 0) return NYS_OK;
  hipLaunchKernelGGL(k_unit_sketch, dim3(unit_blocks(k * (int64_t)ell)), dim3(NYS_BLOCK), 0, h->stream, k, A->m,
                     ell, A->unit_row, A->unit_val, d + A->n, Omega, Y);
  NYS_LAUNCH_CHECK(h);
  return NYS_OK;
}

int check_units(nys_handle h, const nys_matrix* A, const char* who) {
  if (A->n_unit < 0) return set_error(h, NYS_EINVAL, "%s: n_unit < 0", who);
  if (A->n_unit == 0) return NYS_OK;
  if (!A->unit_row || !A->unit_val) return set_error(h, NYS_EINVAL, "%s: NULL unit-column arrays", who);
  if (A->n_unit > A->m)
    return set_error(h, NYS_EINVAL, "%s: %lld unit columns for %lld rows (rows must be distinct)", who,
                     (long long)A->n_unit, (long long)A->m);
  NYS_HIP(h, hipSetDevice(h->device));
  double* sc = h->dscal;
  NYS_CHECK((map_reduce<1, 0>(h, A->n_unit, UnitCheck{A->unit_row, A->unit_val, A->m}, sc + SC_RED0)));
  NYS_CHECK(read_scalars(h, SC_RED0, 1));
  if (h->hscal[SC_RED0] != 0.0)
    return set_error(h, NYS_EINVAL,
                     "%s: unit columns need rows strictly increasing within [0, m) and finite values", who);
  return NYS_OK;
}

}  // namespace nys
