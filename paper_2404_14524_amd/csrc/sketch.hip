// The sketch Y = N Omega = A diag(d) A^T Omega of Algorithm 1 (second step),
// computed as the GEMM pair W = d .* (A^T Omega) (n x ell, reduction over m)
// and Y = A W (m x ell, reduction over n).

#include "common.hpp"
#include "kernels.hpp"

namespace nys {

int sketch_bf16(nys_handle h, const nys_matrix* A, const double* d, const double* Omega, int ell,
                double* Y);

int sketch_product(nys_handle h, const nys_matrix* A, const double* d, const double* Omega,
                   int ell, nys_dtype mode, double* Y) {
  if (mode == NYS_BF16) {
    NYS_CHECK(sketch_bf16(h, A, d, Omega, ell, Y));
    return unit_sketch(h, A, d, Omega, ell, Y);     // unit columns: exact FP64 terms
  }
  if (A->dtype == NYS_BF16)
    return set_error(h, NYS_EINVAL, "FP64 sketch needs an FP64 or FP32 matrix");
  double* W;
  NYS_CHECK(ws(h, WS_SK_W, (size_t)A->n * ell, &W));
  // W (n x ell) = diag(d) A^T Omega : op(A) = A^T, K = m
  NYS_CHECK(gemm_f64(h, true, false, A->n, ell, A->m, A->data, A->dtype, A->ld, Omega, ell, W, ell, d));
  // Y (m x ell) = A W : K = n
  NYS_CHECK(gemm_f64(h, false, false, A->m, ell, A->n, A->data, A->dtype, A->ld, W, ell, Y, ell, nullptr));
  return unit_sketch(h, A, d, Omega, ell, Y);
}

}  // namespace nys
