// Internal launchers of libnysipm.  Every function enqueues on h->stream and
// returns an NYS_* code; none synchronises unless its comment says so.
#pragma once

#include "handle.hpp"

namespace nys {

// ---------------------------------------------------------------- GEMV pair
// Pass 1 (reduction over the m rows of A; over the rows of A->data_t when set):
//   w[j] = d[j] * (sA * sum_i A[i,j] v_i + x0[j])     (d, x0 may be NULL)
// where v_i = v[i], or, when `s` is non-NULL, the fused CG direction update
//   v_i = s[i] + beta * pold[i]   (beta read from the device word *beta),
// which is also stored to pnew[i].
// Both passes return at once, doing nothing, when `skip` is non-NULL and the
// device word *skip is non-zero (a finished PCG solve).
struct GemvT {
  const nys_matrix* A;
  const double* skip = nullptr;
  const double* v = nullptr;
  const double* s = nullptr;
  const double* pold = nullptr;
  double* pnew = nullptr;
  const double* beta = nullptr;
  const double* d = nullptr;
  const double* x0 = nullptr;
  double sA = 1.0;
  double* w = nullptr;
};
int gemv_t(nys_handle h, const GemvT& a);

// Pass 2 (reduction over the n columns of A):
//   out[i] = sA * sum_j A[i,j] w[j] + sV * v[i] + x0[i] + shift   (v, x0 may be NULL)
// and, when dot_out is non-NULL, *dot_out = sum_i out[i] * v[i].  With
// square, A[i,j] is replaced by A[i,j]^2 (the diagonal of A diag(w) A^T).
struct GemvN {
  const nys_matrix* A;
  const double* skip = nullptr;
  const double* w = nullptr;
  const double* v = nullptr;
  const double* x0 = nullptr;
  double sA = 1.0, sV = 0.0, shift = 0.0;
  bool square = false;
  double* out = nullptr;
  double* dot_out = nullptr;
};
int gemv_n(nys_handle h, const GemvN& a);
// Both passes include the unit columns of A (nys_matrix.n_unit): pass 1 writes
// w[n + t] as well, pass 2 adds their terms (squared with square) in FP64.
// (Internal to the two passes: unit_pass1 writes w[n + t] from v; unit_pass2_base
// returns in *x0_eff the per-row vector x0 + unit terms for the dense pass 2.)
int unit_pass1(nys_handle h, const GemvT& a, const double* v);
int unit_pass2_base(nys_handle h, const GemvN& a, const double** x0_eff);
// e[i] = sum over unit columns t in row i of val_t^2 d[n + t] (zero elsewhere):
// the unit columns' part of the diagonal of A diag(d) A^T.
int unit_diag(nys_handle h, const nys_matrix* A, const double* d, double* e);
// Y[row_t, :] += val_t^2 d[n + t] Omega[row_t, :] for every unit column t
// (their part of the sketch N Omega; Y and Omega m x ell row-major).
int unit_sketch(nys_handle h, const nys_matrix* A, const double* d, const double* Omega, int ell, double* Y);
// Device check of the unit arrays (rows strictly increasing in [0, m), values
// finite); NYS_EINVAL with a message naming `who` otherwise.  Synchronises.
int check_units(nys_handle h, const nys_matrix* A, const char* who);

// At (n x m, leading dimension ld_t >= m elements, A's dtype) = A^T.
int transpose(nys_handle h, const nys_matrix* A, void* At, int64_t ld_t);
// *out = *A with data_t pointing at a transposed copy in workspace slot `slot`
// (made here unless A already has one or `allowed` is false; without memory
// for it, *out = *A and the kernels read A as it is).
int with_transpose(nys_handle h, const nys_matrix* A, bool allowed, int slot, nys_matrix* out);

// Doubles of partial sums the two passes request from the workspace: pass 1
// on column stripes of A (WS_PART; 0 with a transposed copy), pass 2's fused
// dot product (WS_PART2).
size_t gemv_t_part_doubles(const nys_matrix* A);
size_t gemv_n_part_doubles(int64_t m);

// Sketch tiles of A (transposed = false: rows m, k along n) or of A^T (rows n,
// k along m) for the BF16 sketch, and their size in bytes.
int64_t sketch_tiles_bytes(int64_t rows, int64_t cols);
int sketch_tiles(nys_handle h, const nys_matrix* A, bool transposed, void* out);

// out = (A diag(d) A^T + delta I) v, with optional *dot_out = v^T out.
int normal_apply(nys_handle h, const nys_matrix* A, const double* d, double delta,
                 const double* v, double* out, double* dot_out);

// Read-stream reference (16-byte non-temporal loads over `bytes`, a multiple of
// 16) in one of stream_read_shapes() shapes; launch stream_read_blocks(bytes,
// shape) blocks; part receives nblocks * 4 words.
int stream_read_shapes();
int stream_read_blocks(int64_t bytes, int shape);
int stream_read(nys_handle h, const void* data, int64_t bytes, unsigned* part, int shape);

// ---------------------------------------------------------------- vectors
int fill(nys_handle h, double* x, int64_t n, double value);
int copy(nys_handle h, double* dst, const double* src, int64_t n);
// dst = a*x + b*y (y may be NULL)
int axpby(nys_handle h, double* dst, double a, const double* x, double b, const double* y, int64_t n);
// *out = sum x_i y_i (device word)
int dot(nys_handle h, const double* x, const double* y, int64_t n, double* out);
// Checks a matrix for non-finite entries; *out = count (device word, as double)
int count_nonfinite_matrix(nys_handle h, const nys_matrix* A, double* out);
// out[0] = #non-finite in x, out[1] = #entries < 0 (device words)
int count_bad(nys_handle h, const double* x, int64_t n, double* out);

// ---------------------------------------------------------------- preconditioner
// Partial t = U^T r over row blocks, finished by the last block:
// t[k] = f_k * sum_i U[i,k] r[i] with f_k = (lam_l + delta)/(lam_k + delta) - 1,
// lam_l = min_k lam_k.  Also ||r||^2 -> h->dscal[SC_RR].
int precond_reduce(nys_handle h, const double* U, const double* lam, int64_t m, int ell,
                   double delta, const double* r, double* t);
// out[i] = r[i] + sum_k U[i,k] t[k]; optional *dot_out = sum_i r[i] out[i].
int precond_expand(nys_handle h, const double* U, int64_t m, int ell, const double* r,
                   const double* t, double* out, double* dot_out);

// Doubles of partial sums requested by the update kernels (WS_PART: pcg_update,
// precond_reduce) and by the expand kernel (WS_PART2).
size_t update_part_doubles(int64_t m, int ell, bool precond);
size_t expand_part_doubles(int64_t m);

// ---------------------------------------------------------------- PCG kernels
// y += alpha p, r -= alpha q with alpha = rs/pq from the device words (zero
// once done); then (with a Nystrom preconditioner) the partial U^T r
// reduction, or (without, unless ext: another preconditioner follows)
// rs_new = ||r||^2 and beta.  Sets done when ||r||^2 <= tol2.
int pcg_update(nys_handle h, int64_t m, double* y, double* r, const double* p,
               const double* q, const double* U, const double* lam, int ell, double delta,
               double* t, bool ext = false);

// ---------------------------------------------------------------- Newton step data
// Box and free variables of Algorithm 5 (all NULL: every variable non-negative).
// vt: index kinds (NYS_VAR_*); w, s: slack and its dual; ru, rws: the r_u and
// r_ws right-hand sides (ru may be NULL: zero); dw, ds: outputs.
struct BoxNewton {
  const int8_t* vt = nullptr;
  const double* w = nullptr;
  const double* s = nullptr;
  const double* ru = nullptr;
  const double* rws = nullptr;
  double* dw = nullptr;
  double* ds = nullptr;
};

// ---------------------------------------------------------------- partial Cholesky (comparator)
// Builds P (caller-sized: P->m = A->m, P->ell) for N + delta I, N = A diag(d) A^T.
// Synchronises (checks the Cholesky of the pivot block).
int pchol_build(nys_handle h, const nys_matrix* A, const double* d, double delta, nys_pchol* P);
// out = P^{-1} r.  pcg: the PCG form (skip once done; rs_new = r^T out, beta,
// rs written to the device scalars); else *dot_out = r^T out when non-NULL.
int pchol_apply(nys_handle h, const nys_pchol* P, const double* r, double* out, bool pcg,
                double* dot_out);
// ||r||^2 -> h->dscal[SC_RR] (no update).
int residual_norm(nys_handle h, int64_t m, double* r);
// With a preconditioner: s = r + U t, rs_new = r^T s, beta = rs_new/rs (zero once done).
int pcg_expand(nys_handle h, int64_t m, const double* U, int ell, const double* r,
               const double* t, double* s);

// ---------------------------------------------------------------- small dense FP64
// C (M x N, ldc) = op(A) op(B) with FP64 accumulation, op = transpose if flag.
// A elements may be FP64/FP32/BF16 (adt); B is FP64.  Row scale: C[i,:] *= rs[i].
// b_upper: B (K x N, not transposed) is upper triangular with zeros below its
// diagonal, so that rows k >= j of B do not reach column j of C.
int gemm_f64(nys_handle h, bool transA, bool transB, int64_t M, int64_t N, int64_t K,
             const void* A, nys_dtype adt, int64_t lda, const double* B, int64_t ldb,
             double* C, int64_t ldc, const double* row_scale, bool b_upper = false);
// In-place Cholesky G = C^T C of an ell x ell matrix (symmetrised first, plus
// shift_abs + shift_rel * trace(G) on the diagonal); result C upper (lower
// part zeroed).  Sets the device word *fail to 1.0 when a pivot is not positive.
int chol_upper(nys_handle h, double* G, int ell, double shift_abs, double shift_rel, double* fail);
// Cinv = C^{-1} for upper-triangular C (ell x ell), zeros below the diagonal.
// With work (ell * ell / 4 doubles) and ell > 256, by diagonal blocks joined
// pairwise with matrix-core products; otherwise column by column.
int tri_inv_upper(nys_handle h, const double* C, double* Cinv, int ell, double* work = nullptr);
// C3 = C1 * C2 for ell x ell (upper triangular products allowed).
int small_mm(nys_handle h, const double* C1, const double* C2, double* C3, int ell);
// One-sided Jacobi SVD of X (ell x ell, row-major, overwritten): on return the
// columns of X are the left singular vectors sorted by descending singular
// value and sig2[k] the squared singular values.  work: ell*ell + ell + 2
// doubles.  Synchronises (sweep polls).
int jacobi_svd(nys_handle h, double* X, int ell, double* sig2, double* work);
// Philox4x32-10 Gaussian matrix (see nys_test_matrix).
int philox_gaussian(nys_handle h, int64_t m, int ell, uint64_t seed, uint64_t counter, double* out);
// out = bf16(fp32(x)) (round to nearest even), count elements.
int to_bf16(nys_handle h, const double* x, uint16_t* out, int64_t count);
int f32_to_bf16(nys_handle h, const float* x, int64_t rows, int64_t cols, int64_t ld,
                uint16_t* out);
// unsigned words to zero (graph-capture safe, no memset node)
int zero_u32(nys_handle h, unsigned* p, int64_t count);
// ||X||_F^2 of a dense FP64 array -> device word
int sumsq(nys_handle h, const double* x, int64_t count, double* out);

// ---------------------------------------------------------------- sketch
// Y = A diag(d) A^T Omega  (m x ell, FP64 out).  mode NYS_F64: FP64 arithmetic
// (A FP64 or FP32 storage).  NYS_BF16: A BF16, Omega and W rounded to BF16,
// matrix-core products with FP32 accumulation.
int sketch_product(nys_handle h, const nys_matrix* A, const double* d, const double* Omega,
                   int ell, nys_dtype mode, double* Y);

}  // namespace nys
