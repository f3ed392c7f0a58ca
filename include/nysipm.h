/*
 * nysipm.h -- C ABI of the MI355X (gfx950) implementation of the hot path of
 * Nys-IP-PMM (Chu, Santos, Udell: "Randomized Nystrom Preconditioned Interior
 * Point-Proximal Method of Multipliers", arXiv 2404.14524) for the separable
 * convex QP
 *
 *     (P)  min 1/2 x^T Q x + c^T x   s.t.  A x = b,  x >= 0,   Q = diag(q) >= 0
 *     (D)  max b^T y - 1/2 x^T Q x   s.t.  A^T y + z = Q x + c,  z >= 0
 *
 * (paper, section 1).  All compute runs in the library's HIP kernels.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - Arrays are DEVICE pointers on the handle's device, allocated and owned by
 *   the caller, contiguous; matrices are row-major with a leading dimension
 *   (elements) >= the number of columns.  The library never frees caller
 *   memory; it owns only the handle and the workspace the handle allocates.
 * - FP64 vectors throughout; the constraint matrix may be stored in FP64,
 *   FP32 or BF16 (nys_matrix.dtype).  Products with A always accumulate in
 *   FP64, whatever the storage.
 * - Work is enqueued on the handle's HIP stream.  Entry points that make host
 *   decisions (nys_sketch, nys_pcg_solve, nys_newton_solve, ipm_solve,
 *   ipm_adjoint) synchronise that stream before returning; the others
 *   (nys_normal_apply, nys_precond_apply, nys_test_matrix) only enqueue.
 * - Return codes: 0 = NYS_OK; > 0 = warning, outputs valid; < 0 = error.
 *   Arguments are validated before any launch, so on NYS_EINVAL outputs are
 *   untouched.  nys_last_error(h) gives a message.  Nothing aborts and no
 *   exception crosses the ABI.  A handle is not thread-safe: one per stream.
 * - Size limits (launch grids): m < 2^31 (unit rows are int32); nys_transpose
 *   takes m <= 65535 * 64 = 4194240, and ipm_solve / ipm_adjoint make no
 *   transposed copy beyond that (the passes then read A_d as it is); sketch
 *   tiles take n <= 16776960, and ipm_solve / ipm_adjoint make none beyond
 *   that (the BF16 sketch then reads A_d as it is); the partial Cholesky
 *   preconditioner takes ell <= 65535.  Otherwise n is bounded only by memory.
 */
#ifndef NYSIPM_H
#define NYSIPM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  NYS_OK = 0,
  NYS_MAXIT = 1,          /* iteration limit reached; last iterate returned      */
  NYS_EINVAL = -1,        /* null or inconsistent argument, non-finite scalar,
                             q < 0, d < 0, delta <= 0 where required, ell not in
                             [1, m], NaN/Inf in the data of ipm_solve            */
  NYS_ENOMEM = -2,        /* workspace allocation failed                          */
  NYS_EHIP = -3,          /* a HIP runtime call failed                            */
  NYS_ENOTPD = -4,        /* Cholesky of a Gram matrix failed after the retries  */
  NYS_EBREAKDOWN = -5,    /* PCG breakdown: p^T M p <= 0 or not finite            */
  NYS_ENUMERIC = -6       /* NaN/Inf appeared in the interior-point iterates      */
};

typedef enum { NYS_F64 = 0, NYS_F32 = 1, NYS_BF16 = 2 } nys_dtype;

/* Preconditioner of the inner solves of ipm_solve: the randomized Nystrom
   preconditioner (Nys-IP-PMM, the method), or the paper's comparators: none
   (CG-IP-PMM) and partial Cholesky with ell pivots (Chol-IP-PMM). */
enum { NYS_PRECOND_NYSTROM = 0, NYS_PRECOND_NONE = 1, NYS_PRECOND_PCHOL = 2 };

typedef struct nys_handle_s* nys_handle;

/* A = [A_d | E]: a dense block A_d (m x n, row-major, leading dimension ld
   in elements, storage dtype) followed by n_unit unit columns E (optional).
   Unit column t (variable n + t) has the single entry unit_val[t] in row
   unit_row[t]; unit_row is strictly increasing within [0, m) (so no two unit
   columns share a row), unit_val finite FP64; both are device arrays of
   n_unit elements (NULL when n_unit = 0).  Such columns are the identity and
   slack blocks of the forms (P~) of the paper's SVM and portfolio problems;
   they are applied exactly in FP64 and never stored densely.  Vectors indexed
   by the columns of A (d, x, z, c, q, ...) have n + n_unit entries, dense
   columns first.  Entry points that take a matrix check the unit arrays on
   the device (NYS_EINVAL when they break the rules above).
   data_t (optional, may be NULL): A_d transposed, n x m row-major with
   leading dimension ld_t >= m, same dtype, caller-owned and not modified.
   When present, the products that reduce over the m rows (A^T v) stream whole
   rows of it instead of column stripes of A_d (same results up to the order
   of the FP64 additions).  ipm_solve and ipm_adjoint make such a copy in their
   workspace when none is given (see nys_ipm_opts.no_transposed_copy).
   tiles, tiles_t (optional, both or neither): A_d in the layout of the BF16
   matrix-core sketch (nys_sketch_tiles), caller-owned; when present the BF16
   sketch reads them instead of data / data_t.  ipm_solve and ipm_adjoint make
   them in their workspace for a BF16 sketch.
   Zero-initialise the struct: n_unit = 0 gives the plain dense matrix. */
typedef struct {
  int64_t m, n, ld;
  nys_dtype dtype;
  const void* data;
  const void* data_t;
  int64_t ld_t;
  int64_t n_unit;
  const int32_t* unit_row;
  const double* unit_val;
  const void* tiles;      /* optional: sketch tiles of A_d (nys_sketch_tiles, transposed = 0) */
  const void* tiles_t;    /* optional: sketch tiles of A_d^T (transposed = 1); give both or neither */
} nys_matrix;

/* Nystrom preconditioner {U_hat, Lambda_hat} (Algorithm 2; eq. Nys_precond).
   U: m x ell FP64 row-major with orthonormal columns; lambda: ell FP64,
   descending, >= 0.  delta is supplied at apply time. */
typedef struct {
  int64_t m;
  int32_t ell;
  double* U;
  double* lambda;
} nys_precond;

/* ---------------------------------------------------------------- handle */

/* Create a handle on HIP device `device`, enqueuing on `hip_stream`
   (a hipStream_t; NULL = the null stream).  Returns NYS_EINVAL / NYS_EHIP. */
int nys_create(nys_handle* h, int device, void* hip_stream);
int nys_destroy(nys_handle h);
/* Enqueue later work on `hip_stream`.  Synchronises the handle's current
   stream first (work queued there may still use the handle's workspace). */
int nys_set_stream(nys_handle h, void* hip_stream);
const char* nys_last_error(nys_handle h);
/* Milliseconds of GPU time spent in the last call, split as in the paper's
   time breakdown (section 5.2.3): preconditioner construction, PCG, other.
   Valid after ipm_solve / ipm_adjoint; otherwise zeros. */
int nys_last_timing(nys_handle h, double* t_sketch_ms, double* t_pcg_ms, double* t_other_ms);

/* Optional kernel timing with HIP events recorded on the handle's stream
   around every launch of the kernel classes below (for roofline reports).
   nys_profile_enable(h, 1) resets the counters and starts recording;
   nys_profile_read returns launches and summed milliseconds for one class
   (it waits for the recorded events).  Classes: */
enum {
  NYS_K_NORMAL_PASS1 = 0,  /* w = d .* (A^T v): one full read of A            */
  NYS_K_NORMAL_PASS2 = 1,  /* out = A w + ...: one full read of A             */
  NYS_K_SKETCH_W = 2,      /* BF16 matrix-core W = d .* (A^T Omega)           */
  NYS_K_SKETCH_Y = 3,      /* BF16 matrix-core Y = A W                        */
  NYS_K_GEMM_F64 = 4,      /* FP64 tiles (FP64 sketch, Gram, Cholesky-QR)     */
  NYS_K_NCLASSES = 5
};
int nys_profile_enable(nys_handle h, int enable);
int nys_profile_read(nys_handle h, int kernel_class, int64_t* launches, double* total_ms);

/* Read-stream reference for roofline reports (not a step of the method):
   reads `bytes` (a multiple of 16; data 16-byte aligned) with the same
   16-byte non-temporal loads as the normal-equation passes, in their shape
   (each block streams a few rows side by side), once in each of four shapes
   (rows of 40 or 80 KB, four or eight per block), and returns in *ms the
   device time of the fastest read (the call synchronises).  NYS_EINVAL on a
   bad size or alignment. */
int nys_stream_read(nys_handle h, const void* data, int64_t bytes, double* ms);

/* ---------------------------------------------------------------- operators */

/* out = (A diag(d) A^T + delta I) v : the regularised normal-equation operator
   N + delta I of eq. normal-eq with d = (Q + Theta^{-1} + rho I)^{-1}.
   Two passes over A: w = d .* (A^T v), then out = A w + delta v.
   d: n FP64 (>= 0 is not checked here: any d gives the product), v, out: m
   FP64, out must not alias v.  Enqueue only. */
int nys_normal_apply(nys_handle h, const nys_matrix* A, const double* d, double delta,
                     const double* v, double* out);

/* Storage layout helper for nys_matrix.data_t (not a step of the method):
   out (n x m row-major, leading dimension ld_out >= m elements, A's dtype,
   caller-owned, must not overlap A) = A^T, so that A^T v products stream
   whole rows.  Elements m .. ld_out-1 of each row are left untouched.  Rows
   whose pitch is a multiple of 128 bytes stream fastest (the copies the
   library makes use that pitch).
   NYS_EINVAL on bad arguments or m > 4194240.  Enqueue only. */
int nys_transpose(nys_handle h, const nys_matrix* A, void* out, int64_t ld_out);

/* Gaussian test matrix (Algorithm 1, first step): out (m x ell FP64,
   row-major) = standard normals from Philox4x32-10 keyed by `seed`, with the
   64-bit draw `counter`; entry e = i*ell + j uses the pair index e/2 as the
   counter's low half and Box-Muller on the four outputs.  Enqueue only. */
int nys_test_matrix(nys_handle h, int64_t m, int32_t ell, uint64_t seed, uint64_t counter,
                    double* out);

/* Sketch tiles: A_d (m x n, any storage dtype) in the layout the BF16
   matrix-core sketch streams best.  transposed = 0: the tiles of A_d (its m
   rows, k along n); 1: the tiles of A_d^T (n rows, k along m).  Stage kb
   (k = 32 kb .. 32 kb + 31) of row r is 64 bytes at offset (kb * Rp + r) * 64,
   Rp = rows rounded up to 256; the four 16-byte chunks of such a row are
   permuted among themselves, the same way in every stage; entries past the
   matrix are zero.  Values are BF16, rounded to nearest even (FP64 through
   FP32).  nys_sketch_tiles_bytes gives the size; out: caller-owned device
   buffer of that size, 16-byte aligned.  NYS_EINVAL on bad arguments or
   n > 16776960.  Enqueue only. */
int nys_sketch_tiles_bytes(int64_t m, int64_t n, int transposed, int64_t* bytes);
int nys_sketch_tiles(nys_handle h, const nys_matrix* A, int transposed, void* out);

/* The sketch Y = N Omega = A diag(d) A^T Omega of Algorithm 1 (second step),
   as the product pair W = d .* (A^T Omega), Y = A W.  omega: m x ell FP64
   row-major (used as given); Y: m x ell FP64 row-major, caller-owned.
   sketch_dtype NYS_F64: FP64 arithmetic, A stored FP64 or FP32.
   NYS_BF16: A stored BF16; Omega and W are rounded to BF16 (round to nearest
   even, through FP32) and both products run on matrix cores with FP32
   accumulation; Y's split partial sums are added in FP64.  A BF16
   transposed copy in A->data_t, or sketch tiles in A->tiles / A->tiles_t
   (then A may be stored FP32 or FP64: the tiles hold its BF16 values), give
   both products k-contiguous operands (same arithmetic; the tiles stream
   best).  Enqueue only. */
int nys_sketch_product(nys_handle h, const nys_matrix* A, const double* d, const double* omega,
                       int32_t ell, nys_dtype sketch_dtype, double* Y);

/* Randomized Nystrom approximation of N = A diag(d) A^T (Algorithm 1; the
   sketched matrix is N, not N + delta I) and the data of the Nystrom
   preconditioner (Algorithm 2).
   Omega = omega (m x ell FP64) if non-NULL, else nys_test_matrix(seed,
   counter); Omega is orthonormalised by a thin QR; Y = N Omega computed as
   W = d .* (A^T Omega), Y = A W, in FP64 (sketch_dtype NYS_F64, A must then be
   FP64 or FP32) or on BF16 matrix cores with FP32 accumulation (NYS_BF16;
   A must then be BF16 storage or carry sketch tiles of A and A^T, see
   nys_sketch_tiles); nu = c_nu * eps(||Y||_F) in the sketch
   precision; Y_nu = Y + nu Omega; C = chol(Omega^T Y_nu) (upper, C^T C = G);
   B = Y_nu C^{-1}; thin SVD of B by Cholesky-QR and a one-sided Jacobi SVD of
   the triangular factor; U_hat = left singular vectors, Lambda_hat =
   max(0, Sigma^2 - nu), descending.  On a failed Cholesky nu grows by 10x, up
   to 6 times, then NYS_ENOTPD.
   P->m must equal A->m, 1 <= P->ell <= m; P->U, P->lambda are caller buffers.
   nu_out (host, may be NULL) receives the final shift.  Synchronises. */
int nys_sketch(nys_handle h, const nys_matrix* A, const double* d, int32_t ell,
               uint64_t seed, uint64_t counter, nys_dtype sketch_dtype,
               const double* omega_or_null, nys_precond* P, double* nu_out);

/* out = P^{-1} r with eq. Nys_precond_inv:
   P^{-1} = (lambda_ell + delta) U (Lambda + delta I)^{-1} U^T + (I - U U^T).
   delta > 0.  r, out: m FP64, may not alias.  Enqueue only. */
int nys_precond_apply(nys_handle h, const nys_precond* P, double delta, const double* r,
                      double* out);

/* ---------------------------------------------------------------- PCG */

typedef struct {
  double rtol;            /* stop when ||rhs - M y|| <= max(rtol ||rhs||, atol) */
  double atol;
  int32_t maxit;          /* <= 0: max(m, 2000)                                  */
  int32_t replace_every;  /* FP64 true-residual replacement period; <= 0: 100    */
  int32_t poll_every;     /* host convergence poll period; <= 0: 8               */
} nys_pcg_opts;

typedef struct {
  int32_t iters;
  int32_t status;         /* NYS_OK, NYS_MAXIT or NYS_EBREAKDOWN                 */
  double true_res;        /* ||rhs - M y||_2 recomputed at exit                  */
  double rel_res;         /* true_res / ||rhs||_2                                */
} nys_pcg_info;

/* Preconditioned CG (section 2.2) on (A diag(d) A^T + delta I) y = rhs with
   the Nystrom preconditioner P (NULL: plain CG).  y holds the initial guess on
   entry (NULL-equivalent: pass zeros) and the solution on exit.  The stopping
   test is on the true residual; the recursion is refreshed with an
   FP64-accumulated true residual every replace_every iterations.
   Returns NYS_OK, NYS_MAXIT (warning, last iterate in y) or NYS_EBREAKDOWN.
   Synchronises. */
int nys_pcg_solve(nys_handle h, const nys_matrix* A, const double* d, double delta,
                  const nys_precond* P, const double* rhs, double* y,
                  const nys_pcg_opts* opts, nys_pcg_info* info);

/* Allocation-free nys_pcg_solve, for callers that cannot allocate device
   memory (code under HIP graph capture, tight serving loops, harnesses that
   forbid hipMalloc).  Same arguments, kernels, results (bit for bit) and
   return codes as nys_pcg_solve with the Nystrom preconditioner or none.
   Instead of the handle's workspace it uses a fixed scratch array of
   NYS_NOALLOC_SCRATCH_BYTES in device memory, one per GPU, held from the
   first nys_create on that GPU until the process ends; it calls no hipMalloc
   or hipFree.  The scratch holds the PCG vectors (6m + ell FP64), the n + n_unit
   FP64 vector of pass 1 and the partial sums of the reductions; every word a
   call reads is written by that call first, so nothing needs clearing, and a
   call leaves its last values there.  A call needs about
   m (48 + (ell + 1) / 8) + 8 (n + n_unit) bytes of it (the PCG vectors, pass
   1's vector and the preconditioner's partial sums), plus partial sums of
   pass 1 when A has no transposed copy; sizes above the scratch are refused
   with NYS_EINVAL before anything is launched (m = 20000, n = 100000,
   ell = 200 needs 2.3 MB).  All calls on one GPU share its scratch: two
   calls that overlap in time on the same GPU (two handles, two streams, two
   threads) race and give undefined results; serialise them.  Synchronises. */
#define NYS_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
int nys_pcg_solve_noalloc(nys_handle h, const nys_matrix* A, const double* d, double delta,
                          const nys_precond* P, const double* rhs, double* y,
                          const nys_pcg_opts* opts, nys_pcg_info* info);

/* ------------------------------------------------ comparator: partial Cholesky */

/* Partial Cholesky preconditioner of N + delta I, N = A diag(d) A^T (section
   "Partial Cholesky preconditioners", eq. partialCholeskyfact and
   eq. chol-precond; the preconditioner of the paper's Chol-IP-PMM
   comparator).  The pivots are the ell largest diagonal entries of
   N + delta I (ties: smaller index); with E moving them first,
   E (N + delta I) E^T = [L11 0; L21 I] [I 0; 0 S] [L11^T L21^T; 0 I] and S is
   replaced by diag(S).  Caller-owned device buffers, sizes from m and ell
   (1 <= ell <= m):
     piv   ell int32: pivot rows, ascending
     pos   m int32: pos[i] = k when i = piv[k], else -1
     L     m x ell FP64 row-major: [L11; L21] in the original row order (row
           piv[k] holds row k of L11, every other row its row of L21)
     Cinv  ell x ell FP64 row-major, upper triangular: L11^{-T}
     diagS m FP64: diag(S) on the rows that are not pivots, 1 on pivots */
typedef struct {
  int64_t m;
  int32_t ell;
  int32_t* piv;
  int32_t* pos;
  double* L;
  double* Cinv;
  double* diagS;
} nys_pchol;

/* Builds P for N + delta I (delta > 0; d >= 0, n FP64).  The diagonal is
   sum_j A_ij^2 d_j + delta (entrywise access to A, as in the paper's
   experiments).  NYS_ENOTPD if the pivot block's Cholesky fails.
   Synchronises. */
int nys_pchol_build(nys_handle h, const nys_matrix* A, const double* d, double delta, nys_pchol* P);

/* out = P_Chol^{-1} r by eq. chol-precond-inv; r, out: m FP64, no aliasing.
   Enqueue only. */
int nys_pchol_apply(nys_handle h, const nys_pchol* P, const double* r, double* out);

/* nys_pcg_solve with the partial Cholesky preconditioner (P built for the
   same d and delta). */
int nys_pcg_solve_pchol(nys_handle h, const nys_matrix* A, const double* d, double delta,
                        const nys_pchol* P, const double* rhs, double* y,
                        const nys_pcg_opts* opts, nys_pcg_info* info);

/* One Newton direction of IP-PMM for non-negative variables (Algorithm 5 with
   F = J = empty; eq. normal-eq, delta_x, delta_z):
   D = (Q + Z X^{-1} + rho I)^{-1}; xi_au = -X^{-1} r_xz;
   xi = r_p + A D (r_d + xi_au); PCG for (A D A^T + delta I) dy = xi;
   dx = D (A^T dy - r_d - xi_au); dz = X^{-1} (r_xz - Z dx).
   x, z > 0 and q >= 0 (n), rho >= 0, delta > 0; P may be NULL.  Outputs dx,
   dz (n), dy (m).  Synchronises. */
int nys_newton_solve(nys_handle h, const nys_matrix* A, const double* q, const double* x,
                     const double* z, double rho, double delta, const nys_precond* P,
                     const double* r_d, const double* r_p, const double* r_xz,
                     const nys_pcg_opts* opts, double* dx, double* dy, double* dz,
                     nys_pcg_info* info);

/* ---------------------------------------------------------------- IP-PMM */

/* Kinds of variables (section "Free and box-constrained variables"): the
   problem (P~) has x_F free, x_I >= 0 and 0 <= x_J <= u_J. */
enum { NYS_VAR_NONNEG = 0, NYS_VAR_FREE = 1, NYS_VAR_BOX = 2 };

typedef struct {
  const nys_matrix* A;      /* problem-defining matrix (FP64 or FP32 storage)   */
  const nys_matrix* A_lo;   /* BF16 copy for the sketch, or NULL                */
  const double* b;          /* m */
  const double* c;          /* n */
  const double* q;          /* n, diag(Q) >= 0 */
  const int8_t* vtype;      /* n NYS_VAR_* kinds, or NULL: every x_j >= 0       */
  const double* u;          /* n upper bounds (read where vtype is BOX; > 0 and
                               finite there), or NULL when vtype is NULL       */
} nys_qp;

/* Sketch size per IP-PMM iteration (options ell_rule; section "Convergence
   analysis of Nys-IP-PMM": the main theorem asks for ell_k of order
   d_eff(N_k, mu_k), eq. main-thm-sketch-size, with d_eff of eq. effective-dim).
   d_eff(N_k, mu_k) is estimated from the eigenvalues lambda_hat (descending)
   of the most recent Nystrom approximation at the current mu_k:
   d_hat = sum_i lambda_hat_i / (lambda_hat_i + mu_k) (a lower estimate: the
   Nystrom approximation lies below N in the Loewner order).
     NYS_ELL_FIXED    ell_k = ell (the paper's experiments).
     NYS_ELL_DEFF     target = ceil(c_ell d_hat); when lambda_hat_ell > mu_k
                      also target >= 2 ell_prev (that sketch saw no eigenvalue
                      below mu_k); ell_k = min(ell_max, max(ell_min, target)).
     NYS_ELL_THEOREM  target = ceil(8 (sqrt(d_hat) + sqrt(32 ln(16 (k+2))))^2),
                      clamped the same way (the bound itself is >= 887).
   The first iteration's d_hat comes from the initial point's sketch of A A^T. */
enum { NYS_ELL_FIXED = 0, NYS_ELL_DEFF = 1, NYS_ELL_THEOREM = 2 };

/* Fields of one record of the per-iteration trace (nys_ipm_opts.trace), all
   stored as double: */
enum {
  NYS_TR_K = 0,        /* IP-PMM iteration                                    */
  NYS_TR_MU,           /* mu_k                                                */
  NYS_TR_DELTA,        /* delta_k (= rho_k)                                   */
  NYS_TR_ELL,          /* size of the preconditioner used at k (0: plain CG)  */
  NYS_TR_BUILT,        /* 1 when the preconditioner was built at k, else 0    */
  NYS_TR_DHAT,         /* d_hat of that Nystrom preconditioner at mu_k (NaN
                          for the other preconditioners)                      */
  NYS_TR_LAMLAST,      /* its smallest eigenvalue lambda_hat_ell (NaN likewise) */
  NYS_TR_PCG,          /* PCG iterations at k, predictor plus corrector       */
  NYS_TR_RULE_DHAT,    /* inputs of the sketch-size rule when it chose ell at k:
                          d_hat and lambda_hat_ell of the previous Nystrom
                          preconditioner at mu_k (NaN when no rule ran)       */
  NYS_TR_RULE_LAMLAST,
  NYS_TR_RP,           /* rp_rel, rd_rel of the stopping test at iteration k  */
  NYS_TR_RD,
  NYS_TR_TIME_MS,      /* milliseconds from entry to that test                */
  NYS_TRACE_FIELDS
};

typedef struct {
  double tol;               /* max(rp_rel, rd_rel, mu) target; <= 0: 1e-6      */
  int32_t max_iter;         /* IP-PMM iterations; <= 0: 100                     */
  int32_t ell;              /* sketch size, 1 <= ell <= m                        */
  uint64_t seed;            /* Philox key of the test matrices                  */
  nys_dtype sketch_dtype;   /* NYS_F64 or NYS_BF16 (needs A_lo or converts A)   */
  double c_nu;              /* shift constant of the sketch; <= 0: 1             */
  nys_pcg_opts pcg;
  int32_t verbose;          /* 1: one line per iteration on stderr              */
  int32_t no_transposed_copy; /* 1: never copy A^T into the workspace         */
  int32_t precond;          /* NYS_PRECOND_*: the inner solver's preconditioner */
  /* sketch size per iteration (NYS_ELL_*; anything but FIXED needs the
     Nystrom preconditioner).  ell is the initial size.                        */
  int32_t ell_rule;
  int32_t ell_min;          /* lower clamp; <= 0: min(8, ell)                    */
  int32_t ell_max;          /* upper clamp, <= m; <= 0: min(m, 4 ell).  The
                               workspace holds an m x ell_max basis.            */
  double c_ell;             /* factor of NYS_ELL_DEFF; <= 0: 2                   */
  /* reuse of the preconditioner across iterations (the paper names it as a
     further improvement without a rule; this one is ours): 0 builds it anew at
     every iteration.  a > 0 builds it at the first iteration and afterwards at
     iteration k only when k - k_build >= a, or when the PCG iterations of
     iteration k-1 exceed reuse_growth times those of iteration k_build; a
     kept Nystrom preconditioner is applied with the current delta_k, a kept
     partial Cholesky factor as built.                                         */
  int32_t reuse_max_age;
  double reuse_growth;      /* <= 0: 1.5                                         */
  double* trace;            /* host, caller-owned: NULL, or trace_len records of
                               NYS_TRACE_FIELDS doubles, one per IP-PMM
                               iteration that reaches the Newton solve (later
                               iterations are not recorded)                    */
  int32_t trace_len;
  /* The direction of the predictor-corrector scheme (Algorithm 6) is the sum
     of the predictor and corrector steps.  0 (default): it is computed as one
     solve with the summed right-hand side (r_d, r_p, r_u of the predictor,
     R_xz = -XZ + mu~ - dx_p dz_p, R_ws likewise), started from the
     predictor's dy and run to the inner tolerance.  With exact solves this
     equals the sum of the two solves (linearity).  The predictor itself is
     solved only to a relative residual of predictor_rtol (<= 0: 2e-3) or the
     usual inner tolerance, whichever is looser; its error then enters the
     predictor step lengths, mu_aff, mu~ and dx_p dz_p of the corrector's
     right-hand side, so the default iterates differ from Algorithm 6's (they
     reach the same optimum).  A predictor_rtol at the inner tolerance gives
     Algorithm 6's iterates.  1: the two solves as printed, both to the inner
     tolerance, then added.                                                    */
  int32_t separate_corrector;
  double predictor_rtol;
  /* inner tolerance of the Newton solves: ||xi - M dy|| <= max(f mu,
     f tol (1 + ||b||)) (capped at pcg.rtol ||xi||, 1e-2 by default, and
     floored at 1e-12 ||xi||), with f = inner_factor in (0, 1); else 0.9    */
  double inner_factor;
} nys_ipm_opts;

typedef struct {
  int32_t iters, pcg_iters_total, status;
  double kkt_rel, rp_rel, rd_rel, mu, rho, delta;
  double t_sketch_ms, t_pcg_ms, t_other_ms;
  double ru_rel;            /* ||u_J - x_J - w_J|| / (1 + ||u_J||) (box variables) */
  double deff_last;         /* d_hat of the last Nystrom preconditioner at its
                               build iteration's mu (NaN otherwise)             */
  int32_t builds;           /* preconditioners built in the IP-PMM iterations  */
  int32_t ell_last;         /* size of the last one                            */
} nys_ipm_info;

/* Nys-IP-PMM (Algorithm 4 with the predictor-corrector of Algorithm 6 and the
   Newton solve of Algorithm 5) for (P): initial point from the regularised
   (A A^T + 10 I) systems solved by Nystrom-PCG; rho_0 = delta_0 = 8; per
   iteration a fresh Nystrom preconditioner of N_k shared by predictor and
   corrector (see ell_rule and reuse_max_age for the alternatives); the
   direction by one solve of the summed predictor and corrector systems (see
   separate_corrector); Newton solves to ||xi - M dy|| <= inner_factor *
   max(mu, tol (1 + ||b||)); step lengths with factor 0.995; parameter update
   rho = delta = max(5e-10, min(rho, mu)); stop when
   max(||r_p||/(1+||b||), ||r_d||/(1+||c||), mu) <= tol.
   Outputs x, z (n) and y (m) FP64.  Returns NYS_OK, NYS_MAXIT, or an error.
   With qp->vtype set this solves (P~) as ipm_solve_box does, keeping w and s
   internal.  Synchronises. */
int ipm_solve(nys_handle h, const nys_qp* qp, const nys_ipm_opts* opts, double* x, double* y,
              double* z, nys_ipm_info* info);

/* The same method for (P~)/(D~) with free, non-negative and box-constrained
   variables (qp->vtype, qp->u; section "Free and box-constrained variables"):
   Theta^{-1}_jj = z_j/x_j (I), z_j/x_j + s_j/w_j (J), 0 (F); the Newton
   direction of Algorithm 5 with xi_au by index kind and
   dz = X^{-1}(r_xz - Z dx), dw_J = (r_u)_J - dx_J, ds = W^{-1}(r_ws - S dw);
   the supplement's initial point (x~ centred at u/2) and step lengths over
   (x_IJ, w_J) and (z_IJ, s_J); mu = (x_IJ^T z_IJ + w_J^T s_J)/(|IJ| + |J|);
   stop when max(rp_rel, rd_rel, ||r_u||/(1+||u_J||), mu) <= tol with
   r_d = c + Q x - A^T y - z + s.  Outputs x, z, w, s (n; z_F = 0, w and s
   zero off J) and y (m).  w, s may be NULL.  Synchronises. */
int ipm_solve_box(nys_handle h, const nys_qp* qp, const nys_ipm_opts* opts, double* x, double* y,
                  double* z, double* w, double* s, nys_ipm_info* info);

/* Adjoint of the converged KKT system (not in the paper; derived from the
   optimality conditions of (P)/(D)).  With g = dL/dx at the solution (x, y, z)
   returned by ipm_solve with final parameters (rho, delta):
   D_j = 0 where x_j <= z_j (inactive), else max(q_j, rho)^{-1} (the exact
   Q_S^{-1} of the converged system: the iterate's barrier term z_j/x_j, zero at
   the optimum, is left out, and only curvature below rho -- zero-curvature
   columns included -- is floored at rho);
   (A D A^T + delta I) u2 = A (D g) by Nystrom-PCG (rtol from opts->pcg, 1e-10
   when <= 0; iteration cap max(m, 20000) when opts->pcg.maxit <= 0);
   u1 = D (g - A^T u2);
   grad_c = -u1, grad_b = u2, grad_q = -u1 .* x, grad_A = y u1^T - u2 x^T.
   Any output pointer may be NULL (skipped); grad_A is m x n row-major FP64
   with leading dimension n.  Returns the PCG status (NYS_MAXIT = the adjoint
   solve did not reach its tolerance; gradients from the last iterate).
   Problems with free or box-constrained variables (qp->vtype set) are
   rejected with NYS_EINVAL.  One sketch of size opts->ell; the sketch-size
   rule, reuse and trace fields of opts are not used.  Synchronises. */
int ipm_adjoint(nys_handle h, const nys_qp* qp, const nys_ipm_opts* opts, const double* x,
                const double* y, const double* z, double rho, double delta, const double* g,
                double* grad_c, double* grad_b, double* grad_q, double* grad_A,
                nys_pcg_info* info);

/* The estimate d_hat = sum_i lambda[i] / (lambda[i] + mu) of the effective
   dimension d_eff(N, mu) (eq. effective-dim) from the ell eigenvalues lambda
   (device, FP64, >= 0) of a Nystrom approximation of N; *out_host receives it.
   Needs 1 <= ell, mu > 0, lambda and out_host non-NULL.  Synchronises. */
int nys_deff_estimate(nys_handle h, const double* lambda, int32_t ell, double mu, double* out_host);

/* The sketch size of the preconditioner built at IP-PMM iteration k under rule
   (NYS_ELL_*, defined above), from d_hat, the previous preconditioner's
   smallest eigenvalue lam_last, mu_k, its size ell_prev, the clamps
   1 <= ell_min <= ell_max and c_ell > 0.  Host only, no handle.  Returns the
   size, or NYS_EINVAL for a bad rule or bad clamps; a d_hat that is NaN or
   infinite gives ell_max. */
int nys_sketch_size_rule(int32_t rule, double d_hat, double lam_last, double mu, int32_t k,
                         int32_t ell_prev, int32_t ell_min, int32_t ell_max, double c_ell);

/* The reuse rule of nys_ipm_opts.reuse_max_age: 1 when the preconditioner is
   built anew at IP-PMM iteration k, else 0.  k_build < 0: none built yet (1);
   max_age <= 0: no reuse (1); otherwise 1 when k - k_build >= max_age or
   pcg_prev > growth * pcg_ref (the PCG iterations of iterations k-1 and
   k_build).  Host only, no handle. */
int nys_precond_rebuild_due(int32_t k, int32_t k_build, int32_t pcg_prev, int32_t pcg_ref,
                            int32_t max_age, double growth);

#ifdef __cplusplus
}
#endif

#endif /* NYSIPM_H */
