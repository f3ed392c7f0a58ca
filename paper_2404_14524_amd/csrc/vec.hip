// Vector kernels: BLAS-1 helpers, data validation, the Nystrom
// preconditioner apply (eq. Nys_precond_inv) and the fused PCG updates.

#include <cmath>

#include "common.hpp"
#include "kernels.hpp"
#include "mapreduce.hpp"

namespace nys {
namespace {

struct FillF {
  double* x;
  double v;
  __device__ void operator()(int64_t j, double*, double*) const { x[j] = v; }
};
struct CopyF {
  double* d;
  const double* s;
  __device__ void operator()(int64_t j, double*, double*) const { d[j] = s[j]; }
};
struct AxpbyF {
  double* d;
  double a, b;
  const double* x;
  const double* y;
  __device__ void operator()(int64_t j, double*, double*) const {
    d[j] = a * x[j] + (y ? b * y[j] : 0.0);
  }
};
struct DotF {
  const double* x;
  const double* y;
  __device__ void operator()(int64_t j, double* s, double*) const { s[0] = fma(x[j], y[j], s[0]); }
};
struct SumsqF {
  const double* x;
  __device__ void operator()(int64_t j, double* s, double*) const { s[0] = fma(x[j], x[j], s[0]); }
};
struct BadF {
  const double* x;
  __device__ void operator()(int64_t j, double* s, double*) const {
    const double v = x[j];
    if (!isfinite(v)) s[0] += 1.0;
    if (v < 0.0) s[1] += 1.0;
  }
};

template <class T>
__global__ __launch_bounds__(NYS_BLOCK) void k_nonfinite(const char* A, int64_t m, int64_t n,
                                                         int64_t row_bytes, double* part) {
  using raw = typename T::raw;
  __shared__ double smem[NYS_BLOCK / NYS_WAVE];
  double c[1] = {0.0};
  for (int64_t i = blockIdx.x; i < m; i += gridDim.x) {
    const raw* row = (const raw*)(A + i * row_bytes);
    for (int64_t j = threadIdx.x; j < n; j += NYS_BLOCK)
      if (!isfinite(to_f64(row[j]))) c[0] += 1.0;
  }
  block_sum<1>(c, smem);
  if (threadIdx.x == 0) part[blockIdx.x] = c[0];
}

// Read-stream reference: the buffer read once with the 16-byte non-temporal
// loads of the GEMV passes, in their shape: each block streams RB rows of
// ROWB bytes side by side, every thread keeping one load per row in flight (a
// wave covers 1 KB of a row per load); the words are XOR-folded so that the
// reads cannot be elided.  A tail shorter than a block is read by the last
// block piece by piece.  The spacing of a block's rows matters on HBM3E
// (rows 80 KB apart stream faster than 64 or 100 KB apart), so the reference
// is the fastest of a few shapes (SR_SHAPES).
template <int64_t ROWB, int RB>
__global__ __launch_bounds__(NYS_BLOCK) void k_stream_read(const char* p, int64_t n16, unsigned* part) {
  constexpr int64_t ROW16 = ROWB / 16;
  const int64_t r0 = (int64_t)blockIdx.x * RB;
  const int64_t nrows = n16 / ROW16;
  unsigned acc = 0u;
  if (r0 + RB <= nrows) {
    const char* base = p + r0 * ROWB;
    for (int64_t c = threadIdx.x; c < ROW16; c += NYS_BLOCK) {
      u32x4 u[RB];
#pragma unroll
      for (int r = 0; r < RB; ++r) u[r] = ld_stream16(base + r * ROWB + 16 * c);
#pragma unroll
      for (int r = 0; r < RB; ++r) acc ^= u[r].x ^ u[r].y ^ u[r].z ^ u[r].w;
    }
  } else {
    for (int64_t i = r0 * ROW16 + threadIdx.x; i < n16; i += NYS_BLOCK) {
      const u32x4 v = ld_stream16(p + 16 * i);
      acc ^= v.x ^ v.y ^ v.z ^ v.w;
    }
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) acc ^= __shfl_xor(acc, off, NYS_WAVE);
  if ((threadIdx.x & (NYS_WAVE - 1)) == 0) part[blockIdx.x * (NYS_BLOCK / NYS_WAVE) + threadIdx.x / NYS_WAVE] = acc;
}

struct SrShape {
  int64_t row_bytes;
  int rb;
};
constexpr SrShape SR_SHAPES[] = {{80 * 1024, 8}, {40 * 1024, 8}, {80 * 1024, 4}, {40 * 1024, 4}};
constexpr int SR_NSHAPES = sizeof(SR_SHAPES) / sizeof(SR_SHAPES[0]);

// ---------------------------------------------------------------- PCG / P^{-1}
// Every reduction below is two launches: per-block partials, then a one-block
// kernel that combines them in block order (deterministic) and advances the
// scalar recurrences held in device words.
// Rows per block of the update/reduce kernel (one row per thread in phase 1).
constexpr int RBU = 64;

struct UpdArgs {
  int64_t m;
  int ell;
  double* y;            // UPDATE: y += alpha p
  double* r;            // UPDATE: r -= alpha q (else read only)
  const double* p;
  const double* q;
  const double* U;      // PRECOND: m x ell
  const double* lam;
  double delta;
  double* t;            // PRECOND: ell-vector result
  double* scal;         // device scalar block
  double* part;         // per block: ell partial sums of U^T r, then ||r||^2
  int ext;              // a separate preconditioner sets rs and beta (no-PRECOND form)
};

// alpha = rs/pq, zero once done; breakdown when pq <= 0 or alpha not finite.
__device__ __forceinline__ double pcg_alpha(const double* scal, bool* done0, bool* brk) {
  *done0 = scal[SC_DONE] != 0.0;
  *brk = false;
  if (*done0) return 0.0;
  const double pq = scal[SC_PQ], rs = scal[SC_RS];
  const double al = rs / pq;
  if (!(pq > 0.0) || !isfinite(al)) {
    *brk = true;
    return 0.0;
  }
  return al;
}

// UPDATE:  y += alpha p; r -= alpha q.
// PRECOND: partial sums of U^T r over this block's rows.
// Always:  partial ||r||^2.
template <bool UPDATE, bool PRECOND>
__global__ __launch_bounds__(NYS_BLOCK) void k_pcg_update(UpdArgs a) {
  __shared__ double rl[RBU];
  __shared__ double smem[NYS_BLOCK / NYS_WAVE];
  const int64_t r0 = (int64_t)blockIdx.x * RBU;
  const int nr = (int)min((int64_t)RBU, a.m - r0);
  double alpha = 0.0;
  if constexpr (UPDATE) {
    bool done0, brk;
    alpha = pcg_alpha(a.scal, &done0, &brk);
  }
  double rr[1] = {0.0};
  if (threadIdx.x < nr) {
    const int64_t i = r0 + threadIdx.x;
    double ri = a.r[i];
    if constexpr (UPDATE) {
      if (alpha != 0.0) {
        a.y[i] = fma(alpha, a.p[i], a.y[i]);
        ri = fma(-alpha, a.q[i], ri);
        a.r[i] = ri;
      }
    }
    rl[threadIdx.x] = ri;
    rr[0] = ri * ri;
  }
  __syncthreads();
  block_sum<1>(rr, smem);
  const int ell = PRECOND ? a.ell : 0;
  if constexpr (PRECOND) {
    for (int k = threadIdx.x; k < ell; k += NYS_BLOCK) {
      double acc = 0.0;
      const double* u = a.U + r0 * ell + k;
      for (int i = 0; i < nr; ++i) acc = fma(u[(int64_t)i * ell], rl[i], acc);
      a.part[(int64_t)blockIdx.x * (ell + 1) + k] = acc;
    }
  }
  if (threadIdx.x == 0) a.part[(int64_t)blockIdx.x * (ell + 1) + ell] = rr[0];
}

// One block per column of the partials (ell + 1 blocks).  Block k < ell:
// t_k = f_k * sum_b part[b][k], f_k = (lam_ell + delta)/(lam_k + delta) - 1 with
// lam_ell the last (smallest) entry of the descending lambda.  Block ell:
// ||r||^2 -> SC_RR; UPDATE: iteration count, done when ||r||^2 <= tol2,
// breakdown flag; without a preconditioner also rs = ||r||^2 and
// beta = rs_new/rs (zero once done).
template <bool UPDATE, bool PRECOND>
__global__ __launch_bounds__(NYS_BLOCK) void k_pcg_update_finish(UpdArgs a, int nb) {
  __shared__ double smem[NYS_BLOCK / NYS_WAVE];
  const int ell = PRECOND ? a.ell : 0;
  const int col = blockIdx.x;
  double s1[1] = {0.0};
  for (int b = threadIdx.x; b < nb; b += NYS_BLOCK) s1[0] += a.part[(int64_t)b * (ell + 1) + col];
  block_sum<1>(s1, smem);
  if constexpr (PRECOND) {
    if (col < ell) {
      if (threadIdx.x == 0) {
        const double laml = a.lam[ell - 1];
        a.t[col] = ((laml + a.delta) / (a.lam[col] + a.delta) - 1.0) * s1[0];
      }
      return;
    }
  }
  if (threadIdx.x == 0) {
    const double rrt = s1[0];
    a.scal[SC_RR] = rrt;
    if constexpr (UPDATE) {
      bool done0, brk;
      (void)pcg_alpha(a.scal, &done0, &brk);
      if (!done0) a.scal[SC_ITERS] += 1.0;
      if (brk) {
        a.scal[SC_BREAK] = 1.0;
        a.scal[SC_DONE] = 1.0;
      } else if (!done0 && rrt <= a.scal[SC_TOL2]) {
        a.scal[SC_DONE] = 1.0;
      }
      if (!PRECOND && !a.ext) {
        const bool dn = a.scal[SC_DONE] != 0.0;
        const double rs = a.scal[SC_RS];
        a.scal[SC_BETA] = dn ? 0.0 : rrt / rs;
        a.scal[SC_RS] = rrt;
      }
    }
  }
}

struct ExpArgs {
  int64_t m;
  int ell;
  const double* U;
  const double* r;
  const double* t;
  double* out;
  double* scal;         // PCG: rs_new, beta (else NULL)
  double* dot_out;      // standalone dot (may be NULL)
  double* part;
};

// out_i = r_i + sum_k U[i,k] t_k (one wave per row); per-block partial r^T out.
__global__ __launch_bounds__(NYS_BLOCK) void k_precond_expand(ExpArgs a) {
  extern __shared__ double tl[];
  __shared__ double smem[NYS_BLOCK / NYS_WAVE];
  for (int k = threadIdx.x; k < a.ell; k += NYS_BLOCK) tl[k] = a.t[k];
  __syncthreads();
  const int lane = threadIdx.x & (NYS_WAVE - 1);
  const int wid = threadIdx.x / NYS_WAVE;
  const int64_t wstride = (int64_t)gridDim.x * (NYS_BLOCK / NYS_WAVE);
  double dotc[1] = {0.0};
  for (int64_t i = (int64_t)blockIdx.x * (NYS_BLOCK / NYS_WAVE) + wid; i < a.m; i += wstride) {
    const double* u = a.U + i * a.ell;
    double acc = 0.0;
    for (int k = lane; k < a.ell; k += NYS_WAVE) acc = fma(u[k], tl[k], acc);
    acc = wave_sum(acc);
    if (lane == 0) {
      const double ri = a.r[i];
      const double o = ri + acc;
      a.out[i] = o;
      dotc[0] = fma(ri, o, dotc[0]);
    }
  }
  if (!a.scal && !a.dot_out) return;
  block_sum<1>(dotc, smem);
  if (threadIdx.x == 0) a.part[blockIdx.x] = dotc[0];
}

// One block: r^T s -> dot_out and/or (PCG) beta = rs_new/rs (zero once done), rs = rs_new.
__global__ __launch_bounds__(NYS_BLOCK) void k_precond_expand_finish(ExpArgs a, int nb) {
  __shared__ double smem[NYS_BLOCK / NYS_WAVE];
  double s[1] = {0.0};
  for (int b = threadIdx.x; b < nb; b += NYS_BLOCK) s[0] += a.part[b];
  block_sum<1>(s, smem);
  if (threadIdx.x == 0) {
    if (a.dot_out) *a.dot_out = s[0];
    if (a.scal) {
      const bool dn = a.scal[SC_DONE] != 0.0;
      const double rs = a.scal[SC_RS];
      a.scal[SC_BETA] = dn ? 0.0 : s[0] / rs;
      a.scal[SC_RS] = s[0];
    }
  }
}

unsigned expand_blocks(int64_t m) {
  int64_t b = (m + (NYS_BLOCK / NYS_WAVE) - 1) / (NYS_BLOCK / NYS_WAVE);
  if (b > 2048) b = 2048;
  if (b < 1) b = 1;
  return (unsigned)b;
}

int launch_update(nys_handle h, bool update, bool precond, UpdArgs& k) {
  const unsigned nb = (unsigned)std::max<int64_t>(1, (k.m + RBU - 1) / RBU);
  NYS_CHECK(ws(h, WS_PART, (size_t)nb * ((precond ? k.ell : 0) + 1), &k.part));
  k.scal = h->dscal;
  // finish: one block per column of the partials (ell entries of t, then ||r||^2)
  dim3 g(nb), b(NYS_BLOCK), fin((unsigned)((precond ? k.ell : 0) + 1));
  if (update && precond) {
    hipLaunchKernelGGL((k_pcg_update<true, true>), g, b, 0, h->stream, k);
    hipLaunchKernelGGL((k_pcg_update_finish<true, true>), fin, b, 0, h->stream, k, (int)nb);
  } else if (update) {
    hipLaunchKernelGGL((k_pcg_update<true, false>), g, b, 0, h->stream, k);
    hipLaunchKernelGGL((k_pcg_update_finish<true, false>), fin, b, 0, h->stream, k, (int)nb);
  } else if (precond) {
    hipLaunchKernelGGL((k_pcg_update<false, true>), g, b, 0, h->stream, k);
    hipLaunchKernelGGL((k_pcg_update_finish<false, true>), fin, b, 0, h->stream, k, (int)nb);
  } else {
    hipLaunchKernelGGL((k_pcg_update<false, false>), g, b, 0, h->stream, k);
    hipLaunchKernelGGL((k_pcg_update_finish<false, false>), fin, b, 0, h->stream, k, (int)nb);
  }
  NYS_LAUNCH_CHECK(h);
  return NYS_OK;
}

int launch_expand(nys_handle h, ExpArgs& k) {
  const unsigned nb = expand_blocks(k.m);
  NYS_CHECK(ws(h, WS_PART2, (size_t)nb, &k.part));
  hipLaunchKernelGGL(k_precond_expand, dim3(nb), dim3(NYS_BLOCK), (size_t)k.ell * sizeof(double),
                     h->stream, k);
  if (k.scal || k.dot_out)
    hipLaunchKernelGGL(k_precond_expand_finish, dim3(1), dim3(NYS_BLOCK), 0, h->stream, k, (int)nb);
  NYS_LAUNCH_CHECK(h);
  return NYS_OK;
}

}  // namespace

size_t update_part_doubles(int64_t m, int ell, bool precond) {
  const int64_t nb = std::max<int64_t>(1, (m + RBU - 1) / RBU);
  return (size_t)nb * (size_t)((precond ? ell : 0) + 1);
}

size_t expand_part_doubles(int64_t m) { return expand_blocks(m); }

int stream_read_shapes() { return SR_NSHAPES; }

int stream_read_blocks(int64_t bytes, int shape) {
  // full blocks of rb rows, plus one block for the tail
  const SrShape sh = SR_SHAPES[shape];
  return (int)(bytes / sh.row_bytes / sh.rb + 1);
}

int stream_read(nys_handle h, const void* data, int64_t bytes, unsigned* part, int shape) {
  const int nb = stream_read_blocks(bytes, shape);
  const char* p = (const char*)data;
  const int64_t n16 = bytes / 16;
  switch (shape) {
    case 0: hipLaunchKernelGGL((k_stream_read<80 * 1024, 8>), dim3((unsigned)nb), dim3(NYS_BLOCK), 0, h->stream, p, n16, part); break;
    case 1: hipLaunchKernelGGL((k_stream_read<40 * 1024, 8>), dim3((unsigned)nb), dim3(NYS_BLOCK), 0, h->stream, p, n16, part); break;
    case 2: hipLaunchKernelGGL((k_stream_read<80 * 1024, 4>), dim3((unsigned)nb), dim3(NYS_BLOCK), 0, h->stream, p, n16, part); break;
    default: hipLaunchKernelGGL((k_stream_read<40 * 1024, 4>), dim3((unsigned)nb), dim3(NYS_BLOCK), 0, h->stream, p, n16, part); break;
  }
  NYS_LAUNCH_CHECK(h);
  return NYS_OK;
}

int fill(nys_handle h, double* x, int64_t n, double value) {
  return map_reduce<0, 0>(h, n, FillF{x, value}, nullptr);
}
int copy(nys_handle h, double* dst, const double* src, int64_t n) {
  return map_reduce<0, 0>(h, n, CopyF{dst, src}, nullptr);
}
int axpby(nys_handle h, double* dst, double a, const double* x, double b, const double* y, int64_t n) {
  return map_reduce<0, 0>(h, n, AxpbyF{dst, a, b, x, y}, nullptr);
}
int dot(nys_handle h, const double* x, const double* y, int64_t n, double* out) {
  return map_reduce<1, 0>(h, n, DotF{x, y}, out);
}
int sumsq(nys_handle h, const double* x, int64_t count, double* out) {
  return map_reduce<1, 0>(h, count, SumsqF{x}, out);
}
int count_bad(nys_handle h, const double* x, int64_t n, double* out) {
  return map_reduce<2, 0>(h, n, BadF{x}, out);
}

int count_nonfinite_matrix(nys_handle h, const nys_matrix* A, double* out) {
  const int es = A->dtype == NYS_F64 ? 8 : A->dtype == NYS_F32 ? 4 : 2;
  unsigned nb = (unsigned)std::min<int64_t>(std::max<int64_t>(A->m, 1), 4096);
  double* part;
  NYS_CHECK(ws(h, WS_PART2, nb, &part));
  const char* p = (const char*)A->data;
  const int64_t rb = A->ld * es;
  switch (A->dtype) {
    case NYS_F64: hipLaunchKernelGGL(k_nonfinite<F64>, dim3(nb), dim3(NYS_BLOCK), 0, h->stream, p, A->m, A->n, rb, part); break;
    case NYS_F32: hipLaunchKernelGGL(k_nonfinite<F32>, dim3(nb), dim3(NYS_BLOCK), 0, h->stream, p, A->m, A->n, rb, part); break;
    default: hipLaunchKernelGGL(k_nonfinite<BF16>, dim3(nb), dim3(NYS_BLOCK), 0, h->stream, p, A->m, A->n, rb, part); break;
  }
  hipLaunchKernelGGL((k_map_reduce_finish<1, 0>), dim3(1), dim3(NYS_BLOCK), 0, h->stream, (int)nb,
                     (const double*)part, out);
  NYS_LAUNCH_CHECK(h);
  return NYS_OK;
}

int precond_reduce(nys_handle h, const double* U, const double* lam, int64_t m, int ell,
                   double delta, const double* r, double* t) {
  UpdArgs k{};
  k.m = m;
  k.ell = ell;
  k.r = const_cast<double*>(r);
  k.U = U;
  k.lam = lam;
  k.delta = delta;
  k.t = t;
  return launch_update(h, false, true, k);
}

int precond_expand(nys_handle h, const double* U, int64_t m, int ell, const double* r,
                   const double* t, double* out, double* dot_out) {
  ExpArgs k{};
  k.m = m;
  k.ell = ell;
  k.U = U;
  k.r = r;
  k.t = t;
  k.out = out;
  k.dot_out = dot_out;
  return launch_expand(h, k);
}

int pcg_update(nys_handle h, int64_t m, double* y, double* r, const double* p, const double* q,
               const double* U, const double* lam, int ell, double delta, double* t, bool ext) {
  UpdArgs k{};
  k.ext = ext ? 1 : 0;
  k.m = m;
  k.ell = ell;
  k.y = y;
  k.r = r;
  k.p = p;
  k.q = q;
  k.U = U;
  k.lam = lam;
  k.delta = delta;
  k.t = t;
  return launch_update(h, true, U != nullptr, k);
}

int pcg_expand(nys_handle h, int64_t m, const double* U, int ell, const double* r,
               const double* t, double* s) {
  ExpArgs k{};
  k.m = m;
  k.ell = ell;
  k.U = U;
  k.r = r;
  k.t = t;
  k.out = s;
  k.scal = h->dscal;
  return launch_expand(h, k);
}

// ||r||^2 and, without a preconditioner, rs = ||r||^2 (start of a solve).
int residual_norm(nys_handle h, int64_t m, double* r) {
  UpdArgs k{};
  k.m = m;
  k.r = r;
  return launch_update(h, false, false, k);
}

}  // namespace nys
