// Small and tall-skinny dense FP64 kernels of the Nystrom construction
// (Algorithm 1): tiled GEMM with split-K, Cholesky, triangular inverse,
// one-sided Jacobi SVD, the Philox test matrix and BF16 rounding.

#include <cmath>

#include "common.hpp"
#include "kernels.hpp"
#include "mapreduce.hpp"

namespace nys {
namespace {

// ---------------------------------------------------------------- GEMM (VALU FP64)
constexpr int GBM = 64, GBN = 64, GBK = 16;

template <class TA, bool TRA, bool TRB>
__global__ __launch_bounds__(NYS_BLOCK) void k_gemm64(int64_t M, int64_t N, int64_t K,
                                                      const void* Av, int64_t lda, const double* B,
                                                      int64_t ldb, double* C, int64_t ldc,
                                                      const double* rs, int64_t klen) {
  using raw = typename TA::raw;
  const raw* A = (const raw*)Av;
  __shared__ double As[GBK][GBM];
  __shared__ double Bs[GBK][GBN];
  const int tid = threadIdx.x;
  const int tx = tid % 16, ty = tid / 16;
  const int64_t m0 = (int64_t)blockIdx.y * GBM, n0 = (int64_t)blockIdx.x * GBN;
  const int64_t kb = (int64_t)blockIdx.z * klen;
  const int64_t ke = min(K, kb + klen);
  double c[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) c[i][j] = 0.0;

  for (int64_t k0 = kb; k0 < ke; k0 += GBK) {
    // A tile: op(A)[m0 + i][k0 + k]
    if (!TRA) {
      const int i = tid / 4, kk = (tid % 4) * 4;
      const int64_t gi = m0 + i;
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int64_t gk = k0 + kk + e;
        As[kk + e][i] = (gi < M && gk < ke) ? to_f64(A[gi * lda + gk]) : 0.0;
      }
    } else {
      const int kk = tid / 16, i = (tid % 16) * 4;
      const int64_t gk = k0 + kk;
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int64_t gi = m0 + i + e;
        As[kk][i + e] = (gi < M && gk < ke) ? to_f64(A[gk * lda + gi]) : 0.0;
      }
    }
    // B tile: op(B)[k0 + k][n0 + j]
    if (!TRB) {
      const int kk = tid / 16, j = (tid % 16) * 4;
      const int64_t gk = k0 + kk;
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int64_t gj = n0 + j + e;
        Bs[kk][j + e] = (gj < N && gk < ke) ? B[gk * ldb + gj] : 0.0;
      }
    } else {
      const int j = tid / 4, kk = (tid % 4) * 4;
      const int64_t gj = n0 + j;
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int64_t gk = k0 + kk + e;
        Bs[kk + e][j] = (gj < N && gk < ke) ? B[gj * ldb + gk] : 0.0;
      }
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < GBK; ++k) {
      double a[4], b[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) a[i] = As[k][ty * 4 + i];
#pragma unroll
      for (int j = 0; j < 4; ++j) b[j] = Bs[k][tx * 4 + j];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) c[i][j] = fma(a[i], b[j], c[i][j]);
    }
    __syncthreads();
  }
  // split-K writes raw partial tiles to C + z * M * ldc (no scaling)
  double* Cz = C + (int64_t)blockIdx.z * M * ldc;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int64_t gi = m0 + ty * 4 + i;
    if (gi >= M) continue;
    const double sc = (rs && gridDim.z == 1) ? rs[gi] : 1.0;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int64_t gj = n0 + tx * 4 + j;
      if (gj < N) Cz[gi * ldc + gj] = c[i][j] * sc;
    }
  }
}

__global__ __launch_bounds__(NYS_BLOCK) void k_splitk_reduce(int64_t M, int64_t N, int nsplit,
                                                             const double* part, double* C,
                                                             int64_t ldc, const double* rs) {
  const int64_t total = M * N;
  for (int64_t idx = (int64_t)blockIdx.x * NYS_BLOCK + threadIdx.x; idx < total;
       idx += (int64_t)gridDim.x * NYS_BLOCK) {
    const int64_t i = idx / N, j = idx % N;
    double s = 0.0;
    for (int z = 0; z < nsplit; ++z) s += part[(int64_t)z * total + idx];
    C[i * ldc + j] = rs ? s * rs[i] : s;
  }
}

template <class TA>
int gemm_dispatch(nys_handle h, bool ta, bool tb, dim3 g, int64_t M, int64_t N, int64_t K,
                  const void* A, int64_t lda, const double* B, int64_t ldb, double* C, int64_t ldc,
                  const double* rs, int64_t klen) {
  dim3 b(NYS_BLOCK);
  if (!ta && !tb) hipLaunchKernelGGL((k_gemm64<TA, false, false>), g, b, 0, h->stream, M, N, K, A, lda, B, ldb, C, ldc, rs, klen);
  else if (ta && !tb) hipLaunchKernelGGL((k_gemm64<TA, true, false>), g, b, 0, h->stream, M, N, K, A, lda, B, ldb, C, ldc, rs, klen);
  else if (!ta && tb) hipLaunchKernelGGL((k_gemm64<TA, false, true>), g, b, 0, h->stream, M, N, K, A, lda, B, ldb, C, ldc, rs, klen);
  else hipLaunchKernelGGL((k_gemm64<TA, true, true>), g, b, 0, h->stream, M, N, K, A, lda, B, ldb, C, ldc, rs, klen);
  NYS_LAUNCH_CHECK(h);
  return NYS_OK;
}

// ---------------------------------------------------------------- GEMM (FP64 matrix cores)
// C = op(A) B for FP64 A and B on v_mfma_f64_16x16x4f64.  Lane l of the
// instruction holds A[l%16][l/16] and B[l/16][l%16] and returns
// D[l/16 + 4r][l%16] in its register r.  A block computes a 128 x 128 tile
// with four waves of 64 x 64 (4 x 4 instruction tiles); stages of 16 k go
// through registers into two LDS buffers (one barrier per stage).
// SYM: C = X^T X (A == B, transposed A): only tiles on or above the diagonal
// are computed and each is stored with its mirror.  TRIB: B upper triangular,
// so the k range of a column tile ends at its last column.  Split-K writes raw
// partial tiles to C + z * M * ldc as k_gemm64 does.
constexpr int MBM = 128, MBN = 128, MBK = 16, MPAD = 4;
typedef double f64x4 __attribute__((ext_vector_type(4)));

template <bool TRA, bool TRIB, bool SYM>
__global__ __launch_bounds__(NYS_BLOCK, 2) void k_gemm64_mfma(int64_t M, int64_t N, int64_t K, const double* A,
                                                              int64_t lda, const double* B, int64_t ldb, double* C,
                                                              int64_t ldc, const double* rs, int64_t klen) {
  static_assert(NYS_BLOCK == 256, "four waves");
  const int bm = blockIdx.y, bn = blockIdx.x;
  if (SYM && bm > bn) return;
  __shared__ double As[2][MBK][MBM + MPAD];
  __shared__ double Bs[2][MBK][MBN + MPAD];
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int wm = wave >> 1, wn = wave & 1;
  const int64_t m0 = (int64_t)bm * MBM, n0 = (int64_t)bn * MBN;
  const int64_t kb = (int64_t)blockIdx.z * klen;
  int64_t ke = min(K, kb + klen);
  if (TRIB) ke = min(ke, n0 + MBN);
  const int nst = ke > kb ? (int)((ke - kb + MBK - 1) / MBK) : 0;

  // one stage of loads: 8 elements of A and 8 of B per thread
  double ra[8], rb[8];
  auto load = [&](int64_t k0) {
    if (!TRA) {                          // A row-major M x K: row tid/2, k (tid%2)*8 ..
      const int i = tid >> 1, kk = (tid & 1) * 8;
      const int64_t gi = m0 + i;
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const int64_t gk = k0 + kk + e;
        ra[e] = (gi < M && gk < ke) ? A[gi * lda + gk] : 0.0;
      }
    } else {                             // A stored K x M: k tid/16, rows (tid%16)*8 ..
      const int kk = tid >> 4, i = (tid & 15) * 8;
      const int64_t gk = k0 + kk;
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const int64_t gi = m0 + i + e;
        ra[e] = (gk < ke && gi < M) ? A[gk * lda + gi] : 0.0;
      }
    }
    const int kk = tid >> 4, j = (tid & 15) * 8;   // B row-major K x N
    const int64_t gk = k0 + kk;
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const int64_t gj = n0 + j + e;
      rb[e] = (gk < ke && gj < N) ? B[gk * ldb + gj] : 0.0;
    }
  };
  auto store = [&](int buf) {
    if (!TRA) {
      const int i = tid >> 1, kk = (tid & 1) * 8;
#pragma unroll
      for (int e = 0; e < 8; ++e) As[buf][kk + e][i] = ra[e];
    } else {
      const int kk = tid >> 4, i = (tid & 15) * 8;
#pragma unroll
      for (int e = 0; e < 8; ++e) As[buf][kk][i + e] = ra[e];
    }
    const int kk = tid >> 4, j = (tid & 15) * 8;
#pragma unroll
    for (int e = 0; e < 8; ++e) Bs[buf][kk][j + e] = rb[e];
  };

  f64x4 acc[4][4];
#pragma unroll
  for (int ti = 0; ti < 4; ++ti)
#pragma unroll
    for (int tj = 0; tj < 4; ++tj) acc[ti][tj] = f64x4{0.0, 0.0, 0.0, 0.0};
  if (nst > 0) {
    load(kb);
    store(0);
  }
  __syncthreads();
  const int lr = lane >> 4, lc = lane & 15;
  for (int s = 0; s < nst; ++s) {
    const int buf = s & 1;
    if (s + 1 < nst) load(kb + (int64_t)(s + 1) * MBK);
#pragma unroll
    for (int ks = 0; ks < MBK / 4; ++ks) {
      double a[4], b[4];
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        a[t] = As[buf][ks * 4 + lr][wm * 64 + t * 16 + lc];
        b[t] = Bs[buf][ks * 4 + lr][wn * 64 + t * 16 + lc];
      }
#pragma unroll
      for (int ti = 0; ti < 4; ++ti)
#pragma unroll
        for (int tj = 0; tj < 4; ++tj)
          acc[ti][tj] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[ti], b[tj], acc[ti][tj], 0, 0, 0);
    }
    // the other buffer was last read before the previous barrier
    if (s + 1 < nst) store(buf ^ 1);
    __syncthreads();
  }

  double* Cz = C + (int64_t)blockIdx.z * M * ldc;
  const bool scale = rs && gridDim.z == 1;
#pragma unroll
  for (int ti = 0; ti < 4; ++ti)
#pragma unroll
    for (int tj = 0; tj < 4; ++tj)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t gi = m0 + wm * 64 + ti * 16 + lr + 4 * r;
        const int64_t gj = n0 + wn * 64 + tj * 16 + lc;
        if (gi >= M || gj >= N) continue;
        const double v = acc[ti][tj][r];
        Cz[gi * ldc + gj] = scale ? v * rs[gi] : v;
        if (SYM && bm != bn) Cz[gj * ldc + gi] = v;
      }
}

// ---------------------------------------------------------------- Cholesky (one block)
constexpr int DB = 1024;   // threads of the one-block dense kernels

// G (ell x ell, row-major) -> upper C with C^T C = sym(G) + (shift_abs + shift_rel*trace) I.
__global__ __launch_bounds__(DB) void k_chol_upper(double* G, int ell, double shift_abs,
                                                   double shift_rel, double* fail) {
  __shared__ double piv;
  __shared__ int bad;
  __shared__ double red[DB / NYS_WAVE];
  const int tid = threadIdx.x;
  // symmetrise into the upper triangle, trace
  double tr[1] = {0.0};
  for (int64_t idx = tid; idx < (int64_t)ell * ell; idx += DB) {
    const int i = (int)(idx / ell), j = (int)(idx % ell);
    if (i < j) G[idx] = 0.5 * (G[idx] + G[(int64_t)j * ell + i]);
    if (i == j) tr[0] += G[idx];
  }
  block_sum<1>(tr, red);
  const double shift = shift_abs + shift_rel * tr[0];
  for (int i = tid; i < ell; i += DB) G[(int64_t)i * ell + i] += shift;
  if (tid == 0) bad = 0;
  __syncthreads();
  for (int k = 0; k < ell; ++k) {
    if (tid == 0) {
      const double g = G[(int64_t)k * ell + k];
      if (!(g > 0.0) || !isfinite(g)) {
        bad = 1;
        piv = 1.0;
      } else {
        piv = sqrt(g);
      }
    }
    __syncthreads();
    if (bad) break;
    const double p = piv;
    for (int j = k + 1 + tid; j < ell; j += DB) G[(int64_t)k * ell + j] /= p;
    if (tid == 0) G[(int64_t)k * ell + k] = p;
    __syncthreads();
    const int r = ell - k - 1;
    for (int64_t idx = tid; idx < (int64_t)r * r; idx += DB) {
      const int i = k + 1 + (int)(idx / r), j = k + 1 + (int)(idx % r);
      if (j >= i) G[(int64_t)i * ell + j] -= G[(int64_t)k * ell + i] * G[(int64_t)k * ell + j];
    }
    __syncthreads();
  }
  for (int64_t idx = tid; idx < (int64_t)ell * ell; idx += DB) {
    const int i = (int)(idx / ell), j = (int)(idx % ell);
    if (i > j) G[idx] = 0.0;
  }
  if (tid == 0) *fail = bad ? 1.0 : 0.0;
}

// Cinv = C^{-1}, C upper triangular: rows of Cinv from the bottom up, each row
// in parallel over its columns: Cinv[i][j] = -(sum_{k=i+1..j} C[i][k] Cinv[k][j]) / C[i][i].
__global__ __launch_bounds__(DB) void k_tri_inv_upper(const double* C, double* X, int ell) {
  const int tid = threadIdx.x;
  for (int64_t idx = tid; idx < (int64_t)ell * ell; idx += DB) X[idx] = 0.0;
  __syncthreads();
  for (int i = ell - 1; i >= 0; --i) {
    const double cii = C[(int64_t)i * ell + i];
    for (int j = i + tid; j < ell; j += DB) {
      if (j == i) {
        X[(int64_t)i * ell + i] = 1.0 / cii;
      } else {
        double s = 0.0;
        for (int k = i + 1; k <= j; ++k) s = fma(C[(int64_t)i * ell + k], X[(int64_t)k * ell + j], s);
        X[(int64_t)i * ell + j] = -s / cii;
      }
    }
    __syncthreads();
  }
}

// Blocked form of k_chol_upper for ell >= 2*NB: panels of NB rows are factored
// in LDS (the unblocked steps touch only the panel), and the trailing upper
// triangle is updated once per panel from the LDS copy.  G is symmetrised and
// shifted first, exactly as in k_chol_upper.
__global__ __launch_bounds__(DB) void k_chol_upper_blocked(double* G, int ell, int NB, double shift_abs,
                                                           double shift_rel, double* fail) {
  extern __shared__ double P[];          // NB x ell panel (row pitch ell)
  __shared__ double red[DB / NYS_WAVE];
  __shared__ int bad;
  const int tid = threadIdx.x;
  double tr[1] = {0.0};
  for (int64_t idx = tid; idx < (int64_t)ell * ell; idx += DB) {
    const int i = (int)(idx / ell), j = (int)(idx % ell);
    if (i < j) G[idx] = 0.5 * (G[idx] + G[(int64_t)j * ell + i]);
    if (i == j) tr[0] += G[idx];
  }
  block_sum<1>(tr, red);
  const double shift = shift_abs + shift_rel * tr[0];
  for (int i = tid; i < ell; i += DB) G[(int64_t)i * ell + i] += shift;
  if (tid == 0) bad = 0;
  __syncthreads();
  for (int k0 = 0; k0 < ell; k0 += NB) {
    const int nb = min(NB, ell - k0);
    const int w = ell - k0;              // panel columns k0 .. ell-1
    for (int idx = tid; idx < nb * w; idx += DB) {
      const int r = idx / w, c = idx % w;
      P[r * ell + c] = G[(int64_t)(k0 + r) * ell + k0 + c];
    }
    __syncthreads();
    bool badl = false;
    for (int kk = 0; kk < nb; ++kk) {
      const double g = P[kk * ell + kk];
      if (!(g > 0.0) || !isfinite(g)) {  // uniform: every thread read the same g
        badl = true;
        break;
      }
      const double piv = sqrt(g);
      __syncthreads();
      for (int c = kk + 1 + tid; c < w; c += DB) P[kk * ell + c] /= piv;
      if (tid == 0) P[kk * ell + kk] = piv;
      __syncthreads();
      // rows kk+1 .. nb-1 of the panel, columns c >= r
      const int rows = nb - kk - 1;
      for (int idx = tid; idx < rows * w; idx += DB) {
        const int r = kk + 1 + idx / w, c = idx % w;
        if (c >= r) P[r * ell + c] -= P[kk * ell + r] * P[kk * ell + c];
      }
      __syncthreads();
    }
    if (badl) {
      if (tid == 0) bad = 1;
      break;
    }
    for (int idx = tid; idx < nb * w; idx += DB) {
      const int r = idx / w, c = idx % w;
      G[(int64_t)(k0 + r) * ell + k0 + c] = c >= r ? P[r * ell + c] : 0.0;
    }
    // trailing update of the upper triangle rows/cols >= k0 + nb
    const int t = w - nb;
    for (int64_t idx = tid; idx < (int64_t)t * t; idx += DB) {
      const int i = nb + (int)(idx / t), j = nb + (int)(idx % t);
      if (j < i) continue;
      double acc = 0.0;
      for (int kk = 0; kk < nb; ++kk) acc = fma(P[kk * ell + i], P[kk * ell + j], acc);
      G[(int64_t)(k0 + i) * ell + k0 + j] -= acc;
    }
    __syncthreads();
  }
  for (int64_t idx = tid; idx < (int64_t)ell * ell; idx += DB) {
    const int i = (int)(idx / ell), j = (int)(idx % ell);
    if (i > j) G[idx] = 0.0;
  }
  if (tid == 0) *fail = bad ? 1.0 : 0.0;
}

// X = C^{-1} for upper-triangular C, one wave per column: column j solves
// C x = e_j by back substitution, x_i = -(sum_{k=i+1..j} C[i][k] x_k) / C[i][i].
// Lane l keeps x_k for k = l, l+64, ... in registers (ell <= 64*CH); the row
// of C for the next step is loaded while the current one is reduced.
constexpr int TRI_WAVES = 4;
template <int CH>
__global__ __launch_bounds__(TRI_WAVES * NYS_WAVE) void k_tri_inv_cols(const double* C, double* X, int ell) {
  const int lane = threadIdx.x % NYS_WAVE;
  const int j = blockIdx.x * TRI_WAVES + threadIdx.x / NYS_WAVE;
  if (j >= ell) return;                  // no block-level synchronisation below
  double x[CH];
#pragma unroll
  for (int t = 0; t < CH; ++t) x[t] = 0.0;
  const double xj = 1.0 / C[(int64_t)j * ell + j];
#pragma unroll
  for (int t = 0; t < CH; ++t)
    if (t * NYS_WAVE + lane == j) x[t] = xj;
  double cn[CH];
  auto load_row = [&](int i, double* cr) {
#pragma unroll
    for (int t = 0; t < CH; ++t) {
      const int k = t * NYS_WAVE + lane;
      cr[t] = (k > i && k <= j) ? C[(int64_t)i * ell + k] : 0.0;
    }
  };
  if (j > 0) load_row(j - 1, cn);
  for (int i = j - 1; i >= 0; --i) {
    double cr[CH];
#pragma unroll
    for (int t = 0; t < CH; ++t) cr[t] = cn[t];
    const double cii = C[(int64_t)i * ell + i];
    if (i > 0) load_row(i - 1, cn);
    double s = 0.0;
#pragma unroll
    for (int t = 0; t < CH; ++t) s = fma(cr[t], x[t], s);
    s = wave_sum_dpp(s);
    const double xi = -s / cii;
#pragma unroll
    for (int t = 0; t < CH; ++t)
      if (t * NYS_WAVE + lane == i) x[t] = xi;
  }
#pragma unroll
  for (int t = 0; t < CH; ++t) {
    const int k = t * NYS_WAVE + lane;
    if (k < ell) X[(int64_t)k * ell + j] = x[t];
  }
}

// Inverse of the nb x nb diagonal blocks of an upper-triangular C (nb <= 64):
// block (b, g) of the grid takes columns 4 g .. 4 g + 3 of diagonal block b,
// one wave per column, by the back substitution of k_tri_inv_cols with one
// element per lane.  X (zeroed beforehand) receives the blocks in place.
__global__ __launch_bounds__(TRI_WAVES * NYS_WAVE) void k_tri_inv_diag(const double* C, double* X, int ell, int nb) {
  const int lane = threadIdx.x % NYS_WAVE;
  const int b = blockIdx.x;
  const int jl = blockIdx.y * TRI_WAVES + threadIdx.x / NYS_WAVE;
  const int o = b * nb;
  const int sb = min(nb, ell - o);
  if (jl >= sb) return;
  const int64_t ld = ell;
  double x = lane == jl ? 1.0 / C[(int64_t)(o + jl) * ld + o + jl] : 0.0;
  for (int i = jl - 1; i >= 0; --i) {
    const double cik = (lane > i && lane <= jl) ? C[(int64_t)(o + i) * ld + o + lane] : 0.0;
    const double sum = wave_sum_dpp(cik * x);
    if (lane == i) x = -sum / C[(int64_t)(o + i) * ld + o + i];
  }
  if (lane < sb) X[(int64_t)(o + lane) * ld + o + jl] = x;
}

__global__ __launch_bounds__(NYS_BLOCK) void k_scale_block(double* X, int64_t ld, int rows, int cols, double alpha) {
  const int64_t total = (int64_t)rows * cols;
  for (int64_t idx = (int64_t)blockIdx.x * NYS_BLOCK + threadIdx.x; idx < total; idx += (int64_t)gridDim.x * NYS_BLOCK) {
    const int64_t r = idx / cols, c = idx % cols;
    X[r * ld + c] *= alpha;
  }
}

// ---------------------------------------------------------------- Cholesky across workgroups
// G = C^T C, C upper, for larger ell: right-looking by panels of CP rows.  Per
// panel: the CP x CP diagonal block is factored by one wave in registers, the row
// panel C[k0:k0+nb, k0+nb:] = C_kk^{-T} G[k0:k0+nb, k0+nb:] is solved one
// column per thread, and the trailing upper triangle is updated in 64 x 64
// tiles by as many blocks as there are tiles.  Arithmetic per entry is the
// same as the one-block kernels; only the order of the panel sums differs.
constexpr int CP = 32;                   // panel rows
constexpr int CT = 64;                   // trailing-update tile

// upper triangle := (G + G^T)/2 (the lower triangle is only read)
__global__ __launch_bounds__(NYS_BLOCK) void k_chol_sym(double* G, int ell) {
  const int64_t total = (int64_t)ell * ell;
  for (int64_t idx = (int64_t)blockIdx.x * NYS_BLOCK + threadIdx.x; idx < total;
       idx += (int64_t)gridDim.x * NYS_BLOCK) {
    const int i = (int)(idx / ell), j = (int)(idx % ell);
    if (i < j) G[idx] = 0.5 * (G[idx] + G[(int64_t)j * ell + i]);
  }
}

// diagonal += shift_abs + shift_rel * trace; *fail = 0 (one block)
__global__ __launch_bounds__(NYS_BLOCK) void k_chol_shift(double* G, int ell, double shift_abs, double shift_rel,
                                                          double* fail) {
  __shared__ double red[NYS_BLOCK / NYS_WAVE];
  double tr[1] = {0.0};
  for (int i = threadIdx.x; i < ell; i += NYS_BLOCK) tr[0] += G[(int64_t)i * ell + i];
  block_sum<1>(tr, red);
  const double shift = shift_abs + shift_rel * tr[0];
  for (int i = threadIdx.x; i < ell; i += NYS_BLOCK) G[(int64_t)i * ell + i] += shift;
  if (threadIdx.x == 0) *fail = 0.0;
}

// Broadcast of lane l's double (l wave-uniform) through two scalar reads.
__device__ __forceinline__ double lane_bcast(double v, int l) {
  const uint64_t b = (uint64_t)__double_as_longlong(v);
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)b, l);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(b >> 32), l);
  return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
}

// factor the nb x nb diagonal block at k0 (nb <= CP) by one wave, without
// barriers: lane c < nb keeps column c of the block (rows 0..c) in registers,
// and each pivot row reaches the other lanes by lane broadcasts.  *fail = 1 on
// a pivot that is not positive and finite.
__global__ __launch_bounds__(NYS_WAVE) void k_chol_diag(double* G, int ell, int k0, int nb, double* fail) {
  const int c = threadIdx.x;
  const bool col = c < nb;
  double x[CP];
#pragma unroll
  for (int r = 0; r < CP; ++r) x[r] = (col && r <= c) ? G[(int64_t)(k0 + r) * ell + k0 + c] : 0.0;
  bool bad = false;
#pragma unroll
  for (int k = 0; k < CP; ++k) {
    if (k < nb && !bad) {                      // uniform
      const double g = lane_bcast(x[k], k);
      if (!(g > 0.0) || !isfinite(g)) {
        bad = true;
      } else {
        const double piv = sqrt(g);
        if (c == k) x[k] = piv;
        else if (c > k) x[k] = x[k] / piv;
        // rows r > k: C[r][c] -= C[k][r] C[k][c] for c >= r
#pragma unroll
        for (int r = k + 1; r < CP; ++r) {
          if (r < nb) {
            const double ckr = lane_bcast(x[k], r);
            const double xr = fma(-ckr, x[k], x[r]);
            x[r] = c >= r ? xr : x[r];              // a select, not a branch
          }
        }
      }
    }
  }
  if (bad) {
    if (c == 0) *fail = 1.0;
    return;
  }
  if (col) {
#pragma unroll
    for (int r = 0; r < CP; ++r)
      if (r < nb) G[(int64_t)(k0 + r) * ell + k0 + c] = r <= c ? x[r] : 0.0;
  }
}

// row panel: for every column c >= k0 + nb, x = C_kk^{-T} G[k0:k0+nb, c] by
// forward substitution (C_kk^T is lower triangular), one column per thread;
// the column's nb entries are all read before the first is written back
__global__ __launch_bounds__(NYS_BLOCK) void k_chol_row(double* G, int ell, int k0, int nb) {
  __shared__ double Ck[CP * CP];
  for (int idx = threadIdx.x; idx < nb * nb; idx += NYS_BLOCK) {
    const int r = idx / nb, c = idx % nb;
    Ck[r * CP + c] = G[(int64_t)(k0 + r) * ell + k0 + c];
  }
  __syncthreads();
  const int c = k0 + nb + blockIdx.x * NYS_BLOCK + threadIdx.x;
  if (c >= ell) return;
  double x[CP];
#pragma unroll
  for (int r = 0; r < CP; ++r) x[r] = r < nb ? G[(int64_t)(k0 + r) * ell + c] : 0.0;
#pragma unroll
  for (int r = 0; r < CP; ++r) {
    if (r < nb) {
      double s = x[r];
#pragma unroll
      for (int q = 0; q < r; ++q) s -= Ck[q * CP + r] * x[q];
      x[r] = s / Ck[r * CP + r];
    }
  }
#pragma unroll
  for (int r = 0; r < CP; ++r)
    if (r < nb) G[(int64_t)(k0 + r) * ell + c] = x[r];
}

// trailing update: G[i][j] -= sum_q C[k0+q][i] C[k0+q][j] for t0 <= i <= j < ell,
// t0 = k0 + nb, over the upper tiles (ti <= tj) of a CT x CT tiling; each
// thread owns a 4 x 4 piece of its block's tile
__global__ __launch_bounds__(NYS_BLOCK) void k_chol_update(double* G, int ell, int k0, int nb) {
  static_assert(NYS_BLOCK == (CT / 4) * (CT / 4), "one 4 x 4 piece of the tile per thread");
  __shared__ double Pi[CP * CT];
  __shared__ double Pj[CP * CT];
  const int t0 = k0 + nb;
  const int nt = (ell - t0 + CT - 1) / CT;
  // blockIdx.x -> (ti, tj), ti <= tj, row by row of the upper tile triangle
  int b = blockIdx.x, ti = 0;
  while (b >= nt - ti) {
    b -= nt - ti;
    ++ti;
  }
  const int tj = ti + b;
  const int i0 = t0 + ti * CT, j0 = t0 + tj * CT;
  for (int idx = threadIdx.x; idx < nb * CT; idx += NYS_BLOCK) {
    const int q = idx / CT, a = idx % CT;
    const int64_t row = (int64_t)(k0 + q) * ell;
    Pi[q * CT + a] = i0 + a < ell ? G[row + i0 + a] : 0.0;
    Pj[q * CT + a] = j0 + a < ell ? G[row + j0 + a] : 0.0;
  }
  __syncthreads();
  const int ai = (threadIdx.x / 16) * 4, bj = (threadIdx.x % 16) * 4;
  double acc[4][4] = {};
  for (int q = 0; q < nb; ++q) {
    double u[4], v[4];
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      u[e] = Pi[q * CT + ai + e];
      v[e] = Pj[q * CT + bj + e];
    }
#pragma unroll
    for (int e = 0; e < 4; ++e)
#pragma unroll
      for (int f = 0; f < 4; ++f) acc[e][f] = fma(u[e], v[f], acc[e][f]);
  }
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    const int i = i0 + ai + e;
    if (i >= ell) continue;
#pragma unroll
    for (int f = 0; f < 4; ++f) {
      const int j = j0 + bj + f;
      if (j < ell && j >= i) G[(int64_t)i * ell + j] -= acc[e][f];
    }
  }
}

__global__ __launch_bounds__(NYS_BLOCK) void k_chol_lower_zero(double* G, int ell) {
  const int64_t total = (int64_t)ell * ell;
  for (int64_t idx = (int64_t)blockIdx.x * NYS_BLOCK + threadIdx.x; idx < total;
       idx += (int64_t)gridDim.x * NYS_BLOCK) {
    const int i = (int)(idx / ell), j = (int)(idx % ell);
    if (i > j) G[idx] = 0.0;
  }
}

// ---------------------------------------------------------------- one-sided Jacobi SVD
// Xc holds the columns contiguously (column k at Xc + k*ell).  One launch per
// round of the round-robin ordering; one wave per column pair.
__device__ __forceinline__ int rr_player(int p, int round, int np) {
  // np players 0..np-1 (np even); player 0 fixed, others rotate
  return p == 0 ? 0 : 1 + (p - 1 + round) % (np - 1);
}

// Rotation of the column pair (xp, xq) (length ell) that makes them
// orthogonal, by one wave; returns whether it rotated.
__device__ __forceinline__ bool jacobi_pair(double* xp, double* xq, int ell, double tol, int lane) {
  double al = 0.0, be = 0.0, ga = 0.0;
  for (int i = lane; i < ell; i += NYS_WAVE) {
    const double u = xp[i], v = xq[i];
    al = fma(u, u, al);
    be = fma(v, v, be);
    ga = fma(u, v, ga);
  }
  al = wave_sum_dpp(al);
  be = wave_sum_dpp(be);
  ga = wave_sum_dpp(ga);
  if (!(fabs(ga) > tol * sqrt(al * be))) return false;
  const double zeta = (be - al) / (2.0 * ga);
  const double t = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
  const double c = 1.0 / sqrt(1.0 + t * t);
  const double s = c * t;
  for (int i = lane; i < ell; i += NYS_WAVE) {
    const double u = xp[i], v = xq[i];
    xp[i] = c * u - s * v;
    xq[i] = s * u + c * v;
  }
  return true;
}

__global__ __launch_bounds__(NYS_WAVE) void k_jacobi_round(double* Xc, int ell, int np, int round,
                                                           double tol, unsigned* rotations) {
  const int k = blockIdx.x;                 // pair index 0 .. np/2-1
  const int a = rr_player(k, round, np);
  const int b = rr_player(np - 1 - k, round, np);
  int p = min(a, b), q = max(a, b);
  if (q >= ell) return;                     // pairs with the padding player
  double* xp = Xc + (int64_t)p * ell;
  double* xq = Xc + (int64_t)q * ell;
  const int lane = threadIdx.x;
  if (jacobi_pair(xp, xq, ell, tol, lane) && lane == 0) atomicAdd(rotations, 1u);
}

// Rotation of a column pair held in registers: lane l holds elements
// l, l + 64, ... (CH per lane, ell <= 64 CH) of both columns; same arithmetic
// as jacobi_pair, with every load of the pair in flight together.
template <int CH>
__device__ __forceinline__ bool jacobi_pair_regs(double* xp, double* xq, int ell, double tol, int lane) {
  double u[CH], v[CH];
#pragma unroll
  for (int t = 0; t < CH; ++t) {
    const int i = lane + t * NYS_WAVE;
    u[t] = i < ell ? xp[i] : 0.0;
    v[t] = i < ell ? xq[i] : 0.0;
  }
  double al = 0.0, be = 0.0, ga = 0.0;
#pragma unroll
  for (int t = 0; t < CH; ++t) {
    al = fma(u[t], u[t], al);
    be = fma(v[t], v[t], be);
    ga = fma(u[t], v[t], ga);
  }
  al = wave_sum_dpp(al);
  be = wave_sum_dpp(be);
  ga = wave_sum_dpp(ga);
  if (!(fabs(ga) > tol * sqrt(al * be))) return false;
  const double zeta = (be - al) / (2.0 * ga);
  const double t = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
  const double c = 1.0 / sqrt(1.0 + t * t);
  const double s = c * t;
#pragma unroll
  for (int k = 0; k < CH; ++k) {
    const int i = lane + k * NYS_WAVE;
    if (i < ell) {
      xp[i] = c * u[k] - s * v[k];
      xq[i] = s * u[k] + c * v[k];
    }
  }
  return true;
}

// Rotation of a column pair whose first column stays in registers across
// rounds (u: pairs of doubles, lane l holding elements 2 i, 2 i + 1 for
// i = l, l + 64, ...; even ell <= 128 C2); the second is read from LDS and
// written back when the pair rotates.  Same arithmetic as jacobi_pair.
typedef double f64x2 __attribute__((ext_vector_type(2)));
template <int C2>
__device__ __forceinline__ bool jacobi_pair_held(f64x2 (&u)[C2], double* xq, int ell, double tol, int lane) {
  const int half = ell / 2;
  f64x2 v[C2];
#pragma unroll
  for (int t = 0; t < C2; ++t) {
    const int i = lane + t * NYS_WAVE;
    v[t] = i < half ? ((const f64x2*)xq)[i] : f64x2{0.0, 0.0};
  }
  double al = 0.0, be = 0.0, ga = 0.0;
#pragma unroll
  for (int t = 0; t < C2; ++t) {
    al = fma(u[t][0], u[t][0], al);
    be = fma(v[t][0], v[t][0], be);
    ga = fma(u[t][0], v[t][0], ga);
    al = fma(u[t][1], u[t][1], al);
    be = fma(v[t][1], v[t][1], be);
    ga = fma(u[t][1], v[t][1], ga);
  }
  al = wave_sum_dpp(al);
  be = wave_sum_dpp(be);
  ga = wave_sum_dpp(ga);
  if (!(fabs(ga) > tol * sqrt(al * be))) return false;
  const double zeta = (be - al) / (2.0 * ga);
  const double t = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
  const double c = 1.0 / sqrt(1.0 + t * t);
  const double s = c * t;
#pragma unroll
  for (int k = 0; k < C2; ++k) {
    const f64x2 uu = u[k], vv = v[k];
    u[k] = f64x2{c * uu[0] - s * vv[0], c * uu[1] - s * vv[1]};
    const int i = lane + k * NYS_WAVE;
    if (i < half) ((f64x2*)xq)[i] = f64x2{s * uu[0] + c * vv[0], s * uu[1] + c * vv[1]};
  }
  return true;
}

// Block variant: the columns form groups of JG (the last ones padded), and a
// launch is one round of the round-robin over groups; each block takes one
// group pair and keeps its 2*JG columns in LDS.  FULL (the first round of a
// sweep): a full round-robin over the 2*JG columns (2*JG - 1 rounds, one wave
// per column pair), which also covers the pairs inside each group; otherwise
// only the JG * JG pairs across the two groups (JG rounds, wave w pairs
// column w of the first group with column (w + r) % JG of the second).  Every
// column pair meets at least once per sweep, so the convergence test (a sweep
// without rotations) is unchanged.  Columns move between memory and LDS eight
// elements per thread at a time; CH > 0 holds a pair in registers while it
// is rotated (ell <= 64 CH).  A negative round pairs groups 2b and 2b + 1 in
// block b (the pairs inside the 2*JG-column groups of the wide variant).
template <int JG, int CH, bool FULL>
__device__ __forceinline__ void jacobi_block_body(double* Xc, int ell, int ngp, int round, double tol,
                                                  unsigned* rotations, double* cols) {
  constexpr int NT = JG * NYS_WAVE, U = 8;
  const int ga = round < 0 ? 2 * (int)blockIdx.x : rr_player(blockIdx.x, round, ngp);
  const int gb = round < 0 ? ga + 1 : rr_player(ngp - 1 - blockIdx.x, round, ngp);
  auto gcol = [&](int c) { return c < JG ? ga * JG + c : gb * JG + (c - JG); };
  const int total = 2 * JG * ell;
  const int wid = threadIdx.x / NYS_WAVE, lane = threadIdx.x % NYS_WAVE;
  if ((ell & 1) == 0) {
    // even ell: every column starts 16-byte aligned; each wave moves whole
    // columns straight into LDS, a kilobyte per instruction, all in flight
    const int cb = ell * 8;                // bytes per column
    for (int c = wid; c < 2 * JG; c += JG) {
      const int g = gcol(c);
      char* dst = (char*)(cols + (int64_t)c * ell);
      if (g < ell) {
        const char* src = (const char*)(Xc + (int64_t)g * ell);
        for (int off = 0; off < cb; off += 1024)
          if (off + lane * 16 < cb)
            __builtin_amdgcn_global_load_lds((const void*)(src + off + lane * 16),
                                             (__attribute__((address_space(3))) void*)(dst + off), 16, 0, 0);
      } else {
        for (int i = lane; i < ell; i += NYS_WAVE) cols[(int64_t)c * ell + i] = 0.0;
      }
    }
    __builtin_amdgcn_s_waitcnt(0);
  } else {
    for (int base = threadIdx.x; base < total; base += NT * U) {
      double v[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int idx = base + u * NT;
        v[u] = 0.0;
        if (idx < total) {
          const int c = idx / ell, i = idx - c * ell;
          const int g = gcol(c);
          if (g < ell) v[u] = Xc[(int64_t)g * ell + i];
        }
      }
#pragma unroll
      for (int u = 0; u < U; ++u)
        if (base + u * NT < total) cols[base + u * NT] = v[u];
    }
  }
  __syncthreads();
  unsigned nrot = 0;
  auto rotate = [&](int p, int q) {
    if (gcol(p) >= ell || gcol(q) >= ell) return;
    bool r;
    if constexpr (CH > 0) r = jacobi_pair_regs<CH>(cols + p * ell, cols + q * ell, ell, tol, lane);
    else r = jacobi_pair(cols + p * ell, cols + q * ell, ell, tol, lane);
    if (r) ++nrot;
  };
  if constexpr (FULL) {
    for (int r = 0; r < 2 * JG - 1; ++r) {
      const int a = rr_player(wid, r, 2 * JG), b = rr_player(2 * JG - 1 - wid, r, 2 * JG);
      rotate(min(a, b), max(a, b));
      __syncthreads();
    }
  } else if (CH > 0 && (ell & 1) == 0) {
    // column wid of the first group stays with wave wid for all JG rounds
    constexpr int C2 = CH > 0 ? (CH + 1) / 2 : 1;
    const int half = ell / 2;
    const bool live = gcol(wid) < ell;
    f64x2 u[C2];
    const f64x2* up = (const f64x2*)(cols + (int64_t)wid * ell);
#pragma unroll
    for (int t = 0; t < C2; ++t) {
      const int i = lane + t * NYS_WAVE;
      u[t] = i < half ? up[i] : f64x2{0.0, 0.0};
    }
    for (int r = 0; r < JG; ++r) {
      const int q = JG + (wid + r) % JG;
      if (live && gcol(q) < ell && jacobi_pair_held<C2>(u, cols + (int64_t)q * ell, ell, tol, lane)) ++nrot;
      __syncthreads();
    }
    f64x2* upw = (f64x2*)(cols + (int64_t)wid * ell);
#pragma unroll
    for (int t = 0; t < C2; ++t) {
      const int i = lane + t * NYS_WAVE;
      if (i < half) upw[i] = u[t];
    }
    __syncthreads();
  } else {
    for (int r = 0; r < JG; ++r) {
      rotate(wid, JG + (wid + r) % JG);
      __syncthreads();
    }
  }
  if ((ell & 1) == 0) {
    // pairs of doubles: 16-byte stores
    const int half = ell / 2;
    for (int c = wid; c < 2 * JG; c += JG) {
      const int g = gcol(c);
      if (g >= ell) continue;
      const f64x2* srcl = (const f64x2*)(cols + (int64_t)c * ell);
      f64x2* dstg = (f64x2*)(Xc + (int64_t)g * ell);
      for (int i = lane; i < half; i += NYS_WAVE) dstg[i] = srcl[i];
    }
  } else {
    for (int base = threadIdx.x; base < total; base += NT * U) {
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int idx = base + u * NT;
        if (idx < total) {
          const int c = idx / ell, i = idx - c * ell;
          const int g = gcol(c);
          if (g < ell) Xc[(int64_t)g * ell + i] = cols[idx];
        }
      }
    }
  }
  if (lane == 0 && nrot) atomicAdd(rotations, nrot);
}

template <int JG, int CH, bool FULL>
__global__ __launch_bounds__(JG * NYS_WAVE) void k_jacobi_block_round(double* Xc, int ell, int ngp, int round,
                                                                      double tol, unsigned* rotations) {
  extern __shared__ double cols[];       // 2*JG columns of length ell
  jacobi_block_body<JG, CH, FULL>(Xc, ell, ngp, round, tol, rotations, cols);
}

// Wide variant (even ell): groups of G columns, twice the block variant's JG
// at the same LDS size.  A launch is one round of the round-robin over these
// groups; each block takes one group pair with G waves.  Wave w keeps column w
// of the first group in registers for the whole launch (C2 pairs of doubles
// per lane, ell <= 128 C2) and meets every column of the second group, which
// sits in LDS, once: G rounds of G pairs, against JG rounds of JG pairs for
// the same columns moved.  The pairs inside each group are left to a launch of
// the block variant's FULL round with a negative round (one per sweep).
template <int G, int C2>
__global__ __launch_bounds__(G * NYS_WAVE) void k_jacobi_wide_round(double* Xc, int ell, int ngw, int round,
                                                                    double tol, unsigned* rotations) {
  extern __shared__ double cols[];       // G columns of length ell
  const int wid = __builtin_amdgcn_readfirstlane(threadIdx.x / NYS_WAVE), lane = threadIdx.x % NYS_WAVE;
  const int ga = rr_player(blockIdx.x, round, ngw);
  const int gb = rr_player(ngw - 1 - blockIdx.x, round, ngw);
  const int half = ell / 2, cu = ga * G + wid, cv = gb * G + wid;
  // column wid of the second group straight into LDS (16 bytes per lane)
  if (cv < ell) {
    const int cb = ell * 8;
    const char* src = (const char*)(Xc + (int64_t)cv * ell);
    char* dst = (char*)(cols + (int64_t)wid * ell);
    for (int off = 0; off < cb; off += 1024)
      if (off + lane * 16 < cb)
        __builtin_amdgcn_global_load_lds((const void*)(src + off + lane * 16),
                                         (__attribute__((address_space(3))) void*)(dst + off), 16, 0, 0);
  }
  // column wid of the first group into registers
  const bool live = cu < ell;
  f64x2 u[C2];
  const f64x2* up = (const f64x2*)(Xc + (int64_t)(live ? cu : 0) * ell);
#pragma unroll
  for (int t = 0; t < C2; ++t) {
    const int i = lane + t * NYS_WAVE;
    u[t] = live && i < half ? up[i] : f64x2{0.0, 0.0};
  }
  // round 0 pairs each wave with the LDS column it loaded itself, so its own
  // wait suffices; the barrier after each round orders the rest
  __builtin_amdgcn_s_waitcnt(0);
  unsigned nrot = 0;
  for (int r = 0; r < G; ++r) {
    const int q = (wid + r) % G;
    if (live && gb * G + q < ell && jacobi_pair_held<C2>(u, cols + (int64_t)q * ell, ell, tol, lane)) ++nrot;
    __syncthreads();
  }
  if (live) {
    f64x2* uw = (f64x2*)(Xc + (int64_t)cu * ell);
#pragma unroll
    for (int t = 0; t < C2; ++t) {
      const int i = lane + t * NYS_WAVE;
      if (i < half) uw[i] = u[t];
    }
  }
  if (cv < ell) {
    const f64x2* srcl = (const f64x2*)(cols + (int64_t)wid * ell);
    f64x2* dstg = (f64x2*)(Xc + (int64_t)cv * ell);
    for (int i = lane; i < half; i += NYS_WAVE) dstg[i] = srcl[i];
  }
  if (lane == 0 && nrot) atomicAdd(rotations, nrot);
}

template <int JG, int CH>
void launch_jacobi_round(hipStream_t st, int ngp, size_t lds, double* Xc, int ell, int round, double tol, unsigned* rot) {
  if (round == 0)
    hipLaunchKernelGGL((k_jacobi_block_round<JG, CH, true>), dim3(ngp / 2), dim3(JG * NYS_WAVE), lds, st, Xc, ell, ngp, round, tol, rot);
  else
    hipLaunchKernelGGL((k_jacobi_block_round<JG, CH, false>), dim3(ngp / 2), dim3(JG * NYS_WAVE), lds, st, Xc, ell, ngp, round, tol, rot);
}
template <int JG, int CH>
hipError_t jacobi_lds_attr(size_t lds) {
  hipError_t e = hipFuncSetAttribute((const void*)k_jacobi_block_round<JG, CH, true>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  return hipFuncSetAttribute((const void*)k_jacobi_block_round<JG, CH, false>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
}
// One sweep of the wide variant: the pairs inside each group of 2*JG columns,
// then the ngw - 1 rounds across groups.
template <int JG, int C2>
void launch_jacobi_wide_sweep(hipStream_t st, int ngw, size_t lds, double* Xc, int ell, double tol, unsigned* rot) {
  hipLaunchKernelGGL((k_jacobi_block_round<JG, 32, true>), dim3(ngw), dim3(JG * NYS_WAVE), lds, st, Xc, ell, 2 * ngw, -1, tol, rot);
  for (int round = 0; round < ngw - 1; ++round)
    hipLaunchKernelGGL((k_jacobi_wide_round<2 * JG, C2>), dim3(ngw / 2), dim3(2 * JG * NYS_WAVE), lds, st, Xc, ell, ngw, round, tol, rot);
}
template <int JG, int C2>
hipError_t jacobi_wide_attr(size_t lds) {
  hipError_t e = hipFuncSetAttribute((const void*)k_jacobi_block_round<JG, 32, true>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  return hipFuncSetAttribute((const void*)k_jacobi_wide_round<2 * JG, C2>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
}

__global__ __launch_bounds__(DB) void k_transpose_sq(const double* X, double* Y, int ell) {
  for (int64_t idx = (int64_t)blockIdx.x * DB + threadIdx.x; idx < (int64_t)ell * ell;
       idx += (int64_t)gridDim.x * DB) {
    const int i = (int)(idx / ell), j = (int)(idx % ell);
    Y[(int64_t)j * ell + i] = X[idx];
  }
}

// Squared column norms, one wave per column.
__global__ __launch_bounds__(NYS_BLOCK) void k_jacobi_norms(const double* Xc, int ell, double* nrm) {
  const int k = blockIdx.x * (NYS_BLOCK / NYS_WAVE) + threadIdx.x / NYS_WAVE;
  const int lane = threadIdx.x % NYS_WAVE;
  if (k >= ell) return;
  double s = 0.0;
  for (int i = lane; i < ell; i += NYS_WAVE) s = fma(Xc[(int64_t)k * ell + i], Xc[(int64_t)k * ell + i], s);
  s = wave_sum_dpp(s);
  if (lane == 0) nrm[k] = s;
}

// Column k of the result: its rank in descending norm (ties by index) is its
// position; U (row-major) receives the normalised column there, sig2 its norm.
__global__ __launch_bounds__(NYS_BLOCK) void k_jacobi_place(const double* Xc, int ell, const double* nrm,
                                                            double* U, double* sig2) {
  __shared__ int cnt[NYS_BLOCK / NYS_WAVE];
  const int k = blockIdx.x;
  const double nk = nrm[k];
  int c = 0;
  for (int j = threadIdx.x; j < ell; j += NYS_BLOCK) c += (nrm[j] > nk || (nrm[j] == nk && j < k)) ? 1 : 0;
  for (int off = NYS_WAVE / 2; off > 0; off >>= 1) c += __shfl_down(c, off, NYS_WAVE);
  if (threadIdx.x % NYS_WAVE == 0) cnt[threadIdx.x / NYS_WAVE] = c;
  __syncthreads();
  int rank = 0;
  for (int w = 0; w < NYS_BLOCK / NYS_WAVE; ++w) rank += cnt[w];
  const double inv = nk > 0.0 ? 1.0 / sqrt(nk) : 0.0;
  if (threadIdx.x == 0) sig2[rank] = nk;
  for (int i = threadIdx.x; i < ell; i += NYS_BLOCK) U[(int64_t)i * ell + rank] = Xc[(int64_t)k * ell + i] * inv;
}

// ---------------------------------------------------------------- Philox4x32-10
__device__ __forceinline__ void philox10(uint32_t c[4], uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r > 0) {
      k0 += 0x9E3779B9u;
      k1 += 0xBB67AE85u;
    }
    const uint64_t p0 = (uint64_t)0xD2511F53u * c[0];
    const uint64_t p1 = (uint64_t)0xCD9E8D57u * c[2];
    const uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    const uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    const uint32_t n0 = hi1 ^ c[1] ^ k0, n2 = hi0 ^ c[3] ^ k1;
    c[0] = n0;
    c[1] = lo1;
    c[2] = n2;
    c[3] = lo0;
  }
}

__device__ __forceinline__ double u53(uint32_t a, uint32_t b) {
  const uint64_t v = ((uint64_t)a << 32) | b;
  return (double)(v >> 11) * 0x1.0p-53 + 0x1.0p-54;
}

__global__ __launch_bounds__(NYS_BLOCK) void k_philox_gauss(int64_t count, uint64_t seed,
                                                            uint64_t counter, double* out) {
  const int64_t npairs = (count + 1) / 2;
  for (int64_t pi = (int64_t)blockIdx.x * NYS_BLOCK + threadIdx.x; pi < npairs;
       pi += (int64_t)gridDim.x * NYS_BLOCK) {
    uint32_t c[4] = {(uint32_t)pi, (uint32_t)((uint64_t)pi >> 32), (uint32_t)counter,
                     (uint32_t)(counter >> 32)};
    philox10(c, (uint32_t)seed, (uint32_t)(seed >> 32));
    const double u1 = u53(c[0], c[1]), u2 = u53(c[2], c[3]);
    const double r = sqrt(-2.0 * log(u1));
    double sn, cs;
    sincos(2.0 * M_PI * u2, &sn, &cs);
    const int64_t e = 2 * pi;
    out[e] = r * cs;
    if (e + 1 < count) out[e + 1] = r * sn;
  }
}

// ---------------------------------------------------------------- BF16 rounding
__device__ __forceinline__ uint16_t f32_bf16_rne(float f) {
  uint32_t u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

__global__ __launch_bounds__(NYS_BLOCK) void k_to_bf16(const double* x, uint16_t* out, int64_t n) {
  for (int64_t j = (int64_t)blockIdx.x * NYS_BLOCK + threadIdx.x; j < n; j += (int64_t)gridDim.x * NYS_BLOCK)
    out[j] = f32_bf16_rne((float)x[j]);
}

__global__ __launch_bounds__(NYS_BLOCK) void k_f32_to_bf16(const float* x, int64_t rows, int64_t cols,
                                                           int64_t ld, uint16_t* out) {
  const int64_t total = rows * cols;
  for (int64_t idx = (int64_t)blockIdx.x * NYS_BLOCK + threadIdx.x; idx < total;
       idx += (int64_t)gridDim.x * NYS_BLOCK) {
    const int64_t i = idx / cols, j = idx % cols;
    out[i * cols + j] = f32_bf16_rne(x[i * ld + j]);
  }
}

__global__ void k_zero_u32(unsigned* p, int64_t n) {
  for (int64_t j = (int64_t)blockIdx.x * NYS_BLOCK + threadIdx.x; j < n; j += (int64_t)gridDim.x * NYS_BLOCK) p[j] = 0u;
}

unsigned grid_for(int64_t n) {
  int64_t b = (n + NYS_BLOCK - 1) / NYS_BLOCK;
  return (unsigned)std::max<int64_t>(1, std::min<int64_t>(b, 8192));
}

}  // namespace

// FP64 operands, B not transposed: the matrix-core kernel
int gemm_f64_mfma(nys_handle h, bool transA, int64_t M, int64_t N, int64_t K, const double* A, int64_t lda,
                  const double* B, int64_t ldb, double* C, int64_t ldc, const double* row_scale, bool b_upper) {
  const bool sym = transA && A == B && lda == ldb && M == N && !row_scale && !b_upper;
  const int64_t tm = (M + MBM - 1) / MBM, tn = (N + MBN - 1) / MBN;
  const int64_t active = sym ? tm * (tm + 1) / 2 : tm * tn;
  // split K so that the blocks fill whole rounds of 512 (two per compute
  // unit) as far as possible, each split at least 512 long
  int64_t nsplit = 1;
  if (active < 512 && K > 1024) {
    double best_eff = 0.0;
    for (int64_t sp = 1; sp <= std::min<int64_t>(64, K / 512); ++sp) {
      const int64_t blocks = active * sp;
      const double eff = (double)blocks / (512.0 * (double)((blocks + 511) / 512));
      if (eff > best_eff + 0.02) {
        best_eff = eff;
        nsplit = sp;
      }
      if (best_eff >= 0.85) break;
    }
  }
  int64_t klen = (K + nsplit - 1) / nsplit;
  klen = std::max<int64_t>(MBK, (klen + MBK - 1) / MBK * MBK);
  nsplit = std::max<int64_t>(1, (K + klen - 1) / klen);
  double* out = C;
  int64_t ldo = ldc;
  if (nsplit > 1) {
    NYS_CHECK(ws(h, WS_SK_SPLIT, (size_t)nsplit * M * N, &out));
    ldo = N;
  }
  const dim3 g((unsigned)tn, (unsigned)tm, (unsigned)nsplit), b(NYS_BLOCK);
  const double* rs = nsplit > 1 ? nullptr : row_scale;
  const int ps = prof_begin(h, NYS_K_GEMM_F64);
  if (sym)
    hipLaunchKernelGGL((k_gemm64_mfma<true, false, true>), g, b, 0, h->stream, M, N, K, A, lda, B, ldb, out, ldo, rs, klen);
  else if (transA && b_upper)
    hipLaunchKernelGGL((k_gemm64_mfma<true, true, false>), g, b, 0, h->stream, M, N, K, A, lda, B, ldb, out, ldo, rs, klen);
  else if (transA)
    hipLaunchKernelGGL((k_gemm64_mfma<true, false, false>), g, b, 0, h->stream, M, N, K, A, lda, B, ldb, out, ldo, rs, klen);
  else if (b_upper)
    hipLaunchKernelGGL((k_gemm64_mfma<false, true, false>), g, b, 0, h->stream, M, N, K, A, lda, B, ldb, out, ldo, rs, klen);
  else
    hipLaunchKernelGGL((k_gemm64_mfma<false, false, false>), g, b, 0, h->stream, M, N, K, A, lda, B, ldb, out, ldo, rs, klen);
  NYS_LAUNCH_CHECK(h);
  prof_end(h, ps);
  if (nsplit > 1) {
    hipLaunchKernelGGL(k_splitk_reduce, dim3(grid_for(M * N)), dim3(NYS_BLOCK), 0, h->stream, M, N,
                       (int)nsplit, out, C, ldc, row_scale);
    NYS_LAUNCH_CHECK(h);
  }
  return NYS_OK;
}

int gemm_f64(nys_handle h, bool transA, bool transB, int64_t M, int64_t N, int64_t K,
             const void* A, nys_dtype adt, int64_t lda, const double* B, int64_t ldb, double* C,
             int64_t ldc, const double* row_scale, bool b_upper) {
  if (M == 0 || N == 0) return NYS_OK;
  // the grid's y dimension counts GBM-row tiles and stops at 65535: taller
  // products run as one launch per chunk of rows
  constexpr int64_t kMaxRows = 65535LL * GBM;
  if (M > kMaxRows) {
    const int64_t es = adt == NYS_F64 ? 8 : adt == NYS_F32 ? 4 : 2;
    for (int64_t r0 = 0; r0 < M; r0 += kMaxRows) {
      const int64_t mc = std::min(kMaxRows, M - r0);
      const char* Ac = (const char*)A + (transA ? r0 : r0 * lda) * es;
      NYS_CHECK(gemm_f64(h, transA, transB, mc, N, K, Ac, adt, lda, B, ldb, C + r0 * ldc, ldc,
                         row_scale ? row_scale + r0 : nullptr, b_upper));
    }
    return NYS_OK;
  }
  if (adt == NYS_F64 && !transB && K > 0)
    return gemm_f64_mfma(h, transA, M, N, K, (const double*)A, lda, B, ldb, C, ldc, row_scale, b_upper);
  const int64_t tiles = ((M + GBM - 1) / GBM) * ((N + GBN - 1) / GBN);
  int64_t nsplit = 1;
  if (tiles < 512 && K > 512) {
    nsplit = std::min<int64_t>((1024 + tiles - 1) / tiles, (K + 255) / 256);
    nsplit = std::max<int64_t>(1, std::min<int64_t>(nsplit, 256));
  }
  int64_t klen = (K + nsplit - 1) / nsplit;
  klen = std::max<int64_t>(GBK, (klen + GBK - 1) / GBK * GBK);
  nsplit = std::max<int64_t>(1, (K + klen - 1) / klen);
  double* out = C;
  int64_t ldo = ldc;
  if (nsplit > 1) {
    NYS_CHECK(ws(h, WS_SK_SPLIT, (size_t)nsplit * M * N, &out));
    ldo = N;
  }
  dim3 g((unsigned)((N + GBN - 1) / GBN), (unsigned)((M + GBM - 1) / GBM), (unsigned)nsplit);
  const double* rs = nsplit > 1 ? nullptr : row_scale;
  if (K == 0) {
    // empty contraction: C = 0
    dim3 g1((unsigned)((N + GBN - 1) / GBN), (unsigned)((M + GBM - 1) / GBM), 1);
    NYS_CHECK(gemm_dispatch<F64>(h, transA, transB, g1, M, N, K, A, lda, B, ldb, C, ldc, nullptr, GBK));
    return NYS_OK;
  }
  const int ps = prof_begin(h, NYS_K_GEMM_F64);
  switch (adt) {
    case NYS_F64: NYS_CHECK(gemm_dispatch<F64>(h, transA, transB, g, M, N, K, A, lda, B, ldb, out, ldo, rs, klen)); break;
    case NYS_F32: NYS_CHECK(gemm_dispatch<F32>(h, transA, transB, g, M, N, K, A, lda, B, ldb, out, ldo, rs, klen)); break;
    default: NYS_CHECK(gemm_dispatch<BF16>(h, transA, transB, g, M, N, K, A, lda, B, ldb, out, ldo, rs, klen)); break;
  }
  prof_end(h, ps);
  if (nsplit > 1) {
    hipLaunchKernelGGL(k_splitk_reduce, dim3(grid_for(M * N)), dim3(NYS_BLOCK), 0, h->stream, M, N,
                       (int)nsplit, out, C, ldc, row_scale);
    NYS_LAUNCH_CHECK(h);
  }
  return NYS_OK;
}

int chol_upper(nys_handle h, double* G, int ell, double shift_abs, double shift_rel, double* fail) {
  if (ell >= 128) {
    // across workgroups (one block would update the whole trailing triangle
    // for each of ell/CP panels)
    const unsigned gsq = (unsigned)std::min<int64_t>(((int64_t)ell * ell + NYS_BLOCK - 1) / NYS_BLOCK, 4096);
    hipLaunchKernelGGL(k_chol_sym, dim3(gsq), dim3(NYS_BLOCK), 0, h->stream, G, ell);
    hipLaunchKernelGGL(k_chol_shift, dim3(1), dim3(NYS_BLOCK), 0, h->stream, G, ell, shift_abs, shift_rel, fail);
    for (int k0 = 0; k0 < ell; k0 += CP) {
      const int nb = std::min(CP, ell - k0);
      hipLaunchKernelGGL(k_chol_diag, dim3(1), dim3(NYS_WAVE), 0, h->stream, G, ell, k0, nb, fail);
      const int rest = ell - k0 - nb;
      if (rest > 0) {
        hipLaunchKernelGGL(k_chol_row, dim3((unsigned)((rest + NYS_BLOCK - 1) / NYS_BLOCK)), dim3(NYS_BLOCK), 0,
                           h->stream, G, ell, k0, nb);
        const int nt = (rest + CT - 1) / CT;
        hipLaunchKernelGGL(k_chol_update, dim3((unsigned)(nt * (nt + 1) / 2)), dim3(NYS_BLOCK), 0, h->stream, G,
                           ell, k0, nb);
      }
    }
    hipLaunchKernelGGL(k_chol_lower_zero, dim3(gsq), dim3(NYS_BLOCK), 0, h->stream, G, ell);
    NYS_LAUNCH_CHECK(h);
    return NYS_OK;
  }
  // panel height: the largest power of two <= 32 whose NB x ell panel fits in
  // 60 KB of LDS (the kernel's static LDS and 64 KB per block stay clear)
  int nb = 32;
  while (nb > 1 && (size_t)nb * ell * sizeof(double) > 61440) nb /= 2;
  if (ell >= 2 * nb && nb >= 4) {
    hipLaunchKernelGGL(k_chol_upper_blocked, dim3(1), dim3(DB), (size_t)nb * ell * sizeof(double), h->stream,
                       G, ell, nb, shift_abs, shift_rel, fail);
  } else {
    hipLaunchKernelGGL(k_chol_upper, dim3(1), dim3(DB), 0, h->stream, G, ell, shift_abs, shift_rel, fail);
  }
  NYS_LAUNCH_CHECK(h);
  return NYS_OK;
}

int tri_inv_upper(nys_handle h, const double* C, double* Cinv, int ell, double* work) {
  if (ell > 256 && work) {
    // blocked: diagonal blocks of 64 in parallel, then pairs of inverted
    // blocks of size s joined into blocks of 2 s for s = 64, 128, ...:
    // [A B; 0 D]^-1 = [A^-1, -A^-1 (B D^-1); 0, D^-1]
    constexpr int NBD = 64;
    const int nblk = (ell + NBD - 1) / NBD;
    NYS_CHECK(fill(h, Cinv, (int64_t)ell * ell, 0.0));
    hipLaunchKernelGGL(k_tri_inv_diag, dim3((unsigned)nblk, (unsigned)(NBD / TRI_WAVES)), dim3(TRI_WAVES * NYS_WAVE), 0,
                       h->stream, C, Cinv, ell, NBD);
    NYS_LAUNCH_CHECK(h);
    for (int sz = NBD; sz < ell; sz *= 2) {
      for (int r0 = 0; r0 + sz < ell; r0 += 2 * sz) {
        const int r1 = r0 + sz, r2 = std::min(r0 + 2 * sz, ell), n2 = r2 - r1;
        // work (sz x n2, ld n2) = B D^-1, B = C[r0:r1, r1:r2], D^-1 = Cinv[r1:r2, r1:r2]
        NYS_CHECK(gemm_f64(h, false, false, sz, n2, n2, C + (int64_t)r0 * ell + r1, NYS_F64, ell,
                           Cinv + (int64_t)r1 * ell + r1, ell, work, n2, nullptr, true));
        // Cinv[r0:r1, r1:r2] = -A^-1 work, A^-1 = Cinv[r0:r1, r0:r1]
        NYS_CHECK(gemm_f64(h, false, false, sz, n2, sz, Cinv + (int64_t)r0 * ell + r0, NYS_F64, ell, work, n2,
                           Cinv + (int64_t)r0 * ell + r1, ell, nullptr));
        hipLaunchKernelGGL(k_scale_block, dim3(grid_for((int64_t)sz * n2)), dim3(NYS_BLOCK), 0, h->stream,
                           Cinv + (int64_t)r0 * ell + r1, (int64_t)ell, sz, n2, -1.0);
        NYS_LAUNCH_CHECK(h);
      }
    }
    return NYS_OK;
  }
  const dim3 g((unsigned)((ell + TRI_WAVES - 1) / TRI_WAVES)), b(TRI_WAVES * NYS_WAVE);
  if (ell <= 16 * NYS_WAVE) {
    hipLaunchKernelGGL(k_tri_inv_cols<16>, g, b, 0, h->stream, C, Cinv, ell);
  } else if (ell <= 32 * NYS_WAVE) {
    hipLaunchKernelGGL(k_tri_inv_cols<32>, g, b, 0, h->stream, C, Cinv, ell);
  } else if (ell <= 64 * NYS_WAVE) {
    hipLaunchKernelGGL(k_tri_inv_cols<64>, g, b, 0, h->stream, C, Cinv, ell);
  } else {
    hipLaunchKernelGGL(k_tri_inv_upper, dim3(1), dim3(DB), 0, h->stream, C, Cinv, ell);
  }
  NYS_LAUNCH_CHECK(h);
  return NYS_OK;
}

int small_mm(nys_handle h, const double* C1, const double* C2, double* C3, int ell) {
  return gemm_f64(h, false, false, ell, ell, ell, C1, NYS_F64, ell, C2, ell, C3, ell, nullptr);
}

int jacobi_svd(nys_handle h, double* X, int ell, double* sig2, double* work) {
  // work: ell*ell doubles (column storage), a counter word, a spare word and
  // ell doubles of column norms
  double* Xc = work;
  unsigned* rot = reinterpret_cast<unsigned*>(work + (int64_t)ell * ell);
  hipLaunchKernelGGL(k_transpose_sq, dim3(grid_for((int64_t)ell * ell)), dim3(DB), 0, h->stream, X, Xc, ell);
  NYS_LAUNCH_CHECK(h);
  const int np = ell + (ell & 1);
  // rotation threshold ell * eps: the computed cosine of two columns of length
  // ell carries a rounding error up to about ell * eps, so a smaller threshold
  // keeps rotating on noise and only stops when a sweep happens to find none
  const double tol = (double)ell * 2.220446049250313e-16;
  // Group sizes, from sweep timings on gfx950 (ell = 64 to 1600): eight
  // waves per block beat sixteen (fewer waves per SIMD shorten each round
  // more than the extra launches cost) and match twelve at ell = 1600.
  // Block variant: JG = 8 (16 columns in LDS) when they fit in the 160 KB of
  // LDS (ell <= 1280), else the largest of 6, 4, 2 that fits (0: per-pair
  // launches).  Pairs are held in registers up to ell = 64 * CH, with CH = 4,
  // 8, 16 or 32 by ell so that no wave rotates padding; beyond, in LDS.
  int jg = 0;
  for (int c : {8, 6, 4, 2})
    if ((size_t)2 * c * ell * sizeof(double) <= (size_t)160 * 1024) {
      jg = c;
      break;
    }
  const int ng = jg ? (ell + jg - 1) / jg : 0;
  const int ngp = ng + (ng & 1);
  const size_t lds = (size_t)2 * jg * ell * sizeof(double);
  const bool regs = ell <= 32 * NYS_WAVE;
  const int ch = ell <= 4 * NYS_WAVE ? 4 : ell <= 8 * NYS_WAVE ? 8 : ell <= 16 * NYS_WAVE ? 16 : 32;
  auto dispatch = [&](int round) {
    switch (jg) {
      case 8:
        if (ch == 4) launch_jacobi_round<8, 4>(h->stream, ngp, lds, Xc, ell, round, tol, rot);
        else if (ch == 8) launch_jacobi_round<8, 8>(h->stream, ngp, lds, Xc, ell, round, tol, rot);
        else if (ch == 16) launch_jacobi_round<8, 16>(h->stream, ngp, lds, Xc, ell, round, tol, rot);
        else launch_jacobi_round<8, 32>(h->stream, ngp, lds, Xc, ell, round, tol, rot);
        break;
      case 6:
        if (regs) launch_jacobi_round<6, 32>(h->stream, ngp, lds, Xc, ell, round, tol, rot);
        else launch_jacobi_round<6, 0>(h->stream, ngp, lds, Xc, ell, round, tol, rot);
        break;
      case 4:
        if (regs) launch_jacobi_round<4, 32>(h->stream, ngp, lds, Xc, ell, round, tol, rot);
        else launch_jacobi_round<4, 0>(h->stream, ngp, lds, Xc, ell, round, tol, rot);
        break;
      default:
        if (regs) launch_jacobi_round<2, 32>(h->stream, ngp, lds, Xc, ell, round, tol, rot);
        else launch_jacobi_round<2, 0>(h->stream, ngp, lds, Xc, ell, round, tol, rot);
        break;
    }
  };
  // wide variant for even 256 < ell <= 2048: groups of G = 8 columns, each
  // wave of a block holding one in registers (C2 pairs per lane, ell <= 128
  // C2, C2 = 4, 8, 10, 12, 14 or 16 by ell), the other group in LDS
  const bool wide = (ell & 1) == 0 && ell > 4 * NYS_WAVE && ell <= 2048;
  const int ngwide = wide ? (ell + 7) / 8 : 0;
  const int ngw = ngwide + (ngwide & 1);
  const size_t ldsw = (size_t)8 * ell * sizeof(double);
  const int c2w = ell <= 512 ? 4 : ell <= 1024 ? 8 : ell <= 1280 ? 10 : ell <= 1536 ? 12 : ell <= 1792 ? 14 : 16;
  if (wide) {
    hipError_t e = c2w == 4    ? jacobi_wide_attr<4, 4>(ldsw)
                   : c2w == 8  ? jacobi_wide_attr<4, 8>(ldsw)
                   : c2w == 10 ? jacobi_wide_attr<4, 10>(ldsw)
                   : c2w == 12 ? jacobi_wide_attr<4, 12>(ldsw)
                   : c2w == 14 ? jacobi_wide_attr<4, 14>(ldsw)
                               : jacobi_wide_attr<4, 16>(ldsw);
    if (e != hipSuccess) return set_error(h, NYS_EHIP, "Jacobi SVD: LDS attribute: %s", hipGetErrorString(e));
  } else if (jg && lds > 65536) {
    hipError_t e = hipSuccess;
    switch (jg) {
      case 8: e = ch == 16 ? jacobi_lds_attr<8, 16>(lds) : jacobi_lds_attr<8, 32>(lds); break;
      case 6: e = regs ? jacobi_lds_attr<6, 32>(lds) : jacobi_lds_attr<6, 0>(lds); break;
      case 4: e = regs ? jacobi_lds_attr<4, 32>(lds) : jacobi_lds_attr<4, 0>(lds); break;
      default: e = regs ? jacobi_lds_attr<2, 32>(lds) : jacobi_lds_attr<2, 0>(lds); break;
    }
    if (e != hipSuccess) return set_error(h, NYS_EHIP, "Jacobi SVD: LDS attribute: %s", hipGetErrorString(e));
  }
  int sweep = 0;
  const int max_sweeps = 40;
  if (np >= 2) {
    for (; sweep < max_sweeps; ++sweep) {
      NYS_CHECK(zero_u32(h, rot, 1));
      if (wide) {
        if (c2w == 4) launch_jacobi_wide_sweep<4, 4>(h->stream, ngw, ldsw, Xc, ell, tol, rot);
        else if (c2w == 8) launch_jacobi_wide_sweep<4, 8>(h->stream, ngw, ldsw, Xc, ell, tol, rot);
        else if (c2w == 10) launch_jacobi_wide_sweep<4, 10>(h->stream, ngw, ldsw, Xc, ell, tol, rot);
        else if (c2w == 12) launch_jacobi_wide_sweep<4, 12>(h->stream, ngw, ldsw, Xc, ell, tol, rot);
        else if (c2w == 14) launch_jacobi_wide_sweep<4, 14>(h->stream, ngw, ldsw, Xc, ell, tol, rot);
        else launch_jacobi_wide_sweep<4, 16>(h->stream, ngw, ldsw, Xc, ell, tol, rot);
      } else if (jg) {
        for (int round = 0; round < ngp - 1; ++round) dispatch(round);
      } else {
        for (int round = 0; round < np - 1; ++round) {
          hipLaunchKernelGGL(k_jacobi_round, dim3(np / 2), dim3(NYS_WAVE), 0, h->stream, Xc, ell, np,
                             round, tol, rot);
        }
      }
      NYS_LAUNCH_CHECK(h);
      unsigned hrot = 0;
      NYS_HIP(h, hipMemcpyAsync(&hrot, rot, sizeof(unsigned), hipMemcpyDeviceToHost, h->stream));
      NYS_HIP(h, hipStreamSynchronize(h->stream));
      if (hrot == 0) break;
    }
  }
  // normalise the columns and order them by descending norm: U (row-major, in X) and sig2
  double* nrm = work + (int64_t)ell * ell + 2;
  hipLaunchKernelGGL(k_jacobi_norms, dim3((ell + NYS_BLOCK / NYS_WAVE - 1) / (NYS_BLOCK / NYS_WAVE)), dim3(NYS_BLOCK), 0,
                     h->stream, Xc, ell, nrm);
  hipLaunchKernelGGL(k_jacobi_place, dim3(ell), dim3(NYS_BLOCK), 0, h->stream, Xc, ell, nrm, X, sig2);
  NYS_LAUNCH_CHECK(h);
  if (sweep == max_sweeps) return set_error(h, NYS_ENOTPD, "Jacobi SVD did not converge in %d sweeps", max_sweeps);
  return NYS_OK;
}

int zero_u32(nys_handle h, unsigned* p, int64_t count) {
  hipLaunchKernelGGL(k_zero_u32, dim3(grid_for(count)), dim3(NYS_BLOCK), 0, h->stream, p, count);
  NYS_LAUNCH_CHECK(h);
  return NYS_OK;
}

int philox_gaussian(nys_handle h, int64_t m, int ell, uint64_t seed, uint64_t counter, double* out) {
  const int64_t count = m * ell;
  hipLaunchKernelGGL(k_philox_gauss, dim3(grid_for((count + 1) / 2)), dim3(NYS_BLOCK), 0, h->stream,
                     count, seed, counter, out);
  NYS_LAUNCH_CHECK(h);
  return NYS_OK;
}

int to_bf16(nys_handle h, const double* x, uint16_t* out, int64_t count) {
  hipLaunchKernelGGL(k_to_bf16, dim3(grid_for(count)), dim3(NYS_BLOCK), 0, h->stream, x, out, count);
  NYS_LAUNCH_CHECK(h);
  return NYS_OK;
}

int f32_to_bf16(nys_handle h, const float* x, int64_t rows, int64_t cols, int64_t ld, uint16_t* out) {
  hipLaunchKernelGGL(k_f32_to_bf16, dim3(grid_for(rows * cols)), dim3(NYS_BLOCK), 0, h->stream, x, rows,
                     cols, ld, out);
  NYS_LAUNCH_CHECK(h);
  return NYS_OK;
}

}  // namespace nys
