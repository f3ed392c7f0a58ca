// The fused two-pass normal-equation operator v -> A diag(d) A^T v + delta v
// (eq. normal-eq).  Both passes stream A from HBM once with 16-byte
// non-temporal loads and accumulate in FP64 whatever the storage of A.
//
// Pass 1 (w = d .* A^T v): a 2-D grid of (column tile) x (row chunk) blocks.
//   Thread t of a block owns VEC consecutive columns (16 bytes of a row) and
//   walks the rows of its chunk, four rows in flight; v_i is a wave-uniform
//   value.  Partial column sums go to a workspace array and a small second
//   launch sums the chunks in a fixed order (deterministic).  No device-wide
//   fence is used anywhere: on gfx950 an agent-scope fence writes back and
//   invalidates the L2, which would evict w and v for every block.
// Pass 2 (out = A w + delta v): each block owns RB consecutive rows; every
//   16-byte piece of w it loads is reused for RB rows.  Row sums are finished
//   by wave shuffles and LDS.  An optional p^T (M p) dot product is fused as
//   per-block partials summed by a one-block launch.
// Pass 1 over a transposed copy (A^T stored n x m row-major): the same
//   row-streaming shape as pass 2, with rows of A^T in place of rows of A, so
//   each block reads RB whole rows (contiguous runs of m elements) instead of
//   16-byte pieces of ~m rows that lie a full row of A apart.  With 288 GB of
//   HBM the second copy of A is cheap, and the copy itself costs about one
//   pass.

#include "common.hpp"
#include "kernels.hpp"

// Pass-1 launch shape: rows in flight per thread, and the block count the
// row chunking aims for (a few blocks per CU).
#ifndef NYS_T_UNROLL
#define NYS_T_UNROLL 4
#endif
#ifndef NYS_T_TARGET_BLOCKS
#define NYS_T_TARGET_BLOCKS 2048
#endif
// Rows per block of the row-streaming passes on large matrices (pass 2 on A,
// pass 1 on A^T): 1, 2, 4, 8 or 16.
#ifndef NYS_N_RB
#define NYS_N_RB 8
#endif
#ifndef NYS_GEMV_UNROLL
#define NYS_GEMV_UNROLL 1
#endif
#ifndef NYS_N_SPACE
#define NYS_N_SPACE 1
#endif
#ifndef NYS_TT_RB
#define NYS_TT_RB 8
#endif

namespace nys {
namespace {

struct T1Args {
  const double* skip;
  const char* A;
  int64_t m, n, row_bytes;
  const double* v;
  const double* s;
  const double* pold;
  double* pnew;
  const double* beta;
  const double* d;
  const double* x0;
  double sA;
  double* w;
  double* part;
  int rows_per_chunk;
  int nchunks;
};

template <class T, bool FUSEDP, bool VECLOAD>
__global__ __launch_bounds__(NYS_BLOCK) void k_gemv_t(T1Args a) {
  using raw = typename T::raw;
  constexpr int VEC = T::vec;
  if (a.skip && *a.skip != 0.0) return;
  const int64_t col0 = ((int64_t)blockIdx.x * NYS_BLOCK + threadIdx.x) * VEC;
  const int64_t r0 = (int64_t)blockIdx.y * a.rows_per_chunk;
  const int64_t r1 = min(a.m, r0 + (int64_t)a.rows_per_chunk);
  const double beta = FUSEDP ? *a.beta : 0.0;
  auto rowv = [&](int64_t i) -> double {
    if constexpr (FUSEDP) return a.s[i] + beta * a.pold[i];
    else return a.v[i];
  };
  double acc[VEC];
#pragma unroll
  for (int e = 0; e < VEC; ++e) acc[e] = 0.0;

  if (VECLOAD && col0 + VEC <= a.n) {
    const char* p = a.A + r0 * a.row_bytes + col0 * (int64_t)sizeof(raw);
    int64_t i = r0;
    constexpr int U = NYS_T_UNROLL;     // rows in flight per thread
    for (; i + U <= r1; i += U) {
      u32x4 uu[U];
#pragma unroll
      for (int t = 0; t < U; ++t) uu[t] = ld_stream16(p + t * a.row_bytes);
      double vv[U];
#pragma unroll
      for (int t = 0; t < U; ++t) vv[t] = rowv(i + t);
#pragma unroll
      for (int t = 0; t < U; ++t) {
        double e0[VEC];
        Unpack<T>::run(uu[t], e0);
#pragma unroll
        for (int e = 0; e < VEC; ++e) acc[e] = fma(e0[e], vv[t], acc[e]);
      }
      p += U * a.row_bytes;
    }
    for (; i < r1; ++i) {
      const u32x4 u0 = ld_stream16(p);
      double e0[VEC];
      Unpack<T>::run(u0, e0);
      const double v0 = rowv(i);
#pragma unroll
      for (int e = 0; e < VEC; ++e) acc[e] = fma(e0[e], v0, acc[e]);
      p += a.row_bytes;
    }
  } else if (col0 < a.n) {
    for (int64_t i = r0; i < r1; ++i) {
      const raw* row = (const raw*)(a.A + i * a.row_bytes);
      const double v0 = rowv(i);
#pragma unroll
      for (int e = 0; e < VEC; ++e)
        if (col0 + e < a.n) acc[e] = fma(to_f64(row[col0 + e]), v0, acc[e]);
    }
  }

  if constexpr (FUSEDP) {
    if (blockIdx.x == 0)
      for (int64_t i = r0 + threadIdx.x; i < r1; i += NYS_BLOCK) a.pnew[i] = a.s[i] + beta * a.pold[i];
  }

  if (a.nchunks == 1) {
#pragma unroll
    for (int e = 0; e < VEC; ++e) {
      const int64_t j = col0 + e;
      if (j < a.n) {
        double val = a.sA * acc[e] + (a.x0 ? a.x0[j] : 0.0);
        if (a.d) val *= a.d[j];
        a.w[j] = val;
      }
    }
    return;
  }
  double* mypart = a.part + (int64_t)blockIdx.y * a.n;
#pragma unroll
  for (int e = 0; e < VEC; ++e)
    if (col0 + e < a.n) mypart[col0 + e] = acc[e];
}

// Second stage of pass 1: w[j] = d[j] * (sA * sum_c part[c][j] + x0[j]), chunks
// summed in a fixed order (deterministic).  A separate launch: the kernel
// boundary orders the partial sums, so no device-wide fence is needed.
__global__ __launch_bounds__(NYS_BLOCK) void k_gemv_t_finish(T1Args a) {
  if (a.skip && *a.skip != 0.0) return;
  for (int64_t j = (int64_t)blockIdx.x * NYS_BLOCK + threadIdx.x; j < a.n;
       j += (int64_t)gridDim.x * NYS_BLOCK) {
    double s = 0.0;
    for (int c = 0; c < a.nchunks; ++c) s += a.part[(int64_t)c * a.n + j];
    double val = a.sA * s + (a.x0 ? a.x0[j] : 0.0);
    if (a.d) val *= a.d[j];
    a.w[j] = val;
  }
}

// Sum of per-block partials into one device word (one block, fixed order).
__global__ __launch_bounds__(NYS_BLOCK) void k_sum_partials(const double* skip, const double* part,
                                                            int nb, double* out) {
  __shared__ double smem[NYS_BLOCK / NYS_WAVE];
  if (skip && *skip != 0.0) return;
  double s[1] = {0.0};
  for (int b = threadIdx.x; b < nb; b += NYS_BLOCK) s[0] += part[b];
  block_sum<1>(s, smem);
  if (threadIdx.x == 0) *out = s[0];
}

struct T2Args {
  const double* skip;
  const char* A;
  int64_t m, n, row_bytes;
  const double* w;
  const double* v;
  const double* x0;
  double sA, sV;
  double* out;
  double* dot_out;
  double* dpart;
  double shift;         // added to every output
};

// SQ: the entries of A are squared (sum_j A_ij^2 w_j: the diagonal of A diag(w) A^T).
template <class T, int RB, bool VECLOAD, bool SQ>
__global__ __launch_bounds__(NYS_BLOCK) void k_gemv_n(T2Args a) {
  using raw = typename T::raw;
  constexpr int VEC = T::vec;
  __shared__ double smem[RB * (NYS_BLOCK / NYS_WAVE) + NYS_BLOCK / NYS_WAVE];
  if (a.skip && *a.skip != 0.0) return;
  // rows i0, i0 + SP, ..., i0 + (RB - 1) SP: blocks of SP consecutive indices
  // interleave their rows within groups of RB SP rows
  constexpr int64_t SP = RB > 1 ? NYS_N_SPACE : 1;
  const int64_t i0 = ((int64_t)blockIdx.x / SP) * RB * SP + (int64_t)blockIdx.x % SP;
  int nr = i0 < a.m ? (int)min((int64_t)RB, (a.m - i0 + SP - 1) / SP) : 0;
  double acc[RB];
#pragma unroll
  for (int r = 0; r < RB; ++r) acc[r] = 0.0;

  int64_t jtail = 0;
  if (VECLOAD) {
    const int64_t nv = a.n / VEC;   // full 16-byte pieces per row
    const char* base = a.A + i0 * a.row_bytes;
#pragma unroll NYS_GEMV_UNROLL
    for (int64_t jv = threadIdx.x; jv < nv; jv += NYS_BLOCK) {
      const int64_t j = jv * VEC;
      u32x4 u[RB];
#pragma unroll
      for (int r = 0; r < RB; ++r)
        if (r < nr) u[r] = ld_stream16(base + r * SP * a.row_bytes + j * (int64_t)sizeof(raw));
      double wv[VEC];
      ld_f64s<VEC>(a.w + j, wv);
#pragma unroll
      for (int r = 0; r < RB; ++r) {
        if (r < nr) {
          double e[VEC];
          Unpack<T>::run(u[r], e);
#pragma unroll
          for (int k = 0; k < VEC; ++k) acc[r] = fma(SQ ? e[k] * e[k] : e[k], wv[k], acc[r]);
        }
      }
    }
    jtail = nv * VEC;
  }
  for (int64_t j = jtail + threadIdx.x; j < a.n; j += NYS_BLOCK) {
    const double wj = a.w[j];
#pragma unroll
    for (int r = 0; r < RB; ++r)
      if (r < nr) {
        const double e = to_f64(((const raw*)(a.A + (i0 + r * SP) * a.row_bytes))[j]);
        acc[r] = fma(SQ ? e * e : e, wj, acc[r]);
      }
  }
  block_sum<RB>(acc, smem);
  double dotc = 0.0;
  if (threadIdx.x == 0) {
#pragma unroll
    for (int r = 0; r < RB; ++r) {
      if (r < nr) {
        const int64_t i = i0 + r * SP;
        const double vi = a.v ? a.v[i] : 0.0;
        const double o = a.sA * acc[r] + a.sV * vi + (a.x0 ? a.x0[i] : 0.0) + a.shift;
        a.out[i] = o;
        dotc += o * vi;
      }
    }
  }
  if (a.dot_out && threadIdx.x == 0) a.dpart[blockIdx.x] = dotc;
}

// Pass 1 on A^T (rows = n rows of A^T, cols = m):
//   w[j] = d[j] * (sA * sum_i At[j,i] v_i + x0[j]).
// (The CG direction update runs before it as its own small kernel: fusing it
// here makes every block read two vectors instead of one, which measured ~4%
// slower than the extra launch.)
struct TTArgs {
  const double* skip;
  const char* At;
  int64_t rows, cols, row_bytes;
  const double* v;
  const double* d;
  const double* x0;
  double sA;
  double* w;
};

template <class T, int RB, bool VECLOAD>
__global__ __launch_bounds__(NYS_BLOCK) void k_gemv_tt(TTArgs a) {
  using raw = typename T::raw;
  constexpr int VEC = T::vec;
  __shared__ double smem[RB * (NYS_BLOCK / NYS_WAVE)];
  if (a.skip && *a.skip != 0.0) return;
  const int64_t j0 = (int64_t)blockIdx.x * RB;
  const int nr = (int)max((int64_t)0, min((int64_t)RB, a.rows - j0));
  double acc[RB];
#pragma unroll
  for (int r = 0; r < RB; ++r) acc[r] = 0.0;

  int64_t itail = 0;
  if (VECLOAD) {
    const int64_t nv = a.cols / VEC;
    const char* base = a.At + j0 * a.row_bytes;
#pragma unroll NYS_GEMV_UNROLL
    for (int64_t iv = threadIdx.x; iv < nv; iv += NYS_BLOCK) {
      const int64_t i = iv * VEC;
      u32x4 u[RB];
#pragma unroll
      for (int r = 0; r < RB; ++r)
        if (r < nr) u[r] = ld_stream16(base + r * a.row_bytes + i * (int64_t)sizeof(raw));
      double vv[VEC];
      ld_f64s<VEC>(a.v + i, vv);
#pragma unroll
      for (int r = 0; r < RB; ++r) {
        if (r < nr) {
          double e[VEC];
          Unpack<T>::run(u[r], e);
#pragma unroll
          for (int k = 0; k < VEC; ++k) acc[r] = fma(e[k], vv[k], acc[r]);
        }
      }
    }
    itail = nv * VEC;
  }
  for (int64_t i = itail + threadIdx.x; i < a.cols; i += NYS_BLOCK) {
    const double vi = a.v[i];
#pragma unroll
    for (int r = 0; r < RB; ++r)
      if (r < nr) acc[r] = fma(to_f64(((const raw*)(a.At + (j0 + r) * a.row_bytes))[i]), vi, acc[r]);
  }
  block_sum<RB>(acc, smem);
  if (threadIdx.x == 0) {
#pragma unroll
    for (int r = 0; r < RB; ++r) {
      if (r < nr) {
        const int64_t j = j0 + r;
        double val = a.sA * acc[r] + (a.x0 ? a.x0[j] : 0.0);
        if (a.d) val *= a.d[j];
        a.w[j] = val;
      }
    }
  }
}

// pnew = s + beta * pold (beta from a device word), skip-aware.
__global__ __launch_bounds__(NYS_BLOCK) void k_dir_update(const double* skip, const double* s,
                                                          const double* pold, const double* beta,
                                                          double* pnew, int64_t m) {
  if (skip && *skip != 0.0) return;
  const double b = *beta;
  for (int64_t i = (int64_t)blockIdx.x * NYS_BLOCK + threadIdx.x; i < m; i += (int64_t)gridDim.x * NYS_BLOCK)
    pnew[i] = s[i] + b * pold[i];
}

// At (n x m, row pitch ldt_bytes) = A^T through a 64 x 64 LDS tile.
template <class raw>
__global__ __launch_bounds__(NYS_BLOCK) void k_transpose(const char* A, int64_t m, int64_t n,
                                                         int64_t lda_bytes, char* At, int64_t ldt_bytes) {
  __shared__ raw tile[64][65];
  const int64_t j0 = (int64_t)blockIdx.x * 64, i0 = (int64_t)blockIdx.y * 64;
  const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
  for (int r = ty; r < 64; r += NYS_BLOCK / 64) {
    const int64_t i = i0 + r, j = j0 + tx;
    if (i < m && j < n) tile[r][tx] = ((const raw*)(A + i * lda_bytes))[j];
  }
  __syncthreads();
  for (int r = ty; r < 64; r += NYS_BLOCK / 64) {
    const int64_t j = j0 + r, i = i0 + tx;
    if (j < n && i < m) ((raw*)(At + j * ldt_bytes))[i] = tile[tx][r];
  }
}

int elem_size(nys_dtype dt) { return dt == NYS_F64 ? 8 : dt == NYS_F32 ? 4 : 2; }

bool vec_ok(const nys_matrix* A) {
  const int es = elem_size(A->dtype);
  return ((uintptr_t)A->data % 16 == 0) && ((A->ld * es) % 16 == 0);
}

template <class T, bool FUSEDP, bool VECLOAD>
void launch_t(dim3 g, T1Args& k, hipStream_t st) {
  hipLaunchKernelGGL((k_gemv_t<T, FUSEDP, VECLOAD>), g, dim3(NYS_BLOCK), 0, st, k);
}

template <class T>
void dispatch_t(dim3 g, T1Args& k, bool fused, bool vecload, hipStream_t st) {
  if (fused) {
    if (vecload) launch_t<T, true, true>(g, k, st);
    else launch_t<T, true, false>(g, k, st);
  } else {
    if (vecload) launch_t<T, false, true>(g, k, st);
    else launch_t<T, false, false>(g, k, st);
  }
}

template <class T, int RB, bool SQ>
void launch_n_rb(T2Args& k, bool vecload, hipStream_t st) {
  constexpr int64_t SP = RB > 1 ? NYS_N_SPACE : 1;
  dim3 g((unsigned)((k.m + RB * SP - 1) / (RB * SP) * SP));
  if (vecload) hipLaunchKernelGGL((k_gemv_n<T, RB, true, SQ>), g, dim3(NYS_BLOCK), 0, st, k);
  else hipLaunchKernelGGL((k_gemv_n<T, RB, false, SQ>), g, dim3(NYS_BLOCK), 0, st, k);
}

template <class T, bool SQ>
void dispatch_n_sq(T2Args& k, bool vecload, hipStream_t st) {
  const int64_t m = k.m;
  if (m >= 8 * 1536) launch_n_rb<T, NYS_N_RB, SQ>(k, vecload, st);
  else if (m >= 4 * 1024) launch_n_rb<T, 4, SQ>(k, vecload, st);
  else if (m >= 2 * 1024) launch_n_rb<T, 2, SQ>(k, vecload, st);
  else launch_n_rb<T, 1, SQ>(k, vecload, st);
}

template <class T>
void dispatch_n(T2Args& k, bool vecload, bool sq, hipStream_t st) {
  if (sq) dispatch_n_sq<T, true>(k, vecload, st);
  else dispatch_n_sq<T, false>(k, vecload, st);
}

template <class T, int RB>
void launch_tt_rb(TTArgs& k, bool vecload, hipStream_t st) {
  dim3 g((unsigned)std::max<int64_t>(1, (k.rows + RB - 1) / RB));
  if (vecload) hipLaunchKernelGGL((k_gemv_tt<T, RB, true>), g, dim3(NYS_BLOCK), 0, st, k);
  else hipLaunchKernelGGL((k_gemv_tt<T, RB, false>), g, dim3(NYS_BLOCK), 0, st, k);
}

template <class T>
void dispatch_tt(TTArgs& k, bool vecload, hipStream_t st) {
  const int64_t r = k.rows;
  if (r >= 8 * 1536) launch_tt_rb<T, NYS_TT_RB>(k, vecload, st);
  else if (r >= 4 * 1024) launch_tt_rb<T, 4>(k, vecload, st);
  else if (r >= 2 * 1024) launch_tt_rb<T, 2>(k, vecload, st);
  else launch_tt_rb<T, 1>(k, vecload, st);
}

bool al16(const void* p) { return ((uintptr_t)p % 16) == 0; }

// Pass 1 over the caller's (or the workspace's) transposed copy of A; a
// fused direction update runs first as k_dir_update.
int gemv_t_rows(nys_handle h, const GemvT& a) {
  const nys_matrix* A = a.A;
  const int es = elem_size(A->dtype);
  const double* v = a.v;
  if (a.s) {
    const int64_t nb = std::max<int64_t>(1, std::min<int64_t>((A->m + NYS_BLOCK - 1) / NYS_BLOCK, 1024));
    hipLaunchKernelGGL(k_dir_update, dim3((unsigned)nb), dim3(NYS_BLOCK), 0, h->stream, a.skip, a.s, a.pold,
                       a.beta, a.pnew, A->m);
    NYS_LAUNCH_CHECK(h);
    v = a.pnew;
  }
  if (A->n == 0) return NYS_OK;
  TTArgs k{};
  k.skip = a.skip;
  k.At = (const char*)A->data_t;
  k.rows = A->n;
  k.cols = A->m;
  k.row_bytes = A->ld_t * es;
  k.v = v;
  k.d = a.d;
  k.x0 = a.x0;
  k.sA = a.sA;
  k.w = a.w;
  const bool vl = al16(A->data_t) && (k.row_bytes % 16 == 0) && al16(v);
  const int ps = prof_begin(h, NYS_K_NORMAL_PASS1);
  switch (A->dtype) {
    case NYS_F64: dispatch_tt<F64>(k, vl, h->stream); break;
    case NYS_F32: dispatch_tt<F32>(k, vl, h->stream); break;
    case NYS_BF16: dispatch_tt<BF16>(k, vl, h->stream); break;
    default: return set_error(h, NYS_EINVAL, "gemv_t: bad dtype");
  }
  prof_end(h, ps);
  NYS_LAUNCH_CHECK(h);
  return NYS_OK;
}

// Grid of the pass-1 kernel on column stripes of A (no transposed copy):
// ncol column tiles of NYS_BLOCK * vec columns, nch row chunks of rpc rows,
// enough blocks to cover the chip several times with rows per chunk >= 32.
void t_chunks(const nys_matrix* A, int64_t* ncol_out, int64_t* nch_out, int64_t* rpc_out) {
  const int vec = 16 / elem_size(A->dtype);
  const int64_t ncol =
      std::max<int64_t>(1, (A->n + (int64_t)NYS_BLOCK * vec - 1) / ((int64_t)NYS_BLOCK * vec));
  int64_t nch = std::max<int64_t>(
      1, std::min<int64_t>((A->m + 31) / 32, (NYS_T_TARGET_BLOCKS + ncol - 1) / ncol));
  int64_t rpc = (A->m + nch - 1) / nch;
  rpc = std::max<int64_t>(NYS_T_UNROLL, (rpc + NYS_T_UNROLL - 1) / NYS_T_UNROLL * NYS_T_UNROLL);
  nch = std::max<int64_t>(1, (A->m + rpc - 1) / rpc);
  *ncol_out = ncol;
  *nch_out = nch;
  *rpc_out = rpc;
}

int n_blocks_pass2(int64_t m) {
  const int rb = m >= 8 * 1536 ? NYS_N_RB : m >= 4 * 1024 ? 4 : m >= 2 * 1024 ? 2 : 1;
  const int64_t sp = rb > 1 ? NYS_N_SPACE : 1;
  return (int)((m + rb * sp - 1) / (rb * sp) * sp);
}

}  // namespace

int gemv_t_dense(nys_handle h, const GemvT& a);

int gemv_t(nys_handle h, const GemvT& a) {
  NYS_CHECK(gemv_t_dense(h, a));
  return unit_pass1(h, a, a.s ? a.pnew : a.v);
}

int gemv_t_dense(nys_handle h, const GemvT& a) {
  const nys_matrix* A = a.A;
  const int es = elem_size(A->dtype);
  const bool fused = a.s != nullptr;
  // n == 0: nothing to reduce; the fused direction update still has to run
  if (A->n == 0 && !fused) return NYS_OK;
  if (A->m == 0) return NYS_OK;
  if (A->data_t) return gemv_t_rows(h, a);
  int64_t ncol, nch, rpc;
  t_chunks(A, &ncol, &nch, &rpc);
  T1Args k{};
  k.skip = a.skip;
  k.A = (const char*)A->data;
  k.m = A->m;
  k.n = A->n;
  k.row_bytes = A->ld * es;
  k.v = a.v;
  k.s = a.s;
  k.pold = a.pold;
  k.pnew = a.pnew;
  k.beta = a.beta;
  k.d = a.d;
  k.x0 = a.x0;
  k.sA = a.sA;
  k.w = a.w;
  k.rows_per_chunk = (int)rpc;
  k.nchunks = (int)nch;
  if (nch > 1) NYS_CHECK(ws(h, WS_PART, (size_t)nch * A->n, &k.part));
  dim3 g((unsigned)ncol, (unsigned)nch);
  const bool vl = vec_ok(A);
  const int ps = prof_begin(h, NYS_K_NORMAL_PASS1);
  switch (A->dtype) {
    case NYS_F64: dispatch_t<F64>(g, k, fused, vl, h->stream); break;
    case NYS_F32: dispatch_t<F32>(g, k, fused, vl, h->stream); break;
    case NYS_BF16: dispatch_t<BF16>(g, k, fused, vl, h->stream); break;
    default: return set_error(h, NYS_EINVAL, "gemv_t: bad dtype");
  }
  prof_end(h, ps);
  NYS_LAUNCH_CHECK(h);
  if (nch > 1 && A->n > 0) {
    const int64_t nb = std::min<int64_t>((A->n + NYS_BLOCK - 1) / NYS_BLOCK, 4096);
    hipLaunchKernelGGL(k_gemv_t_finish, dim3((unsigned)nb), dim3(NYS_BLOCK), 0, h->stream, k);
    NYS_LAUNCH_CHECK(h);
  }
  return NYS_OK;
}

size_t gemv_t_part_doubles(const nys_matrix* A) {
  if (A->data_t || A->m == 0 || A->n == 0) return 0;
  int64_t ncol, nch, rpc;
  t_chunks(A, &ncol, &nch, &rpc);
  return nch > 1 ? (size_t)nch * (size_t)A->n : 0;
}

size_t gemv_n_part_doubles(int64_t m) { return m > 0 ? (size_t)n_blocks_pass2(m) : 0; }

int gemv_n(nys_handle h, const GemvN& a) {
  const nys_matrix* A = a.A;
  if (A->m == 0) return NYS_OK;
  const int es = elem_size(A->dtype);
  const double* x0 = a.x0;
  NYS_CHECK(unit_pass2_base(h, a, &x0));
  T2Args k{};
  k.skip = a.skip;
  k.A = (const char*)A->data;
  k.m = A->m;
  k.n = A->n;
  k.row_bytes = A->ld * es;
  k.w = a.w;
  k.v = a.v;
  k.x0 = x0;
  k.sA = a.sA;
  k.sV = a.sV;
  k.out = a.out;
  k.dot_out = a.dot_out;
  k.shift = a.shift;
  const int nbp = n_blocks_pass2(A->m);
  if (a.dot_out) NYS_CHECK(ws(h, WS_PART2, (size_t)nbp, &k.dpart));
  const bool vl = vec_ok(A) && ((uintptr_t)a.w % 16 == 0);
  const int ps = a.square ? -1 : prof_begin(h, NYS_K_NORMAL_PASS2);
  switch (A->dtype) {
    case NYS_F64: dispatch_n<F64>(k, vl, a.square, h->stream); break;
    case NYS_F32: dispatch_n<F32>(k, vl, a.square, h->stream); break;
    case NYS_BF16: dispatch_n<BF16>(k, vl, a.square, h->stream); break;
    default: return set_error(h, NYS_EINVAL, "gemv_n: bad dtype");
  }
  if (ps >= 0) prof_end(h, ps);
  NYS_LAUNCH_CHECK(h);
  if (a.dot_out) {
    hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(NYS_BLOCK), 0, h->stream, a.skip,
                       (const double*)k.dpart, nbp, a.dot_out);
    NYS_LAUNCH_CHECK(h);
  }
  return NYS_OK;
}

int transpose(nys_handle h, const nys_matrix* A, void* At, int64_t ld_t) {
  if (A->m == 0 || A->n == 0) return NYS_OK;
  const int es = elem_size(A->dtype);
  const int64_t gy = (A->m + 63) / 64;
  if (gy > 65535) return set_error(h, NYS_EINVAL, "transpose: m=%lld too large", (long long)A->m);
  dim3 g((unsigned)((A->n + 63) / 64), (unsigned)gy);
  const char* src = (const char*)A->data;
  char* dst = (char*)At;
  switch (A->dtype) {
    case NYS_F64: hipLaunchKernelGGL(k_transpose<double>, g, dim3(NYS_BLOCK), 0, h->stream, src, A->m, A->n, A->ld * es, dst, ld_t * es); break;
    case NYS_F32: hipLaunchKernelGGL(k_transpose<float>, g, dim3(NYS_BLOCK), 0, h->stream, src, A->m, A->n, A->ld * es, dst, ld_t * es); break;
    case NYS_BF16: hipLaunchKernelGGL(k_transpose<uint16_t>, g, dim3(NYS_BLOCK), 0, h->stream, src, A->m, A->n, A->ld * es, dst, ld_t * es); break;
    default: return set_error(h, NYS_EINVAL, "transpose: bad dtype");
  }
  NYS_LAUNCH_CHECK(h);
  return NYS_OK;
}

int with_transpose(nys_handle h, const nys_matrix* A, bool allowed, int slot, nys_matrix* out) {
  *out = *A;
  if (A->data_t || !allowed || A->m == 0 || A->n == 0) return NYS_OK;
  // rows start on 128-byte boundaries: a row pitch off by 64 bytes makes every
  // 1 KB wave load of a row touch nine cache lines instead of eight (measured
  // 5 % on pass 1 at m = 50000 FP32)
  const int es = elem_size(A->dtype);
  const int64_t per = 128 / es;
  const int64_t ld_t = (A->m + per - 1) / per * per;
  void* p = nullptr;
  const int rc = ws_get(h, slot, (size_t)A->n * ld_t * es, &p);
  if (rc == NYS_ENOMEM) {
    h->err.clear();   // not enough memory for the copy: the kernels read A as it is
    return NYS_OK;
  }
  NYS_CHECK(rc);
  NYS_CHECK(transpose(h, A, p, ld_t));
  out->data_t = p;
  out->ld_t = ld_t;
  return NYS_OK;
}

int normal_apply(nys_handle h, const nys_matrix* A, const double* d, double delta,
                 const double* v, double* out, double* dot_out) {
  double* w;
  NYS_CHECK(ws(h, WS_W, (size_t)std::max<int64_t>(ncols(A), 1), &w));
  GemvT t;
  t.A = A;
  t.v = v;
  t.d = d;
  t.w = w;
  NYS_CHECK(gemv_t(h, t));
  GemvN nn;
  nn.A = A;
  nn.w = w;
  nn.v = v;
  nn.sV = delta;
  nn.out = out;
  nn.dot_out = dot_out;
  return gemv_n(h, nn);
}

}  // namespace nys
