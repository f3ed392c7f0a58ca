// The sketch Y = A diag(d) A^T Omega (Algorithm 1, second step) on BF16
// matrix cores with FP32 accumulation (v_mfma_f32_32x32x16_bf16, gfx950).
//
//   Ot   = bf16(Omega)^T                      ell x m  (k-contiguous operand)
//   Wt   = bf16(d .* (A^T Omega))^T = bf16((Ot A) .* d)   ell x n
//   Y    = A Wt^T                              m x ell (FP32 partial sums,
//                                               reduced in FP64 across split-K)
//
// One kernel template computes C = Aop * Bop for Aop stored M x K (K
// contiguous) and Bop stored either N x K (K contiguous, "NT") or K x N (N
// contiguous, "NN"; transposed on its way into LDS).  Block tile 128 x 128 x
// 32, four waves in a 2 x 2 arrangement, each wave a 64 x 64 tile made of
// 2 x 2 MFMA 32 x 32 x 16 tiles.  Operands are staged through LDS in
// [row][k] order so every MFMA operand is one 16-byte LDS read per lane.
//
// MFMA 32x32x16 lane layout (lane l, 8 bf16 per operand, 16 floats out):
//   A operand: row l%32, k = 8*(l/32) .. +7;  B operand: column l%32, same k;
//   D: column l%32, row 8*(r/4) + 4*(l/32) + r%4 for output register r.

#include "common.hpp"
#include "kernels.hpp"

namespace nys {
namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef unsigned short u16x8 __attribute__((ext_vector_type(8)));

constexpr int TBM = 128, TBN = 128, TBK = 64;
constexpr int LDK = TBK + 8;   // padded LDS row (bf16 elements): 144 bytes
constexpr int KCH = TBK / 8;   // 16-byte chunks along k per tile row
constexpr int APT = TBM * KCH / NYS_BLOCK;   // A chunks per thread (4)
constexpr int BPT = TBN * KCH / NYS_BLOCK;   // B chunks per thread (4)

__device__ __forceinline__ uint16_t bf16_rne(float f) {
  uint32_t u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

// Load 8 consecutive K-direction elements of row `row` starting at k (zero
// outside [0, rows) x [0, K)).
__device__ __forceinline__ u16x8 load_k8(const uint16_t* P, int64_t ld, int64_t row, int64_t rows,
                                         int64_t k, int64_t K, bool vec) {
  u16x8 v = {0, 0, 0, 0, 0, 0, 0, 0};
  if (row >= rows) return v;
  const uint16_t* p = P + row * ld + k;
  if (vec && k + 8 <= K) return *(const u16x8*)p;
#pragma unroll
  for (int e = 0; e < 8; ++e)
    if (k + e < K) v[e] = p[e];
  return v;
}

struct EpiWt {      // Wt[c][j] = bf16(acc * d[j]); M = ell (c), N = n (j)
  uint16_t* Wt;
  int64_t ldw;
  const double* d;
  __device__ void operator()(int64_t c, int64_t j, float v) const {
    Wt[c * ldw + j] = bf16_rne((float)((double)v * d[j]));
  }
};
struct EpiPart {    // part[z][i][c] = acc; M = m (i), N = ell (c)
  float* part;
  int64_t M, N;
  __device__ void operator()(int64_t i, int64_t c, float v) const {
    part[((int64_t)blockIdx.z * M + i) * N + c] = v;
  }
};

template <bool B_NK, class Epi>
__global__ __launch_bounds__(NYS_BLOCK) void k_mfma_gemm(int64_t M, int64_t N, int64_t K,
                                                         const uint16_t* A, int64_t lda,
                                                         const uint16_t* B, int64_t ldb,
                                                         int64_t klen, bool veca, bool vecb, Epi epi) {
  __shared__ __attribute__((aligned(16))) uint16_t As[TBM * LDK];
  __shared__ __attribute__((aligned(16))) uint16_t Bs[TBN * LDK];
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  const int64_t m0 = (int64_t)blockIdx.y * TBM, n0 = (int64_t)blockIdx.x * TBN;
  const int64_t kb = (int64_t)blockIdx.z * klen;
  const int64_t ke = min(K, kb + klen);
  f32x16 acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[a][b][r] = 0.0f;

  // Register-prefetch pipeline: the next k-tile's global loads are issued
  // before the current tile's MFMAs, so their latency hides behind the math.
  u16x8 ra[APT], rb[BPT];
  auto load_tiles = [&](int64_t k0) {
#pragma unroll
    for (int p = 0; p < APT; ++p) {
      const int idx = tid + p * NYS_BLOCK;
      ra[p] = load_k8(A, lda, m0 + idx / KCH, M, k0 + (idx % KCH) * 8, ke, veca);
    }
    if constexpr (B_NK) {
#pragma unroll
      for (int p = 0; p < BPT; ++p) {
        const int idx = tid + p * NYS_BLOCK;
        rb[p] = load_k8(B, ldb, n0 + idx / KCH, N, k0 + (idx % KCH) * 8, ke, vecb);
      }
    } else {
      // B stored K x N (N contiguous): 8 consecutive columns of one k-row
#pragma unroll
      for (int p = 0; p < BPT; ++p) {
        const int idx = tid + p * NYS_BLOCK;
        const int kr = idx / (TBN / 8), nc = (idx % (TBN / 8)) * 8;
        const int64_t gk = k0 + kr;
        u16x8 v = {0, 0, 0, 0, 0, 0, 0, 0};
        if (gk < ke) {
          const uint16_t* src = B + gk * ldb + n0 + nc;
          if (vecb && n0 + nc + 8 <= N) {
            v = *(const u16x8*)src;
          } else {
#pragma unroll
            for (int e = 0; e < 8; ++e)
              if (n0 + nc + e < N) v[e] = src[e];
          }
        }
        rb[p] = v;
      }
    }
  };
  auto store_tiles = [&]() {
#pragma unroll
    for (int p = 0; p < APT; ++p) {
      const int idx = tid + p * NYS_BLOCK;
      *(u16x8*)(As + (idx / KCH) * LDK + (idx % KCH) * 8) = ra[p];
    }
    if constexpr (B_NK) {
#pragma unroll
      for (int p = 0; p < BPT; ++p) {
        const int idx = tid + p * NYS_BLOCK;
        *(u16x8*)(Bs + (idx / KCH) * LDK + (idx % KCH) * 8) = rb[p];
      }
    } else {
#pragma unroll
      for (int p = 0; p < BPT; ++p) {
        const int idx = tid + p * NYS_BLOCK;
        const int kr = idx / (TBN / 8), nc = (idx % (TBN / 8)) * 8;
#pragma unroll
        for (int e = 0; e < 8; ++e) Bs[(nc + e) * LDK + kr] = rb[p][e];   // transpose into [n][k]
      }
    }
  };

  if (kb < ke) load_tiles(kb);
  for (int64_t k0 = kb; k0 < ke; k0 += TBK) {
    store_tiles();
    __syncthreads();
    if (k0 + TBK < ke) load_tiles(k0 + TBK);
#pragma unroll
    for (int ks = 0; ks < TBK; ks += 16) {
      const int kk = ks + 8 * (lane >> 5);
      bf16x8 a[2], b[2];
#pragma unroll
      for (int t = 0; t < 2; ++t) {
        const int ar = wm * 64 + t * 32 + (lane & 31);
        const int bc = wn * 64 + t * 32 + (lane & 31);
        a[t] = __builtin_bit_cast(bf16x8, *(const u16x8*)(As + ar * LDK + kk));
        b[t] = __builtin_bit_cast(bf16x8, *(const u16x8*)(Bs + bc * LDK + kk));
      }
#pragma unroll
      for (int ti = 0; ti < 2; ++ti)
#pragma unroll
        for (int tj = 0; tj < 2; ++tj)
          acc[ti][tj] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[ti], b[tj], acc[ti][tj], 0, 0, 0);
    }
    __syncthreads();
  }
#pragma unroll
  for (int ti = 0; ti < 2; ++ti)
#pragma unroll
    for (int tj = 0; tj < 2; ++tj)
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int64_t row = m0 + wm * 64 + ti * 32 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
        const int64_t col = n0 + wn * 64 + tj * 32 + (lane & 31);
        if (row < M && col < N) epi(row, col, acc[ti][tj][r]);
      }
}

// Wide NT form, used when the BF16 matrix has a transposed copy: both
// operands are K-contiguous (Aop M x K, Bop N x K), block tile 128 x 256 x 64
// with eight waves in 2 x 4, each wave 64 x 64 (2 x 2 MFMA tiles).  A block
// covers 256 columns of the output, so for ell <= 256 every 16-byte piece of
// the big operand is read from HBM once per product.
//
// STAGE_T: the output is written transposed, Out[c][j] = bf16(acc * d[j]) for
// row j < M and column c < N, through an LDS tile so that the stores run
// along j (coalesced) instead of one 2-byte store per (j, c).
// Otherwise the epilogue functor stores split-K partials as in k_mfma_gemm.
constexpr int WBN = 256;                     // block tile N of the wide form
constexpr int WTHREADS = 512;                // eight waves
constexpr int WAPT = TBM * KCH / WTHREADS;   // A chunks per thread (2)
constexpr int WBPT = WBN * KCH / WTHREADS;   // B chunks per thread (4)
constexpr int TLD = TBM + 8;                 // LDS row of the staged transpose (bf16)
static_assert(WBN / 2 * TLD <= WBN * LDK, "staged half tile fits in the B tile");

template <bool STAGE_T, class Epi>
__global__ __launch_bounds__(WTHREADS) void k_mfma_nt_wide(int64_t M, int64_t N, int64_t K,
                                                           const uint16_t* A, int64_t lda,
                                                           const uint16_t* B, int64_t ldb, int64_t klen,
                                                           bool veca, bool vecb, Epi epi,
                                                           uint16_t* Out, int64_t ldout, const double* d) {
  __shared__ __attribute__((aligned(16))) uint16_t As[TBM * LDK];
  __shared__ __attribute__((aligned(16))) uint16_t Bs[WBN * LDK];
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 2, wn = wave & 3;
  const int64_t n0 = (int64_t)blockIdx.x * WBN, m0 = (int64_t)blockIdx.y * TBM;
  const int64_t kb = (int64_t)blockIdx.z * klen;
  const int64_t ke = min(K, kb + klen);
  f32x16 acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[a][b][r] = 0.0f;

  // Two register sets, loaded two k-steps ahead: one block per CU (150+
  // VGPRs), so the loads of the step after next are what cover HBM latency.
  u16x8 ra0[WAPT], rb0[WBPT], ra1[WAPT], rb1[WBPT];
  auto load_tiles = [&](int64_t k0, u16x8* ra, u16x8* rb) {
#pragma unroll
    for (int p = 0; p < WAPT; ++p) {
      const int idx = tid + p * WTHREADS;
      ra[p] = load_k8(A, lda, m0 + idx / KCH, M, k0 + (idx % KCH) * 8, ke, veca);
    }
#pragma unroll
    for (int p = 0; p < WBPT; ++p) {
      const int idx = tid + p * WTHREADS;
      rb[p] = load_k8(B, ldb, n0 + idx / KCH, N, k0 + (idx % KCH) * 8, ke, vecb);
    }
  };
  auto store_tiles = [&](const u16x8* ra, const u16x8* rb) {
#pragma unroll
    for (int p = 0; p < WAPT; ++p) {
      const int idx = tid + p * WTHREADS;
      *(u16x8*)(As + (idx / KCH) * LDK + (idx % KCH) * 8) = ra[p];
    }
#pragma unroll
    for (int p = 0; p < WBPT; ++p) {
      const int idx = tid + p * WTHREADS;
      *(u16x8*)(Bs + (idx / KCH) * LDK + (idx % KCH) * 8) = rb[p];
    }
  };
  auto compute = [&]() {
#pragma unroll
    for (int ks = 0; ks < TBK; ks += 16) {
      const int kk = ks + 8 * (lane >> 5);
      bf16x8 a[2], b[2];
#pragma unroll
      for (int t = 0; t < 2; ++t) {
        const int ar = wm * 64 + t * 32 + (lane & 31);
        const int bc = wn * 64 + t * 32 + (lane & 31);
        a[t] = __builtin_bit_cast(bf16x8, *(const u16x8*)(As + ar * LDK + kk));
        b[t] = __builtin_bit_cast(bf16x8, *(const u16x8*)(Bs + bc * LDK + kk));
      }
#pragma unroll
      for (int ti = 0; ti < 2; ++ti)
#pragma unroll
        for (int tj = 0; tj < 2; ++tj)
          acc[ti][tj] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[ti], b[tj], acc[ti][tj], 0, 0, 0);
    }
  };

  if (kb < ke) load_tiles(kb, ra0, rb0);
  if (kb + TBK < ke) load_tiles(kb + TBK, ra1, rb1);
  for (int64_t k0 = kb; k0 < ke; k0 += 2 * TBK) {
    store_tiles(ra0, rb0);
    __syncthreads();
    if (k0 + 2 * TBK < ke) load_tiles(k0 + 2 * TBK, ra0, rb0);
    compute();
    __syncthreads();
    if (k0 + TBK >= ke) break;
    store_tiles(ra1, rb1);
    __syncthreads();
    if (k0 + 3 * TBK < ke) load_tiles(k0 + 3 * TBK, ra1, rb1);
    compute();
    __syncthreads();
  }
  if constexpr (STAGE_T) {
    // two halves of 128 output columns; Bs holds Ts[c][j] (row pitch TLD)
    uint16_t* Ts = Bs;
#pragma unroll
    for (int half = 0; half < 2; ++half) {
      if ((wn >> 1) == half) {
#pragma unroll
        for (int ti = 0; ti < 2; ++ti)
#pragma unroll
          for (int tj = 0; tj < 2; ++tj)
#pragma unroll
            for (int r = 0; r < 16; ++r) {
              const int jl = wm * 64 + ti * 32 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
              const int cl = (wn & 1) * 64 + tj * 32 + (lane & 31);
              const int64_t j = m0 + jl;
              const double dj = j < M ? d[j] : 0.0;
              Ts[cl * TLD + jl] = bf16_rne((float)((double)acc[ti][tj][r] * dj));
            }
      }
      __syncthreads();
      // 128 columns x 128 rows of bf16: 16 chunks of 8 per column
      for (int idx = tid; idx < 128 * (TBM / 8); idx += WTHREADS) {
        const int cl = idx / (TBM / 8), jc = (idx % (TBM / 8)) * 8;
        const int64_t c = n0 + half * 128 + cl;
        const int64_t j = m0 + jc;
        if (c >= N || j >= M) continue;
        const uint16_t* src = Ts + cl * TLD + jc;
        uint16_t* dst = Out + c * ldout + j;
        if (j + 8 <= M && ((uintptr_t)dst % 16) == 0) {
          *(u16x8*)dst = *(const u16x8*)src;
        } else {
          for (int e = 0; e < 8 && j + e < M; ++e) dst[e] = src[e];
        }
      }
      __syncthreads();
    }
  } else {
#pragma unroll
    for (int ti = 0; ti < 2; ++ti)
#pragma unroll
      for (int tj = 0; tj < 2; ++tj)
#pragma unroll
        for (int r = 0; r < 16; ++r) {
          const int64_t row = m0 + wm * 64 + ti * 32 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
          const int64_t col = n0 + wn * 64 + tj * 32 + (lane & 31);
          if (row < M && col < N) epi(row, col, acc[ti][tj][r]);
        }
  }
}

// Ot[c][i] = bf16(fp32(Omega[i][c])), i < m; ld of Ot = ldo
__global__ __launch_bounds__(NYS_BLOCK) void k_omega_t(const double* Om, int64_t m, int ell,
                                                       uint16_t* Ot, int64_t ldo) {
  const int64_t total = (int64_t)ell * m;
  for (int64_t idx = (int64_t)blockIdx.x * NYS_BLOCK + threadIdx.x; idx < total;
       idx += (int64_t)gridDim.x * NYS_BLOCK) {
    const int64_t c = idx / m, i = idx % m;
    Ot[c * ldo + i] = bf16_rne((float)Om[i * ell + c]);
  }
}

__global__ __launch_bounds__(NYS_BLOCK) void k_split_sum(const float* part, int nsplit, int64_t count,
                                                         double* Y) {
  for (int64_t idx = (int64_t)blockIdx.x * NYS_BLOCK + threadIdx.x; idx < count;
       idx += (int64_t)gridDim.x * NYS_BLOCK) {
    double s = 0.0;
    for (int z = 0; z < nsplit; ++z) s += (double)part[(int64_t)z * count + idx];
    Y[idx] = s;
  }
}

unsigned grid1d(int64_t n) {
  int64_t b = (n + NYS_BLOCK - 1) / NYS_BLOCK;
  return (unsigned)std::max<int64_t>(1, std::min<int64_t>(b, 8192));
}

}  // namespace

int sketch_bf16(nys_handle h, const nys_matrix* A, const double* d, const double* Omega, int ell,
                double* Y) {
  if (A->dtype != NYS_BF16) return set_error(h, NYS_EINVAL, "BF16 sketch needs BF16 storage of A");
  const int64_t m = A->m, n = A->n;
  // grid y counts TBM-row tiles (of A's m rows in the Y product, of A^T's n
  // rows in the wide W product) and stops at 65535
  if ((m + TBM - 1) / TBM > 65535)
    return set_error(h, NYS_EINVAL, "BF16 sketch: m=%lld above %lld rows", (long long)m, 65535LL * TBM);
  if (n == 0) return fill(h, Y, m * ell, 0.0);
  const int64_t ldo = (m + 7) / 8 * 8, ldw = (n + 7) / 8 * 8;
  uint16_t *Ot, *Wt;
  NYS_CHECK(ws(h, WS_SK_LO, (size_t)ell * ldo, &Ot));
  NYS_CHECK(ws(h, WS_SK_W, (size_t)ell * ldw, &Wt));
  hipLaunchKernelGGL(k_omega_t, dim3(grid1d(m * ell)), dim3(NYS_BLOCK), 0, h->stream, Omega, m, ell, Ot, ldo);
  NYS_LAUNCH_CHECK(h);
  const uint16_t* Ad = (const uint16_t*)A->data;
  const bool vecA = ((uintptr_t)Ad % 16 == 0) && (A->ld % 8 == 0);
  const bool wide = A->data_t != nullptr && (n + TBM - 1) / TBM <= 65535;
  if (wide) {
    // Wt (ell x n) written transposed from W = At (n x m) * Ot^T: both operands k-contiguous
    const uint16_t* Atd = (const uint16_t*)A->data_t;
    const bool vecAt = ((uintptr_t)Atd % 16 == 0) && (A->ld_t % 8 == 0);
    dim3 g((unsigned)((ell + WBN - 1) / WBN), (unsigned)((n + TBM - 1) / TBM), 1);
    EpiPart none{nullptr, 0, 0};
    const int ps = prof_begin(h, NYS_K_SKETCH_W);
    hipLaunchKernelGGL((k_mfma_nt_wide<true, EpiPart>), g, dim3(WTHREADS), 0, h->stream, n, (int64_t)ell, m,
                       Atd, A->ld_t, (const uint16_t*)Ot, ldo, m, vecAt, true, none, Wt, ldw, d);
    prof_end(h, ps);
    NYS_LAUNCH_CHECK(h);
  } else {
    // Wt (ell x n) = Ot (ell x m) * A (m x n, "NN"), scaled by d and rounded to BF16
    dim3 g((unsigned)((n + TBN - 1) / TBN), (unsigned)((ell + TBM - 1) / TBM), 1);
    EpiWt epi{Wt, ldw, d};
    const int ps = prof_begin(h, NYS_K_SKETCH_W);
    hipLaunchKernelGGL((k_mfma_gemm<false, EpiWt>), g, dim3(NYS_BLOCK), 0, h->stream, (int64_t)ell, n, m,
                       (const uint16_t*)Ot, ldo, Ad, A->ld, m, true, vecA, epi);
    prof_end(h, ps);
    NYS_LAUNCH_CHECK(h);
  }
  // Y (m x ell) = A (m x n) * Wt^T ("NT"), split over n
  {
    const int bn = wide ? WBN : TBN;
    const int64_t tiles = ((m + TBM - 1) / TBM) * ((ell + bn - 1) / bn);
    int64_t nsplit = std::max<int64_t>(1, std::min<int64_t>((1024 + tiles - 1) / tiles, 16));
    int64_t klen = (n + nsplit - 1) / nsplit;
    klen = std::max<int64_t>(4096, (klen + TBK - 1) / TBK * TBK);
    nsplit = std::max<int64_t>(1, (n + klen - 1) / klen);
    float* part;
    NYS_CHECK(ws_get(h, WS_SK_SPLIT, (size_t)nsplit * m * ell * sizeof(float), (void**)&part));
    EpiPart epi{part, m, ell};
    const int ps = prof_begin(h, NYS_K_SKETCH_Y);
    if (wide) {
      dim3 g((unsigned)((ell + WBN - 1) / WBN), (unsigned)((m + TBM - 1) / TBM), (unsigned)nsplit);
      hipLaunchKernelGGL((k_mfma_nt_wide<false, EpiPart>), g, dim3(WTHREADS), 0, h->stream, m, (int64_t)ell, n,
                         Ad, A->ld, (const uint16_t*)Wt, ldw, klen, vecA, true, epi, (uint16_t*)nullptr,
                         (int64_t)0, (const double*)nullptr);
    } else {
      dim3 g((unsigned)((ell + TBN - 1) / TBN), (unsigned)((m + TBM - 1) / TBM), (unsigned)nsplit);
      hipLaunchKernelGGL((k_mfma_gemm<true, EpiPart>), g, dim3(NYS_BLOCK), 0, h->stream, m, (int64_t)ell, n,
                         Ad, A->ld, (const uint16_t*)Wt, ldw, klen, vecA, true, epi);
    }
    prof_end(h, ps);
    NYS_LAUNCH_CHECK(h);
    hipLaunchKernelGGL(k_split_sum, dim3(grid1d(m * ell)), dim3(NYS_BLOCK), 0, h->stream, part, (int)nsplit,
                       m * ell, Y);
    NYS_LAUNCH_CHECK(h);
  }
  return NYS_OK;
}

}  // namespace nys
