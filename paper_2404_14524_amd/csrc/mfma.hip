// The sketch Y = A diag(d) A^T Omega (Algorithm 1, second step) on BF16
// matrix cores with FP32 accumulation (gfx950).
//
//   Ot   = bf16(Omega)^T                      ell x m  (k-contiguous operand)
//   Wt   = bf16(d .* (A^T Omega))^T           ell x n
//   Y    = A Wt^T                              m x ell (FP32 partial sums of
//                                               split-K, summed in FP64)
//
// Both products have the same shape: C (M x N) = Aop (M x K) Bop (N x K)^T with
// M and K large (n and m of A) and N = ell small.  Aop is the big operand,
// streamed once from HBM; Bop (ell x K) is re-read by every row block, from
// L2.  k_sketch_mfma is built for that shape:
//
// * v_mfma_f32_16x16x32_bf16.  Lane l holds row l%16 of a 16 x 32 A tile
//   (8 consecutive k at 8*(l/16)), column l%16 of the B tile likewise, and
//   rows 4*(l/16)..+3 of column l%16 of the 16 x 16 result.
// * The big operand goes from HBM straight into registers in that layout
//   (each lane reads 16 bytes per row and k-step, four lanes cover 64
//   contiguous bytes of a row): no LDS traffic for it.  Loads run two k-tiles
//   ahead in three rotating register sets.
// * The small operand is staged through LDS (double-buffered, one barrier per
//   k-tile of 64), shared by the block's four waves.
// * A wave owns 64 rows (4 MFMA row tiles) and CTW column tiles of 16; a
//   block is four waves arranged WR x WC, so it covers 64 WR rows and
//   16 CTW WC columns.  With WC = 1 (ell <= 208) a block holds all ell
//   columns and 256 rows; with WC = 2 (ell <= 416) 128 rows, and the two waves
//   of a row pair read the same rows of Aop (the second read is an L2 hit).
//   Beyond that the grid's y dimension runs over column groups.  Per MFMA, a
//   wave reads 1 KB of LDS for four MFMAs (16 B per SIMD cycle at full rate).
// * Split-K over grid z writes FP32 partial tiles [z][c][j] (rows
//   contiguous); finish kernels sum them in FP64.  The W product without
//   split writes Wt = bf16(acc * d) directly.
//
// Without a transposed copy of A, the W product's operand A^T is not
// k-contiguous; k_mfma_nn then stages A's tiles through LDS transposed
// (32 x 32 x 16 MFMA, 128 x 128 tiles).

#include "common.hpp"
#include "kernels.hpp"

namespace nys {
namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef unsigned short u16x8 __attribute__((ext_vector_type(8)));
typedef unsigned short u16x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ uint16_t bf16_rne(float f) {
  uint32_t u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

// ------------------------------------------------------------------ streaming kernel

constexpr int SK_THREADS = 256;     // four waves
constexpr int SK_TK = 32;           // k per stage (one MFMA k-step)
constexpr int SK_ROWB = SK_TK * 2;  // bytes of a slab row

typedef __attribute__((address_space(3))) void lds_void;

// s_waitcnt with vmcnt(N) and lgkmcnt(0) (expcnt unconstrained): this wave's
// direct-to-LDS loads but the last N have landed, and its LDS reads are done.
template <int N>
__device__ __forceinline__ void wait_vm_lgkm0() {
  static_assert(N >= 0 && N < 64, "vmcnt has six bits");
  __builtin_amdgcn_s_waitcnt((N & 15) | (7 << 4) | (0 << 8) | ((N >> 4) << 14));
}

struct SkArgs {
  int64_t M, N, K;                  // C (M x N) = Aop (M x K) Bop (N x K)^T
  const uint16_t* A;
  int64_t lda;
  const uint16_t* B;                // 16-byte aligned rows (ldb % 8 == 0)
  int64_t ldb;
  int64_t klen;                     // k per split; a multiple of SK_TK
  uint16_t* out;                    // direct: out[c * ldout + j] = bf16(acc * d[j])
  int64_t ldout;
  const double* d;
  float* part;                      // split: part[(z * N + c) * Mp + j] = acc
  int64_t Mp;                       // partial row pitch, a multiple of 4
};

template <int CTW, int WC>
struct SkGeom {
  static constexpr int WR = 4 / WC;
  static constexpr int BM = WR * 64;                 // rows of Aop (and C) per block
  static constexpr int BN = WC * CTW * 16;           // columns of C per block
  static constexpr int BNP = (BN + 63) / 64 * 64;    // rows of the B slab: whole load rounds per wave
  static constexpr int QA = BM / 64;                 // A loads per wave and stage (16 rows each)
  static constexpr int QB = BNP / 64;                // B loads per wave and stage
  static constexpr int A_BYTES = BM * SK_ROWB;       // one A slab
  static constexpr int B_BYTES = BNP * SK_ROWB;      // one B slab
};

// LDS slab layout: row r of 64 bytes holds the 32 k of one row of an operand
// as four 16-byte chunks; chunk c sits at position c ^ ((r >> 2) & 3), so that
// the 16 rows an MFMA operand read touches fall on distinct banks.  A load
// instruction fills 16 rows (1 KB): lane l writes row l >> 2, position l & 3.
//
// Pipeline: the big operand (from HBM) runs SK_DA stages ahead in SK_DA + 1
// slabs, the small one (from L2) SK_DB stages ahead in SK_DB + 1 slabs.  Before
// computing stage `it` a wave has issued, in this order, ... B(it), A(it + 3),
// B(it + 1), A(it + 4); vector-memory counts complete in order, so waiting
// until at most that many later loads are pending makes stage `it` resident.
constexpr int SK_DA = 5, SK_DB = 2;

template <int CTW, int WC, bool VEC, bool DIRECT>
__global__ __launch_bounds__(SK_THREADS, 1) __attribute__((amdgpu_waves_per_eu(1, 1))) void k_sketch_mfma(SkArgs a) {
  using G = SkGeom<CTW, WC>;
  constexpr int NA = SK_DA + 1, NB = SK_DB + 1;
  __shared__ __attribute__((aligned(1024))) char lds[NA * G::A_BYTES + NB * G::B_BYTES];
  char* const ldsA = lds;
  char* const ldsB = lds + NA * G::A_BYTES;

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wr = wave / WC, wc = wave % WC;
  const int li = lane & 15;
  const int pos = (lane >> 4) ^ (li >> 2);            // position of this lane's MFMA chunk
  const int64_t rowb = (int64_t)blockIdx.x * G::BM;
  const int64_t colb = (int64_t)blockIdx.y * G::BN;
  const int64_t kb = (int64_t)blockIdx.z * a.klen;
  const int64_t ke = min(a.K, kb + a.klen);
  const int nfull = (int)((ke - kb) / SK_TK);
  const bool ragged = ((ke - kb) % SK_TK) != 0;

  // sources of this lane's direct-to-LDS loads (rows clamped into range:
  // rows of Aop past M and of Bop past N feed only results that are not stored)
  const int dchunk = (lane & 3) ^ ((lane >> 4) & 3);   // chunk loaded by this lane
  const uint16_t* ga[G::QA];
  const uint16_t* gb[G::QB];
#pragma unroll
  for (int u = 0; u < G::QA; ++u) {
    const int64_t r = min(rowb + (wave * G::QA + u) * 16 + (lane >> 2), a.M - 1);
    ga[u] = a.A + r * a.lda + kb + dchunk * 8;
  }
#pragma unroll
  for (int u = 0; u < G::QB; ++u) {
    const int64_t r = min(colb + (wave * G::QB + u) * 16 + (lane >> 2), a.N - 1);
    gb[u] = a.B + r * a.ldb + kb + dchunk * 8;
  }

  f32x4 acc[4][CTW];
#pragma unroll
  for (int t = 0; t < 4; ++t)
#pragma unroll
    for (int j = 0; j < CTW; ++j) acc[t][j] = f32x4{0.f, 0.f, 0.f, 0.f};

  // stage `it` (k = kb + it * 32) of one operand into its slab, straight from memory
  auto issue_a = [&](int it) {
    char* base = ldsA + (it % NA) * G::A_BYTES;
    const int64_t ko = (int64_t)it * SK_TK;
#pragma unroll
    for (int u = 0; u < G::QA; ++u)
      __builtin_amdgcn_global_load_lds((const void*)(ga[u] + ko), (lds_void*)(base + (wave * G::QA + u) * 1024),
                                       16, 0, 0);
  };
  auto issue_b = [&](int it) {
    char* base = ldsB + (it % NB) * G::B_BYTES;
    const int64_t ko = (int64_t)it * SK_TK;
#pragma unroll
    for (int u = 0; u < G::QB; ++u)
      __builtin_amdgcn_global_load_lds((const void*)(gb[u] + ko), (lds_void*)(base + (wave * G::QB + u) * 1024),
                                       16, 0, 0);
  };
  // stage at k0 into the slabs sa, sb through registers, element by element
  // where a chunk is unaligned or crosses ke, zero past ke
  auto fill = [&](int sa, int sb, int64_t k0) {
    for (int q = tid; q < (G::BM + G::BNP) * 4; q += SK_THREADS) {
      const int r = q >> 2, c = (q & 3) ^ ((r >> 2) & 3);
      const bool isA = r < G::BM;
      const int64_t grow = isA ? min(rowb + r, a.M - 1) : min(colb + (r - G::BM), a.N - 1);
      const uint16_t* src = isA ? a.A + grow * a.lda : a.B + grow * a.ldb;
      const int64_t k = k0 + c * 8;
      u16x8 v = {0, 0, 0, 0, 0, 0, 0, 0};
      if (k + 8 <= ke && (!isA || VEC)) {
        v = *(const u16x8*)(src + k);
      } else {
#pragma unroll
        for (int e = 0; e < 8; ++e)
          if (k + e < ke) v[e] = src[k + e];
      }
      char* dst = isA ? ldsA + sa * G::A_BYTES + r * SK_ROWB : ldsB + sb * G::B_BYTES + (r - G::BM) * SK_ROWB;
      *(u16x8*)(dst + (q & 3) * 16) = v;
    }
  };
  // MFMA operands of one stage: all read from LDS first, then the MFMAs
  bf16x8 fa[4], fb[CTW];
  auto compute = [&](int sa, int sb) {
    const char* baseA = ldsA + sa * G::A_BYTES;
    const char* baseB = ldsB + sb * G::B_BYTES;
#pragma unroll
    for (int t = 0; t < 4; ++t) fa[t] = *(const bf16x8*)(baseA + (wr * 64 + t * 16 + li) * SK_ROWB + pos * 16);
#pragma unroll
    for (int j = 0; j < CTW; ++j) fb[j] = *(const bf16x8*)(baseB + ((wc * CTW + j) * 16 + li) * SK_ROWB + pos * 16);
#pragma unroll
    for (int j = 0; j < CTW; ++j)
#pragma unroll
      for (int t = 0; t < 4; ++t) acc[t][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fa[t], fb[j], acc[t][j], 0, 0, 0);
    // schedule: every LDS read of the stage, then the MFMAs (the reads land
    // in order while the first MFMAs run)
    __builtin_amdgcn_sched_group_barrier(0x0100, 4 + CTW, 0);
    __builtin_amdgcn_sched_group_barrier(0x0008, 4 * CTW, 0);
  };

  if constexpr (VEC) {
    // prologue: the issues of iterations -SK_DA .. -1 (B(j + SK_DB), then A(j + SK_DA))
#pragma unroll
    for (int j = -SK_DA; j < 0; ++j) {
      if (j + SK_DB >= 0 && j + SK_DB < nfull) issue_b(j + SK_DB);
      if (j + SK_DA < nfull) issue_a(j + SK_DA);
    }
    for (int it = 0; it < nfull; ++it) {
      // pending after B(it): A(it + 3), B(it + 1), A(it + 4), those that exist
      if (it + 4 < nfull) wait_vm_lgkm0<2 * G::QA + G::QB>();
      else if (it + 3 < nfull) wait_vm_lgkm0<G::QA + G::QB>();
      else if (it + 1 < nfull) wait_vm_lgkm0<G::QB>();
      else wait_vm_lgkm0<0>();
      __builtin_amdgcn_s_barrier();
      if (it + SK_DB < nfull) issue_b(it + SK_DB);
      if (it + SK_DA < nfull) issue_a(it + SK_DA);
      compute(it % NA, it % NB);
    }
    if (ragged) {
      wait_vm_lgkm0<0>();
      __builtin_amdgcn_s_barrier();
      fill(0, 0, kb + (int64_t)nfull * SK_TK);
      wait_vm_lgkm0<0>();
      __builtin_amdgcn_s_barrier();
      compute(0, 0);
    }
  } else {
    // unaligned rows of Aop: every stage through registers, two slabs alternating
    const int ntile = nfull + (ragged ? 1 : 0);
    for (int it = 0; it < ntile; ++it) {
      fill(it & 1, it & 1, kb + (int64_t)it * SK_TK);
      wait_vm_lgkm0<0>();
      __builtin_amdgcn_s_barrier();
      compute(it & 1, it & 1);
    }
  }

  // epilogue: lane holds C[j0 + i][c] for i < 4
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    const int64_t j0 = rowb + wr * 64 + t * 16 + 4 * (lane >> 4);
    if (j0 >= a.M) continue;
#pragma unroll
    for (int jt = 0; jt < CTW; ++jt) {
      const int64_t c = colb + (wc * CTW + jt) * 16 + li;
      if (c >= a.N) continue;
      const f32x4 v = acc[t][jt];
      if constexpr (DIRECT) {
        uint16_t* dst = a.out + c * a.ldout + j0;
        if (j0 + 4 <= a.M) {
          u16x4 o;
#pragma unroll
          for (int i = 0; i < 4; ++i) o[i] = bf16_rne((float)((double)v[i] * a.d[j0 + i]));
          *(u16x4*)dst = o;
        } else {
#pragma unroll
          for (int i = 0; i < 4; ++i)
            if (j0 + i < a.M) dst[i] = bf16_rne((float)((double)v[i] * a.d[j0 + i]));
        }
      } else {
        *(f32x4*)(a.part + ((int64_t)blockIdx.z * a.N + c) * a.Mp + j0) = v;
      }
    }
  }
}

// Wt[c][j] = bf16(d[j] * sum_z part[z][c][j]), j < M (= n), c < N (= ell)
__global__ __launch_bounds__(NYS_BLOCK) void k_sketch_finish_w(const float* part, int nsplit, int64_t M,
                                                               int64_t N, int64_t Mp, const double* d,
                                                               uint16_t* Wt, int64_t ldw) {
  const int64_t total = N * M;
  for (int64_t idx = (int64_t)blockIdx.x * NYS_BLOCK + threadIdx.x; idx < total;
       idx += (int64_t)gridDim.x * NYS_BLOCK) {
    const int64_t c = idx / M, j = idx % M;
    double s = 0.0;
    for (int z = 0; z < nsplit; ++z) s += (double)part[((int64_t)z * N + c) * Mp + j];
    Wt[c * ldw + j] = bf16_rne((float)(s * d[j]));
  }
}

// Y[i][c] = sum_z part[z][c][i] (FP64), through a 64 (i) x 32 (c) LDS tile so
// that reads run along i and writes along c
__global__ __launch_bounds__(NYS_BLOCK) void k_sketch_finish_y(const float* part, int nsplit, int64_t M,
                                                               int64_t N, int64_t Mp, double* Y) {
  __shared__ double T[32][64 + 1];
  const int64_t i0 = (int64_t)blockIdx.x * 64, c0 = (int64_t)blockIdx.y * 32;
  const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;   // 64 x 4
  for (int cc = ty; cc < 32; cc += 4) {
    const int64_t i = i0 + tx, c = c0 + cc;
    double s = 0.0;
    if (i < M && c < N)
      for (int z = 0; z < nsplit; ++z) s += (double)part[((int64_t)z * N + c) * Mp + i];
    T[cc][tx] = s;
  }
  __syncthreads();
  const int cx = threadIdx.x & 31, iy = threadIdx.x >> 5;   // 32 x 8
  for (int ii = iy; ii < 64; ii += 8) {
    const int64_t i = i0 + ii, c = c0 + cx;
    if (i < M && c < N) Y[i * N + c] = T[cx][ii];
  }
}

// Ot[c][i] = bf16(fp32(Omega[i][c])): a 64 (i) x 64 (c) tile through LDS, read
// along c and written along i
__global__ __launch_bounds__(NYS_BLOCK) void k_omega_t(const double* Om, int64_t m, int ell, uint16_t* Ot,
                                                       int64_t ldo) {
  __shared__ uint16_t T[64][64 + 2];
  const int64_t i0 = (int64_t)blockIdx.x * 64;
  const int c0 = blockIdx.y * 64;
  const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
  for (int ii = ty; ii < 64; ii += 4) {
    const int64_t i = i0 + ii;
    const int c = c0 + tx;
    T[tx][ii] = (i < m && c < ell) ? bf16_rne((float)Om[i * ell + c]) : (uint16_t)0;
  }
  __syncthreads();
  for (int cc = ty; cc < 64; cc += 4) {
    const int64_t i = i0 + tx;
    const int c = c0 + cc;
    if (i < m && c < ell) Ot[(int64_t)c * ldo + i] = T[cc][tx];
  }
}

// ------------------------------------------------------------------ W product on A alone
// Wt (ell x n) = Ot (ell x m) * A (m x n, n contiguous): A's tiles are
// transposed on their way into LDS.  Block tile 128 x 128 x 64, four waves in
// 2 x 2, each a 64 x 64 tile of 2 x 2 MFMA 32 x 32 x 16 tiles.
// MFMA 32x32x16 lane layout (lane l, 8 bf16 per operand, 16 floats out):
//   A operand: row l%32, k = 8*(l/32) .. +7;  B operand: column l%32, same k;
//   D: column l%32, row 8*(r/4) + 4*(l/32) + r%4 for output register r.
constexpr int NN_TM = 128, NN_TN = 128, NN_TK = 64;
constexpr int NN_LDK = NN_TK + 8;
constexpr int NN_KCH = NN_TK / 8;
constexpr int NN_APT = NN_TM * NN_KCH / NYS_BLOCK;
constexpr int NN_BPT = NN_TN * NN_KCH / NYS_BLOCK;

__global__ __launch_bounds__(NYS_BLOCK) void k_mfma_nn(int64_t ell, int64_t n, int64_t m, const uint16_t* Ot,
                                                       int64_t ldo, const uint16_t* A, int64_t lda, bool veca,
                                                       const double* d, uint16_t* Wt, int64_t ldw) {
  __shared__ __attribute__((aligned(16))) uint16_t As[NN_TM * NN_LDK];
  __shared__ __attribute__((aligned(16))) uint16_t Bs[NN_TN * NN_LDK];
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  const int64_t r0 = (int64_t)blockIdx.y * NN_TM, n0 = (int64_t)blockIdx.x * NN_TN;
  f32x16 acc[2][2];
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y)
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[x][y][r] = 0.0f;

  u16x8 ra[NN_APT], rb[NN_BPT];
  auto load_tiles = [&](int64_t k0) {
#pragma unroll
    for (int p = 0; p < NN_APT; ++p) {       // Ot rows (ell), k-contiguous, 16-byte aligned
      const int idx = tid + p * NYS_BLOCK;
      const int64_t row = r0 + idx / NN_KCH, k = k0 + (idx % NN_KCH) * 8;
      u16x8 v = {0, 0, 0, 0, 0, 0, 0, 0};
      if (row < ell) {
        const uint16_t* src = Ot + row * ldo + k;
        if (k + 8 <= m) {
          v = *(const u16x8*)src;
        } else {
#pragma unroll
          for (int e = 0; e < 8; ++e)
            if (k + e < m) v[e] = src[e];
        }
      }
      ra[p] = v;
    }
#pragma unroll
    for (int p = 0; p < NN_BPT; ++p) {       // A rows (k = m index), 8 consecutive columns
      const int idx = tid + p * NYS_BLOCK;
      const int kr = idx / (NN_TN / 8), nc = (idx % (NN_TN / 8)) * 8;
      const int64_t gk = k0 + kr;
      u16x8 v = {0, 0, 0, 0, 0, 0, 0, 0};
      if (gk < m) {
        const uint16_t* src = A + gk * lda + n0 + nc;
        if (veca && n0 + nc + 8 <= n) {
          v = *(const u16x8*)src;
        } else {
#pragma unroll
          for (int e = 0; e < 8; ++e)
            if (n0 + nc + e < n) v[e] = src[e];
        }
      }
      rb[p] = v;
    }
  };
  auto store_tiles = [&]() {
#pragma unroll
    for (int p = 0; p < NN_APT; ++p) {
      const int idx = tid + p * NYS_BLOCK;
      *(u16x8*)(As + (idx / NN_KCH) * NN_LDK + (idx % NN_KCH) * 8) = ra[p];
    }
#pragma unroll
    for (int p = 0; p < NN_BPT; ++p) {
      const int idx = tid + p * NYS_BLOCK;
      const int kr = idx / (NN_TN / 8), nc = (idx % (NN_TN / 8)) * 8;
#pragma unroll
      for (int e = 0; e < 8; ++e) Bs[(nc + e) * NN_LDK + kr] = rb[p][e];   // transpose into [n][k]
    }
  };

  load_tiles(0);
  for (int64_t k0 = 0; k0 < m; k0 += NN_TK) {
    store_tiles();
    __syncthreads();
    if (k0 + NN_TK < m) load_tiles(k0 + NN_TK);
#pragma unroll
    for (int ks = 0; ks < NN_TK; ks += 16) {
      const int kk = ks + 8 * (lane >> 5);
      bf16x8 av[2], bv[2];
#pragma unroll
      for (int t = 0; t < 2; ++t) {
        av[t] = __builtin_bit_cast(bf16x8, *(const u16x8*)(As + (wm * 64 + t * 32 + (lane & 31)) * NN_LDK + kk));
        bv[t] = __builtin_bit_cast(bf16x8, *(const u16x8*)(Bs + (wn * 64 + t * 32 + (lane & 31)) * NN_LDK + kk));
      }
#pragma unroll
      for (int ti = 0; ti < 2; ++ti)
#pragma unroll
        for (int tj = 0; tj < 2; ++tj)
          acc[ti][tj] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(av[ti], bv[tj], acc[ti][tj], 0, 0, 0);
    }
    __syncthreads();
  }
#pragma unroll
  for (int ti = 0; ti < 2; ++ti)
#pragma unroll
    for (int tj = 0; tj < 2; ++tj)
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int64_t c = r0 + wm * 64 + ti * 32 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
        const int64_t j = n0 + wn * 64 + tj * 32 + (lane & 31);
        if (c < ell && j < n) Wt[c * ldw + j] = bf16_rne((float)((double)acc[ti][tj][r] * d[j]));
      }
}

unsigned grid1d(int64_t n) {
  int64_t b = (n + NYS_BLOCK - 1) / NYS_BLOCK;
  return (unsigned)std::max<int64_t>(1, std::min<int64_t>(b, 8192));
}

// ------------------------------------------------------------------ host side

// Column tiles per wave and waves per row pair for ell columns: the smallest
// instantiated width that covers ell in one column group (two waves across
// the columns above 208), else column groups of 416.
struct SkShape {
  int ctw, wc, groups;
};
constexpr int kCtw[] = {1, 2, 4, 7, 10, 13};
SkShape sk_shape(int64_t N) {
  const int64_t tiles = (N + 15) / 16;
  for (int wc = 1; wc <= 2; ++wc)
    for (int c : kCtw)
      if ((int64_t)c * wc >= tiles) return {c, wc, 1};
  return {13, 2, (int)((tiles + 25) / 26)};
}

// Splits of K for a grid of `tiles` blocks: enough blocks to keep the 256
// compute units busy in whole rounds (one resident block per unit), each
// split at least 32 k-tiles (1024 k) long.
int sk_splits(int64_t tiles, int64_t K) {
  const int64_t kt = (K + SK_TK - 1) / SK_TK;
  const int maxs = (int)std::max<int64_t>(1, std::min<int64_t>(32, kt / 32));
  int best = 1;
  double best_eff = 0.0;
  for (int s = 1; s <= maxs; ++s) {
    const int64_t blocks = tiles * s;
    const double eff = (double)blocks / (256.0 * (double)((blocks + 255) / 256));
    if (eff > best_eff + 0.02) {
      best = s;
      best_eff = eff;
    }
    if (best_eff >= 0.9) break;
  }
  return best;
}

template <int CTW, int WC>
void launch_sk(const SkArgs& a, dim3 g, bool vec, bool direct, hipStream_t st) {
  if (direct) {
    if (vec) hipLaunchKernelGGL((k_sketch_mfma<CTW, WC, true, true>), g, dim3(SK_THREADS), 0, st, a);
    else hipLaunchKernelGGL((k_sketch_mfma<CTW, WC, false, true>), g, dim3(SK_THREADS), 0, st, a);
  } else {
    if (vec) hipLaunchKernelGGL((k_sketch_mfma<CTW, WC, true, false>), g, dim3(SK_THREADS), 0, st, a);
    else hipLaunchKernelGGL((k_sketch_mfma<CTW, WC, false, false>), g, dim3(SK_THREADS), 0, st, a);
  }
}

template <int WC>
void launch_sk_ctw(int ctw, const SkArgs& a, dim3 g, bool vec, bool direct, hipStream_t st) {
  switch (ctw) {
    case 1: launch_sk<1, WC>(a, g, vec, direct, st); break;
    case 2: launch_sk<2, WC>(a, g, vec, direct, st); break;
    case 4: launch_sk<4, WC>(a, g, vec, direct, st); break;
    case 7: launch_sk<7, WC>(a, g, vec, direct, st); break;
    case 10: launch_sk<10, WC>(a, g, vec, direct, st); break;
    default: launch_sk<13, WC>(a, g, vec, direct, st); break;
  }
}

// C (M x N) = Aop (M x K) Bop (N x K)^T.  With out != NULL and one split, C is
// written as out[c][j] = bf16(C[j][c] d[j]); otherwise split-K partials go to
// the workspace and *part / *nsplit / *Mp describe them.
int sketch_gemm(nys_handle h, int64_t M, int64_t N, int64_t K, const uint16_t* A, int64_t lda,
                const uint16_t* B, int64_t ldb, uint16_t* out, int64_t ldout, const double* d, bool allow_direct,
                float** part_out, int* nsplit_out, int64_t* Mp_out) {
  const SkShape sh = sk_shape(N);
  const int64_t bm = 64 * (4 / sh.wc);
  const int64_t tiles = (M + bm - 1) / bm;
  int nsplit = sk_splits(tiles * sh.groups, K);
  const bool direct = allow_direct && nsplit == 1;
  int64_t klen = (K + nsplit - 1) / nsplit;
  klen = (klen + SK_TK - 1) / SK_TK * SK_TK;
  nsplit = (int)std::max<int64_t>(1, (K + klen - 1) / klen);
  SkArgs a{};
  a.M = M;
  a.N = N;
  a.K = K;
  a.A = A;
  a.lda = lda;
  a.B = B;
  a.ldb = ldb;
  a.klen = klen;
  a.out = out;
  a.ldout = ldout;
  a.d = d;
  a.Mp = (M + 3) / 4 * 4;
  if (!direct) {
    NYS_CHECK(ws_get(h, WS_SK_SPLIT, (size_t)nsplit * N * a.Mp * sizeof(float), (void**)&a.part));
    *part_out = a.part;
    *nsplit_out = nsplit;
    *Mp_out = a.Mp;
  } else {
    *part_out = nullptr;
  }
  if ((uint64_t)tiles > 0x7FFFFFFFull)
    return set_error(h, NYS_EINVAL, "BF16 sketch: %lld row tiles", (long long)tiles);
  const bool vec = ((uintptr_t)A % 16 == 0) && (lda % 8 == 0);
  dim3 g((unsigned)tiles, (unsigned)sh.groups, (unsigned)nsplit);
  if (sh.wc == 1) launch_sk_ctw<1>(sh.ctw, a, g, vec, direct, h->stream);
  else launch_sk_ctw<2>(sh.ctw, a, g, vec, direct, h->stream);
  NYS_LAUNCH_CHECK(h);
  return NYS_OK;
}

}  // namespace

int sketch_bf16(nys_handle h, const nys_matrix* A, const double* d, const double* Omega, int ell,
                double* Y) {
  if (A->dtype != NYS_BF16) return set_error(h, NYS_EINVAL, "BF16 sketch needs BF16 storage of A");
  const int64_t m = A->m, n = A->n;
  if ((m + NN_TM - 1) / NN_TM > 65535)
    return set_error(h, NYS_EINVAL, "BF16 sketch: m=%lld above %lld rows", (long long)m, 65535LL * NN_TM);
  if (n == 0) return fill(h, Y, m * ell, 0.0);
  const int64_t ldo = (m + 7) / 8 * 8, ldw = (n + 7) / 8 * 8;
  uint16_t *Ot, *Wt;
  NYS_CHECK(ws(h, WS_SK_LO, (size_t)ell * ldo, &Ot));
  NYS_CHECK(ws(h, WS_SK_W, (size_t)ell * ldw, &Wt));
  {
    dim3 g((unsigned)((m + 63) / 64), (unsigned)((ell + 63) / 64));
    hipLaunchKernelGGL(k_omega_t, g, dim3(NYS_BLOCK), 0, h->stream, Omega, m, ell, Ot, ldo);
    NYS_LAUNCH_CHECK(h);
  }
  const uint16_t* Ad = (const uint16_t*)A->data;
  // W product: Wt (ell x n) = bf16(d .* (A^T Ot^T))^T
  {
    const int ps = prof_begin(h, NYS_K_SKETCH_W);
    if (A->data_t) {
      float* part = nullptr;
      int nsplit = 1;
      int64_t Mp = 0;
      NYS_CHECK(sketch_gemm(h, n, ell, m, (const uint16_t*)A->data_t, A->ld_t, Ot, ldo, Wt, ldw, d, true, &part,
                            &nsplit, &Mp));
      if (part) {
        hipLaunchKernelGGL(k_sketch_finish_w, dim3(grid1d(n * ell)), dim3(NYS_BLOCK), 0, h->stream, part, nsplit,
                           n, (int64_t)ell, Mp, d, Wt, ldw);
        NYS_LAUNCH_CHECK(h);
      }
    } else {
      const bool vecA = ((uintptr_t)Ad % 16 == 0) && (A->ld % 8 == 0);
      dim3 g((unsigned)((n + NN_TN - 1) / NN_TN), (unsigned)((ell + NN_TM - 1) / NN_TM));
      hipLaunchKernelGGL(k_mfma_nn, g, dim3(NYS_BLOCK), 0, h->stream, (int64_t)ell, n, m, Ot, ldo, Ad, A->ld,
                         vecA, d, Wt, ldw);
      NYS_LAUNCH_CHECK(h);
    }
    prof_end(h, ps);
  }
  // Y product: Y (m x ell) = A (m x n) Wt^T, split over n, partials summed in FP64
  {
    const int ps = prof_begin(h, NYS_K_SKETCH_Y);
    float* part = nullptr;
    int nsplit = 1;
    int64_t Mp = 0;
    NYS_CHECK(sketch_gemm(h, m, ell, n, Ad, A->ld, Wt, ldw, nullptr, 0, nullptr, false, &part, &nsplit, &Mp));
    dim3 g((unsigned)((m + 63) / 64), (unsigned)((ell + 31) / 32));
    hipLaunchKernelGGL(k_sketch_finish_y, g, dim3(NYS_BLOCK), 0, h->stream, part, nsplit, m, (int64_t)ell, Mp, Y);
    NYS_LAUNCH_CHECK(h);
    prof_end(h, ps);
  }
  return NYS_OK;
}

}  // namespace nys
