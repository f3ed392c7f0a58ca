// The sketch Y = A diag(d) A^T Omega (Algorithm 1, second step) on BF16
// matrix cores with FP32 accumulation (gfx950).
//
//   W  = d .* (A^T Omega)   n x ell, rounded to BF16 (the operand of Y)
//   Y  = A W                m x ell (FP32 partial sums of split-K, summed in FP64)
//
// Both products have the shape C (M x N) = Aop (M x K) Bop (N x K)^T with M
// and K large (n and m of A) and N = ell small: Aop streams once from HBM,
// Bop (ell x K) is re-read by every row block from L2.  k_sketch_mfma:
//
// * v_mfma_f32_32x32x16_bf16: a single wave per SIMD keeps it at its full
//   rate, which the 16 x 16 x 32 form does not reach.  Lane l holds row l%32
//   of a 32 x 16 operand tile (8 consecutive k at 8*(l/32)) and column l%32 of
//   the result, rows 8*(r/4) + 4*(l/32) + r%4 for its register r.
// * A wave owns 64 rows (two row tiles) and CTW column tiles of 32; a block
//   is four waves arranged WR x WC: all ell columns with WC = 1 (ell <= 224)
//   and 256 rows, or WC = 2 (ell <= 448) and 128 rows, the two waves of a row
//   pair reading the same rows of Aop.  Beyond that the grid's y dimension
//   runs over column groups.
// * Both operands reach LDS through direct-to-LDS loads (global_load_lds,
//   16 bytes per lane, no registers in flight), in stages of 32 k: Bop two
//   stages ahead in three slabs, Aop as far ahead as the rest of the 160 KB
//   allows (at most five); a wave waits by its vector-memory count, then one
//   barrier per stage.  The wave index is made scalar so that the per-wave
//   parts of every address stay in scalar registers.
// * Software pipeline by k-steps of 16: the products of one k-step run while
//   the operands of the next are read from LDS (two register sets), so LDS
//   reads hide behind the matrix cores; the stage's barrier sits between
//   the two k-steps.
// * Limits measured on MI355X: the matrix cores alone run these products at
//   about 2 PFLOP/s; streaming alone (no products) reaches about 28 bytes per
//   clock and compute unit when Aop comes from HBM and Bop from L2 in the
//   same unit (54 with both from L2): a unit's outstanding requests are
//   shared by the two streams and the HBM ones hold them longest.
// * Operands are either row-major (the caller's matrix or its transposed
//   copy: a stage reads 64 bytes of each of the block's rows) or "sketch
//   tiles" (see below: a stage is one contiguous run of memory, the pattern
//   HBM streams best; K is zero-padded to whole stages).
// * Split-K over grid z writes FP32 partial tiles [z][c][j]; finish kernels
//   sum them in FP64.  Without split, the W product writes BF16 W directly.
//
// Sketch tiles of an R x K operand X: stage kb (k = 32 kb .. 32 kb + 31) of
// row r is 64 bytes at offset (kb * Rp + r) * 64, Rp = R rounded up to 256
// rows, its four 16-byte chunks permuted within the row as in LDS (see
// sk_swz); rows >= R and k >= K are zero.  A DMA of 16 rows is then one
// contiguous kilobyte, and a block's stage one contiguous run.
//
// Without a transposed copy, the W product's operand A^T is not k-contiguous;
// k_mfma_nn then stages A's tiles through LDS transposed (128 x 128 tiles).

#include <utility>

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
// BF16 of a stored element: BF16 as is, FP32 rounded to nearest even, FP64
// through FP32 (two roundings, as the mixed path defines its BF16 copy)
__device__ __forceinline__ uint16_t to_bf16(uint16_t v) { return v; }
__device__ __forceinline__ uint16_t to_bf16(float v) { return bf16_rne(v); }
__device__ __forceinline__ uint16_t to_bf16(double v) { return bf16_rne((float)v); }
// 8 consecutive elements from a 16-byte aligned address, as BF16
typedef double f64x2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ u16x8 load8_bf16(const uint16_t* p) { return *(const u16x8*)p; }
__device__ __forceinline__ u16x8 load8_bf16(const float* p) {
  const f32x4 a = *(const f32x4*)p, b = *(const f32x4*)(p + 4);
  return u16x8{bf16_rne(a[0]), bf16_rne(a[1]), bf16_rne(a[2]), bf16_rne(a[3]),
               bf16_rne(b[0]), bf16_rne(b[1]), bf16_rne(b[2]), bf16_rne(b[3])};
}
__device__ __forceinline__ u16x8 load8_bf16(const double* p) {
  u16x8 v;
#pragma unroll
  for (int e = 0; e < 8; e += 2) {
    const f64x2 x = *(const f64x2*)(p + e);
    v[e] = to_bf16(x[0]);
    v[e + 1] = to_bf16(x[1]);
  }
  return v;
}

// ------------------------------------------------------------------ layouts

constexpr int SK_THREADS = 256;     // four waves
constexpr int SK_TK = 32;           // k per stage (two MFMA k-steps of 16)
constexpr int SK_ROWB = SK_TK * 2;  // bytes of a slab row
constexpr int SK_TILE_ROWS = 256;   // row padding of sketch tiles (the largest block)

typedef __attribute__((address_space(3))) void lds_void;

// Chunk position permutation of a slab row (r < 16): rows 2i and 2i + 1
// share a 128-byte bank line, so the four row pairs of each half of 16 rows
// take the four positions, the second half shifted by one.  An operand read
// (16 or 32 rows, one 16-byte chunk each) then touches distinct banks in
// every LDS cycle, for 8 lanes over 32 four-byte banks or 16 over 64.
__device__ __forceinline__ int sk_swz(int r) { return ((r >> 1) & 3) ^ ((r >> 3) & 1); }

// s_waitcnt with vmcnt(N) and lgkmcnt(0) (expcnt unconstrained): this wave's
// direct-to-LDS loads but the last N have landed, and its LDS reads are done.
template <int N>
__device__ __forceinline__ void wait_vm_lgkm0() {
  static_assert(N >= 0 && N < 64, "vmcnt has six bits");
  __builtin_amdgcn_s_waitcnt((N & 15) | (7 << 4) | (0 << 8) | ((N >> 4) << 14));
}

// Scheduling of one pipelined step: NR operand reads (of the next stage)
// spread evenly between the NM matrix-core instructions (of this stage).
template <int NR, int NM, int... I>
__device__ __forceinline__ void sk_interleave(std::integer_sequence<int, I...>) {
  ((__builtin_amdgcn_sched_group_barrier(0x0100, 1, 0),
    __builtin_amdgcn_sched_group_barrier(0x0008, (NM * (I + 1)) / NR - (NM * I) / NR, 0)),
   ...);
}

// Output of k_sketch_mfma.
enum { SK_OUT_PART = 0, SK_OUT_WT = 1, SK_OUT_WT_TILES = 2 };

struct SkArgs {
  int64_t M, N, K;                  // C (M x N) = Aop (M x K) Bop (N x K)^T
  const uint16_t* A;                // row-major (lda) or sketch tiles (rpa rows)
  int64_t lda, rpa;
  const uint16_t* B;                // row-major (ldb, 16-byte aligned rows) or tiles (rpb rows)
  int64_t ldb, rpb;
  int64_t klen;                     // k per split; a multiple of SK_TK
  uint16_t* out;                    // W: bf16(C[j][c] d[j]) at out[c * ldout + j], or in tiles of rpo rows
  int64_t ldout, rpo, kout;         // kout: rows j written in the tiled output (its K, rounded to 32)
  const double* d;
  float* part;                      // split: part[(z * N + c) * Mp + j] = C[j][c]
  int64_t Mp;                       // partial row pitch, a multiple of 4
  int64_t ntile;                    // row tiles; with ngroup > 1 the grid's x runs over
  int ngroup;                       // (row tile, column group) in XCD order
  int64_t tile0;                    // first row tile of the grid (ngroup == 1)
};

#ifndef SK_DA_MAX
#define SK_DA_MAX 5
#endif
constexpr int SK_LDS_MAX = 160 * 1024;   // LDS of a compute unit (gfx950)

// Pipeline depths: Bop (from L2) DB stages ahead in DB + 1 slabs, Aop (from
// HBM) DA ahead in DA + 1, DA as deep as the remaining LDS allows (capped).
// A wave issues, per iteration j, B(j + DB) then A(j + DA); loads complete in
// order, so once B(it) has landed, so has A(it), and at most the loads issued
// after B(it) are pending: A(it + DA - DB .. it + DA - 1) and B(it + 1 ..
// it + DB - 1), those that exist.
template <int CTW, int WC>
struct SkGeom {
  static constexpr int WR = 4 / WC;
  static constexpr int BM = WR * 64;                 // rows of Aop (and C) per block
  static constexpr int BN = WC * CTW * 32;           // columns of C per block
  static constexpr int BNP = (BN + 63) / 64 * 64;    // rows of the B slab: whole load rounds per wave
  static constexpr int QA = BM / 64;                 // A loads per wave and stage (16 rows each)
  static constexpr int QB = BNP / 64;                // B loads per wave and stage
  static constexpr int A_BYTES = BM * SK_ROWB;
  static constexpr int B_BYTES = BNP * SK_ROWB;
  static constexpr int DB = 2;
  static constexpr int DA_FIT = (SK_LDS_MAX - (DB + 1) * B_BYTES) / A_BYTES - 1;
  static constexpr int DA = DA_FIT < SK_DA_MAX ? DA_FIT : SK_DA_MAX;
  static constexpr int PEND = DB * QA + (DB - 1) * QB;   // pending after B(it) in the steady state
  static_assert(DA > DB, "Aop must be prefetched deeper than Bop");
  static_assert((DA + 1) * A_BYTES + (DB + 1) * B_BYTES <= SK_LDS_MAX, "LDS");
};

template <int CTW, int WC, bool TILED, bool VEC, int OUT>
__global__ __launch_bounds__(SK_THREADS, 1) void k_sketch_mfma(SkArgs a) {
  using G = SkGeom<CTW, WC>;
  constexpr int NA = G::DA + 1, NB = G::DB + 1;
  __shared__ __attribute__((aligned(1024))) char lds[NA * G::A_BYTES + NB * G::B_BYTES];
  char* const ldsA = lds;
  char* const ldsB = lds + NA * G::A_BYTES;

  const int tid = threadIdx.x, lane = tid & 63, wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int wr = wave / WC, wc = wave % WC;
  const int l32 = lane & 31;
  const int pos0 = (lane >> 5) ^ sk_swz(lane & 15);   // position of this lane's chunk, k-step 0
  // with several column groups, block x of the grid runs group (x / 8) % ng
  // of row tile (x / (8 ng)) * 8 + x % 8: blocks are dispatched to the eight
  // XCDs in turn, so the groups of one row tile run back to back on one XCD
  // and its Aop stream comes from HBM once, the other groups reading it in L2
  int64_t tile = a.tile0 + blockIdx.x, group = blockIdx.y;
  if (a.ngroup > 1) {
    const int64_t x = blockIdx.x, q = x >> 3;
    group = q % a.ngroup;
    tile = (q / a.ngroup) * 8 + (x & 7);
    if (tile >= a.ntile) return;
  }
  const int64_t rowb = tile * G::BM;
  const int64_t colb = group * G::BN;
  const int64_t kb = (int64_t)blockIdx.z * a.klen;
  const int64_t ke = min(a.K, kb + a.klen);
  const int nfull = TILED ? (int)((ke - kb + SK_TK - 1) / SK_TK) : (int)((ke - kb) / SK_TK);
  const bool ragged = !TILED && ((ke - kb) % SK_TK) != 0;

  // sources of this lane's direct-to-LDS loads: in tiles, consecutive
  // kilobytes; row-major, 16 rows x 64 bytes (rows clamped into range: rows of
  // Aop past M and of Bop past N feed only results that are not stored)
  const int dchunk = (lane & 3) ^ sk_swz(lane >> 2);   // chunk this lane loads (row-major)
  const char* ga[G::QA];
  const char* gb[G::QB];
  int64_t stepA, stepB;                               // bytes from one stage to the next
  if constexpr (TILED) {
    stepA = a.rpa * SK_ROWB;
    stepB = a.rpb * SK_ROWB;
#pragma unroll
    for (int u = 0; u < G::QA; ++u)
      ga[u] = (const char*)a.A + (kb / SK_TK) * stepA + (rowb + (wave * G::QA + u) * 16) * SK_ROWB + lane * 16;
#pragma unroll
    for (int u = 0; u < G::QB; ++u)
      gb[u] = (const char*)a.B + (kb / SK_TK) * stepB + (colb + (wave * G::QB + u) * 16) * SK_ROWB + lane * 16;
  } else {
    stepA = stepB = SK_ROWB;
#pragma unroll
    for (int u = 0; u < G::QA; ++u) {
      const int64_t r = min(rowb + (wave * G::QA + u) * 16 + (lane >> 2), a.M - 1);
      ga[u] = (const char*)(a.A + r * a.lda + kb + dchunk * 8);
    }
#pragma unroll
    for (int u = 0; u < G::QB; ++u) {
      const int64_t r = min(colb + (wave * G::QB + u) * 16 + (lane >> 2), a.N - 1);
      gb[u] = (const char*)(a.B + r * a.ldb + kb + dchunk * 8);
    }
  }

  f32x16 acc[2][CTW];
#pragma unroll
  for (int t = 0; t < 2; ++t)
#pragma unroll
    for (int j = 0; j < CTW; ++j)
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[t][j][r] = 0.0f;

  // stage `it` (k = kb + 32 it) of one operand into its slab, straight from memory
  auto issue_a = [&](int it) {
    char* base = ldsA + (it % NA) * G::A_BYTES;
#pragma unroll
    for (int u = 0; u < G::QA; ++u)
      __builtin_amdgcn_global_load_lds((const void*)(ga[u] + it * stepA),
                                       (lds_void*)(base + (wave * G::QA + u) * 1024), 16, 0, 0);
  };
  auto issue_b = [&](int it) {
    char* base = ldsB + (it % NB) * G::B_BYTES;
#pragma unroll
    for (int u = 0; u < G::QB; ++u)
      __builtin_amdgcn_global_load_lds((const void*)(gb[u] + it * stepB),
                                       (lds_void*)(base + (wave * G::QB + u) * 1024), 16, 0, 0);
  };
  // (row-major operands) stage at k0 into slabs sa, sb through registers,
  // element by element where a chunk is unaligned or crosses ke, zero past ke
  auto fill = [&](int sa, int sb, int64_t k0) {
    for (int q = tid; q < (G::BM + G::BNP) * 4; q += SK_THREADS) {
      const int r = q >> 2, c = (q & 3) ^ sk_swz(r & 15);
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
  // MFMA operands of k-step S (16 k) of a stage from its slabs (FA[t]: rows
  // of tile t; FB[j]: columns of tile j), and the products of one k-step
#define SK_READ(FA, FB, sa, sb, S)                                                              \
  do {                                                                                          \
    const char* baseA_ = ldsA + (sa) * G::A_BYTES;                                              \
    const char* baseB_ = ldsB + (sb) * G::B_BYTES;                                              \
    const int po_ = (pos0 ^ (2 * (S))) * 16;                                                    \
    _Pragma("unroll") for (int t_ = 0; t_ < 2; ++t_)                                            \
      FA[t_] = *(const bf16x8*)(baseA_ + (wr * 64 + t_ * 32 + l32) * SK_ROWB + po_);            \
    _Pragma("unroll") for (int j_ = 0; j_ < CTW; ++j_)                                          \
      FB[j_] = *(const bf16x8*)(baseB_ + ((wc * CTW + j_) * 32 + l32) * SK_ROWB + po_);         \
  } while (0)
#define SK_MMA(FA, FB)                                                                          \
  do {                                                                                          \
    _Pragma("unroll") for (int j_ = 0; j_ < CTW; ++j_)                                          \
      _Pragma("unroll") for (int t_ = 0; t_ < 2; ++t_)                                          \
        acc[t_][j_] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(FA[t_], FB[j_], acc[t_][j_], 0, 0, 0); \
  } while (0)
  constexpr int NRD = 2 + CTW, NMM = 2 * CTW;   // reads and products per k-step
  bf16x8 fa0[2], fb0[CTW], fa1[2], fb1[CTW];
  // unpipelined stage (ragged tail, register-staged operands): reads, then products
  auto compute = [&](int sa, int sb) {
    SK_READ(fa0, fb0, sa, sb, 0);
    SK_READ(fa1, fb1, sa, sb, 1);
    SK_MMA(fa0, fb0);
    SK_MMA(fa1, fb1);
    __builtin_amdgcn_sched_group_barrier(0x0100, 2 * NRD, 0);
    __builtin_amdgcn_sched_group_barrier(0x0008, 2 * NMM, 0);
  };

  if constexpr (TILED || VEC) {
    // Pipelined by k-steps: the products of one k-step run while the operands
    // of the next are read.  Per iteration j a wave issues B(j + DB + 1) then
    // A(j + DA + 1), into the slabs of stage j, once every wave has read them;
    // the prologue issues those of j = -DA - 1 .. -1 in the same order.
#pragma unroll
    for (int j = -G::DA - 1; j < 0; ++j) {
      if (j + G::DB + 1 >= 0 && j + G::DB + 1 < nfull) issue_b(j + G::DB + 1);
      if (j + G::DA + 1 < nfull) issue_a(j + G::DA + 1);
    }
    // stage x is resident once B(x) has landed: at most PEND later loads pending
    // (all of them issued only while x + DA - 1 < nfull; otherwise wait for all);
    // the barrier also orders every wave's reads of the stage before (lgkmcnt 0)
    // ahead of the loads that overwrite its slabs
#define SK_WAIT_STAGE(x)                                   \
  do {                                                     \
    if ((x) + G::DA - 1 < nfull) wait_vm_lgkm0<G::PEND>(); \
    else wait_vm_lgkm0<0>();                               \
    __builtin_amdgcn_s_barrier();                          \
  } while (0)
    if (nfull > 0) {
      SK_WAIT_STAGE(0);
      SK_READ(fa0, fb0, 0, 0, 0);
    }
    for (int it = 0; it < nfull; ++it) {
      // k-step 1 of stage it read during the products of k-step 0
      SK_READ(fa1, fb1, it % NA, it % NB, 1);
      SK_MMA(fa0, fb0);
      if constexpr (NMM >= NRD) sk_interleave<NRD, NMM>(std::make_integer_sequence<int, NRD>{});
      SK_WAIT_STAGE(it + 1);
      if (it + G::DB + 1 < nfull) issue_b(it + G::DB + 1);
      if (it + G::DA + 1 < nfull) issue_a(it + G::DA + 1);
      // k-step 0 of stage it + 1 (of stage it again on the last: a harmless re-read)
      const int nx = it + 1 < nfull ? it + 1 : it;
      SK_READ(fa0, fb0, nx % NA, nx % NB, 0);
      SK_MMA(fa1, fb1);
      if constexpr (NMM >= NRD) sk_interleave<NRD, NMM>(std::make_integer_sequence<int, NRD>{});
    }
#undef SK_WAIT_STAGE
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

  // epilogue: register group g of tile (t, jt) holds C[j0 + i][c], i < 4
#pragma unroll
  for (int t = 0; t < 2; ++t)
#pragma unroll
    for (int g = 0; g < 4; ++g) {
      const int64_t j0 = rowb + wr * 64 + t * 32 + 8 * g + 4 * (lane >> 5);
      const int64_t jlim = OUT == SK_OUT_WT_TILES ? a.kout : a.M;
      if (j0 >= jlim) continue;
#pragma unroll
      for (int jt = 0; jt < CTW; ++jt) {
        const int64_t c = colb + (wc * CTW + jt) * 32 + l32;
        if (c >= a.N) continue;
        const f32x16& v = acc[t][jt];
        if constexpr (OUT == SK_OUT_PART) {
          *(f32x4*)(a.part + ((int64_t)blockIdx.z * a.N + c) * a.Mp + j0) =
              f32x4{v[4 * g], v[4 * g + 1], v[4 * g + 2], v[4 * g + 3]};
        } else {
          u16x4 o;
#pragma unroll
          for (int i = 0; i < 4; ++i)
            o[i] = (j0 + i < a.M) ? bf16_rne((float)((double)v[4 * g + i] * a.d[j0 + i])) : (uint16_t)0;
          if constexpr (OUT == SK_OUT_WT_TILES) {
            // row c of the tiles, k = j0 .. j0 + 3 (within one chunk)
            const int64_t kb2 = j0 >> 5;
            const int ch = (int)((j0 & 31) >> 3) ^ sk_swz((int)(c & 15));
            *(u16x4*)((char*)a.out + (kb2 * a.rpo + c) * SK_ROWB + ch * 16 + (j0 & 7) * 2) = o;
          } else {
            uint16_t* dst = a.out + c * a.ldout + j0;
            if (j0 + 4 <= a.M) {
              *(u16x4*)dst = o;
            } else {
#pragma unroll
              for (int i = 0; i < 4; ++i)
                if (j0 + i < a.M) dst[i] = o[i];
            }
          }
        }
      }
    }
}

// ------------------------------------------------------------------ tiles, conversions, finishes

// Sketch tiles of X (R x K, row-major, leading dimension ld; T(r, k) = X[r][k]).
// A block covers 64 rows and 8 stages (256 k): four threads per row read 512
// contiguous bytes of it; each stage's 64 rows are written as 4 KB.
template <class SRC>
__global__ __launch_bounds__(NYS_BLOCK) void k_tile_rows(const SRC* X, int64_t R, int64_t K, int64_t ld,
                                                         bool vec, char* T, int64_t Rp, int64_t nkb) {
  const int r = threadIdx.x >> 2, p = threadIdx.x & 3;
  const int64_t row = (int64_t)blockIdx.x * 64 + r;
  const int c = p ^ sk_swz(r & 15);
  for (int s = 0; s < 8; ++s) {
    const int64_t kb = (int64_t)blockIdx.y * 8 + s;
    if (kb >= nkb) break;
    const int64_t k = kb * SK_TK + c * 8;
    u16x8 v = {0, 0, 0, 0, 0, 0, 0, 0};
    if (row < R) {
      const SRC* src = X + row * ld + k;
      if (vec && k + 8 <= K) {
        v = load8_bf16(src);
      } else {
#pragma unroll
        for (int e = 0; e < 8; ++e)
          if (k + e < K) v[e] = to_bf16(src[e]);
      }
    }
    *(u16x8*)(T + (kb * Rp + row) * SK_ROWB + p * 16) = v;
  }
}

// Sketch tiles of the transpose of X (X is K x R row-major, leading dimension
// ld; T(r, k) = X[k][r]).  A block covers one stage (32 rows of X) and 256 of
// its columns: coalesced 512-byte reads of X's rows into LDS, then the tile
// rows written as one contiguous 16 KB run.
template <class SRC>
__global__ __launch_bounds__(NYS_BLOCK) void k_tile_cols(const SRC* X, int64_t K, int64_t R, int64_t ld,
                                                         char* T, int64_t Rp) {
  __shared__ uint16_t S[SK_TK][256 + 2];
  const int64_t kb = blockIdx.x;
  const int64_t r0 = (int64_t)blockIdx.y * 256;
  for (int i = 0; i < SK_TK; ++i) {
    const int64_t k = kb * SK_TK + i, r = r0 + threadIdx.x;
    S[i][threadIdx.x] = (k < K && r < R) ? to_bf16(X[k * ld + r]) : (uint16_t)0;
  }
  __syncthreads();
  for (int q = threadIdx.x; q < 256 * 4; q += NYS_BLOCK) {
    const int r = q >> 2, p = q & 3, c = p ^ sk_swz(r & 15);
    u16x8 v;
#pragma unroll
    for (int e = 0; e < 8; ++e) v[e] = S[c * 8 + e][r];
    *(u16x8*)(T + (kb * Rp + r0 + r) * SK_ROWB + p * 16) = v;
  }
}

// Omega's tiles (rows c < rp, k = i < m): T(c, i) = bf16(fp32(Omega[i][c])),
// zero for c >= ell or i >= m.  A block: one stage (32 rows of Omega) and 64
// of its columns, read along c and written as 4 KB.
__global__ __launch_bounds__(NYS_BLOCK) void k_omega_tiles(const double* Om, int64_t m, int ell, char* T,
                                                           int64_t Rp) {
  __shared__ uint16_t S[SK_TK][64 + 2];
  const int64_t kb = blockIdx.x;
  const int c0 = blockIdx.y * 64;
  const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
  for (int i = ty; i < SK_TK; i += 4) {
    const int64_t k = kb * SK_TK + i;
    const int c = c0 + tx;
    S[i][tx] = (k < m && c < ell) ? bf16_rne((float)Om[k * ell + c]) : (uint16_t)0;
  }
  __syncthreads();
  const int r = threadIdx.x >> 2, p = threadIdx.x & 3, ch = p ^ sk_swz(r & 15);
  u16x8 v;
#pragma unroll
  for (int e = 0; e < 8; ++e) v[e] = S[ch * 8 + e][r];
  *(u16x8*)(T + (kb * Rp + c0 + r) * SK_ROWB + p * 16) = v;
}

// Ot[c][i] = bf16(fp32(Omega[i][c])), i < m (row-major operand): a 64 (i) x
// 64 (c) tile through LDS, read along c and written along i
__global__ __launch_bounds__(NYS_BLOCK) void k_omega_t(const double* Om, int64_t m, int ell, uint16_t* Ot,
                                                       int64_t ldo) {
  __shared__ uint16_t S[64][64 + 2];
  const int64_t i0 = (int64_t)blockIdx.x * 64;
  const int c0 = blockIdx.y * 64;
  const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
  for (int ii = ty; ii < 64; ii += 4) {
    const int64_t i = i0 + ii;
    const int c = c0 + tx;
    S[tx][ii] = (i < m && c < ell) ? bf16_rne((float)Om[i * ell + c]) : (uint16_t)0;
  }
  __syncthreads();
  for (int cc = ty; cc < 64; cc += 4) {
    const int64_t i = i0 + tx;
    const int c = c0 + cc;
    if (i < m && c < ell) Ot[(int64_t)c * ldo + i] = S[cc][tx];
  }
}

// W from the split-K partials: bf16(d[j] * sum_z part[z][c][j]) for c < N and
// j0 <= j < jlim, row-major (out[c * ldout + j], jlim = M) or in tiles of rpo
// rows (jlim = the tiles' K, zero for j >= M)
template <bool TILES>
__global__ __launch_bounds__(NYS_BLOCK) void k_sketch_finish_w(const float* part, int nsplit, int64_t M,
                                                               int64_t N, int64_t Mp, int64_t j0, int64_t jlim,
                                                               const double* d, uint16_t* out, int64_t ldout,
                                                               int64_t rpo) {
  const int64_t rows = jlim - j0, total = N * rows;
  for (int64_t idx = (int64_t)blockIdx.x * NYS_BLOCK + threadIdx.x; idx < total;
       idx += (int64_t)gridDim.x * NYS_BLOCK) {
    const int64_t c = idx / rows, j = j0 + idx % rows;
    uint16_t w = 0;
    if (j < M) {
      double s = 0.0;
      for (int z = 0; z < nsplit; ++z) s += (double)part[((int64_t)z * N + c) * Mp + j];
      w = bf16_rne((float)(s * d[j]));
    }
    if constexpr (TILES) {
      const int ch = (int)((j & 31) >> 3) ^ sk_swz((int)(c & 15));
      *(uint16_t*)((char*)out + ((j >> 5) * rpo + c) * SK_ROWB + ch * 16 + (j & 7) * 2) = w;
    } else {
      out[c * ldout + j] = w;
    }
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

// Column tiles (of 32) per wave and waves across the columns for N columns:
// the smallest instantiated width that covers N in one column group (two
// waves across the columns above 224), else column groups of 448.
struct SkShape {
  int ctw, wc, groups;
  int64_t bn() const { return 32LL * ctw * wc; }
  int64_t bnp() const { return (bn() + 63) / 64 * 64; }
  int64_t bm() const { return 64LL * (4 / wc); }
};
constexpr int kCtw[] = {1, 2, 4, 7};
SkShape sk_shape(int64_t N) {
  const int64_t tiles = (N + 31) / 32;
  for (int wc = 1; wc <= 2; ++wc)
    for (int c : kCtw)
      if ((int64_t)c * wc >= tiles) return {c, wc, 1};
  return {7, 2, (int)((tiles + 13) / 14)};
}
// Rows of the tiles of a small operand with N rows (covers every column group's slab)
int64_t sk_rows_small(int64_t N) {
  const SkShape sh = sk_shape(N);
  return sh.groups * sh.bnp();
}
int64_t sk_rows_big(int64_t R) { return (R + SK_TILE_ROWS - 1) / SK_TILE_ROWS * SK_TILE_ROWS; }
int64_t sk_kblocks(int64_t K) { return (K + SK_TK - 1) / SK_TK; }

// Splits of K for a grid of `tiles` blocks: enough blocks to keep the 256
// compute units busy in whole rounds (one resident block per unit), each
// split at least 32 stages (1024 k) long.
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
void launch_sk(const SkArgs& a, dim3 g, bool tiled, bool vec, int out, hipStream_t st) {
  if (tiled) {
    if (out == SK_OUT_PART) hipLaunchKernelGGL((k_sketch_mfma<CTW, WC, true, true, SK_OUT_PART>), g, dim3(SK_THREADS), 0, st, a);
    else hipLaunchKernelGGL((k_sketch_mfma<CTW, WC, true, true, SK_OUT_WT_TILES>), g, dim3(SK_THREADS), 0, st, a);
  } else if (vec) {
    if (out == SK_OUT_PART) hipLaunchKernelGGL((k_sketch_mfma<CTW, WC, false, true, SK_OUT_PART>), g, dim3(SK_THREADS), 0, st, a);
    else hipLaunchKernelGGL((k_sketch_mfma<CTW, WC, false, true, SK_OUT_WT>), g, dim3(SK_THREADS), 0, st, a);
  } else {
    if (out == SK_OUT_PART) hipLaunchKernelGGL((k_sketch_mfma<CTW, WC, false, false, SK_OUT_PART>), g, dim3(SK_THREADS), 0, st, a);
    else hipLaunchKernelGGL((k_sketch_mfma<CTW, WC, false, false, SK_OUT_WT>), g, dim3(SK_THREADS), 0, st, a);
  }
}

template <int WC>
void launch_sk_ctw(int ctw, const SkArgs& a, dim3 g, bool tiled, bool vec, int out, hipStream_t st) {
  switch (ctw) {
    case 1: launch_sk<1, WC>(a, g, tiled, vec, out, st); break;
    case 2: launch_sk<2, WC>(a, g, tiled, vec, out, st); break;
    case 4: launch_sk<4, WC>(a, g, tiled, vec, out, st); break;
    default: launch_sk<7, WC>(a, g, tiled, vec, out, st); break;
  }
}

// One product C (M x N) = Aop (M x K) Bop (N x K)^T.  Operands row-major
// (tiled = false; a.lda, a.ldb) or in sketch tiles (a.rpa, a.rpb).  With
// want_w and one split, C is written as BF16 W (SK_OUT_WT or
// SK_OUT_WT_TILES per a.out...); otherwise split-K partials go to the
// workspace and *part / *nsplit describe them (*part = NULL when W was
// written directly), for rows from *row0 on (the rows before it were
// written as W directly).
int sketch_gemm(nys_handle h, SkArgs a, bool tiled, bool want_w, float** part, int* nsplit_out,
                int64_t* row0 = nullptr) {
  const SkShape sh = sk_shape(a.N);
  const int64_t tiles = (a.M + sh.bm() - 1) / sh.bm();
  if (tiles > 0x7FFFFFFFLL) return set_error(h, NYS_EINVAL, "BF16 sketch: %lld row tiles", (long long)tiles);
  if (row0) *row0 = 0;
  // The W product writes BF16 W directly, without split-K, once its grid has
  // a block for every compute unit: partial sums of n x ell in FP32 per split
  // and their summation cost more than a last, partly filled round of blocks.
  // When that last round (one block per compute unit, tiles % 256 of them)
  // is under half full, it runs as a launch of its own, split over K so that
  // it fills the units: the split s minimises its rounds times the stages
  // per block, plus the partial sums' traffic counted in stages (one stage
  // moves about (BM + BN) * 64 bytes into a unit, 256 units at a time).
  // Measured: W at 50000 x 200000, ell = 400 (27 tiles in the last round)
  // 8.8 ms against 9.8; at 20000 x 100000, ell = 200 (135 tiles) no change.
  const int64_t ncu = 256;
  if (want_w && sh.groups == 1 && tiles > ncu && tiles % ncu != 0 && tiles % ncu <= ncu / 2 && row0) {
    const int64_t full = tiles - tiles % ncu, tail = tiles % ncu;
    const int64_t kt = (a.K + SK_TK - 1) / SK_TK;
    const double stage_bytes = (double)(sh.bm() + sh.bnp()) * SK_ROWB * ncu;
    int best = 1;
    double best_cost = 0.0;
    for (int sp = 1; sp <= 16 && sp <= kt; ++sp) {
      const int64_t rounds = (tail * sp + ncu - 1) / ncu, per = (kt + sp - 1) / sp;
      const double traffic = sp > 1 ? 2.0 * sp * (double)(tail * sh.bm()) * (double)a.N * 4.0 / stage_bytes : 0.0;
      const double cost = (double)(rounds * per) + traffic;
      if (sp == 1 || cost < best_cost) {
        best = sp;
        best_cost = cost;
      }
    }
    if (best > 1) {
      SkArgs b = a;
      b.ntile = full;
      b.ngroup = 1;
      b.tile0 = 0;
      b.klen = kt * SK_TK;
      b.Mp = (a.M + 3) / 4 * 4;
      const bool vec = tiled || (((uintptr_t)a.A % 16 == 0) && (a.lda % 8 == 0));
      const int out_w = tiled ? SK_OUT_WT_TILES : SK_OUT_WT;
      dim3 g1((unsigned)full, 1u, 1u);
      if (sh.wc == 1) launch_sk_ctw<1>(sh.ctw, b, g1, tiled, vec, out_w, h->stream);
      else launch_sk_ctw<2>(sh.ctw, b, g1, tiled, vec, out_w, h->stream);
      NYS_LAUNCH_CHECK(h);
      int64_t klen = (a.K + best - 1) / best;
      klen = (klen + SK_TK - 1) / SK_TK * SK_TK;
      const int nsplit = (int)std::max<int64_t>(1, (a.K + klen - 1) / klen);
      b.klen = klen;
      b.tile0 = full;
      b.ntile = tiles;
      NYS_CHECK(ws_get(h, WS_SK_SPLIT, (size_t)nsplit * a.N * b.Mp * sizeof(float), (void**)&b.part));
      dim3 g2((unsigned)tail, 1u, (unsigned)nsplit);
      if (sh.wc == 1) launch_sk_ctw<1>(sh.ctw, b, g2, tiled, vec, SK_OUT_PART, h->stream);
      else launch_sk_ctw<2>(sh.ctw, b, g2, tiled, vec, SK_OUT_PART, h->stream);
      NYS_LAUNCH_CHECK(h);
      *part = b.part;
      *nsplit_out = nsplit;
      *row0 = full * sh.bm();
      return NYS_OK;
    }
  }
  int nsplit = want_w && tiles * sh.groups >= ncu ? 1 : sk_splits(tiles * sh.groups, a.K);
  const bool direct = want_w && nsplit == 1;
  int64_t klen = (a.K + nsplit - 1) / nsplit;
  klen = (klen + SK_TK - 1) / SK_TK * SK_TK;
  nsplit = (int)std::max<int64_t>(1, (a.K + klen - 1) / klen);
  a.klen = klen;
  a.Mp = (a.M + 3) / 4 * 4;
  *part = nullptr;
  *nsplit_out = nsplit;
  if (!direct) {
    NYS_CHECK(ws_get(h, WS_SK_SPLIT, (size_t)nsplit * a.N * a.Mp * sizeof(float), (void**)&a.part));
    *part = a.part;
  }
  const bool vec = tiled || (((uintptr_t)a.A % 16 == 0) && (a.lda % 8 == 0));
  const int out = !direct ? SK_OUT_PART : (tiled ? SK_OUT_WT_TILES : SK_OUT_WT);
  a.ntile = tiles;
  a.ngroup = sh.groups;
  dim3 g((unsigned)tiles, 1u, (unsigned)nsplit);
  if (sh.groups > 1) {
    const int64_t nx = (tiles + 7) / 8 * 8 * sh.groups;
    if (nx > 0x7FFFFFFFLL) return set_error(h, NYS_EINVAL, "BF16 sketch: %lld blocks", (long long)nx);
    g.x = (unsigned)nx;
  }
  if (sh.wc == 1) launch_sk_ctw<1>(sh.ctw, a, g, tiled, vec, out, h->stream);
  else launch_sk_ctw<2>(sh.ctw, a, g, tiled, vec, out, h->stream);
  NYS_LAUNCH_CHECK(h);
  return NYS_OK;
}

}  // namespace

int64_t sketch_tiles_bytes(int64_t rows, int64_t cols) {
  return sk_kblocks(cols) * sk_rows_big(rows) * SK_ROWB;
}

int sketch_tiles(nys_handle h, const nys_matrix* A, bool transposed, void* out) {
  const int64_t m = A->m, n = A->n;
  if (m == 0 || n == 0) return NYS_OK;
  char* T = (char*)out;
  if (!transposed) {
    // rows m, k = n: from the rows of A
    const int64_t rp = sk_rows_big(m), nkb = sk_kblocks(n);
    if ((nkb + 7) / 8 > 65535)
      return set_error(h, NYS_EINVAL, "sketch tiles: n=%lld above %lld", (long long)n, 65535LL * 8 * SK_TK);
    dim3 g((unsigned)(rp / 64), (unsigned)((nkb + 7) / 8));
    const bool vec = ((uintptr_t)A->data % 16 == 0) && (A->ld % 8 == 0);
    switch (A->dtype) {
      case NYS_BF16: hipLaunchKernelGGL(k_tile_rows<uint16_t>, g, dim3(NYS_BLOCK), 0, h->stream, (const uint16_t*)A->data, m, n, A->ld, vec, T, rp, nkb); break;
      case NYS_F32: hipLaunchKernelGGL(k_tile_rows<float>, g, dim3(NYS_BLOCK), 0, h->stream, (const float*)A->data, m, n, A->ld, vec, T, rp, nkb); break;
      default: hipLaunchKernelGGL(k_tile_rows<double>, g, dim3(NYS_BLOCK), 0, h->stream, (const double*)A->data, m, n, A->ld, vec, T, rp, nkb); break;
    }
  } else {
    // rows n, k = m: from the columns of A
    const int64_t rp = sk_rows_big(n), nkb = sk_kblocks(m);
    if (rp / 256 > 65535)
      return set_error(h, NYS_EINVAL, "sketch tiles: n=%lld above %lld", (long long)n, 65535LL * 256);
    dim3 g((unsigned)nkb, (unsigned)(rp / 256));
    switch (A->dtype) {
      case NYS_BF16: hipLaunchKernelGGL(k_tile_cols<uint16_t>, g, dim3(NYS_BLOCK), 0, h->stream, (const uint16_t*)A->data, m, n, A->ld, T, rp); break;
      case NYS_F32: hipLaunchKernelGGL(k_tile_cols<float>, g, dim3(NYS_BLOCK), 0, h->stream, (const float*)A->data, m, n, A->ld, T, rp); break;
      default: hipLaunchKernelGGL(k_tile_cols<double>, g, dim3(NYS_BLOCK), 0, h->stream, (const double*)A->data, m, n, A->ld, T, rp); break;
    }
  }
  NYS_LAUNCH_CHECK(h);
  return NYS_OK;
}

int sketch_bf16(nys_handle h, const nys_matrix* A, const double* d, const double* Omega, int ell,
                double* Y) {
  const int64_t m = A->m, n = A->n;
  if (n == 0) return fill(h, Y, m * ell, 0.0);
  float* part = nullptr;
  int nsplit = 1;
  if (A->tiles && A->tiles_t) {
    // sketch tiles of A (rows m) and of A^T (rows n); Omega and W in tiles too
    const int64_t rpb = sk_rows_small(ell), kbm = sk_kblocks(m), kbn = sk_kblocks(n);
    char *Ot, *Wt;
    NYS_CHECK(ws_get(h, WS_SK_LO, (size_t)(kbm * rpb * SK_ROWB), (void**)&Ot));
    NYS_CHECK(ws_get(h, WS_SK_W, (size_t)(kbn * rpb * SK_ROWB), (void**)&Wt));
    hipLaunchKernelGGL(k_omega_tiles, dim3((unsigned)kbm, (unsigned)(rpb / 64)), dim3(NYS_BLOCK), 0, h->stream,
                       Omega, m, ell, Ot, rpb);
    NYS_LAUNCH_CHECK(h);
    {
      const int ps = prof_begin(h, NYS_K_SKETCH_W);
      SkArgs a{};
      a.M = n;
      a.N = ell;
      a.K = m;
      a.A = (const uint16_t*)A->tiles_t;
      a.rpa = sk_rows_big(n);
      a.B = (const uint16_t*)Ot;
      a.rpb = rpb;
      a.out = (uint16_t*)Wt;
      a.rpo = rpb;
      a.kout = kbn * SK_TK;
      a.d = d;
      int64_t row0 = 0;
      NYS_CHECK(sketch_gemm(h, a, true, true, &part, &nsplit, &row0));
      if (part) {
        hipLaunchKernelGGL((k_sketch_finish_w<true>), dim3(grid1d((int64_t)ell * (kbn * SK_TK - row0))),
                           dim3(NYS_BLOCK), 0, h->stream, part, nsplit, n, (int64_t)ell, (n + 3) / 4 * 4, row0,
                           kbn * SK_TK, d, (uint16_t*)Wt, (int64_t)0, rpb);
        NYS_LAUNCH_CHECK(h);
      }
      prof_end(h, ps);
    }
    {
      const int ps = prof_begin(h, NYS_K_SKETCH_Y);
      SkArgs a{};
      a.M = m;
      a.N = ell;
      a.K = n;
      a.A = (const uint16_t*)A->tiles;
      a.rpa = sk_rows_big(m);
      a.B = (const uint16_t*)Wt;
      a.rpb = rpb;
      NYS_CHECK(sketch_gemm(h, a, true, false, &part, &nsplit));
      hipLaunchKernelGGL(k_sketch_finish_y, dim3((unsigned)((m + 63) / 64), (unsigned)((ell + 31) / 32)),
                         dim3(NYS_BLOCK), 0, h->stream, part, nsplit, m, (int64_t)ell, (m + 3) / 4 * 4, Y);
      NYS_LAUNCH_CHECK(h);
      prof_end(h, ps);
    }
    return NYS_OK;
  }
  if (A->dtype != NYS_BF16) return set_error(h, NYS_EINVAL, "BF16 sketch needs BF16 storage of A");
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
      SkArgs a{};
      a.M = n;
      a.N = ell;
      a.K = m;
      a.A = (const uint16_t*)A->data_t;
      a.lda = A->ld_t;
      a.B = Ot;
      a.ldb = ldo;
      a.out = Wt;
      a.ldout = ldw;
      a.d = d;
      int64_t row0 = 0;
      NYS_CHECK(sketch_gemm(h, a, false, true, &part, &nsplit, &row0));
      if (part) {
        hipLaunchKernelGGL((k_sketch_finish_w<false>), dim3(grid1d((n - row0) * ell)), dim3(NYS_BLOCK), 0, h->stream,
                           part, nsplit, n, (int64_t)ell, (n + 3) / 4 * 4, row0, n, d, Wt, ldw, (int64_t)0);
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
    SkArgs a{};
    a.M = m;
    a.N = ell;
    a.K = n;
    a.A = Ad;
    a.lda = A->ld;
    a.B = Wt;
    a.ldb = ldw;
    NYS_CHECK(sketch_gemm(h, a, false, false, &part, &nsplit));
    dim3 g((unsigned)((m + 63) / 64), (unsigned)((ell + 31) / 32));
    hipLaunchKernelGGL(k_sketch_finish_y, g, dim3(NYS_BLOCK), 0, h->stream, part, nsplit, m, (int64_t)ell,
                       (m + 3) / 4 * 4, Y);
    NYS_LAUNCH_CHECK(h);
    prof_end(h, ps);
  }
  return NYS_OK;
}

}  // namespace nys
