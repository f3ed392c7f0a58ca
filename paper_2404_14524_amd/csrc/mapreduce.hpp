// A fused element-wise map with a deterministic two-stage reduction, used by
// the vector updates of PCG and of the interior-point driver.  The functor is
// called as f(j, sums, mins) for every index j < n; it may write any outputs
// for index j and add to NS running sums / lower NM running minima.  Each
// block writes its NS + NM results to a partial buffer; a one-block second
// launch combines them in block order into the device words out[0 .. NS+NM).
// (Two launches instead of a "last block" election: on gfx950 the device-wide
// fence such an election needs writes back and invalidates the whole L2.)
#pragma once

#include <cmath>

#include "common.hpp"
#include "handle.hpp"

namespace nys {

template <class F, int NS, int NM>
__global__ __launch_bounds__(NYS_BLOCK) void k_map_reduce(int64_t n, F f, double* part, double* out) {
  constexpr int NR = NS + NM;
  __shared__ double smem[(NR > 0 ? NR : 1) * (NYS_BLOCK / NYS_WAVE)];
  double s[NS > 0 ? NS : 1];
  double mn[NM > 0 ? NM : 1];
#pragma unroll
  for (int k = 0; k < NS; ++k) s[k] = 0.0;
#pragma unroll
  for (int k = 0; k < NM; ++k) mn[k] = HUGE_VAL;
  const int64_t stride = (int64_t)gridDim.x * NYS_BLOCK;
  for (int64_t j = (int64_t)blockIdx.x * NYS_BLOCK + threadIdx.x; j < n; j += stride) f(j, s, mn);
  if constexpr (NR > 0) {
    if constexpr (NS > 0) block_sum<NS>(s, smem);
    if constexpr (NM > 0) block_min<NM>(mn, smem);
    double* dst = gridDim.x == 1 ? out : part + (int64_t)blockIdx.x * NR;
    if (threadIdx.x == 0) {
#pragma unroll
      for (int k = 0; k < NS; ++k) dst[k] = s[k];
#pragma unroll
      for (int k = 0; k < NM; ++k) dst[NS + k] = mn[k];
    }
  }
}

template <int NS, int NM>
__global__ __launch_bounds__(NYS_BLOCK) void k_map_reduce_finish(int nb, const double* part, double* out) {
  constexpr int NR = NS + NM;
  __shared__ double smem[NR * (NYS_BLOCK / NYS_WAVE)];
  double s[NS > 0 ? NS : 1];
  double mn[NM > 0 ? NM : 1];
#pragma unroll
  for (int k = 0; k < NS; ++k) s[k] = 0.0;
#pragma unroll
  for (int k = 0; k < NM; ++k) mn[k] = HUGE_VAL;
  for (int b = threadIdx.x; b < nb; b += NYS_BLOCK) {
#pragma unroll
    for (int k = 0; k < NS; ++k) s[k] += part[(int64_t)b * NR + k];
#pragma unroll
    for (int k = 0; k < NM; ++k) mn[k] = fmin(mn[k], part[(int64_t)b * NR + NS + k]);
  }
  if constexpr (NS > 0) block_sum<NS>(s, smem);
  if constexpr (NM > 0) block_min<NM>(mn, smem);
  if (threadIdx.x == 0) {
#pragma unroll
    for (int k = 0; k < NS; ++k) out[k] = s[k];
#pragma unroll
    for (int k = 0; k < NM; ++k) out[NS + k] = mn[k];
  }
}

inline unsigned map_reduce_blocks(int64_t n) {
  int64_t b = (n + NYS_BLOCK - 1) / NYS_BLOCK;
  if (b > 1024) b = 1024;
  if (b < 1) b = 1;
  return (unsigned)b;
}

// Launch helper: out may be NULL when NS + NM == 0.
template <int NS, int NM, class F>
int map_reduce(nys_handle h, int64_t n, const F& f, double* out) {
  const unsigned nb = map_reduce_blocks(n);
  double* part = nullptr;
  if (NS + NM > 0 && nb > 1) NYS_CHECK(ws(h, WS_PART2, (size_t)nb * (NS + NM), &part));
  hipLaunchKernelGGL((k_map_reduce<F, NS, NM>), dim3(nb), dim3(NYS_BLOCK), 0, h->stream, n, f, part, out);
  NYS_LAUNCH_CHECK(h);
  if constexpr (NS + NM > 0) {
    if (nb > 1) {
      hipLaunchKernelGGL((k_map_reduce_finish<NS, NM>), dim3(1), dim3(NYS_BLOCK), 0, h->stream, (int)nb,
                         (const double*)part, out);
      NYS_LAUNCH_CHECK(h);
    }
  }
  return NYS_OK;
}

}  // namespace nys
