// Device helpers shared by the nysipm kernels (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "nysipm.h"

#define NYS_WAVE 64
#define NYS_BLOCK 256

namespace nys {

// ------------------------------------------------------------------ storage types
// Tag types for the three storage formats of the constraint matrix.
struct F64 { using raw = double;   static constexpr int vec = 2; };   // 16 B = 2 values
struct F32 { using raw = float;    static constexpr int vec = 4; };   // 16 B = 4 values
struct BF16 { using raw = uint16_t; static constexpr int vec = 8; };  // 16 B = 8 values

__device__ __forceinline__ double to_f64(double v) { return v; }
__device__ __forceinline__ double to_f64(float v) { return (double)v; }
__device__ __forceinline__ double to_f64(uint16_t v) {
  return (double)__uint_as_float(((uint32_t)v) << 16);
}

typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

// Unpack a 16-byte vector into VEC doubles.
template <class T> struct Unpack;
template <> struct Unpack<F64> {
  __device__ __forceinline__ static void run(const u32x4& u, double* o) {
    o[0] = __hiloint2double((int)u.y, (int)u.x);
    o[1] = __hiloint2double((int)u.w, (int)u.z);
  }
};
template <> struct Unpack<F32> {
  __device__ __forceinline__ static void run(const u32x4& u, double* o) {
    o[0] = (double)__uint_as_float(u.x);
    o[1] = (double)__uint_as_float(u.y);
    o[2] = (double)__uint_as_float(u.z);
    o[3] = (double)__uint_as_float(u.w);
  }
};
template <> struct Unpack<BF16> {
  __device__ __forceinline__ static void run(const u32x4& u, double* o) {
    o[0] = (double)__uint_as_float(u.x << 16);
    o[1] = (double)__uint_as_float(u.x & 0xFFFF0000u);
    o[2] = (double)__uint_as_float(u.y << 16);
    o[3] = (double)__uint_as_float(u.y & 0xFFFF0000u);
    o[4] = (double)__uint_as_float(u.z << 16);
    o[5] = (double)__uint_as_float(u.z & 0xFFFF0000u);
    o[6] = (double)__uint_as_float(u.w << 16);
    o[7] = (double)__uint_as_float(u.w & 0xFFFF0000u);
  }
};

// Non-temporal 16-byte load of a streamed operand (A is read once per pass).
__device__ __forceinline__ u32x4 ld_stream16(const void* p) {
  return __builtin_nontemporal_load((const u32x4*)p);
}
__device__ __forceinline__ u32x4 ld16(const void* p) { return *(const u32x4*)p; }

// VEC consecutive doubles (VEC even, p 16-byte aligned) through 16-byte loads.
template <int VEC>
__device__ __forceinline__ void ld_f64s(const double* p, double* o) {
#pragma unroll
  for (int e = 0; e < VEC; e += 2) {
    const u32x4 u = ld16(p + e);
    o[e] = __hiloint2double((int)u.y, (int)u.x);
    o[e + 1] = __hiloint2double((int)u.w, (int)u.z);
  }
}

// ------------------------------------------------------------------ reductions
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, NYS_WAVE);
  return v;
}
__device__ __forceinline__ double wave_min(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v = fmin(v, __shfl_xor(v, off, NYS_WAVE));
  return v;
}

// Block-wide sum of K values per thread; result valid in every thread.
// `smem` needs K * (blockDim/64) doubles.  Fixed order: deterministic.
// Wave sum through DPP lane moves and lane reads instead of LDS permutes (for
// latency-bound loops).  Within each row of 16 lanes: swap neighbours, swap
// pairs (quad permutes), then half-row and row mirrors leave every lane of the
// row with the row sum; the four row sums are read from lanes 0/16/32/48 and
// added in a fixed order, so all lanes return the same value.  Needs all 64
// lanes active.
template <int CTRL>
__device__ __forceinline__ double dpp_mov(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)b, CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xF, 0xF, false);
  return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}
__device__ __forceinline__ double lane_read(double v, int lane) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)b, lane);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), lane);
  return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}
__device__ __forceinline__ double wave_sum_dpp(double v) {
  v += dpp_mov<0xB1>(v);    // quad_perm [1,0,3,2]
  v += dpp_mov<0x4E>(v);    // quad_perm [2,3,0,1]
  v += dpp_mov<0x141>(v);   // row_half_mirror
  v += dpp_mov<0x140>(v);   // row_mirror
  return (lane_read(v, 0) + lane_read(v, 16)) + (lane_read(v, 32) + lane_read(v, 48));
}

template <int K>
__device__ __forceinline__ void block_sum(double* v, double* smem) {
  const int lane = threadIdx.x & (NYS_WAVE - 1);
  const int wid = threadIdx.x / NYS_WAVE;
  const int nw = blockDim.x / NYS_WAVE;
#pragma unroll
  for (int k = 0; k < K; ++k) v[k] = wave_sum(v[k]);
  __syncthreads();
  if (lane == 0) {
#pragma unroll
    for (int k = 0; k < K; ++k) smem[k * nw + wid] = v[k];
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < K; ++k) {
    double s = 0.0;
    for (int w = 0; w < nw; ++w) s += smem[k * nw + w];
    v[k] = s;
  }
  __syncthreads();
}

template <int K>
__device__ __forceinline__ void block_min(double* v, double* smem) {
  const int lane = threadIdx.x & (NYS_WAVE - 1);
  const int wid = threadIdx.x / NYS_WAVE;
  const int nw = blockDim.x / NYS_WAVE;
#pragma unroll
  for (int k = 0; k < K; ++k) v[k] = wave_min(v[k]);
  __syncthreads();
  if (lane == 0) {
#pragma unroll
    for (int k = 0; k < K; ++k) smem[k * nw + wid] = v[k];
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < K; ++k) {
    double s = smem[k * nw];
    for (int w = 1; w < nw; ++w) s = fmin(s, smem[k * nw + w]);
    v[k] = s;
  }
  __syncthreads();
}

}  // namespace nys
