// Device helpers shared by the NNLS kernels (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace nnls {

constexpr int kWave = 64;

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x4 __attribute__((ext_vector_type(4)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

// Round-to-nearest-even FP32 -> BF16 bits.  NaN and Inf map to NaN and Inf.
__device__ __forceinline__ uint32_t bf16_bits_rne(float x) {
  uint32_t u = __builtin_bit_cast(uint32_t, x);
  uint32_t lsb = (u >> 16) & 1u;
  return (u + 0x7FFFu + lsb) >> 16;
}

__device__ __forceinline__ float bf16_bits_to_f32(uint32_t b) {
  return __builtin_bit_cast(float, b << 16);
}

template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, kWave);
  return v;
}

// FP32 wave sum without the LDS crossbar: quad sums by DPP quad permutations, row sums by DPP row
// rotations, the four rows by v_permlane16_swap_b32 / v_permlane32_swap_b32 (each exchanges half
// of one register with half of another, so the sum of two swapped copies pairs lanes l and
// l ^ 16, or l ^ 32), then lane 0's total broadcast, so every lane returns the same value.  Every
// lane must be active.  (s_nop 1: the swaps read registers the instructions just before may
// have written.)
template <int CTRL>
__device__ __forceinline__ float dpp_f32(float v) {
  return __builtin_bit_cast(
      float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), CTRL, 0xF, 0xF, false));
}
template <>
__device__ __forceinline__ float wave_sum<float>(float v) {
  v += dpp_f32<0xB1>(v);   // quad_perm [1, 0, 3, 2]
  v += dpp_f32<0x4E>(v);   // quad_perm [2, 3, 0, 1]
  v += dpp_f32<0x124>(v);  // row_ror 4
  v += dpp_f32<0x128>(v);  // row_ror 8
  float a = v, b = v;
  asm volatile("s_nop 1\n\tv_permlane16_swap_b32 %0, %1" : "+v"(a), "+v"(b));
  v = a + b;
  a = v;
  b = v;
  asm volatile("s_nop 1\n\tv_permlane32_swap_b32 %0, %1" : "+v"(a), "+v"(b));
  v = a + b;
  return __builtin_bit_cast(float, __builtin_amdgcn_readfirstlane(__builtin_bit_cast(int, v)));
}

// Sum over the block; every thread gets the result.  `red` is LDS scratch of >= nwaves entries.
// Contains two barriers.
template <typename T, int NT>
__device__ __forceinline__ T block_sum(T v, T* red) {
  constexpr int NW = NT / kWave;
  v = wave_sum(v);
  const int lane = threadIdx.x & (kWave - 1);
  const int w = threadIdx.x / kWave;
  if (lane == 0) red[w] = v;
  __syncthreads();
  T t = 0;
#pragma unroll
  for (int i = 0; i < NW; ++i) t += red[i];
  __syncthreads();
  return t;
}

// Exclusive prefix sum of one int per thread over the block, in thread order; `total` gets the
// block total.  `red` is LDS scratch of >= nwaves ints.  Two barriers.
template <int NT>
__device__ __forceinline__ int block_exclusive_scan(int v, int* red, int& total) {
  constexpr int NW = NT / kWave;
  const int lane = threadIdx.x & (kWave - 1);
  const int w = threadIdx.x / kWave;
  // inclusive scan within each 16-lane row by DPP row shifts (zero fill), then the totals of
  // the rows below from lanes 15, 31 and 47
  int incl = v;
  incl += __builtin_amdgcn_update_dpp(0, incl, 0x111, 0xF, 0xF, false);  // row_shr 1
  incl += __builtin_amdgcn_update_dpp(0, incl, 0x112, 0xF, 0xF, false);  // row_shr 2
  incl += __builtin_amdgcn_update_dpp(0, incl, 0x114, 0xF, 0xF, false);  // row_shr 4
  incl += __builtin_amdgcn_update_dpp(0, incl, 0x118, 0xF, 0xF, false);  // row_shr 8
  const int r0 = __builtin_amdgcn_readlane(incl, 15), r1 = __builtin_amdgcn_readlane(incl, 31),
            r2 = __builtin_amdgcn_readlane(incl, 47);
  const int row = lane >> 4;
  incl += (row >= 1 ? r0 : 0) + (row >= 2 ? r1 : 0) + (row >= 3 ? r2 : 0);
  if (lane == kWave - 1) red[w] = incl;
  __syncthreads();
  int base = 0, tot = 0;
#pragma unroll
  for (int i = 0; i < NW; ++i) {
    int r = red[i];
    base += (i < w) ? r : 0;
    tot += r;
  }
  __syncthreads();
  total = tot;
  return base + incl - v;
}

__device__ __forceinline__ bool is_finite_val(float v) { return __builtin_isfinite(v); }
__device__ __forceinline__ bool is_finite_val(double v) { return __builtin_isfinite(v); }

}  // namespace nnls
