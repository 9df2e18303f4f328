// Device-side types and wave-level helpers shared by the HIP kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "layout.hpp"
#include "nasg_math.hpp"

namespace nasg {

typedef __attribute__((ext_vector_type(8))) __bf16 bf16x8;
typedef __attribute__((ext_vector_type(4))) __bf16 bf16x4;
typedef __attribute__((ext_vector_type(4))) float f32x4;

constexpr int kWave = 64;
constexpr int kTileV = 16;          // vertices per MFMA column block
constexpr int kRecTile = 64;        // vertices per decoded-record tile

__device__ __forceinline__ int lane_id() { return (int)(threadIdx.x & 63); }

// Reductions over the four lanes c, c+16, c+32, c+48 that share a vertex.
__device__ __forceinline__ float quad_max(float x) {
  x = fmaxf(x, __shfl_xor(x, 16));
  return fmaxf(x, __shfl_xor(x, 32));
}
__device__ __forceinline__ float quad_sum(float x) {
  x += __shfl_xor(x, 16);
  return x + __shfl_xor(x, 32);
}
__device__ __forceinline__ int quad_min_i(int x) {
  x = min(x, __shfl_xor(x, 16));
  return min(x, __shfl_xor(x, 32));
}
__device__ __forceinline__ int quad_max_i(int x) {
  x = max(x, __shfl_xor(x, 16));
  return max(x, __shfl_xor(x, 32));
}

__device__ __forceinline__ f32x4 mfma_bf16_32(bf16x8 a, bf16x8 b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ f32x4 mfma_bf16_16(bf16x4 a, bf16x4 b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ f32x4 mfma_f32_4(float a, float b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

// max(x, 0) as one integer max on the bit pattern: negative floats (and -0)
// are negative integers. Avoids the NaN canonicalisation fmaxf needs.
__device__ __forceinline__ float relu(float x) { return __int_as_float(max(__float_as_int(x), 0)); }

__device__ __forceinline__ f32x4 zero4() { return f32x4{0.0f, 0.0f, 0.0f, 0.0f}; }

// Copy `bytes` (multiple of 16) from global to LDS with the whole block.
__device__ __forceinline__ void block_copy_to_lds(void* lds, const void* src, int bytes) {
  const uint4* s = reinterpret_cast<const uint4*>(src);
  uint4* d = reinterpret_cast<uint4*>(lds);
  int n = bytes >> 4;
  for (int i = threadIdx.x; i < n; i += blockDim.x) d[i] = s[i];
}

}  // namespace nasg
