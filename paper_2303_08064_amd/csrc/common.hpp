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

// Asynchronous copy of `bytes` (multiple of 16) from global memory to LDS
// with the whole block, through the gfx950 direct-to-LDS load
// (global_load_lds_dwordx4): every wave moves 1 KiB per instruction, lane i
// landing at LDS offset 16 i of that KiB, without passing through registers.
// All loads are issued before any completes; lds_dma_wait() then waits for
// this wave's copies, and a barrier after it publishes everyone's.
__device__ __forceinline__ void lds_dma(void* lds, const void* src, int bytes) {
  const int wave = (int)(threadIdx.x >> 6), lane = lane_id();
  const int nw = (int)(blockDim.x >> 6);
  const int chunks = (bytes + 1023) >> 10;
  for (int j = wave; j < chunks; j += nw) {
    const int off = j * 1024 + lane * 16;
    if (off < bytes)
      __builtin_amdgcn_global_load_lds(reinterpret_cast<const char*>(src) + off,
                                       (__attribute__((address_space(3))) void*)(reinterpret_cast<char*>(lds) +
                                                                                 j * 1024),
                                       16, 0, 0);
  }
}

// s_waitcnt vmcnt(0): every vector-memory load of this wave, including the
// direct-to-LDS copies, has completed (expcnt and lgkmcnt left unconstrained).
__device__ __forceinline__ void lds_dma_wait() { __builtin_amdgcn_s_waitcnt(0x0F70); }

}  // namespace nasg
