// Device-side types and wave-level helpers shared by the HIP kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <mutex>

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
// The same reductions by the gfx950 lane swaps (VALU, no LDS round trip):
// v_permlane16_swap of x with itself leaves x and its xor-16 partner in the
// two results of every lane, v_permlane32_swap the xor-32 partner; the
// operations are the same commutative pairs as above, so the results are
// bitwise the same.
__device__ __forceinline__ float xchg_max(float x) {
  auto a = __builtin_amdgcn_permlane16_swap(__float_as_uint(x), __float_as_uint(x), false, false);
  x = fmaxf(__uint_as_float(a[0]), __uint_as_float(a[1]));
  auto b = __builtin_amdgcn_permlane32_swap(__float_as_uint(x), __float_as_uint(x), false, false);
  return fmaxf(__uint_as_float(b[0]), __uint_as_float(b[1]));
}
__device__ __forceinline__ float xchg_sum(float x) {
  auto a = __builtin_amdgcn_permlane16_swap(__float_as_uint(x), __float_as_uint(x), false, false);
  x = __uint_as_float(a[0]) + __uint_as_float(a[1]);
  auto b = __builtin_amdgcn_permlane32_swap(__float_as_uint(x), __float_as_uint(x), false, false);
  return __uint_as_float(b[0]) + __uint_as_float(b[1]);
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

// acc[nb][mt] = sum over kb of A[mt][kb] b[nb][kb] for MT row tiles and KB
// 32-wide contraction blocks, the A fragments [MT][KB][64 lanes] at `frag`
// (LDS). The steps run block-major (kb outer, row tiles inner), so
// consecutive MFMAs accumulate into different tiles instead of waiting on
// each other, and the fragment of step s + PF is requested before step s is
// multiplied, so PF LDS reads are in flight behind the MFMAs.
// bop(nb, kb) returns the B operand b[nb][kb].
template <int MT, int KB, int NB, int PF = 4, typename BOp>
__device__ __forceinline__ void mfma_rows(const bf16x8* frag, BOp bop, f32x4 (&acc)[NB][MT], int lane) {
  constexpr int N = MT * KB;
  constexpr int D = PF < N ? PF : N;
  bf16x8 a[D + 1];
#pragma unroll
  for (int s = 0; s < D; ++s) a[s] = frag[((s % MT) * KB + s / MT) * 64 + lane];
#pragma unroll
  for (int s = 0; s < N; ++s) {
    if (s + D < N) {
      const int t = s + D;
      a[t % (D + 1)] = frag[((t % MT) * KB + t / MT) * 64 + lane];
    }
    const int kb = s / MT, mt = s % MT;
#pragma unroll
    for (int nb = 0; nb < NB; ++nb)
      acc[nb][mt] = mfma_bf16_32(a[s % (D + 1)], bop(nb, kb), kb == 0 ? zero4() : acc[nb][mt]);
  }
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

// Raises KERN's dynamic-LDS limit to `bytes` (the largest footprint any of
// its launches uses) once per process; thread safe, and every later call
// returns the first call's status.
template <auto KERN>
inline hipError_t set_max_lds_once(size_t bytes) {
  static std::once_flag once;
  static hipError_t err = hipSuccess;
  std::call_once(once, [bytes] {
    err = hipFuncSetAttribute((const void*)KERN, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
  });
  return err;
}

}  // namespace nasg
