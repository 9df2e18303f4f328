// MLP backward pieces shared by the training kernels: dgrad in registers,
// staging of a layer's deltas and inputs for the weight gradient, the
// weight-gradient MFMA over a workgroup's staged vertices, and the flush of a
// wave's gradient tiles to its workgroup's partial.
//
// dW_l = sum_v delta_l(v) h_{l-1}(v)^T contracts over vertices, which sit in
// different lanes of the accumulator layout, so the four waves of a
// workgroup stage delta_l and h_{l-1} of its 64 vertices in LDS, and each
// wave accumulates its own row tiles of dW_l.
#pragma once

#include "common.hpp"

namespace nasg {

constexpr int kWGV = 64;   // vertices per workgroup tile

// delta_prev = W_l^T delta (contraction over the RT*16 rows of layer l),
// rows of the result are the previous layer's neurons in accumulator layout.
template <int H, int K, int PREC, int RT>
__device__ __forceinline__ void dgrad(const void* wl, const float (&dl)[RT][4],
                                      float (&dp)[H / 16][4], int lane) {
  constexpr int MTP = H / 16;
  if constexpr (PREC == 1) {
    constexpr int KB = RT / 2;   // 32-wide blocks over the rows of layer l
    const bf16x8* frag = reinterpret_cast<const bf16x8*>(wl);
    bf16x8 b[KB];
#pragma unroll
    for (int kb = 0; kb < KB; ++kb)
#pragma unroll
      for (int j = 0; j < 8; ++j) b[kb][j] = (__bf16)dl[2 * kb + (j >> 2)][j & 3];
    // an odd last row tile (the selection tile) contracts with 16x16x16
    // fragments stored after the 32-wide ones: lane (g, c) holds its rows
    // 4g .. 4g+3, which are this lane's accumulators dl[RT-1][0..3]. Its
    // product has an accumulator of its own, added with VALU: chaining a
    // 16x16x16 MFMA onto a 16x16x32 accumulator gave non-reproducible
    // results with this toolchain.
    const bf16x4* frag_s = reinterpret_cast<const bf16x4*>(frag + MTP * KB * 64);
    bf16x4 bs;
    if constexpr (RT % 2 == 1) {
#pragma unroll
      for (int j = 0; j < 4; ++j) bs[j] = (__bf16)dl[RT - 1][j];
    }
    // block-major with prefetched fragments (mfma_rows): the chains of the
    // MTP row tiles interleave instead of waiting on each other
    f32x4 acc[1][MTP];
    mfma_rows<MTP, KB, 1>(frag, [&](int, int kb) { return b[kb]; }, acc, lane);
#pragma unroll
    for (int mt = 0; mt < MTP; ++mt) {
      if constexpr (RT % 2 == 1) {
        const f32x4 sel = mfma_bf16_16(frag_s[mt * 64 + lane], bs, zero4());
#pragma unroll
        for (int i = 0; i < 4; ++i) acc[0][mt][i] += sel[i];
      }
#pragma unroll
      for (int i = 0; i < 4; ++i) dp[mt][i] = acc[0][mt][i];
    }
  } else {
    const float* W = reinterpret_cast<const float*>(wl);
    constexpr int P = H + 1;
    const int g = lane >> 4, c = lane & 15;
#pragma unroll
    for (int mt = 0; mt < MTP; ++mt) {
      f32x4 acc = zero4();
#pragma unroll
      for (int kb = 0; kb < 4 * RT; ++kb) {
        // row R of layer l fed by slot (kb, g): accumulator dl[kb/4][kb%4]
        const int R = (kb >> 2) * 16 + 4 * g + (kb & 3);
        acc = mfma_f32_4(W[R * P + mt * 16 + c], dl[kb >> 2][kb & 3], acc);
      }
#pragma unroll
      for (int i = 0; i < 4; ++i) dp[mt][i] = acc[i];
    }
  }
}

// One row tile of BF16 staging, [row][vertex] at `tile` (its row 0, the
// wave's vertex column 0): lane (g, c) holds rows 4g..4g+3 of vertex c as
// two packed words, w0 (rows 4g, 4g+1) and w1 (rows 4g+2, 4g+3). Lanes c and
// c^1 (neighbouring vertices) swap half of them through one DPP move, so
// each writes two rows of both vertices as two 4-byte stores (the even lane
// rows 4g, 4g+1, the odd lane rows 4g+2, 4g+3; one ds_write2_b32) instead
// of four 2-byte stores.
template <int SP>
__device__ __forceinline__ void stage_tile_bf16(__bf16* tile, uint32_t w0, uint32_t w1, int g, int c) {
  const bool odd = c & 1;
  const uint32_t send = odd ? w0 : w1;   // the rows the partner writes
  const uint32_t mine = odd ? w1 : w0;
  // quad_perm [1, 0, 3, 2]: the value of lane c^1
  const uint32_t recv = (uint32_t)__builtin_amdgcn_mov_dpp((int)send, 0xB1, 0xF, 0xF, false);
  // v_perm_b32 byte selectors over (recv: bytes 4..7, mine: bytes 0..3):
  // even lane (recv = vertex c+1) [mine.lo, recv.lo], [mine.hi, recv.hi];
  // odd lane (recv = vertex c-1) [recv.lo, mine.lo], [recv.hi, mine.hi]
  __bf16* const p = tile + (4 * g + (odd ? 2 : 0)) * SP + (c & ~1);
  *reinterpret_cast<uint32_t*>(p) = __builtin_amdgcn_perm(recv, mine, odd ? 0x01000504u : 0x05040100u);
  *reinterpret_cast<uint32_t*>(p + SP) = __builtin_amdgcn_perm(recv, mine, odd ? 0x03020706u : 0x07060302u);
}

// Write a wave's accumulator-layout block [RT*16 rows][16 vertices] into the
// staging buffer at vertex column wave*16 (BF16 through stage_tile_bf16).
template <typename S, int RT, int SP>
__device__ __forceinline__ void stage_rows(S* buf, const float (&x)[RT][4], int wave, int lane) {
  const int g = lane >> 4, c = lane & 15;
  if constexpr (sizeof(S) == 2) {
    typedef __attribute__((ext_vector_type(2))) __bf16 bf16x2;
    typedef __attribute__((ext_vector_type(2))) float f32x2;
#pragma unroll
    for (int mt = 0; mt < RT; ++mt) {
      const uint32_t w0 = __builtin_bit_cast(uint32_t, __builtin_convertvector((f32x2){x[mt][0], x[mt][1]}, bf16x2));
      const uint32_t w1 = __builtin_bit_cast(uint32_t, __builtin_convertvector((f32x2){x[mt][2], x[mt][3]}, bf16x2));
      stage_tile_bf16<SP>(reinterpret_cast<__bf16*>(buf) + mt * 16 * SP + wave * 16, w0, w1, g, c);
    }
  } else {
#pragma unroll
    for (int mt = 0; mt < RT; ++mt)
#pragma unroll
      for (int i = 0; i < 4; ++i) buf[(mt * 16 + 4 * g + i) * SP + wave * 16 + c] = (S)x[mt][i];
  }
}

// BF16 rows of a block packed in pairs (as the MFMA operands hold them):
// w[mt][0] = rows mt*16 + 4g, + 4g + 1 and w[mt][1] = rows + 4g + 2, + 4g + 3
// of vertex c, low half first; rounded to nearest even.
template <int RT>
__device__ __forceinline__ void pack_rows(const float (&x)[RT][4], uint32_t (&w)[RT][2]) {
  typedef __attribute__((ext_vector_type(2))) __bf16 bf16x2;
  typedef __attribute__((ext_vector_type(2))) float f32x2;
#pragma unroll
  for (int mt = 0; mt < RT; ++mt)
#pragma unroll
    for (int k = 0; k < 2; ++k)
      w[mt][k] = __builtin_bit_cast(uint32_t, __builtin_convertvector((f32x2){x[mt][2 * k], x[mt][2 * k + 1]}, bf16x2));
}

// d *= (h != 0) per BF16 half: the ReLU derivative, h being packed ReLU
// outputs (non-negative, so min(h, 1) as a 16-bit integer is the indicator)
template <int RT>
__device__ __forceinline__ void mask_rows(uint32_t (&d)[RT][2], const uint32_t (&h)[RT][2]) {
  typedef __attribute__((ext_vector_type(2))) unsigned short u16x2;
#pragma unroll
  for (int mt = 0; mt < RT; ++mt)
#pragma unroll
    for (int k = 0; k < 2; ++k) {
      const u16x2 ind = __builtin_elementwise_min(__builtin_bit_cast(u16x2, h[mt][k]), (u16x2)1);
      d[mt][k] = __builtin_bit_cast(uint32_t, __builtin_bit_cast(u16x2, d[mt][k]) * ind);
    }
}

// Packed rows into the staging buffer at vertex column wave*16.
template <int RT, int SP>
__device__ __forceinline__ void stage_words(__bf16* buf, const uint32_t (&w)[RT][2], int wave, int lane) {
  const int g = lane >> 4, c = lane & 15;
#pragma unroll
  for (int mt = 0; mt < RT; ++mt) stage_tile_bf16<SP>(buf + mt * 16 * SP + wave * 16, w[mt][0], w[mt][1], g, c);
}

// dgrad (BF16) with the deltas already packed: the packed words are the B
// operands as they are (an even number of row tiles, no selection tile).
template <int H, int RT>
__device__ __forceinline__ void dgrad_words(const void* wl, const uint32_t (&dw)[RT][2], float (&dp)[H / 16][4],
                                            int lane) {
  static_assert(RT % 2 == 0, "whole 32-wide blocks");
  constexpr int MTP = H / 16, KB = RT / 2;
  typedef __attribute__((ext_vector_type(4))) uint32_t u32x4_;
  bf16x8 b[KB];
#pragma unroll
  for (int kb = 0; kb < KB; ++kb)
    b[kb] = __builtin_bit_cast(bf16x8, u32x4_{dw[2 * kb][0], dw[2 * kb][1], dw[2 * kb + 1][0], dw[2 * kb + 1][1]});
  f32x4 acc[1][MTP];
  mfma_rows<MTP, KB, 1>(reinterpret_cast<const bf16x8*>(wl), [&](int, int kb) { return b[kb]; }, acc, lane);
#pragma unroll
  for (int mt = 0; mt < MTP; ++mt)
#pragma unroll
    for (int i = 0; i < 4; ++i) dp[mt][i] = acc[0][mt][i];
}

// acc[rt][ct] += D[rows rt*16..][v] * Hs[cols ct*16..][v]^T over the NV staged vertices
template <int PREC, typename S, int SP, int NR, int NC, int NV = kWGV>
__device__ __forceinline__ void wgrad_tiles(const S* dst, const S* hst, const int (&rt)[NR], int nrt,
                                            f32x4 (&acc)[NR][NC], int lane) {
  const int g = lane >> 4, c = lane & 15;
  if constexpr (PREC == 1) {
#pragma unroll
    for (int vb = 0; vb < NV / 32; ++vb) {
      bf16x8 hb[NC];
#pragma unroll
      for (int ct = 0; ct < NC; ++ct)
        hb[ct] = *reinterpret_cast<const bf16x8*>(hst + (ct * 16 + c) * SP + vb * 32 + 8 * g);
#pragma unroll
      for (int r = 0; r < NR; ++r) {
        if (r < nrt) {
          bf16x8 da = *reinterpret_cast<const bf16x8*>(dst + (rt[r] * 16 + c) * SP + vb * 32 + 8 * g);
#pragma unroll
          for (int ct = 0; ct < NC; ++ct) acc[r][ct] = mfma_bf16_32(da, hb[ct], acc[r][ct]);
        }
      }
    }
  } else {
#pragma unroll
    for (int vb = 0; vb < NV / 4; ++vb) {
      float hb[NC];
#pragma unroll
      for (int ct = 0; ct < NC; ++ct) hb[ct] = hst[(ct * 16 + c) * SP + vb * 4 + g];
#pragma unroll
      for (int r = 0; r < NR; ++r) {
        if (r < nrt) {
          float da = dst[(rt[r] * 16 + c) * SP + vb * 4 + g];
#pragma unroll
          for (int ct = 0; ct < NC; ++ct) acc[r][ct] = mfma_f32_4(da, hb[ct], acc[r][ct]);
        }
      }
    }
  }
}

// Ownership of a layer's dW tiles (RT row tiles x CT column tiles) among the
// NW waves of a workgroup, tile j of a wave being (rt(w, j), ct(w, j)):
// * RT a multiple of NW (row mode): wave w owns row tiles w, w + NW, ... and
//   every column tile (per staged block: CT column operands, one row operand
//   per row tile);
// * otherwise (column mode, NW a multiple of CT): wave w owns column tile
//   w % CT and row tiles w / CT + (NW / CT) j below RT (one column operand,
//   one row operand per tile), so that an odd row tile (the selection
//   output's) adds one tile to some waves rather than CT to one.
template <int RT, int CT, int NW>
struct Own {
  static constexpr bool ROW = RT >= NW && RT % NW == 0;
  static_assert(ROW || NW % CT == 0, "waves must split evenly over the column tiles");
  static constexpr int STEP = ROW ? NW : NW / CT;
  static constexpr int NRW = (RT + STEP - 1) / STEP;        // row tiles per wave
  static constexpr int TPW = ROW ? NRW * CT : NRW;          // tiles per wave
  __device__ __forceinline__ static int rt(int wave, int j) { return ROW ? wave + NW * (j / CT) : wave / CT + STEP * j; }
  __device__ __forceinline__ static int ct(int wave, int j) { return ROW ? j % CT : wave % CT; }
};

template <int PREC, typename S, int SP>
__device__ __forceinline__ auto stage_operand(const S* st, int row, int vb, int g, int c) {
  if constexpr (PREC == 1) return *reinterpret_cast<const bf16x8*>(st + (row * 16 + c) * SP + vb * 32 + 8 * g);
  else return st[(row * 16 + c) * SP + vb * 4 + g];
}

// acc[j] += D[rows of rt(j)][v] * Hs[cols of ct(j)][v]^T over NV staged vertices
template <int PREC, typename S, int SP, int RT, int CT, int NW, int NV>
__device__ __forceinline__ void wgrad_own(const S* dst, const S* hst, f32x4 (&acc)[Own<RT, CT, NW>::TPW],
                                          int wave, int lane) {
  typedef Own<RT, CT, NW> O;
  typedef decltype(stage_operand<PREC, S, SP>(dst, 0, 0, 0, 0)) Op;
  const int g = lane >> 4, c = lane & 15;
  constexpr int VB = PREC == 1 ? NV / 32 : NV / 4;
  if constexpr (PREC == 1) {
    // BF16: the operands of vertex block vb + 1 are read while block vb is
    // multiplied (two register sets), so the LDS latency overlaps the MFMAs
    constexpr int NH_ = O::ROW ? CT : 1, ND = O::ROW ? O::NRW : O::TPW;
    struct Ops { Op h[NH_]; Op d[ND]; };
    auto load = [&](int vb, Ops& o) {
      if constexpr (O::ROW) {
#pragma unroll
        for (int ct = 0; ct < CT; ++ct) o.h[ct] = stage_operand<PREC, S, SP>(hst, ct, vb, g, c);
#pragma unroll
        for (int r = 0; r < O::NRW; ++r)
          if (O::rt(wave, r * CT) < RT) o.d[r] = stage_operand<PREC, S, SP>(dst, O::rt(wave, r * CT), vb, g, c);
      } else {
        o.h[0] = stage_operand<PREC, S, SP>(hst, O::ct(wave, 0), vb, g, c);
#pragma unroll
        for (int j = 0; j < O::TPW; ++j)
          if (O::rt(wave, j) < RT) o.d[j] = stage_operand<PREC, S, SP>(dst, O::rt(wave, j), vb, g, c);
      }
    };
    Ops ops[2];
    load(0, ops[0]);
#pragma unroll
    for (int vb = 0; vb < VB; ++vb) {
      if (vb + 1 < VB) load(vb + 1, ops[(vb + 1) & 1]);
      const Ops& o = ops[vb & 1];
      if constexpr (O::ROW) {
#pragma unroll
        for (int r = 0; r < O::NRW; ++r)
          if (O::rt(wave, r * CT) < RT)
#pragma unroll
            for (int ct = 0; ct < CT; ++ct) acc[r * CT + ct] = mfma_bf16_32(o.d[r], o.h[ct], acc[r * CT + ct]);
      } else {
#pragma unroll
        for (int j = 0; j < O::TPW; ++j)
          if (O::rt(wave, j) < RT) acc[j] = mfma_bf16_32(o.d[j], o.h[0], acc[j]);
      }
    }
    return;
  }
#pragma unroll
  for (int vb = 0; vb < VB; ++vb) {
    if constexpr (O::ROW) {
      Op hb[CT];
#pragma unroll
      for (int ct = 0; ct < CT; ++ct) hb[ct] = stage_operand<PREC, S, SP>(hst, ct, vb, g, c);
#pragma unroll
      for (int r = 0; r < O::NRW; ++r) {
        if (O::rt(wave, r * CT) < RT) {
          const Op da = stage_operand<PREC, S, SP>(dst, O::rt(wave, r * CT), vb, g, c);
#pragma unroll
          for (int ct = 0; ct < CT; ++ct) {
            if constexpr (PREC == 1) acc[r * CT + ct] = mfma_bf16_32(da, hb[ct], acc[r * CT + ct]);
            else acc[r * CT + ct] = mfma_f32_4(da, hb[ct], acc[r * CT + ct]);
          }
        }
      }
    } else {
      const Op hb = stage_operand<PREC, S, SP>(hst, O::ct(wave, 0), vb, g, c);
#pragma unroll
      for (int j = 0; j < O::TPW; ++j) {
        if (O::rt(wave, j) < RT) {
          const Op da = stage_operand<PREC, S, SP>(dst, O::rt(wave, j), vb, g, c);
          if constexpr (PREC == 1) acc[j] = mfma_bf16_32(da, hb, acc[j]);
          else acc[j] = mfma_f32_4(da, hb, acc[j]);
        }
      }
    }
  }
}

// Flush a wave's owned dW tiles of layer l to the workgroup's canonical partial.
template <int RT, int CT, int NW>
__device__ __forceinline__ void flush_own(float* part, const NetDims& d, int l,
                                          const f32x4 (&acc)[Own<RT, CT, NW>::TPW], int wave, int lane) {
  typedef Own<RT, CT, NW> O;
  const int g = lane >> 4, c = lane & 15;
  const int cols = d.cols(l);
  const int64_t off = d.canon_off(l);
#pragma unroll
  for (int j = 0; j < O::TPW; ++j) {
    const int k = O::ct(wave, j) * 16 + c;
    if (O::rt(wave, j) >= RT || k >= cols) continue;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int R = O::rt(wave, j) * 16 + 4 * g + i;
      const int n = (l == d.NH) ? canon_out_row(R, d.K) : R;
      if (n >= 0) part[off + (int64_t)n * cols + k] = acc[j][i];   // n < 0: padding rows
    }
  }
}

// Flush a wave's dW tiles of layer l to the workgroup's canonical partial.
// PAD: the tiles may hold the selection tile's padding rows (skipped).
template <int NR, int NC, bool PAD = false>
__device__ __forceinline__ void flush_tiles(float* part, const NetDims& d, int l, const int (&rt)[NR], int nrt,
                                            const f32x4 (&acc)[NR][NC], int lane) {
  const int g = lane >> 4, c = lane & 15;
  const int cols = d.cols(l);
  const int64_t off = d.canon_off(l);
#pragma unroll
  for (int r = 0; r < NR; ++r) {
    if (r >= nrt) continue;
#pragma unroll
    for (int ct = 0; ct < NC; ++ct) {
      const int k = ct * 16 + c;
      if (k >= cols) continue;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int R = rt[r] * 16 + 4 * g + i;
        const int n = (l == d.NH) ? canon_out_row(R, d.K) : R;
        if (!PAD || n >= 0) part[off + (int64_t)n * cols + k] = acc[r][ct][i];   // n < 0: padding rows
      }
    }
  }
}

}  // namespace nasg
