// Wave-level MLP layers on MFMA for one block of 16 vertices.
//
// Activations live in the 16x16 accumulator layout: act[mt][i] at lane
// (g, c) is neuron mt*16 + 4g + i of vertex c. Weights are read from LDS in
// the layouts of layout.hpp, so each layer's accumulators feed the next layer
// without any lane exchange (Sec. 4.1: bias-free layers, ReLU between them).
#pragma once

#include "common.hpp"

namespace nasg {

// The encoded input of Tab. "encoding" as the two 16x16x32 B operands of
// layer 0: lane (g, c) holds inputs k = kb*32 + 8g + j (j = 0..7) of vertex
// c. Input k < 57 is one-blob bin k % 19 of position coordinate k / 19: a
// Gaussian of standard deviation 1/19 centred at the coordinate s, evaluated
// at the bin centre (b + 1/2)/19, i.e. exp(-(19 s - b - 1/2)^2 / 2); then
// omega_o (57..59), n (60..62) and the constant one (63). Computed in
// registers from the 9 raw features: 36 bytes per vertex are read, not 256.
struct EncodedInput {
  bf16x8 b[2];
};

__device__ __forceinline__ EncodedInput load_encoded(const float* __restrict__ feat, int64_t ld, int64_t v,
                                                     bool valid, int g) {
  float p[3] = {0.0f, 0.0f, 0.0f}, dn[6] = {0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f};
  if (valid) {
#pragma unroll
    for (int i = 0; i < 3; ++i) p[i] = feat[(int64_t)i * ld + v];
    if (g == 3) {
#pragma unroll
      for (int i = 0; i < 6; ++i) dn[i] = feat[(int64_t)(3 + i) * ld + v];
    }
  }
  constexpr float kHalfLog2e = 0.72134752044448170368f;   // log2(e) / 2
  EncodedInput x;
#pragma unroll
  for (int kb = 0; kb < 2; ++kb)
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      float val;
      if (kb == 1 && j >= 1 && g == 3) {   // k = 57 + (j - 1): omega_o, n, then the one
        val = j == 7 ? 1.0f : dn[j - 1];
      } else {
        const int k = kb * 32 + 8 * g + j;   // < 57
        const int d = (k >= 2 * kBlobBins) ? 2 : (k >= kBlobBins ? 1 : 0);
        const float s = d == 0 ? p[0] : (d == 1 ? p[1] : p[2]);
        const float t = fmaf(s, (float)kBlobBins, -((float)(k - kBlobBins * d) + 0.5f));
        val = __builtin_amdgcn_exp2f(-kHalfLog2e * t * t);
      }
      x.b[kb][j] = (__bf16)(valid ? val : 0.0f);
    }
  return x;
}

template <int H, int K, int PREC, int E = 0>
struct Mlp;

// ---------------------------------------------------------------- BF16 ----
// 16x16x32 bf16 MFMA with FP32 accumulation; layer 0 uses 16x16x16 over the
// 16 padded raw inputs (E = 0) or 16x16x32 over the 64 encoded ones (E = 1).
template <int H, int K, int E>
struct Mlp<H, K, 1, E> {
  static constexpr int MTH = H / 16;     // row tiles of a hidden layer
  static constexpr int MTO = K / 2;      // row tiles of the output layer (8K/16)
  static constexpr int KBH = H / 32;     // 32-wide contraction blocks over a hidden layer
  static constexpr int KBO = K / 4;      // 32-wide contraction blocks over the output (8K/32)
  static constexpr int IN = E ? kInEncoded : kInPadded;   // layer 0's packed input width
  typedef typename std::conditional<E == 1, EncodedInput, bf16x4>::type Input;

  // features 4g..4g+3 of vertex v: p, omega_o, n, then the constant one, then
  // zeros; or the encoded input
  __device__ __forceinline__ static Input load_input(const float* __restrict__ feat, int64_t ld, int64_t v, bool valid, int g) {
    if constexpr (E == 1) return load_encoded(feat, ld, v, valid, g);
    else return load_raw(feat, ld, v, valid, g);
  }
  __device__ __forceinline__ static bf16x4 load_raw(const float* __restrict__ feat, int64_t ld, int64_t v, bool valid, int g) {
    float f[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      int k = 4 * g + j;
      float x = 0.0f;
      if (valid) {
        if (k < kInFeatures) x = feat[(int64_t)k * ld + v];
        else if (k == kInFeatures) x = 1.0f;
      }
      f[j] = x;
    }
    return bf16x4{(__bf16)f[0], (__bf16)f[1], (__bf16)f[2], (__bf16)f[3]};
  }

  // layer 0's input (the values the forward used) into rows 0..IN-1 of a
  // [row][vertex] staging buffer at vertex column wave*16: rows 4g..4g+3, or
  // for the encoded input rows kb*32 + 8g .. + 7
  template <typename S, int SP>
  __device__ __forceinline__ static void stage_input(S* st, const Input& x, int wave, int lane) {
    const int g = lane >> 4, c = lane & 15;
    if constexpr (E == 1) {
#pragma unroll
      for (int kb = 0; kb < 2; ++kb)
#pragma unroll
        for (int j = 0; j < 8; ++j) st[(kb * 32 + 8 * g + j) * SP + wave * 16 + c] = (S)x.b[kb][j];
    } else {
#pragma unroll
      for (int j = 0; j < 4; ++j) st[(4 * g + j) * SP + wave * 16 + c] = (S)x[j];
    }
  }

  __device__ __forceinline__ static bf16x8 operand(const float (&in)[2][4]) {
    bf16x8 b;
#pragma unroll
    for (int j = 0; j < 8; ++j) b[j] = (__bf16)in[j >> 2][j & 3];
    return b;
  }

  // h = relu(W_0 x)
  __device__ __forceinline__ static void layer0(const __bf16* lds, const Input& x, float (&h)[MTH][4], int lane) {
    layer0_linear(lds, x, h, lane);
#pragma unroll
    for (int mt = 0; mt < MTH; ++mt)
#pragma unroll
      for (int i = 0; i < 4; ++i) h[mt][i] = relu(h[mt][i]);
  }

  // Next layer's B operands from a layer's pre-activation accumulators, the
  // ReLU applied to the packed BF16 values (one 16-bit integer max per pair:
  // BF16 keeps the sign bit on top, and rounding never changes a sign, so
  // this equals rounding relu(y)).
  __device__ __forceinline__ static uint32_t relu_pair(float lo, float hi) {
    typedef __attribute__((ext_vector_type(2))) __bf16 bf16x2;
    typedef __attribute__((ext_vector_type(2))) float f32x2;
    typedef __attribute__((ext_vector_type(2))) short s16x2;
    const bf16x2 p = __builtin_convertvector((f32x2){lo, hi}, bf16x2);
    return __builtin_bit_cast(uint32_t, __builtin_elementwise_max(__builtin_bit_cast(s16x2, p), (s16x2)0));
  }
  __device__ __forceinline__ static void relu_operands(const float (&y)[MTH][4], bf16x8 (&b)[KBH]) {
    typedef __attribute__((ext_vector_type(4))) uint32_t u32x4;
#pragma unroll
    for (int kb = 0; kb < KBH; ++kb) {
      const u32x4 w = {relu_pair(y[2 * kb][0], y[2 * kb][1]), relu_pair(y[2 * kb][2], y[2 * kb][3]),
                       relu_pair(y[2 * kb + 1][0], y[2 * kb + 1][1]), relu_pair(y[2 * kb + 1][2], y[2 * kb + 1][3])};
      b[kb] = __builtin_bit_cast(bf16x8, w);
    }
  }

  // W_0 x without the ReLU
  __device__ __forceinline__ static void layer0_linear(const __bf16* lds, const Input& x, float (&y)[MTH][4], int lane) {
#pragma unroll
    for (int mt = 0; mt < MTH; ++mt) {
      f32x4 acc;
      if constexpr (E == 1) {
        const bf16x8* frag = reinterpret_cast<const bf16x8*>(lds);
        acc = mfma_bf16_32(frag[(mt * 2) * 64 + lane], x.b[0], zero4());
        acc = mfma_bf16_32(frag[(mt * 2 + 1) * 64 + lane], x.b[1], acc);
      } else {
        const bf16x4* frag = reinterpret_cast<const bf16x4*>(lds);
        acc = mfma_bf16_16(frag[mt * 64 + lane], x, zero4());
      }
#pragma unroll
      for (int i = 0; i < 4; ++i) y[mt][i] = acc[i];
    }
  }

  // NB vertex blocks at once: each weight fragment read from LDS feeds NB
  // MFMAs, which divides the LDS traffic per FLOP by NB
  template <int NB>
  __device__ __forceinline__ static void layer0_linear_nb(const __bf16* lds, const Input (&x)[NB], float (&y)[NB][MTH][4],
                                          int lane) {
#pragma unroll
    for (int mt = 0; mt < MTH; ++mt) {
      f32x4 acc[NB];
      if constexpr (E == 1) {
        const bf16x8* frag = reinterpret_cast<const bf16x8*>(lds);
        const bf16x8 a0 = frag[(mt * 2) * 64 + lane], a1 = frag[(mt * 2 + 1) * 64 + lane];
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) acc[nb] = mfma_bf16_32(a1, x[nb].b[1], mfma_bf16_32(a0, x[nb].b[0], zero4()));
      } else {
        const bf16x4 a = reinterpret_cast<const bf16x4*>(lds)[mt * 64 + lane];
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) acc[nb] = mfma_bf16_16(a, x[nb], zero4());
      }
#pragma unroll
      for (int nb = 0; nb < NB; ++nb)
#pragma unroll
        for (int i = 0; i < 4; ++i) y[nb][mt][i] = acc[nb][i];
    }
  }
  // out[nb] = W b[nb] over MT row tiles for NB vertex blocks: each A
  // fragment read from LDS feeds NB MFMAs. BM: block-major order with the
  // fragments prefetched (mfma_rows), else row tile by row tile (fewer live
  // registers). Measured on the hidden-128 query: block-major is faster
  // ahead of the NASG epilogue, row-major for the raw forward alone.
  template <int MT, int NB, bool BM>
  __device__ __forceinline__ static void gemm_op_nb(const __bf16* lds, const bf16x8 (&b)[NB][KBH], float (&out)[NB][MT][4],
                                    int lane) {
    if constexpr (BM) {
      f32x4 acc[NB][MT];
      mfma_rows<MT, KBH, NB>(reinterpret_cast<const bf16x8*>(lds), [&](int nb, int kb) { return b[nb][kb]; }, acc,
                             lane);
#pragma unroll
      for (int nb = 0; nb < NB; ++nb)
#pragma unroll
        for (int mt = 0; mt < MT; ++mt)
#pragma unroll
          for (int i = 0; i < 4; ++i) out[nb][mt][i] = acc[nb][mt][i];
    } else {
      const bf16x8* frag = reinterpret_cast<const bf16x8*>(lds);
#pragma unroll
      for (int mt = 0; mt < MT; ++mt) {
        f32x4 acc[NB];
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) acc[nb] = zero4();
#pragma unroll
        for (int kb = 0; kb < KBH; ++kb) {
          const bf16x8 a = frag[(mt * KBH + kb) * 64 + lane];
#pragma unroll
          for (int nb = 0; nb < NB; ++nb) acc[nb] = mfma_bf16_32(a, b[nb][kb], acc[nb]);
        }
#pragma unroll
        for (int nb = 0; nb < NB; ++nb)
#pragma unroll
          for (int i = 0; i < 4; ++i) out[nb][mt][i] = acc[nb][i];
      }
    }
  }

  // out = W in over MT row tiles from ready B operands. BM: block-major
  // with prefetched fragments (mfma_rows), else row tile by row tile, which
  // keeps fewer registers live (block-major raised the spills of the
  // multi-tile hidden-128 group-1 kernel and measured slower there).
  template <int MT, bool BM = false>
  __device__ __forceinline__ static void gemm_op(const __bf16* lds, const bf16x8 (&b)[KBH], float (&out)[MT][4], int lane) {
    if constexpr (BM) {
      f32x4 acc[1][MT];
      mfma_rows<MT, KBH, 1>(reinterpret_cast<const bf16x8*>(lds), [&](int, int kb) { return b[kb]; }, acc, lane);
#pragma unroll
      for (int mt = 0; mt < MT; ++mt)
#pragma unroll
        for (int i = 0; i < 4; ++i) out[mt][i] = acc[0][mt][i];
    } else {
      const bf16x8* frag = reinterpret_cast<const bf16x8*>(lds);
#pragma unroll
      for (int mt = 0; mt < MT; ++mt) {
        f32x4 acc = zero4();
#pragma unroll
        for (int kb = 0; kb < KBH; ++kb) acc = mfma_bf16_32(frag[(mt * KBH + kb) * 64 + lane], b[kb], acc);
#pragma unroll
        for (int i = 0; i < 4; ++i) out[mt][i] = acc[i];
      }
    }
  }

  // out = W in over MT row tiles, W fragments [MT][KBH][64] at `lds`
  template <int MT>
  __device__ __forceinline__ static void gemm(const __bf16* lds, const float (&in)[MTH][4], float (&out)[MT][4], int lane) {
    const bf16x8* frag = reinterpret_cast<const bf16x8*>(lds);
    bf16x8 b[KBH];
#pragma unroll
    for (int kb = 0; kb < KBH; ++kb) {
      float t[2][4];
#pragma unroll
      for (int i = 0; i < 4; ++i) { t[0][i] = in[2 * kb][i]; t[1][i] = in[2 * kb + 1][i]; }
      b[kb] = operand(t);
    }
#pragma unroll
    for (int mt = 0; mt < MT; ++mt) {
      f32x4 acc = zero4();
#pragma unroll
      for (int kb = 0; kb < KBH; ++kb) acc = mfma_bf16_32(frag[(mt * KBH + kb) * 64 + lane], b[kb], acc);
#pragma unroll
      for (int i = 0; i < 4; ++i) out[mt][i] = acc[i];
    }
  }
};

// ---------------------------------------------------------------- FP32 ----
// 16x16x4 f32 MFMA; weights row-major in LDS with an odd pitch.
template <int H, int K, int E>
struct Mlp<H, K, 0, E> {
  static constexpr int MTH = H / 16;
  static constexpr int MTO = K / 2;
  static constexpr int IN = E ? kInEncoded : kInPadded;   // layer 0's packed input width
  static constexpr int KB0 = E ? kInEncoded / 4 : 3;       // 4-wide contraction blocks of layer 0
  // inputs kb*4 + g for kb < KB0
  struct Input { float x[KB0]; };

  // raw: features, then the constant one, then zeros. Encoded (the same
  // inputs as the BF16 network's): one-blob bin k % 19 of position
  // coordinate k / 19 for k < 57, then omega_o, n and the constant one.
  __device__ __forceinline__ static Input load_input(const float* __restrict__ feat, int64_t ld, int64_t v, bool valid, int g) {
    Input in;
    if constexpr (E == 1) {
      float p[3] = {0.0f, 0.0f, 0.0f};
      float wo = 0.0f, nn = 0.0f;
      if (valid) {
#pragma unroll
        for (int i = 0; i < 3; ++i) p[i] = feat[(int64_t)i * ld + v];
        if (g >= 1) wo = feat[(int64_t)(3 + g - 1) * ld + v];   // k = 56 + g: omega_o[g - 1]
        if (g <= 2) nn = feat[(int64_t)(6 + g) * ld + v];       // k = 60 + g: n[g]
      }
      constexpr float kHalfLog2e = 0.72134752044448170368f;   // log2(e) / 2
#pragma unroll
      for (int kb = 0; kb < KB0; ++kb) {
        const int k = kb * 4 + g;
        float val;
        if (kb == 14 && g >= 1) val = wo;
        else if (kb == 15) val = g == 3 ? 1.0f : nn;
        else {
          const int d = (k >= 2 * kBlobBins) ? 2 : (k >= kBlobBins ? 1 : 0);
          const float s = d == 0 ? p[0] : (d == 1 ? p[1] : p[2]);
          const float t = fmaf(s, (float)kBlobBins, -((float)(k - kBlobBins * d) + 0.5f));
          val = __builtin_amdgcn_exp2f(-kHalfLog2e * t * t);
        }
        in.x[kb] = valid ? val : 0.0f;
      }
    } else {
#pragma unroll
      for (int kb = 0; kb < KB0; ++kb) {
        int k = kb * 4 + g;
        float x = 0.0f;
        if (valid) {
          if (k < kInFeatures) x = feat[(int64_t)k * ld + v];
          else if (k == kInFeatures) x = 1.0f;
        }
        in.x[kb] = x;
      }
    }
    return in;
  }

  // layer 0's input into rows 0..IN-1 of a staging buffer: rows kb*4 + g
  // hold this lane's x.x[kb]; for the raw input rows 12..15 are zero padding
  template <typename S, int SP>
  __device__ __forceinline__ static void stage_input(S* st, const Input& x, int wave, int lane) {
    const int g = lane >> 4, c = lane & 15;
#pragma unroll
    for (int kb = 0; kb < KB0; ++kb) st[(kb * 4 + g) * SP + wave * 16 + c] = (S)x.x[kb];
    if constexpr (E == 0) st[(12 + g) * SP + wave * 16 + c] = (S)0.0f;
  }

  __device__ __forceinline__ static void layer0(const float* lds, const Input& x, float (&h)[MTH][4], int lane) {
    const int g = lane >> 4, c = lane & 15;
    constexpr int P = IN + 1;
#pragma unroll
    for (int mt = 0; mt < MTH; ++mt) {
      f32x4 acc = zero4();
#pragma unroll
      for (int kb = 0; kb < KB0; ++kb) acc = mfma_f32_4(lds[(mt * 16 + c) * P + kb * 4 + g], x.x[kb], acc);
#pragma unroll
      for (int i = 0; i < 4; ++i) h[mt][i] = relu(acc[i]);
    }
  }

  // out = W in; W row-major [MT*16][H+1] at `lds`, input neuron of slot (kb, g)
  // is (kb/4)*16 + 4g + kb%4 = accumulator in[kb/4][kb%4] of this lane
  template <int MT>
  __device__ __forceinline__ static void gemm(const float* lds, const float (&in)[MTH][4], float (&out)[MT][4], int lane) {
    const int g = lane >> 4, c = lane & 15;
    constexpr int P = H + 1;
#pragma unroll
    for (int mt = 0; mt < MT; ++mt) {
      f32x4 acc = zero4();
      const float* row = lds + (mt * 16 + c) * P + 4 * g;
#pragma unroll
      for (int kb = 0; kb < 4 * MTH; ++kb) acc = mfma_f32_4(row[(kb >> 2) * 16 + (kb & 3)], in[kb >> 2][kb & 3], acc);
#pragma unroll
      for (int i = 0; i < 4; ++i) out[mt][i] = acc[i];
    }
  }
};

// Forward through all layers; h[l] keeps hidden activations for the backward.
// S = 1: the output layer has one more 16-row tile whose row 0 is the
// selection logit (rows 8K .. 8K+15; the rest are zero padding).
template <int H, int K, int PREC, int NHMAX, int S = 0, int E = 0>
struct Forward {
  typedef Mlp<H, K, PREC, E> M;
  typedef typename std::conditional<PREC == 1, __bf16, float>::type W;
  static constexpr int MTO = M::MTO + S;   // output row tiles

  // offsets (elements) of each layer's forward weights in LDS
  __device__ __forceinline__ static const W* layer_ptr(const W* lds, int l, int nh) {
    if (PREC == 1) {
      Bf16Layout Lt{NetDims{H, nh, K, S, E}};
      return lds + Lt.fwd_off(l);
    } else {
      F32Layout Lt{NetDims{H, nh, K, S, E}};
      return lds + Lt.off(l);
    }
  }

  // h[l] receives hidden layer l's activation for l < nh; `last` the one the
  // output layer reads (h[nh-1]). Layers past nh are skipped with uniform
  // branches; no array is indexed by a runtime value.
  __device__ __forceinline__ static void run(const W* lds, int nh, const typename M::Input& x,
                             float (&h)[NHMAX][M::MTH][4], float (&last)[M::MTH][4],
                             float (&out)[MTO][4], int lane) {
    M::layer0(layer_ptr(lds, 0, nh), x, h[0], lane);
#pragma unroll
    for (int mt = 0; mt < M::MTH; ++mt)
#pragma unroll
      for (int i = 0; i < 4; ++i) last[mt][i] = h[0][mt][i];
#pragma unroll
    for (int l = 1; l < NHMAX; ++l) {
      if (l < nh) {
        float y[M::MTH][4];
        M::template gemm<M::MTH>(layer_ptr(lds, l, nh), last, y, lane);
#pragma unroll
        for (int mt = 0; mt < M::MTH; ++mt)
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            h[l][mt][i] = relu(y[mt][i]);
            last[mt][i] = h[l][mt][i];
          }
      }
    }
    M::template gemm<MTO>(layer_ptr(lds, nh, nh), last, out, lane);
  }

  // BF16 forward keeping the hidden activations packed: hw[l] receives layer
  // l's ReLU outputs as BF16 pairs (word k of row tile mt: rows mt*16 + 4g +
  // 2k, + 1 of vertex c, low half first), exactly the operands the next layer
  // read; lastw the pairs the output layer reads (hw[nh-1]). Same values as
  // run() rounded to BF16.
  __device__ __forceinline__ static void run_packed(const W* lds, int nh, const typename M::Input& x,
                                                    uint32_t (&hw)[NHMAX][M::MTH][2], uint32_t (&lastw)[M::MTH][2],
                                                    float (&out)[MTO][4], int lane) {
    static_assert(PREC == 1, "BF16 only");
    typedef __attribute__((ext_vector_type(4))) uint32_t u32x4_;
    float y[M::MTH][4];
    bf16x8 b[M::KBH];
    auto keep = [&](uint32_t (&w)[M::MTH][2]) {
#pragma unroll
      for (int kb = 0; kb < M::KBH; ++kb) {
        const u32x4_ q = __builtin_bit_cast(u32x4_, b[kb]);
        w[2 * kb][0] = q[0]; w[2 * kb][1] = q[1]; w[2 * kb + 1][0] = q[2]; w[2 * kb + 1][1] = q[3];
      }
    };
    M::layer0_linear(layer_ptr(lds, 0, nh), x, y, lane);
    M::relu_operands(y, b);
    keep(hw[0]);
#pragma unroll
    for (int l = 1; l < NHMAX; ++l) {
      if (l < nh) {
        M::template gemm_op<M::MTH>(layer_ptr(lds, l, nh), b, y, lane);
        M::relu_operands(y, b);
        keep(hw[l]);
      }
    }
    keep(lastw);
    M::template gemm_op<MTO>(layer_ptr(lds, nh, nh), b, out, lane);
  }

  // BF16 query forward of NB vertex blocks sharing every weight fragment read
  template <int NB, bool BM>
  __device__ __forceinline__ static void run_query_nb(const W* lds, int nh, const typename M::Input (&x)[NB],
                                      float (&out)[NB][MTO][4], int lane) {
    static_assert(PREC == 1, "BF16 only");
    float y[NB][M::MTH][4];
    bf16x8 b[NB][M::KBH];
    M::template layer0_linear_nb<NB>(layer_ptr(lds, 0, nh), x, y, lane);
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) M::relu_operands(y[nb], b[nb]);
#pragma unroll
    for (int l = 1; l < NHMAX; ++l) {
      if (l < nh) {
        M::template gemm_op_nb<M::MTH, NB, BM>(layer_ptr(lds, l, nh), b, y, lane);
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) M::relu_operands(y[nb], b[nb]);
      }
    }
    M::template gemm_op_nb<MTO, NB, BM>(layer_ptr(lds, nh, nh), b, out, lane);
  }

  // Forward for queries (no activations kept): in BF16 the layers pass
  // packed, ReLU'd B operands; the same values as run().
  __device__ __forceinline__ static void run_query(const W* lds, int nh, const typename M::Input& x, float (&out)[MTO][4],
                                   int lane) {
    if constexpr (PREC == 1) {
      float y[M::MTH][4];
      bf16x8 b[M::KBH];
      M::layer0_linear(layer_ptr(lds, 0, nh), x, y, lane);
      M::relu_operands(y, b);
#pragma unroll
      for (int l = 1; l < NHMAX; ++l) {
        if (l < nh) {
          M::template gemm_op<M::MTH>(layer_ptr(lds, l, nh), b, y, lane);
          M::relu_operands(y, b);
        }
      }
      M::template gemm_op<MTO>(layer_ptr(lds, nh, nh), b, out, lane);
    } else {
      float h[NHMAX][M::MTH][4];
      float last[M::MTH][4];
      run(lds, nh, x, h, last, out, lane);
    }
  }
};

}  // namespace nasg
