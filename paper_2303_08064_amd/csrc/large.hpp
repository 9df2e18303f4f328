// Hidden-128 networks (four hidden layers): the query and training kernels
// and their launchers, instantiated by large.hip (K = 32 lobes on the 9 raw
// features, BF16 and FP32) and large_paper.hip (the paper's default network,
// Sec. 4.1, Sec. 6: 128 units, K = 8, the selection output, the encoded input
// of Tab. "encoding", BF16 and FP32).
//
// The K = 32 network's forward weights alone (164 KiB in BF16) exceed one
// CU's 160 KiB of LDS, and its 83,200 FP32 weight-gradient accumulators would
// need ~325 registers per lane in each of four waves. So:
// * weights stream through LDS while the workgroup moves through the layers
//   together (64 vertices per tile). BF16: two 32 KiB buffers in a pipeline;
//   each stage is one layer of MFMA fragments (a K = 32 output layer in two
//   halves), and while the waves compute from one buffer the next stage
//   arrives in the other by asynchronous direct-to-LDS loads. FP32 (the
//   comparison path): one buffer, 64 rows (33 KiB) at a time.
// * training runs as two backward kernels over the batch (FP32: three, a
//   gradient kernel first): one evaluates the weighted-NLL / NASG backward
//   (Sec. 4.2) and keeps only dL/d(raw outputs) (the operand image the other
//   reads: 512 B per sample in BF16, 1 KiB in FP32 at K = 32); each backward
//   kernel recomputes the forward, runs dgrad and accumulates the weight
//   gradient of one group of layers (group 0: the output and last hidden
//   layer; group 1: the rest) in registers. Activations are recomputed,
//   never stored.
#pragma once

#include <type_traits>

#include "backward.hpp"
#include "epilogue.hpp"
#include "kernels.hpp"
#include "mlp.hpp"

namespace nasg {

// ------------------------------------------------------------------ BF16 ----
// RT*16 rows of one 16-vertex block in the accumulator layout as BF16 pairs:
// p[mt][k] holds rows mt*16 + 4g + 2k (low half) and + 1 (high half) of
// vertex c at lane (g, c). Four consecutive words are exactly one 32-wide
// MFMA B operand, so hidden activations, deltas and the raw-output gradient
// move between layers, masks and LDS staging without conversions.
typedef __attribute__((ext_vector_type(4))) uint32_t u32x4;

template <int RT>
struct Pk {
  uint32_t p[RT][2];
  __device__ __forceinline__ void from_ops(const bf16x8 (&b)[RT / 2]) {
#pragma unroll
    for (int kb = 0; kb < RT / 2; ++kb) {
      const u32x4 w = __builtin_bit_cast(u32x4, b[kb]);
      p[2 * kb][0] = w[0]; p[2 * kb][1] = w[1]; p[2 * kb + 1][0] = w[2]; p[2 * kb + 1][1] = w[3];
    }
  }
  // the selection tile (an odd last tile) from its 16x16x16 B operand
  __device__ __forceinline__ void set_last(const bf16x4& b) {
    typedef __attribute__((ext_vector_type(2))) uint32_t u32x2;
    const u32x2 w = __builtin_bit_cast(u32x2, b);
    p[RT - 1][0] = w[0];
    p[RT - 1][1] = w[1];
  }
  __device__ __forceinline__ void ops(bf16x8 (&b)[RT / 2]) const {
#pragma unroll
    for (int kb = 0; kb < RT / 2; ++kb)
      b[kb] = __builtin_bit_cast(bf16x8, u32x4{p[2 * kb][0], p[2 * kb][1], p[2 * kb + 1][0], p[2 * kb + 1][1]});
  }
  // bf16(d) where the activation h of the same row is > 0, else 0 (the ReLU
  // derivative). h holds ReLU outputs, so its halves are non-negative
  // integers: min(h, 1) is the 0/1 indicator and a 16-bit multiply applies it.
  __device__ __forceinline__ void masked(const float (&d)[RT][4], const Pk& h) {
    typedef __attribute__((ext_vector_type(2))) __bf16 bf16x2;
    typedef __attribute__((ext_vector_type(2))) float f32x2;
    typedef __attribute__((ext_vector_type(2))) unsigned short u16x2;
#pragma unroll
    for (int mt = 0; mt < RT; ++mt)
#pragma unroll
      for (int k = 0; k < 2; ++k) {
        const bf16x2 v = __builtin_convertvector((f32x2){d[mt][2 * k], d[mt][2 * k + 1]}, bf16x2);
        const u16x2 ind = __builtin_elementwise_min(__builtin_bit_cast(u16x2, h.p[mt][k]), (u16x2)1);
        p[mt][k] = __builtin_bit_cast(uint32_t, __builtin_bit_cast(u16x2, v) * ind);
      }
  }
  // write row tiles [MT0, MT0 + NMT) of the block into a [row][vertex]
  // staging buffer (as its rows 0 ..) at vertex column wave*16
  template <int SP, int MT0 = 0, int NMT = RT>
  __device__ __forceinline__ void stage(__bf16* buf, int wave, int lane) const {
    const int g = lane >> 4, c = lane & 15;
#pragma unroll
    for (int mt = 0; mt < NMT; ++mt)
      stage_tile_bf16<SP>(buf + mt * 16 * SP + wave * 16, p[MT0 + mt][0], p[MT0 + mt][1], g, c);
  }
};

constexpr int cmax(int a, int b) { return a > b ? a : b; }

// dp[MT0 .. MT0+NMT) of W^T dl from backward fragments [NMT][KB][64] at buf;
// b holds dl as B operands. BM: block-major with prefetched fragments
// (mfma_rows), else row tile by row tile.
template <int KB, int NMT, int MT0, bool BM, int MTP>
__device__ __forceinline__ void dgrad_rows(const __bf16* buf, const bf16x8 (&b)[KB], float (&dp)[MTP][4],
                                           int lane) {
  if constexpr (BM) {
    f32x4 acc[1][NMT];
    mfma_rows<NMT, KB, 1>(reinterpret_cast<const bf16x8*>(buf), [&](int, int kb) { return b[kb]; }, acc, lane);
#pragma unroll
    for (int mt = 0; mt < NMT; ++mt)
#pragma unroll
      for (int i = 0; i < 4; ++i) dp[MT0 + mt][i] = acc[0][mt][i];
  } else {
    const bf16x8* frag = reinterpret_cast<const bf16x8*>(buf);
#pragma unroll
    for (int mt = 0; mt < NMT; ++mt) {
      f32x4 acc = zero4();
#pragma unroll
      for (int kb = 0; kb < KB; ++kb) acc = mfma_bf16_32(frag[(mt * KB + kb) * 64 + lane], b[kb], acc);
#pragma unroll
      for (int i = 0; i < 4; ++i) dp[MT0 + mt][i] = acc[i];
    }
  }
}

// dp += W_sel^T dl_sel for the selection tile: 16x16x16 A operands [MTP][64]
// at buf, bs = the tile's deltas as the B operand. Its own accumulator, added
// with VALU (chaining a 16x16x16 MFMA onto a 16x16x32 accumulator gave
// non-reproducible results with this toolchain).
template <int MTP>
__device__ __forceinline__ void dgrad_sel(const __bf16* buf, const bf16x4& bs, float (&dp)[MTP][4], int lane) {
  const bf16x4* frag = reinterpret_cast<const bf16x4*>(buf);
#pragma unroll
  for (int mt = 0; mt < MTP; ++mt) {
    const f32x4 sel = mfma_bf16_16(frag[mt * 64 + lane], bs, zero4());
#pragma unroll
    for (int i = 0; i < 4; ++i) dp[mt][i] += sel[i];
  }
}

// Stage order of one tile's forward: layer 0, hidden layers 1..NH-1, then the
// output layer in NOUT stages (two halves of its row tiles when its
// fragments exceed a buffer); stage s computes from buffer s % 2 while stage
// s + 1 is copied into the other. The functions take the buffer pointers by
// reference and swap them where a layer ends on the other parity, so that
// "resident in b0" always names the buffer the next stage computes from.
// SEL = 1: one more output tile, the selection logit (row 8K); ENC = 1:
// layer 0 reads the encoded input; BM_: the layers' MFMAs in block-major
// order with prefetched fragments (for kernels with registers to spare).
template <int H, int K, int SEL = 0, int ENC = 0, bool BM_ = false>
struct NetBf16 {
  typedef Mlp<H, K, 1, ENC> M;
  static constexpr bool BM = BM_;
  typedef __bf16 W;
  static constexpr int NH = 4;
  static constexpr int MTH = H / 16, MTO = K / 2 + SEL, KQ = K / 4;
  static constexpr int KBO = K / 4;                        // 32-wide blocks over the 8K lobe rows
  static constexpr int L0 = H * M::IN;                     // layer 0's forward fragments (elements)
  static constexpr int OUT = MTO * 16 * H;                 // the output layer's forward fragments
  static constexpr int OB = 8 * K * H + SEL * 16 * H;      // its backward fragments (+ the selection tile's)
  static constexpr int NOUT = OUT > H * H ? 2 : 1;         // stages of the output layer
  static constexpr int HALF_O = MTO / 2;
  static constexpr int OUT_STAGE = OUT / NOUT, OB_STAGE = OB / NOUT;
  static constexpr int BUF = cmax(cmax(H * H, L0), cmax(OUT_STAGE, OB_STAGE));   // elements per buffer
  static constexpr int SP = kWGV + 8;                      // staging pitch (bf16)
  static constexpr int RMAX = 8 * K;
  static_assert(NH % 2 == 0, "buffer parity assumes an even number of hidden layers");
  static_assert(NOUT == 1 || (SEL == 0 && MTO % 2 == 0 && MTH % 2 == 0), "a two-stage output layer splits evenly");
  static_assert(BUF * 2 <= 16384 * 2, "two 32 KiB weight buffers");

  __device__ __forceinline__ static Bf16Layout layout() { return Bf16Layout{NetDims{H, NH, K, SEL, ENC}}; }
  __device__ __forceinline__ static void dma(W* dst, const W* src, int elems) { lds_dma(dst, src, elems * 2); }
  __device__ __forceinline__ static void sync_stage() {
    lds_dma_wait();
    __syncthreads();
  }
  __device__ __forceinline__ static void swap(W*& a, W*& b) {
    W* t = a;
    a = b;
    b = t;
  }
  // Layer 0 into b0, awaited: the first tile of a workgroup.
  __device__ __forceinline__ static void begin(const W* wg, W* b0) {
    dma(b0, wg + layout().fwd_off(0), L0);
    sync_stage();
  }

  // Hidden layers of one tile with layer 0 resident in b0: hp[l] receives
  // hidden layer l's activations as B operands; `next` (elems) is resident
  // in b0 on return (a full forward puts the output layer's first stage there).
  __device__ __forceinline__ static void hidden(const W* wg, W*& b0, W*& b1, const typename M::Input& x, Pk<MTH> (&hp)[NH],
                                const W* next, int next_elems, int lane) {
    const Bf16Layout Lt = layout();
    float y[MTH][4];
    bf16x8 b[M::KBH];
    dma(b1, wg + Lt.fwd_off(1), H * H);
    M::layer0_linear(b0, x, y, lane);
    M::relu_operands(y, b);
    hp[0].from_ops(b);
    sync_stage();
#pragma unroll
    for (int l = 1; l < NH; ++l) {
      W* cur = (l & 1) ? b1 : b0;
      W* oth = (l & 1) ? b0 : b1;
      if (l + 1 < NH) dma(oth, wg + Lt.fwd_off(l + 1), H * H);
      else dma(oth, next, next_elems);
      M::template gemm_op<MTH, BM>(cur, b, y, lane);
      M::relu_operands(y, b);
      hp[l].from_ops(b);
      sync_stage();
    }
  }

  // Output layer from the last hidden layer's activations, with its first
  // stage resident in b0; leaves `next` (elems) resident in b0 on return.
  __device__ __forceinline__ static void output(const W* wg, W*& b0, W*& b1, const Pk<MTH>& hl, float (&out)[MTO][4],
                                const W* next, int next_elems, int lane) {
    const Bf16Layout Lt = layout();
    bf16x8 b[M::KBH];
    hl.ops(b);
    if constexpr (NOUT == 2) {
      dma(b1, wg + Lt.fwd_off(NH) + OUT_STAGE, OUT_STAGE);
      {
        float part[HALF_O][4];
        M::template gemm_op<HALF_O, BM>(b0, b, part, lane);
#pragma unroll
        for (int mt = 0; mt < HALF_O; ++mt)
#pragma unroll
          for (int i = 0; i < 4; ++i) out[mt][i] = part[mt][i];
      }
      sync_stage();
      dma(b0, next, next_elems);
      {
        float part[HALF_O][4];
        M::template gemm_op<HALF_O, BM>(b1, b, part, lane);
#pragma unroll
        for (int mt = 0; mt < HALF_O; ++mt)
#pragma unroll
          for (int i = 0; i < 4; ++i) out[HALF_O + mt][i] = part[mt][i];
      }
      sync_stage();
    } else {
      dma(b1, next, next_elems);
      M::template gemm_op<MTO, BM>(b0, b, out, lane);
      sync_stage();
      swap(b0, b1);
    }
  }

  // Full forward of one tile with layer 0 resident in b0; the next tile's
  // layer 0 is resident in b0 on return (query).
  __device__ __forceinline__ static void forward(const W* wg, W*& b0, W*& b1, const typename M::Input& x, float (&out)[MTO][4],
                                 int lane) {
    const Bf16Layout Lt = layout();
    Pk<MTH> hp[NH];
    hidden(wg, b0, b1, x, hp, wg + Lt.fwd_off(NH), OUT_STAGE, lane);   // output stage 0 -> b0
    output(wg, b0, b1, hp[NH - 1], out, wg + Lt.fwd_off(0), L0, lane);
  }

  // Forward of one tile with every forward weight resident at `base` in the
  // packed forward order (FWD elements): no stage waits.
  static constexpr int FWD = L0 + (NH - 1) * H * H + OUT;
  __device__ __forceinline__ static void forward_resident(const W* base, const typename M::Input& x, Pk<MTH> (&hp)[NH],
                                          float (&out)[MTO][4], int lane) {
    const Bf16Layout Lt = layout();
    float y[MTH][4];
    bf16x8 b[M::KBH];
    M::layer0_linear(base, x, y, lane);
    M::relu_operands(y, b);
    hp[0].from_ops(b);
#pragma unroll
    for (int l = 1; l < NH; ++l) {
      M::template gemm_op<MTH, BM>(base + Lt.fwd_off(l), b, y, lane);
      M::relu_operands(y, b);
      hp[l].from_ops(b);
    }
    M::template gemm_op<MTO, BM>(base + Lt.fwd_off(NH), b, out, lane);
  }

  // dh = W_out^T dl with the output layer's first backward stage resident in
  // b0: bo holds dl's 8K lobe rows as B operands, bs the selection tile's.
  // `next` (elems) is resident in b0 on return.
  __device__ __forceinline__ static void out_dgrad(const W* out_bwd, W*& b0, W*& b1, const bf16x8 (&bo)[KBO], const bf16x4& bs,
                                   float (&dh)[MTH][4], const W* next, int next_elems, int lane) {
    if constexpr (NOUT == 2) {
      dma(b1, out_bwd + OB_STAGE, OB_STAGE);
      dgrad_rows<KBO, MTH / 2, 0, BM>(b0, bo, dh, lane);
      sync_stage();
      dma(b0, next, next_elems);
      dgrad_rows<KBO, MTH / 2, MTH / 2, BM>(b1, bo, dh, lane);
      sync_stage();
    } else {
      dma(b1, next, next_elems);
      dgrad_rows<KBO, MTH, 0, BM>(b0, bo, dh, lane);
      if constexpr (SEL == 1) dgrad_sel(b0 + 8 * K * H, bs, dh, lane);
      sync_stage();
      swap(b0, b1);
    }
  }
};

// ------------------------------------------------------------------ FP32 ----
// One buffer, 64 rows of a layer at a time (a last, shorter chunk when the
// layer's row tiles are not a multiple of four: the selection tile).
template <int H, int K, int SEL = 0, int ENC = 0>
struct NetF32 {
  typedef Mlp<H, K, 0, ENC> M;
  typedef float W;
  static constexpr int NH = 4;
  static constexpr int MTH = H / 16, MTO = K / 2 + SEL, KQ = K / 4;
  static constexpr int CH = 64;              // rows per LDS chunk
  static constexpr int TPC = CH / 16;        // row tiles per chunk
  static constexpr int PH = H + 1;           // pitch of hidden and output layers
  static constexpr int P0 = M::IN + 1;       // pitch of layer 0
  static constexpr int BUF = (CH * PH > H * P0) ? CH * PH : H * P0;
  static constexpr int SP = kWGV + 4;
  // rows of the backward's delta staging: the output layer's or a hidden layer's
  static constexpr int RMAX = (8 * K + 16 * SEL > H) ? 8 * K + 16 * SEL : H;

  __device__ __forceinline__ static F32Layout layout() { return F32Layout{NetDims{H, NH, K, SEL, ENC}}; }
  // Replace the LDS weight buffer's contents (whole workgroup).
  __device__ __forceinline__ static void wstage(W* buf, const W* src, int elems) {
    __syncthreads();
    lds_dma(buf, src, elems * (int)sizeof(W));
    lds_dma_wait();
    __syncthreads();
  }

  // y = W_l h over all MT_*16 rows of layer l, 64 rows at a time
  template <int MT_>
  __device__ __forceinline__ static void layer(const W* wg, W* buf, int l, const float (&in)[MTH][4], float (&y)[MT_][4],
                               int lane) {
    const F32Layout Lt = layout();
    constexpr int NCH = MT_ / TPC, TAIL = MT_ % TPC;
#pragma unroll
    for (int ch = 0; ch < NCH; ++ch) {
      wstage(buf, wg + Lt.off(l) + (int64_t)ch * CH * PH, CH * PH);
      float part[TPC][4];
      M::template gemm<TPC>(buf, in, part, lane);   // rows ch*CH .. ch*CH + CH - 1
#pragma unroll
      for (int t = 0; t < TPC; ++t)
#pragma unroll
        for (int i = 0; i < 4; ++i) y[ch * TPC + t][i] = part[t][i];
    }
    if constexpr (TAIL > 0) {
      wstage(buf, wg + Lt.off(l) + (int64_t)NCH * CH * PH, TAIL * 16 * PH);
      float part[TAIL][4];
      M::template gemm<TAIL>(buf, in, part, lane);
#pragma unroll
      for (int t = 0; t < TAIL; ++t)
#pragma unroll
        for (int i = 0; i < 4; ++i) y[NCH * TPC + t][i] = part[t][i];
    }
  }

  __device__ __forceinline__ static void forward(const W* wg, W* buf, W* unused, const typename M::Input& x, float (&out)[MTO][4],
                                 int lane) {
    float h[NH][MTH][4];
    forward(wg, buf, unused, x, h, out, lane);
  }

  __device__ __forceinline__ static void forward(const W* wg, W* buf, W*, const typename M::Input& x, float (&h)[NH][MTH][4],
                                 float (&out)[MTO][4], int lane) {
    wstage(buf, wg + layout().off(0), H * P0);
    M::layer0(buf, x, h[0], lane);
#pragma unroll
    for (int l = 1; l < NH; ++l) {
      float y[MTH][4];
      layer<MTH>(wg, buf, l, h[l - 1], y, lane);
#pragma unroll
      for (int mt = 0; mt < MTH; ++mt)
#pragma unroll
        for (int i = 0; i < 4; ++i) h[l][mt][i] = relu(y[mt][i]);
    }
    layer<MTO>(wg, buf, NH, h[NH - 1], out, lane);
  }

  // dp = W_l^T dl (rows of layer l = RT*16), 64 rows of weights at a time;
  // slot (kb, g) of the contraction is row (kb/4)*16 + 4g + kb%4 of layer l,
  // held in dl[kb/4][kb%4]; chunk ch holds rows [CH*ch, CH*ch + CH) (the
  // last chunk the remaining RT % 4 row tiles)
  template <int RT>
  __device__ __forceinline__ static void dgrad_layer(const W* wg, W* buf, int l, const float (&dl)[RT][4], float (&dp)[MTH][4],
                                     int lane) {
    const F32Layout Lt = layout();
    const int g = lane >> 4, c = lane & 15;
    constexpr int NCH = (RT + TPC - 1) / TPC;
    f32x4 acc[MTH];
#pragma unroll
    for (int mt = 0; mt < MTH; ++mt) acc[mt] = zero4();
#pragma unroll
    for (int ch = 0; ch < NCH; ++ch) {
      const int nt = (ch + 1) * TPC <= RT ? TPC : RT - ch * TPC;   // row tiles in this chunk
      wstage(buf, wg + Lt.off(l) + (int64_t)ch * CH * PH, nt * 16 * PH);
#pragma unroll
      for (int mt = 0; mt < MTH; ++mt)
#pragma unroll
        for (int kk = 0; kk < 4 * TPC; ++kk) {
          if (kk < 4 * nt) {
            const int kb = 4 * TPC * ch + kk;
            const int r = ((kb >> 2) - TPC * ch) * 16 + 4 * g + (kb & 3);
            acc[mt] = mfma_f32_4(buf[r * PH + mt * 16 + c], dl[kb >> 2][kb & 3], acc[mt]);
          }
        }
    }
#pragma unroll
    for (int mt = 0; mt < MTH; ++mt)
#pragma unroll
      for (int i = 0; i < 4; ++i) dp[mt][i] = acc[mt][i];
  }
};

template <int H, int K, int PREC, int SEL, int ENC>
using LargeNet = typename std::conditional<PREC == 1, NetBf16<H, K, SEL, ENC>, NetF32<H, K, SEL, ENC>>::type;

// Hidden activations kept by the FP32 backward kernels (the BF16 ones keep
// them packed, as Pk).
template <int PREC, int MTH>
struct Act;

template <int MTH>
struct Act<0, MTH> {
  float v[MTH][4];
  __device__ __forceinline__ void set(const float (&h)[MTH][4]) {
#pragma unroll
    for (int mt = 0; mt < MTH; ++mt)
#pragma unroll
      for (int i = 0; i < 4; ++i) v[mt][i] = h[mt][i];
  }
  __device__ __forceinline__ float get(int mt, int i) const { return v[mt][i]; }
};

template <int PREC, int MTH>
__device__ __forceinline__ void mask_relu(float (&d)[MTH][4], const Act<PREC, MTH>& h) {
#pragma unroll
  for (int mt = 0; mt < MTH; ++mt)
#pragma unroll
    for (int i = 0; i < 4; ++i) d[mt][i] = h.get(mt, i) > 0.0f ? d[mt][i] : 0.0f;
}

template <typename S, int PREC, int MTH, int SP>
__device__ __forceinline__ void stage_act(S* st, const Act<PREC, MTH>& h, int wave, int lane) {
  float x[MTH][4];
#pragma unroll
  for (int mt = 0; mt < MTH; ++mt)
#pragma unroll
    for (int i = 0; i < 4; ++i) x[mt][i] = h.get(mt, i);
  stage_rows<S, MTH, SP>(st, x, wave, lane);
}

// dL/d(raw outputs) of 16 vertices: BF16 as the output layer's dgrad B
// operands (K/4 16-byte slots per lane, then with the selection output one
// 8-byte slot of the selection tile's 16x16x16 operand); FP32 as the
// accumulator image (K/2 16-byte slots per lane, one more for the selection
// tile). Written once and read once, by non-temporal stores and loads, so
// the stream does not displace the weights in L2.
template <int K, int PREC, int SEL = 0>
struct DOut {
  static constexpr int MTO = K / 2 + SEL, KBO = K / 4;     // FP32: every output tile
  static constexpr int BLOCK = 64 * (8 * KBO + 4 * SEL);   // BF16 elements per 16 vertices
  __device__ __forceinline__ static void store(void* base, int64_t tile16, const float (&dl)[MTO][4], int lane) {
    float4* d = reinterpret_cast<float4*>(base) + tile16 * MTO * 64 + lane;
#pragma unroll
    for (int mt = 0; mt < MTO; ++mt)
      __builtin_nontemporal_store(f32x4{dl[mt][0], dl[mt][1], dl[mt][2], dl[mt][3]},
                                  reinterpret_cast<f32x4*>(d + mt * 64));
  }
  __device__ __forceinline__ static void load(const void* base, int64_t tile16, float (&dl)[MTO][4], int lane) {
    const float4* s = reinterpret_cast<const float4*>(base) + tile16 * MTO * 64 + lane;
#pragma unroll
    for (int mt = 0; mt < MTO; ++mt) {
      const f32x4 x = __builtin_nontemporal_load(reinterpret_cast<const f32x4*>(s + mt * 64));
      dl[mt][0] = x[0]; dl[mt][1] = x[1]; dl[mt][2] = x[2]; dl[mt][3] = x[3];
    }
  }
  // BF16: the stored slots are exactly the output layer's dgrad B operands
  __device__ __forceinline__ static void store_operands(void* base, int64_t tile16, const bf16x8 (&b)[KBO], const bf16x4& bs,
                                        int lane) {
    __bf16* blk = reinterpret_cast<__bf16*>(base) + tile16 * BLOCK;
    bf16x8* d = reinterpret_cast<bf16x8*>(blk) + lane;
#pragma unroll
    for (int kb = 0; kb < KBO; ++kb) __builtin_nontemporal_store(b[kb], d + kb * 64);
    if constexpr (SEL == 1) __builtin_nontemporal_store(bs, reinterpret_cast<bf16x4*>(blk + KBO * 512) + lane);
  }
  __device__ __forceinline__ static void load_operands(const void* base, int64_t tile16, bf16x8 (&b)[KBO], bf16x4& bs, int lane) {
    const __bf16* blk = reinterpret_cast<const __bf16*>(base) + tile16 * BLOCK;
    const bf16x8* s = reinterpret_cast<const bf16x8*>(blk) + lane;
#pragma unroll
    for (int kb = 0; kb < KBO; ++kb) b[kb] = __builtin_nontemporal_load(s + kb * 64);
    if constexpr (SEL == 1) bs = __builtin_nontemporal_load(reinterpret_cast<const bf16x4*>(blk + KBO * 512) + lane);
  }
};

// ---------------------------------------------------------------- query ----
// MODE 0: query, 1: raw forward only
template <int H, int K, int PREC, int SEL, int ENC, int MODE>
__global__ __launch_bounds__(256) void large_query_kernel(QueryArgs a) {
  typedef LargeNet<H, K, PREC, SEL, ENC> N;
  typedef typename N::M M;
  typedef typename N::W W;
  constexpr int KQ = N::KQ;
  extern __shared__ __align__(16) unsigned char smem[];
  W* b0 = reinterpret_cast<W*>(smem);
  W* b1 = b0 + N::BUF;
  const W* wg = reinterpret_cast<const W*>(a.wpack);
  const int lane = lane_id();
  const int g = lane >> 4, c = lane & 15;
  const int wave = threadIdx.x >> 6;
  if constexpr (PREC == 1) N::begin(wg, b0);
  const int64_t n_tiles = (a.B + kWGV - 1) / kWGV;
  for (int64_t tile = blockIdx.x; tile < n_tiles; tile += gridDim.x) {
    const int64_t v = tile * kWGV + wave * 16 + c;
    const bool valid = v < a.B;
    typename M::Input x = M::load_input(a.feat, a.ld, v, valid, g);
    float out[N::MTO][4];
    N::forward(wg, b0, b1, x, out, lane);
    if (MODE == 1) {
      if (valid) {
#pragma unroll
        for (int t = 0; t < 2 * K; ++t) {
          const int p = t / KQ, k = g * KQ + t % KQ;
          a.raw_out[(int64_t)(p * K + k) * a.ld + v] = out[t >> 2][t & 3];
        }
        if (SEL == 1 && g == 0) a.raw_out[(int64_t)(8 * K) * a.ld + v] = out[N::MTO - 1][0];
      }
      continue;
    }
    float xi_sel = 0.0f, xi0 = 0.0f, xi1 = 0.0f, xi2 = 0.0f;
    if (valid) {
      xi_sel = a.xi[v];
      xi0 = a.xi[a.ld + v];
      xi1 = a.xi[2 * a.ld + v];
      xi2 = a.xi[3 * a.ld + v];
    }
    Lobe lb[KQ];
    float vx, vy, vz;
    const float logq =
        query_epilogue<KQ, N::MTO>(out, xi_sel, xi0, xi1, xi2, a.eps, g, c, lb, vx, vy, vz, a.amul);
    if (valid && g == 0) {
      a.dir_out[v] = vx;
      a.dir_out[a.ld + v] = vy;
      a.dir_out[2 * a.ld + v] = vz;
      a.pdf_out[v] = fexp(logq);
      // selection probability c = sigmoid(o[8K]) (Tab. "decoding")
      if (SEL == 1 && a.sel_out != nullptr) a.sel_out[v] = frcp(1.0f + fexp(-out[N::MTO - 1][0]));
    }
    if (a.rec_out != nullptr && valid) {
      float* base = a.rec_out + (v / kRecTile) * 9 * K * kRecTile + (v % kRecTile);
#pragma unroll
      for (int q = 0; q < KQ; ++q) {
        const int k = g * KQ + q;
        const float vals[9] = {lb[q].zx, lb[q].zy, lb[q].zz, lb[q].xx, lb[q].xy, lb[q].xz,
                               lb[q].lam, lb[q].a, lb[q].logc};
#pragma unroll
        for (int p = 0; p < 9; ++p) base[(p * K + k) * kRecTile] = vals[p];
      }
    }
  }
}

// ------------------------------------------------------------- gradient ----
// FP32 path: forward and the weighted-NLL / NASG backward, storing dL/d(raw
// outputs) and the loss partials.
template <int H, int K, int SEL, int ENC>
__global__ __launch_bounds__(256) void gradout_kernel(LargeTrainArgs a) {
  typedef NetF32<H, K, SEL, ENC> N;
  typedef typename N::M M;
  typedef typename N::W W;
  constexpr int KQ = N::KQ, MTO = N::MTO;
  extern __shared__ __align__(16) unsigned char smem[];
  W* b0 = reinterpret_cast<W*>(smem);
  W* b1 = b0 + N::BUF;
  const W* wg = reinterpret_cast<const W*>(a.wpack);
  const int lane = lane_id();
  const int g = lane >> 4, c = lane & 15;
  const int wave = threadIdx.x >> 6;
  const float inv_b = 1.0f / (float)a.B;
  double loss_sum = 0.0, w_sum = 0.0;
  const int64_t n_tiles = (a.B + kWGV - 1) / kWGV;
  for (int64_t tile = blockIdx.x; tile < n_tiles; tile += gridDim.x) {
    const int64_t v = tile * kWGV + wave * 16 + c;
    const bool valid = v < a.B;
    typename M::Input x = M::load_input(a.feat, a.ld, v, valid, g);
    float vx = 0.0f, vy = 0.0f, vz = 1.0f, wj = 0.0f, pfs = 0.0f;
    if (valid) {
      vx = a.dir[v]; vy = a.dir[a.ld + v]; vz = a.dir[2 * a.ld + v];
      wj = a.w[v];
      if constexpr (SEL == 1) pfs = a.bsdf_pdf[v];
    }
    float out[MTO][4];
    N::forward(wg, b0, b1, x, out, lane);
    {
      const float inv = frsq(fmaf(vx, vx, fmaf(vy, vy, vz * vz)));
      vx *= inv; vy *= inv; vz *= inv;
    }
    const float gs = valid ? -wj * inv_b : 0.0f;
    float dl[MTO][4];
    const float lterm = train_epilogue<KQ, MTO, SEL>(out, vx, vy, vz, gs, valid, a.eps, dl, pfs, a.mis_e, a.amul);
    if (valid && g == 0) {
      loss_sum += (double)wj * (double)(-lterm);
      w_sum += (double)wj;
    }
    DOut<K, 0, SEL>::store(a.dout, tile * 4 + wave, dl, lane);
  }
  __shared__ double red[4][2];
#pragma unroll
  for (int s = 32; s >= 1; s >>= 1) {
    loss_sum += __shfl_xor(loss_sum, s);
    w_sum += __shfl_xor(w_sum, s);
  }
  if (lane == 0) { red[wave][0] = loss_sum; red[wave][1] = w_sum; }
  __syncthreads();
  if (threadIdx.x == 0) {
    a.loss_partial[2 * blockIdx.x] = ((red[0][0] + red[1][0]) + red[2][0]) + red[3][0];
    a.loss_partial[2 * blockIdx.x + 1] = ((red[0][1] + red[1][1]) + red[2][1]) + red[3][1];
  }
}

// ------------------------------------------------------- backward, BF16 ----
// Eight waves (two per SIMD) over 128-vertex tiles: each wave recomputes the
// hidden layers and runs dgrad for its 16 vertices, and owns row tile `wave`
// (and wave + 8 of the output layer) of every weight gradient it
// accumulates. GROUP 1 (launched first) also runs the output layer and the
// weighted-NLL / NASG backward (Sec. 4.2), stores dL/d(raw outputs) and the
// loss partials, and accumulates the weight gradients of hidden layers
// NH-2 .. 1 and layer 0; the VALU-heavy NASG work of one wave overlaps the
// MFMA work of the other on each SIMD. GROUP 0 reads the stored gradient and
// accumulates those of the output layer and the last hidden layer. The
// weight pipeline runs through every stage of a tile and ends it with the
// next tile's layer 0 resident.
constexpr int kBwdWaves = 8;
constexpr int kBwdV = 16 * kBwdWaves;   // vertices per backward tile
// staging pitch (bf16): 144 values are 18 16-byte units, which makes the
// weight-gradient operand reads free of LDS bank conflicts (units per row
// 2 mod 4; 136 costs ~3 conflict cycles per 16-byte read on gfx950)
constexpr int kBwdSP = kBwdV + 16;

// LDS of the weight buffers, and of the backward kernels (weights + staging)
template <int H, int K, int PREC, int SEL, int ENC>
struct LargeLds {
  typedef LargeNet<H, K, PREC, SEL, ENC> N;
  static constexpr size_t fwd = (size_t)(PREC == 1 ? 2 : 1) * N::BUF * sizeof(typename N::W);
  static constexpr size_t bwd = PREC == 1 ? fwd + (size_t)2 * H * kBwdSP * sizeof(__bf16)
                                          : fwd + (size_t)(N::RMAX + H) * N::SP * sizeof(typename N::W);
  static constexpr int bwd_threads = PREC == 1 ? 64 * kBwdWaves : 256;
  static_assert(bwd <= 160 * 1024, "LDS budget");
};


// One workgroup's share of a backward group: tiles wg, wg + n_wg, ... OWN
// (group 0 only): evaluate the loss gradient itself (the forward's output
// layer and the epilogue) instead of reading group 1's stored one, so that
// the two groups can run at the same time.
// SINGLE: the workgroup has one tile at most, so the tile loop has no back
// edge and the gradient accumulators are live from their first MFMA only
// (not across the forward and the epilogue). RES (SINGLE, loss gradient
// evaluated here): the whole forward image is loaded at once into the LDS
// (the two weight buffers and the staging area, which the forward does not
// use), so the forward waits for memory once instead of once per layer.
template <int H, int K, int SEL, int ENC, int GROUP, bool OWN, bool SINGLE = false, bool RES = false>
__device__ __forceinline__ void bwd_bf16_body(const LargeTrainArgs& a, int wgi, int n_wg) {
  // block-major MFMA order where the registers allow it: everywhere but the
  // multi-tile group-1 kernel, whose gradient accumulators stay live across
  // the forward and the epilogue
  typedef NetBf16<H, K, SEL, ENC, GROUP == 0 || SINGLE> N;
  static_assert(!RES || (SINGLE && (GROUP == 1 || OWN)), "the resident forward: one tile, loss gradient here");
  typedef typename N::M M;
  typedef __bf16 W;
  typedef __bf16 St;   // staging element
  typedef DOut<K, 1, SEL> DO;
  constexpr int NH = N::NH, MTH = N::MTH, MTO = N::MTO, KBO = N::KBO, SP = kBwdSP;
  constexpr int CTH = H / 16, HALF_H = MTH / 2, KBH = MTH / 2;
  constexpr int CT0 = M::IN / 16;                   // column tiles of layer 0
  static_assert(MTH == kBwdWaves, "one hidden row tile per wave");
  static_assert(N::NOUT == 2 ? MTO == 2 * kBwdWaves : MTO <= kBwdWaves, "output row tiles per wave");
  static_assert(MTO / N::NOUT * 16 <= H && M::IN <= H, "staging holds H rows");
  extern __shared__ __align__(16) unsigned char smem[];
  W* bufA = reinterpret_cast<W*>(smem);
  W* bufB = bufA + N::BUF;
  St* dst = reinterpret_cast<St*>(smem + 2 * N::BUF * sizeof(W));   // [H rows][SP]
  St* hst = dst + H * SP;                                            // [H rows][SP]
  const W* wg = reinterpret_cast<const W*>(a.wpack);
  const Bf16Layout Lt = N::layout();
  const NetDims dims = Lt.d;
  const W* out_bwd = wg + Lt.bwd_off(NH);   // the output layer's backward fragments
  const int lane = lane_id();
  const int g = lane >> 4, c = lane & 15;
  const int wave = threadIdx.x >> 6;
  const int rt[1] = {wave};                 // this wave's row tile (+ MTH for a two-stage output layer)
  const int rt_hi[1] = {wave + MTH};
  const int n_out_rt = (N::NOUT == 2 || wave < MTO) ? 1 : 0;   // output row tiles this wave owns

  constexpr int NO = GROUP == 0 ? N::NOUT : 1;      // output layer stages (group 0)
  constexpr int NM = GROUP == 1 ? NH - 2 : 1;       // hidden layers NH-2..1 (group 1)
  f32x4 accO[NO][1][CTH];
  f32x4 accT[1][CTH];                               // layer NH-1 (group 0)
  f32x4 accM[NM][1][CTH];
  f32x4 acc0[1][CT0];                               // layer 0 (group 1)
#pragma unroll
  for (int ct = 0; ct < CT0; ++ct) acc0[0][ct] = zero4();
#pragma unroll
  for (int ct = 0; ct < CTH; ++ct) {
    accT[0][ct] = zero4();
#pragma unroll
    for (int l = 0; l < NM; ++l) accM[l][0][ct] = zero4();
#pragma unroll
    for (int h = 0; h < NO; ++h) accO[h][0][ct] = zero4();
  }

  const float inv_b = 1.0f / (float)a.B;
  double loss_sum = 0.0, w_sum = 0.0;
  W* b0 = bufA;
  W* b1 = bufB;
  if constexpr (!RES) N::begin(wg, b0);
  const int64_t n_tiles = (a.B + kBwdV - 1) / kBwdV;
  for (int64_t tile = wgi; tile < n_tiles; tile += n_wg) {
    const int64_t v = tile * kBwdV + wave * 16 + c;
    const int64_t blk = tile * kBwdWaves + wave;   // this wave's 16-vertex block
    const bool valid = v < a.B;
    typename M::Input x = M::load_input(a.feat, a.ld, v, valid, g);
    Pk<MTH> hp[NH];
    bf16x8 bo[KBO];
    bf16x4 bs = {};
    if constexpr (GROUP == 1 || OWN) {
      float vx = 0.0f, vy = 0.0f, vz = 1.0f, wj = 0.0f, pfs = 0.0f;
      if (valid) {
        vx = a.dir[v]; vy = a.dir[a.ld + v]; vz = a.dir[2 * a.ld + v];
        wj = a.w[v];
        if constexpr (SEL == 1) pfs = a.bsdf_pdf[v];
      }
      float out[MTO][4];
      if constexpr (RES) {
        __syncthreads();                                                        // a previous tile's staging is read
        N::dma(bufA, wg, N::FWD);
        N::sync_stage();
        N::forward_resident(bufA, x, hp, out, lane);
        __syncthreads();                                                        // the forward image is consumed
        N::dma(b0, out_bwd, N::OB_STAGE);                                       // awaited after the epilogue
      } else {
        N::hidden(wg, b0, b1, x, hp, wg + Lt.fwd_off(NH), N::OUT_STAGE, lane);  // output stage 0 -> b0
        N::output(wg, b0, b1, hp[NH - 1], out, out_bwd, N::OB_STAGE, lane);    // output-dgrad stage 0 -> b0
      }
      const float inv = frsq(fmaf(vx, vx, fmaf(vy, vy, vz * vz)));
      vx *= inv; vy *= inv; vz *= inv;
      const float gs = valid ? -wj * inv_b : 0.0f;
      float dl[MTO][4];
      const float lterm =
          train_epilogue<N::KQ, MTO, SEL>(out, vx, vy, vz, gs, valid, a.eps, dl, pfs, a.mis_e, a.amul);
      if (GROUP == 1 && valid && g == 0) {
        loss_sum += (double)wj * (double)(-lterm);
        w_sum += (double)wj;
      }
#pragma unroll
      for (int kb = 0; kb < KBO; ++kb)
#pragma unroll
        for (int j = 0; j < 8; ++j) bo[kb][j] = (__bf16)dl[2 * kb + (j >> 2)][j & 3];
      if constexpr (SEL == 1) {
#pragma unroll
        for (int j = 0; j < 4; ++j) bs[j] = (__bf16)dl[MTO - 1][j];
      }
      // stored for the separate group-0 kernel only (in the one-launch
      // schedule group 0 evaluates its own)
      if constexpr (GROUP == 1 && !SINGLE) DO::store_operands(a.dout, blk, bo, bs, lane);
      if constexpr (RES) N::sync_stage();                                       // output-dgrad stage 0 in b0
    } else {
      N::hidden(wg, b0, b1, x, hp, out_bwd, N::OB_STAGE, lane);   // leaves output-dgrad stage 0 in b0
      DO::load_operands(a.dout, blk, bo, bs, lane);
    }
    float dh[MTH][4];
    Pk<MTH> dhw;
    if constexpr (GROUP == 0) {
      Pk<MTO> dlw;
      dlw.from_ops(bo);
      if constexpr (SEL == 1) dlw.set_last(bs);
      hp[NH - 1].template stage<SP>(hst, wave, lane);
      if constexpr (N::NOUT == 2) {
        dlw.template stage<SP, 0, MTH>(dst, wave, lane);           // output rows [0, 8K/2)
        N::dma(b1, out_bwd + N::OB_STAGE, N::OB_STAGE);
        dgrad_rows<KBO, HALF_H, 0, N::BM>(b0, bo, dh, lane);
        N::sync_stage();                                            // also publishes the staging
        wgrad_tiles<1, St, SP, 1, CTH, kBwdV>(dst, hst, rt, 1, accO[0], lane);
        N::dma(b0, wg + Lt.fwd_off(0), N::L0);                      // the next tile's layer 0
        dgrad_rows<KBO, HALF_H, HALF_H, N::BM>(b1, bo, dh, lane);
        dhw.masked(dh, hp[NH - 1]);
        N::sync_stage();                                            // the first half has been read
        dlw.template stage<SP, MTH, MTH>(dst, wave, lane);          // output rows [8K/2, 8K)
        __syncthreads();
        wgrad_tiles<1, St, SP, 1, CTH, kBwdV>(dst, hst, rt, 1, accO[N::NOUT - 1], lane);
      } else {
        dlw.template stage<SP, 0, MTO>(dst, wave, lane);            // every output row
        if constexpr (!RES) N::dma(b1, wg + Lt.fwd_off(0), N::L0);  // the next tile's layer 0
        dgrad_rows<KBO, MTH, 0, N::BM>(b0, bo, dh, lane);
        if constexpr (SEL == 1) dgrad_sel(b0 + 8 * K * H, bs, dh, lane);
        N::sync_stage();                                            // also publishes the staging
        N::swap(b0, b1);
        wgrad_tiles<1, St, SP, 1, CTH, kBwdV>(dst, hst, rt, n_out_rt, accO[0], lane);
        dhw.masked(dh, hp[NH - 1]);
      }
      __syncthreads();
      dhw.template stage<SP>(dst, wave, lane);
      hp[NH - 2].template stage<SP>(hst, wave, lane);
      __syncthreads();
      wgrad_tiles<1, St, SP, 1, CTH, kBwdV>(dst, hst, rt, 1, accT, lane);
      // the next writes to the staging area follow the next tile's forward,
      // whose barriers order them after these reads
    } else {
      N::out_dgrad(out_bwd, b0, b1, bo, bs, dh, wg + Lt.bwd_off(NH - 1), H * H, lane);   // layer NH-1 -> b0
      dhw.masked(dh, hp[NH - 1]);
      Pk<MTH> d2w;
      {
        bf16x8 op[KBH];
        dhw.ops(op);
        float d2[MTH][4];
        N::dma(b1, wg + Lt.bwd_off(NH - 2), H * H);
        dgrad_rows<KBH, MTH, 0, N::BM>(b0, op, d2, lane);                // through hidden layer NH-1
        d2w.masked(d2, hp[NH - 2]);
        N::sync_stage();
      }
      W* cur = b1;   // holds hidden layer l's backward fragments
      W* oth = b0;
#pragma unroll
      for (int l = NH - 2; l >= 1; --l) {
        d2w.template stage<SP>(dst, wave, lane);
        hp[l - 1].template stage<SP>(hst, wave, lane);
        if (l > 1) N::dma(oth, wg + Lt.bwd_off(l - 1), H * H);
        else if (!RES) N::dma(oth, wg + Lt.fwd_off(0), N::L0);    // the next tile's layer 0
        bf16x8 op[KBH];
        d2w.ops(op);
        float dn[MTH][4];
        dgrad_rows<KBH, MTH, 0, N::BM>(cur, op, dn, lane);
        Pk<MTH> dnw;
        dnw.masked(dn, hp[l - 1]);
        N::sync_stage();                                          // also publishes the staging
        wgrad_tiles<1, St, SP, 1, CTH, kBwdV>(dst, hst, rt, 1, accM[l - 1], lane);
        __syncthreads();
        d2w = dnw;
        W* t = cur; cur = oth; oth = t;
      }
      d2w.template stage<SP>(dst, wave, lane);
      M::template stage_input<St, SP>(hst, x, wave, lane);
      __syncthreads();
      wgrad_tiles<1, St, SP, 1, CT0, kBwdV>(dst, hst, rt, 1, acc0, lane);
      b0 = cur;   // the next tile's layer 0
      b1 = oth;
    }
    if constexpr (SINGLE) break;
  }

  float* part = a.partial + (int64_t)wgi * a.n_weights;
  if constexpr (GROUP == 0) {
    flush_tiles<1, CTH, SEL == 1>(part, dims, NH, rt, n_out_rt, accO[0], lane);
    if constexpr (N::NOUT == 2) flush_tiles<1, CTH>(part, dims, NH, rt_hi, 1, accO[N::NOUT - 1], lane);
    flush_tiles<1, CTH>(part, dims, NH - 1, rt, 1, accT, lane);
  } else {
#pragma unroll
    for (int l = 1; l <= NH - 2; ++l) flush_tiles<1, CTH>(part, dims, l, rt, 1, accM[l - 1], lane);
    flush_tiles<1, CT0>(part, dims, 0, rt, 1, acc0, lane);
    // loss partials: wave reduction, then the waves in order
    __shared__ double red[kBwdWaves][2];
#pragma unroll
    for (int s = 32; s >= 1; s >>= 1) {
      loss_sum += __shfl_xor(loss_sum, s);
      w_sum += __shfl_xor(w_sum, s);
    }
    if (lane == 0) { red[wave][0] = loss_sum; red[wave][1] = w_sum; }
    __syncthreads();
    if (threadIdx.x == 0) {
      double ls = 0.0, ws = 0.0;
#pragma unroll
      for (int w = 0; w < kBwdWaves; ++w) { ls += red[w][0]; ws += red[w][1]; }
      a.loss_partial[2 * wgi] = ls;
      a.loss_partial[2 * wgi + 1] = ws;
    }
  }
}

// GROUP 0 or 1: that group over the whole grid. GROUP 2 (small batches, when
// both groups fit on the GPU at once, one tile per workgroup): group 1 on the
// first half of the grid and group 0, evaluating the loss gradient itself,
// on the second half.
template <int H, int K, int SEL, int ENC, int GROUP>
__global__ __launch_bounds__(64 * kBwdWaves) __attribute__((amdgpu_waves_per_eu(2, 2)))
void bwd_bf16_kernel(LargeTrainArgs a) {
  if constexpr (GROUP == 2) {
    // one tile per workgroup here; the forward image fits the LDS for K = 8
    constexpr bool RES = NetBf16<H, K, SEL, ENC>::FWD <= LargeLds<H, K, 1, SEL, ENC>::bwd / 2;
    const int half = (int)(gridDim.x >> 1);
    if ((int)blockIdx.x < half) bwd_bf16_body<H, K, SEL, ENC, 1, false, true, RES>(a, (int)blockIdx.x, half);
    else bwd_bf16_body<H, K, SEL, ENC, 0, true, true, RES>(a, (int)blockIdx.x - half, half);
  } else {
    bwd_bf16_body<H, K, SEL, ENC, GROUP, false>(a, (int)blockIdx.x, (int)gridDim.x);
  }
}

// ------------------------------------------------------- backward, FP32 ----
template <int H, int K, int SEL, int ENC, int GROUP>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(1, 1)))
void bwd_f32_kernel(LargeTrainArgs a) {
  typedef NetF32<H, K, SEL, ENC> N;
  typedef typename N::M M;
  typedef float W;
  typedef float S;
  constexpr int NH = N::NH, MTH = N::MTH, MTO = N::MTO, SP = N::SP;
  constexpr int RTW_H = (MTH + 3) / 4, RTW_O = (MTO + 3) / 4, CTH = H / 16;
  constexpr int CT0 = M::IN / 16;   // column tiles of layer 0
  extern __shared__ __align__(16) unsigned char smem[];
  W* buf = reinterpret_cast<W*>(smem);
  S* dst = reinterpret_cast<S*>(smem + N::BUF * sizeof(W));
  S* hst = dst + N::RMAX * SP;
  const W* wg = reinterpret_cast<const W*>(a.wpack);
  const NetDims dims = N::layout().d;
  const int lane = lane_id();
  const int g = lane >> 4, c = lane & 15;
  const int wave = threadIdx.x >> 6;

  int rt_h[RTW_H], rt_o[RTW_O];
  int nrt_h = 0, nrt_o = 0;
#pragma unroll
  for (int r = 0; r < RTW_H; ++r) { rt_h[r] = wave + 4 * r; if (rt_h[r] < MTH) nrt_h = r + 1; }
#pragma unroll
  for (int r = 0; r < RTW_O; ++r) { rt_o[r] = wave + 4 * r; if (rt_o[r] < MTO) nrt_o = r + 1; }

  constexpr int NO = GROUP == 0 ? RTW_O : 1;
  constexpr int NM = GROUP == 1 ? NH - 2 : 1;
  f32x4 accO[NO][CTH];
  f32x4 accT[RTW_H][CTH];
  f32x4 accM[NM][RTW_H][CTH];
  f32x4 acc0[RTW_H][CT0];
#pragma unroll
  for (int r = 0; r < RTW_H; ++r) {
#pragma unroll
    for (int ct = 0; ct < CT0; ++ct) acc0[r][ct] = zero4();
#pragma unroll
    for (int ct = 0; ct < CTH; ++ct) {
      accT[r][ct] = zero4();
#pragma unroll
      for (int l = 0; l < NM; ++l) accM[l][r][ct] = zero4();
    }
  }
#pragma unroll
  for (int r = 0; r < NO; ++r)
#pragma unroll
    for (int ct = 0; ct < CTH; ++ct) accO[r][ct] = zero4();

  const int64_t n_tiles = (a.B + kWGV - 1) / kWGV;
  for (int64_t tile = blockIdx.x; tile < n_tiles; tile += gridDim.x) {
    const int64_t v = tile * kWGV + wave * 16 + c;
    const bool valid = v < a.B;
    typename M::Input x = M::load_input(a.feat, a.ld, v, valid, g);
    Act<0, MTH> hp[NH];
    {
      float h[NH][MTH][4];
      float out[MTO][4];
      N::forward(wg, buf, nullptr, x, h, out, lane);
#pragma unroll
      for (int l = 0; l < NH; ++l) hp[l].set(h[l]);
    }
    float dl[MTO][4];
    DOut<K, 0, SEL>::load(a.dout, tile * 4 + wave, dl, lane);
    float dh[MTH][4];
    if constexpr (GROUP == 0) {
      stage_rows<S, MTO, SP>(dst, dl, wave, lane);
      stage_act<S, 0, MTH, SP>(hst, hp[NH - 1], wave, lane);
      N::template dgrad_layer<MTO>(wg, buf, NH, dl, dh, lane);   // its weight staging publishes the above
      mask_relu<0, MTH>(dh, hp[NH - 1]);
      wgrad_tiles<0, S, SP, RTW_O, CTH>(dst, hst, rt_o, nrt_o, accO, lane);
      __syncthreads();
      stage_rows<S, MTH, SP>(dst, dh, wave, lane);
      stage_act<S, 0, MTH, SP>(hst, hp[NH - 2], wave, lane);
      __syncthreads();
      wgrad_tiles<0, S, SP, RTW_H, CTH>(dst, hst, rt_h, nrt_h, accT, lane);
      __syncthreads();
    } else {
      N::template dgrad_layer<MTO>(wg, buf, NH, dl, dh, lane);
      mask_relu<0, MTH>(dh, hp[NH - 1]);
      float d2[MTH][4];
      N::template dgrad_layer<MTH>(wg, buf, NH - 1, dh, d2, lane);
      mask_relu<0, MTH>(d2, hp[NH - 2]);
#pragma unroll
      for (int l = NH - 2; l >= 1; --l) {
        stage_rows<S, MTH, SP>(dst, d2, wave, lane);
        stage_act<S, 0, MTH, SP>(hst, hp[l - 1], wave, lane);
        float dn[MTH][4];
        N::template dgrad_layer<MTH>(wg, buf, l, d2, dn, lane);   // publishes the staging
        mask_relu<0, MTH>(dn, hp[l - 1]);
        wgrad_tiles<0, S, SP, RTW_H, CTH>(dst, hst, rt_h, nrt_h, accM[l - 1], lane);
        __syncthreads();
#pragma unroll
        for (int mt = 0; mt < MTH; ++mt)
#pragma unroll
          for (int i = 0; i < 4; ++i) d2[mt][i] = dn[mt][i];
      }
      stage_rows<S, MTH, SP>(dst, d2, wave, lane);
      M::template stage_input<S, SP>(hst, x, wave, lane);
      __syncthreads();
      wgrad_tiles<0, S, SP, RTW_H, CT0>(dst, hst, rt_h, nrt_h, acc0, lane);
      __syncthreads();
    }
  }

  float* part = a.partial + (int64_t)blockIdx.x * a.n_weights;
  if constexpr (GROUP == 0) {
    flush_tiles<RTW_O, CTH, SEL == 1>(part, dims, NH, rt_o, nrt_o, accO, lane);
    flush_tiles<RTW_H, CTH>(part, dims, NH - 1, rt_h, nrt_h, accT, lane);
  } else {
#pragma unroll
    for (int l = 1; l <= NH - 2; ++l) flush_tiles<RTW_H, CTH>(part, dims, l, rt_h, nrt_h, accM[l - 1], lane);
    flush_tiles<RTW_H, CT0>(part, dims, 0, rt_h, nrt_h, acc0, lane);
  }
}

// ------------------------------------------------------------ launchers ----
template <int H, int K, int PREC, int SEL, int ENC>
static hipError_t launch_large_query_t(const QueryArgs& a, int mode, hipStream_t st) {
  const size_t shmem = LargeLds<H, K, PREC, SEL, ENC>::fwd;
  auto kern = mode == 0 ? large_query_kernel<H, K, PREC, SEL, ENC, 0> : large_query_kernel<H, K, PREC, SEL, ENC, 1>;
  hipError_t e = mode == 0 ? set_max_lds_once<large_query_kernel<H, K, PREC, SEL, ENC, 0>>(shmem)
                           : set_max_lds_once<large_query_kernel<H, K, PREC, SEL, ENC, 1>>(shmem);
  if (e != hipSuccess) return e;
  const int64_t n_tiles = (a.B + kWGV - 1) / kWGV;
  const int64_t cap = 2LL * a.num_cus;
  const int grid = (int)(n_tiles < cap ? (n_tiles < 1 ? 1 : n_tiles) : cap);
  hipLaunchKernelGGL(kern, dim3(grid), dim3(256), shmem, st, a);
  return hipGetLastError();
}

template <int H, int K, int PREC, int SEL, int ENC>
static hipError_t launch_large_train_t(const LargeTrainArgs& a, int n_wg, int n_grad, hipStream_t st) {
  typedef LargeLds<H, K, PREC, SEL, ENC> Lds;
  if constexpr (PREC == 1) {
    auto k_bwd0 = bwd_bf16_kernel<H, K, SEL, ENC, 0>;
    auto k_bwd1 = bwd_bf16_kernel<H, K, SEL, ENC, 1>;
    auto k_both = bwd_bf16_kernel<H, K, SEL, ENC, 2>;
    hipError_t e = set_max_lds_once<bwd_bf16_kernel<H, K, SEL, ENC, 0>>(Lds::bwd);
    if (e == hipSuccess) e = set_max_lds_once<bwd_bf16_kernel<H, K, SEL, ENC, 1>>(Lds::bwd);
    if (e == hipSuccess) e = set_max_lds_once<bwd_bf16_kernel<H, K, SEL, ENC, 2>>(Lds::bwd);
    if (e != hipSuccess) return e;
    const int64_t n_tiles = (a.B + kBwdV - 1) / kBwdV;
    if (n_tiles <= n_wg && 2 * n_wg <= a.num_cus) {
      // a small batch: one tile per workgroup and one workgroup per CU for
      // both groups at once (group 0 repeats the output layer and the NASG
      // gradient instead of waiting for group 1's)
      hipLaunchKernelGGL(k_both, dim3(2 * n_wg), dim3(Lds::bwd_threads), Lds::bwd, st, a);
    } else {
      // the group-1 kernel computes and stores the raw-output gradient first
      hipLaunchKernelGGL(k_bwd1, dim3(n_wg), dim3(Lds::bwd_threads), Lds::bwd, st, a);
      hipLaunchKernelGGL(k_bwd0, dim3(n_wg), dim3(Lds::bwd_threads), Lds::bwd, st, a);
    }
  } else {
    auto k_grad = gradout_kernel<H, K, SEL, ENC>;
    auto k_bwd0 = bwd_f32_kernel<H, K, SEL, ENC, 0>;
    auto k_bwd1 = bwd_f32_kernel<H, K, SEL, ENC, 1>;
    hipError_t e = set_max_lds_once<gradout_kernel<H, K, SEL, ENC>>(Lds::fwd);
    if (e == hipSuccess) e = set_max_lds_once<bwd_f32_kernel<H, K, SEL, ENC, 0>>(Lds::bwd);
    if (e == hipSuccess) e = set_max_lds_once<bwd_f32_kernel<H, K, SEL, ENC, 1>>(Lds::bwd);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_grad, dim3(n_grad), dim3(256), Lds::fwd, st, a);
    hipLaunchKernelGGL(k_bwd0, dim3(n_wg), dim3(Lds::bwd_threads), Lds::bwd, st, a);
    hipLaunchKernelGGL(k_bwd1, dim3(n_wg), dim3(Lds::bwd_threads), Lds::bwd, st, a);
  }
  return hipGetLastError();
}

// Dispatchers of one translation unit's networks (NETS: training, QNETS:
// streamed queries): true when (d, prec) is one of them, with the launch
// status in *err.
#define NASG_LARGE_QCASE(h, k, p, s, e)                                \
  if (d.H == h && d.K == k && prec == p && d.S == s && d.E == e) {     \
    *err = launch_large_query_t<h, k, p, s, e>(a, mode, st);          \
    return true;                                                      \
  }
#define NASG_LARGE_TCASE(h, k, p, s, e)                                \
  if (d.H == h && d.K == k && prec == p && d.S == s && d.E == e) {     \
    *err = launch_large_train_t<h, k, p, s, e>(a, n_wg, n_grad, st);  \
    return true;                                                      \
  }
#define NASG_LARGE_LAUNCHERS(NAME, NETS, QNETS)                                                            \
  bool launch_large_query_##NAME(const QueryArgs& a, const NetDims& d, int prec, int mode, hipStream_t st, \
                                 hipError_t* err) {                                                       \
    QNETS(NASG_LARGE_QCASE)                                                                                \
    return false;                                                                                          \
  }                                                                                                        \
  bool launch_large_train_##NAME(const LargeTrainArgs& a, const NetDims& d, int prec, int n_wg, int n_grad, \
                                 hipStream_t st, hipError_t* err) {                                       \
    NETS(NASG_LARGE_TCASE)                                                                                 \
    return false;                                                                                          \
  }

}  // namespace nasg
