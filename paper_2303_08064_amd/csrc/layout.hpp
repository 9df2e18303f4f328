// Kernel-side weight layouts and the neuron orders the MFMA tiles imply.
//
// A layer computes Y^T[n][v] = sum_k W[n][k] H^T[k][v] with neurons as MFMA
// rows and 16 vertices as MFMA columns. In the 16x16 accumulator layout, lane
// (g = lane/16, c = lane%16) holds rows 4g..4g+3 of every 16-row tile for
// vertex c. The next layer's B operand wants, at lane (g, c), contraction
// indices 8g..8g+7 (bf16 16x16x32) or g (f32 16x16x4) of each block. Instead
// of moving activations between lanes, each layer's input columns are
// permuted so that a lane's accumulators ARE its next B operand:
//   bf16: logical k = kb*32 + 8g + j  <->  neuron (2kb + j/4)*16 + 4g + j%4
//   f32:  logical k = kb*4 + g        <->  neuron (kb/4)*16 + 4g + kb%4
// The output layer's rows are permuted so that lane group g owns whole lobes:
// the lane's accumulator t = mt*4 + i is parameter t / (K/4) of lobe
// g*(K/4) + t % (K/4).
#pragma once

#include <stdint.h>

#if defined(__HIPCC__)
#define NASG_HD __host__ __device__ __forceinline__
#else
#define NASG_HD inline
#endif

namespace nasg {

constexpr int kInFeatures = 9;
constexpr int kInPadded = 16;   // 9 features + constant one, zero-padded
// Tab. "encoding": 19 one-blob bins per position coordinate (57), omega_o (3),
// n (3) and the constant one: 64 inputs, no padding
constexpr int kBlobBins = 19;
constexpr int kInEncoded = 3 * kBlobBins + 6 + 1;

// neuron feeding logical contraction index kl of the next layer
NASG_HD int phys_bf16(int kl) { return (2 * (kl >> 5) + ((kl & 7) >> 2)) * 16 + 4 * ((kl & 31) >> 3) + (kl & 3); }
NASG_HD int phys_f32(int kl) { return (kl >> 4) * 16 + 4 * (kl & 3) + ((kl >> 2) & 3); }

// inverse of phys_bf16 / phys_f32: logical index whose B-operand slot holds neuron n
NASG_HD int inv_phys_bf16(int n) {
  int a = n >> 4, g = (n & 15) >> 2, cc = n & 3;
  return (a >> 1) * 32 + 8 * g + (a & 1) * 4 + cc;
}
NASG_HD int inv_phys_f32(int n) {
  int a = n >> 4, g = (n & 15) >> 2, i = n & 3;
  return (a * 4 + i) * 4 + g;
}

// canonical output row (p*K + k) held at physical output row R; rows from
// 8K form one more 16-row tile when the network has the selection output:
// its row 8K is canonical row 8K, the rest padding (-1)
NASG_HD int canon_out_row(int R, int K) {
  if (R >= 8 * K) return R == 8 * K ? 8 * K : -1;
  int mt = R >> 4, g = (R & 15) >> 2, i = R & 3;
  int t = mt * 4 + i;
  int kq = K / 4;
  return (t / kq) * K + g * kq + (t % kq);
}

// physical output row holding canonical row n = p*K + k (or the selection row 8K)
NASG_HD int inv_canon_out_row(int n, int K) {
  if (n >= 8 * K) return n;
  int kq = K / 4;
  int p = n / K, k = n % K;
  int g = k / kq, q = k % kq;
  int t = p * kq + q;
  return (t >> 2) * 16 + 4 * g + (t & 3);
}

struct NetDims {
  int H, NH, K;
  int S = 0;   // 1: one more output, the selection probability (8K + 1 outputs)
  int E = 0;   // 1: W_0 reads the encoded input (kInEncoded columns), else the 9 features + one
  NASG_HD int nout() const { return 8 * K + S; }
  NASG_HD int out_rows() const { return 8 * K + 16 * S; }   // physical, padded to whole tiles
  NASG_HD int layers() const { return NH + 1; }
  NASG_HD int rows(int l) const { return l == NH ? 8 * K + S : H; }
  NASG_HD int in_cols() const { return E ? kInEncoded : kInFeatures + 1; }
  NASG_HD int in_pad() const { return E ? kInEncoded : kInPadded; }   // layer 0's packed width
  NASG_HD int cols(int l) const { return l == 0 ? in_cols() : H; }
  // canonical flat offset of W_l
  NASG_HD int64_t canon_off(int l) const {
    if (l == 0) return 0;
    return (int64_t)H * in_cols() + (int64_t)(l - 1) * H * H;
  }
  NASG_HD int64_t num_weights() const { return canon_off(NH) + (int64_t)(8 * K + S) * H; }
};

// ---- BF16 fragment layout (elements are bf16) ----
// forward: L0 [H/16][64][4] (16x16x16 operands over the 16 padded inputs) or,
// for the encoded input, [H/16][2][64][8] (16x16x32 operands, input k =
// kb*32 + 8g + j in logical order); hidden l [H/16][H/32][64][8]; out
// [K/2 (+1)][H/32][64][8]
// backward (W^T): hidden l [H/16][H/32][64][8]; out [H/16][8K/32][64][8], then
// for the selection tile the 16x16x16 A operands [H/16][64][4]
struct Bf16Layout {
  NetDims d;
  NASG_HD int64_t fwd_off(int l) const {
    if (l == 0) return 0;
    return (int64_t)d.H * d.in_pad() + (int64_t)(l - 1) * d.H * d.H;
  }
  NASG_HD int64_t fwd_elems() const { return fwd_off(d.NH) + (int64_t)d.out_rows() * d.H; }
  NASG_HD int64_t bwd_off(int l) const {   // l >= 1
    return fwd_elems() + (int64_t)(l - 1) * d.H * d.H;
  }
  NASG_HD int64_t bwd_sel_off() const { return bwd_off(d.NH) + (int64_t)8 * d.K * d.H; }
  NASG_HD int64_t total_elems() const { return bwd_sel_off() + (int64_t)16 * d.S * d.H; }
};

// ---- FP32 row-major layout (elements are float) ----
// layer l: [rows][cols_pad + 1] with cols_pad = 16 or 64 (l == 0) or H; output rows in physical order
struct F32Layout {
  NetDims d;
  NASG_HD int pitch(int l) const { return (l == 0 ? d.in_pad() : d.H) + 1; }
  NASG_HD int64_t off(int l) const {
    if (l == 0) return 0;
    return (int64_t)d.H * pitch(0) + (int64_t)(l - 1) * d.H * pitch(1);
  }
  NASG_HD int64_t total_elems() const { return off(d.NH) + (int64_t)d.out_rows() * pitch(d.NH); }
};

}  // namespace nasg

namespace nasg {

// Packed position of canonical weight W_l[n][k] (element index into the bf16
// buffer): forward fragment, and backward (transposed) fragment for l >= 1.
NASG_HD int64_t bf16_fwd_pos(const Bf16Layout& Lt, int l, int n, int k) {
  const NetDims& d = Lt.d;
  if (l == 0) {
    if (d.E) {
      int mt = n >> 4, c = n & 15, kb = k >> 5, g = (k & 31) >> 3, j = k & 7;
      return Lt.fwd_off(0) + ((int64_t)((mt * 2 + kb) * 64 + g * 16 + c) * 8 + j);
    }
    int mt = n >> 4, c = n & 15, g = k >> 2, j = k & 3;
    return Lt.fwd_off(0) + ((int64_t)(mt * 64 + g * 16 + c) * 4 + j);
  }
  int R = (l == d.NH) ? inv_canon_out_row(n, d.K) : n;
  int kl = inv_phys_bf16(k);
  int KB = d.H / 32;
  int mt = R >> 4, c = R & 15, kb = kl >> 5, g = (kl & 31) >> 3, j = kl & 7;
  return Lt.fwd_off(l) + ((int64_t)((mt * KB + kb) * 64 + g * 16 + c) * 8 + j);
}

NASG_HD int64_t bf16_bwd_pos(const Bf16Layout& Lt, int l, int n, int k) {
  const NetDims& d = Lt.d;
  int R = (l == d.NH) ? inv_canon_out_row(n, d.K) : n;
  if (l == d.NH && R >= 8 * d.K) {   // selection tile: lane (g, c) holds rows 4g..4g+3, column c
    const int r = R - 8 * d.K, mt = k >> 4, c = k & 15;
    return Lt.bwd_sel_off() + ((int64_t)(mt * 64 + (r >> 2) * 16 + c) * 4 + (r & 3));
  }
  int kl = inv_phys_bf16(R);
  int KB = (l == d.NH) ? (8 * d.K) / 32 : d.H / 32;
  int mt = k >> 4, c = k & 15, kb = kl >> 5, g = (kl & 31) >> 3, j = kl & 7;
  return Lt.bwd_off(l) + ((int64_t)((mt * KB + kb) * 64 + g * 16 + c) * 8 + j);
}

NASG_HD int64_t f32_pos(const F32Layout& Lt, int l, int n, int k) {
  int R = (l == Lt.d.NH) ? inv_canon_out_row(n, Lt.d.K) : n;
  return Lt.off(l) + (int64_t)R * Lt.pitch(l) + k;
}

// Gather form: canonical (l, n, k) of packed element e, or k = -1 for padding.
NASG_HD void bf16_source(const Bf16Layout& Lt, int64_t e, int& l, int& n, int& k) {
  const NetDims& d = Lt.d;
  if (e < Lt.fwd_elems()) {
    if (e < Lt.fwd_off(1)) {
      l = 0;
      if (d.E) {
        int j = (int)(e & 7), lane = (int)((e >> 3) & 63), kb = (int)((e >> 9) & 1), mt = (int)(e >> 10);
        n = mt * 16 + (lane & 15);
        k = kb * 32 + (lane >> 4) * 8 + j;
        return;
      }
      int j = (int)(e & 3), lane = (int)((e >> 2) & 63), mt = (int)(e >> 8);
      n = mt * 16 + (lane & 15);
      k = (lane >> 4) * 4 + j;
      if (k >= kInFeatures + 1) k = -1;
      return;
    }
    l = 1 + (int)((e - Lt.fwd_off(1)) / ((int64_t)d.H * d.H));
    if (l > d.NH) l = d.NH;
    int64_t el = e - Lt.fwd_off(l);
    int KB = d.H / 32;
    int j = (int)(el & 7), lane = (int)((el >> 3) & 63);
    int kb = (int)((el >> 9) % KB), mt = (int)((el >> 9) / KB);
    int R = mt * 16 + (lane & 15);
    n = (l == d.NH) ? canon_out_row(R, d.K) : R;
    k = n < 0 ? -1 : phys_bf16(kb * 32 + 8 * (lane >> 4) + j);
    return;
  }
  if (e >= Lt.bwd_sel_off()) {
    l = d.NH;
    const int64_t el = e - Lt.bwd_sel_off();
    const int j = (int)(el & 3), lane = (int)((el >> 2) & 63), mt = (int)(el >> 8);
    n = canon_out_row(8 * d.K + 4 * (lane >> 4) + j, d.K);
    k = n < 0 ? -1 : mt * 16 + (lane & 15);
    return;
  }
  l = 1 + (int)((e - Lt.bwd_off(1)) / ((int64_t)d.H * d.H));
  if (l > d.NH) l = d.NH;
  int64_t el = e - Lt.bwd_off(l);
  int KB = (l == d.NH) ? (8 * d.K) / 32 : d.H / 32;
  int j = (int)(el & 7), lane = (int)((el >> 3) & 63);
  int kb = (int)((el >> 9) % KB), mt = (int)((el >> 9) / KB);
  k = mt * 16 + (lane & 15);
  int R = phys_bf16(kb * 32 + 8 * (lane >> 4) + j);
  n = (l == d.NH) ? canon_out_row(R, d.K) : R;
}

NASG_HD void f32_source(const F32Layout& Lt, int64_t e, int& l, int& n, int& k) {
  const NetDims& d = Lt.d;
  if (e < Lt.off(1)) {
    l = 0;
  } else {
    l = 1 + (int)((e - Lt.off(1)) / ((int64_t)d.H * Lt.pitch(1)));
    if (l > d.NH) l = d.NH;
  }
  int64_t el = e - Lt.off(l);
  int R = (int)(el / Lt.pitch(l));
  k = (int)(el % Lt.pitch(l));
  n = (l == d.NH) ? canon_out_row(R, d.K) : R;
  if (k >= d.cols(l) || n < 0) k = -1;
}

}  // namespace nasg
