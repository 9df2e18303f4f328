// Online training step (Sec. 4.2, Sec. 5): fused forward recompute, weighted
// NLL, closed-form NASG backward, MLP backward on MFMA; then a fixed-order
// reduction of per-workgroup weight gradients and a fused Adam update.
//
// Work split of the fused kernel (one persistent workgroup per CU; eight waves
// over 128-vertex tiles in BF16, four over 64 in FP32): each wave runs
// forward, NASG backward and dgrad for its own 16 vertices with activations
// in registers (nothing is written to HBM); for the weight gradient
// dW_l = sum_v delta_l(v) h_{l-1}(v)^T the waves stage delta_l and h_{l-1}
// of the tile's vertices in LDS and each wave accumulates its own tiles of
// dW_l in registers across every tile the workgroup visits.
// Every sum has a fixed order, so results are bitwise reproducible.
#include <type_traits>

#include "backward.hpp"
#include "epilogue.hpp"
#include "kernels.hpp"
#include "mlp.hpp"

namespace nasg {


// waves per training workgroup (see TrainCfg)
template <int PREC>
constexpr int train_waves() { return PREC == 1 ? 8 : 4; }

template <int H, int K, int PREC, int SEL>
struct TrainCfg {
  typedef Mlp<H, K, PREC> M;
  typedef typename std::conditional<PREC == 1, __bf16, float>::type S;   // staging type
  static constexpr int NHMAX = 4;
  static constexpr int KQ = K / 4;
  static constexpr int MTH = H / 16;
  static constexpr int MTO = K / 2 + SEL;       // output row tiles (+ the selection tile)
  static constexpr int CTH = H / 16;            // column tiles of dW (hidden input)
  // BF16: eight waves (two per SIMD) over 128-vertex tiles; FP32 (larger
  // weights and staging): four waves over 64-vertex tiles
  static constexpr int NW = train_waves<PREC>();
  static constexpr int NV = 16 * NW;            // vertices per tile
  static constexpr int RMAX = (16 * MTO > H) ? 16 * MTO : H;   // rows of the largest delta
  // staging pitch (elements). BF16: a row of NV + 16 = 144 values is 18
  // 16-byte units; the weight-gradient operand reads (lane (g, c): 16 B of
  // row c at unit g) are free of LDS bank conflicts when the row's units are
  // 2 mod 4 (measured on gfx950: 136, 152, 160, 168 and 184 values per row
  // each cost ~3 conflict cycles per read, 144 and 176 none). The selection
  // networks' staging at 144 would exceed the LDS beside their weights, so
  // they keep 136. FP32 reads one value per lane, conflict-free at NV + 4.
  static constexpr int SP = PREC == 1 ? (SEL == 1 ? NV + 8 : NV + 16) : NV + 4;
  typedef Own<MTH, 1, NW> O0;                   // layer 0
  typedef Own<MTH, CTH, NW> OH;                 // hidden layers
  typedef Own<MTO, CTH, NW> OO;                 // output layer
  // BF16: the hidden layers and layer 0 alternate between two staging
  // buffers, so a layer's writes never meet the previous layer's weight-
  // gradient reads and one barrier per layer suffices. The second delta
  // buffer is rows H..2H-1 of the first where the output layer's delta
  // (RMAX rows) leaves room, else rows of its own, like the second input
  // buffer (all BF16 networks fit the 160 KiB of LDS with it).
  static constexpr bool DB = PREC == 1;
  static constexpr int EXTRA = DB ? (RMAX >= 2 * H ? H : 2 * H) : 0;   // staging rows of the second buffer
  static constexpr int stage_elems() { return (RMAX + H + EXTRA) * SP; }
};

// weights of layer l in LDS (forward and, for l >= 1, backward)
template <int H, int K, int PREC, int SEL>
struct TrainLds {
  typedef typename std::conditional<PREC == 1, __bf16, float>::type W;
  __device__ __forceinline__ static const W* fwd(const W* lds, int l, int nh) {
    if (PREC == 1) return lds + Bf16Layout{NetDims{H, nh, K, SEL}}.fwd_off(l);
    return lds + F32Layout{NetDims{H, nh, K, SEL}}.off(l);
  }
  __device__ __forceinline__ static const W* bwd(const W* lds, int l, int nh) {
    if (PREC == 1) return lds + Bf16Layout{NetDims{H, nh, K, SEL}}.bwd_off(l);
    return lds + F32Layout{NetDims{H, nh, K, SEL}}.off(l);
  }
};

// SEL = 1: the network has the selection output and the loss is the blend
// of Sec. 4.2 (the BSDF pdf at each training direction is an input)
template <int H, int K, int PREC, int SEL>
__global__ __launch_bounds__(64 * train_waves<PREC>())
__attribute__((amdgpu_waves_per_eu(train_waves<PREC>() / 4, train_waves<PREC>() / 4)))
void train_kernel(TrainArgs a) {
  typedef TrainCfg<H, K, PREC, SEL> C;
  typedef typename C::M M;
  typedef typename C::S S;
  typedef TrainLds<H, K, PREC, SEL> TL;
  typedef typename TL::W W;
  constexpr int NHMAX = C::NHMAX, KQ = C::KQ, MTH = C::MTH, MTO = C::MTO, SP = C::SP, NW = C::NW, NV = C::NV;
  constexpr int CTH = C::CTH;
  extern __shared__ __align__(16) unsigned char smem[];
  W* lds = reinterpret_cast<W*>(smem);
  S* dst = reinterpret_cast<S*>(smem + a.lds_bytes);     // delta staging [RMAX][SP]
  S* hst = dst + C::RMAX * SP;                            // input staging [H][SP]
  // the second staging buffer (C::DB): delta [H][SP], input [H][SP]
  S* dstB = C::RMAX >= 2 * H ? dst + H * SP : hst + H * SP;
  S* hstB = C::RMAX >= 2 * H ? hst + H * SP : dstB + H * SP;
  lds_dma(lds, a.wpack, a.lds_bytes);
  lds_dma_wait();
  __syncthreads();

  const int lane = lane_id();
  const int g = lane >> 4, c = lane & 15;
  const int wave = threadIdx.x >> 6;
  const int nh = a.nh;
  const NetDims dims{H, nh, K, SEL};
  const float inv_b = 1.0f / (float)a.B;

  f32x4 acc0[C::O0::TPW];
  f32x4 acch[NHMAX - 1][C::OH::TPW];
  f32x4 acco[C::OO::TPW];
#pragma unroll
  for (int j = 0; j < C::O0::TPW; ++j) acc0[j] = zero4();
#pragma unroll
  for (int l = 0; l < NHMAX - 1; ++l)
#pragma unroll
    for (int j = 0; j < C::OH::TPW; ++j) acch[l][j] = zero4();
#pragma unroll
  for (int j = 0; j < C::OO::TPW; ++j) acco[j] = zero4();
  double loss_sum = 0.0, w_sum = 0.0;

  const int64_t n_tiles = (a.B + NV - 1) / NV;
  // this vertex's inputs, loaded one tile ahead so that their latency
  // overlaps the previous tile's work
  struct In {
    typename M::Input x;
    float dx, dy, dz, w, pfs;
  };
  auto load_in = [&](int64_t vv) {
    In r;
    const bool ok = vv < a.B;
    r.x = M::load_input(a.feat, a.ld, vv, ok, g);
    r.dx = 0.0f; r.dy = 0.0f; r.dz = 1.0f; r.w = 0.0f; r.pfs = 0.0f;
    if (ok) {
      r.dx = a.dir[vv]; r.dy = a.dir[a.ld + vv]; r.dz = a.dir[2 * a.ld + vv];
      r.w = a.w[vv];
      if (SEL == 1) r.pfs = a.bsdf_pdf[vv];
    }
    return r;
  };
  In nxt = load_in((int64_t)blockIdx.x * NV + wave * 16 + c);
  for (int64_t tile = blockIdx.x; tile < n_tiles; tile += gridDim.x) {
    const int64_t v = tile * NV + wave * 16 + c;
    const bool valid = v < a.B;
    const In cur = nxt;
    if (tile + gridDim.x < n_tiles) nxt = load_in((tile + gridDim.x) * NV + wave * 16 + c);
    // ---- forward (recomputed) ----
    const typename M::Input x = cur.x;
    // BF16 keeps the activations packed (hw, lastw), FP32 as floats (h, last)
    constexpr int NHF = PREC == 1 ? 1 : NHMAX, MTF = PREC == 1 ? 1 : MTH;
    constexpr int NHP = PREC == 1 ? NHMAX : 1, MTP_ = PREC == 1 ? MTH : 1;
    float h[NHF][MTF][4];
    float last[MTF][4];
    uint32_t hw[NHP][MTP_][2];
    uint32_t lastw[MTP_][2];
    float out[MTO][4];
    if constexpr (PREC == 1) Forward<H, K, PREC, NHMAX, SEL>::run_packed(lds, nh, x, hw, lastw, out, lane);
    else Forward<H, K, PREC, NHMAX, SEL>::run(lds, nh, x, h, last, out, lane);

    // ---- weighted NLL and its gradient w.r.t. the raw outputs ----
    float vx = cur.dx, vy = cur.dy, vz = cur.dz;
    const float wj = cur.w, pfs = cur.pfs;
    {
      const float inv = frsq(fmaf(vx, vx, fmaf(vy, vy, vz * vz)));
      vx *= inv; vy *= inv; vz *= inv;
    }
    const float gs = valid ? -wj * inv_b : 0.0f;   // dL/dlog q (of the log term)
    float dl[MTO][4];
    const float lterm = train_epilogue<KQ, MTO, SEL>(out, vx, vy, vz, gs, valid, a.eps, dl, pfs, a.mis_e, a.amul);
    if (valid && g == 0) {
      loss_sum += (double)wj * (double)(-lterm);
      w_sum += (double)wj;
    }

    // ---- MLP backward: output layer ----
    // BF16: activations and the deltas below the output layer travel as
    // packed words, the staging and the next dgrad's B operands alike, the
    // ReLU derivative a 16-bit mask on them (mask_rows); FP32 keeps floats
    float dh[MTH][4];
    uint32_t dw[MTH][2];
    {
      stage_rows<S, MTO, SP>(dst, dl, wave, lane);
      dgrad<H, K, PREC, MTO>(TL::bwd(lds, nh, nh), dl, dh, lane);
      if constexpr (PREC == 1) {
        stage_words<MTH, SP>(hst, lastw, wave, lane);
        pack_rows(dh, dw);
        mask_rows(dw, lastw);
      } else {
        stage_rows<S, MTH, SP>(hst, last, wave, lane);
#pragma unroll
        for (int mt = 0; mt < MTH; ++mt)
#pragma unroll
          for (int i = 0; i < 4; ++i) dh[mt][i] = last[mt][i] > 0.0f ? dh[mt][i] : 0.0f;
      }
      __syncthreads();
      wgrad_own<PREC, S, SP, MTO, CTH, NW, NV>(dst, hst, acco, wave, lane);
      __syncthreads();
    }
    // ---- hidden layers l = nh-1 .. 1 ----
#pragma unroll
    for (int l = NHMAX - 1; l >= 1; --l) {
      if (l >= nh) continue;
      // the buffers alternate with l (compile-time): a buffer's previous user
      // is two layers back, whose reads every wave finished before the last
      // layer's barrier (the output layer's before its second barrier)
      const bool alt = C::DB && ((NHMAX - 1 - l) & 1);   // folded once the loop unrolls
      S* const ds = alt ? dstB : dst;
      S* const hs = alt ? hstB : hst;
      float dn[MTH][4];
      if constexpr (PREC == 1) {
        stage_words<MTH, SP>(ds, dw, wave, lane);
        stage_words<MTH, SP>(hs, hw[l - 1], wave, lane);
        dgrad_words<H, MTH>(TL::bwd(lds, l, nh), dw, dn, lane);
        pack_rows(dn, dw);
        mask_rows(dw, hw[l - 1]);
      } else {
        const float (&prev)[MTH][4] = h[l - 1];
        stage_rows<S, MTH, SP>(ds, dh, wave, lane);
        stage_rows<S, MTH, SP>(hs, prev, wave, lane);
        dgrad<H, K, PREC, MTH>(TL::bwd(lds, l, nh), dh, dn, lane);
#pragma unroll
        for (int mt = 0; mt < MTH; ++mt)
#pragma unroll
          for (int i = 0; i < 4; ++i) dh[mt][i] = prev[mt][i] > 0.0f ? dn[mt][i] : 0.0f;
      }
      __syncthreads();
      wgrad_own<PREC, S, SP, MTH, CTH, NW, NV>(ds, hs, acch[l - 1], wave, lane);
      if constexpr (!C::DB) __syncthreads();
    }
    // ---- layer 0: input = features, constant one, zero padding ----
    {
      constexpr bool alt = C::DB && ((NHMAX - 1) & 1);
      S* const ds = alt ? dstB : dst;
      S* const hs = alt ? hstB : hst;
      if constexpr (PREC == 1) stage_words<MTH, SP>(ds, dw, wave, lane);
      else stage_rows<S, MTH, SP>(ds, dh, wave, lane);
      M::template stage_input<S, SP>(hs, x, wave, lane);
      __syncthreads();
      wgrad_own<PREC, S, SP, MTH, 1, NW, NV>(ds, hs, acc0, wave, lane);
      __syncthreads();   // the next tile's output layer writes both buffers' rows
    }
  }

  // ---- flush this workgroup's partial sums ----
  float* part = a.partial + (int64_t)blockIdx.x * a.n_weights;
  flush_own<MTH, 1, NW>(part, dims, 0, acc0, wave, lane);
#pragma unroll
  for (int l = 1; l < NHMAX; ++l)
    if (l < nh) flush_own<MTH, CTH, NW>(part, dims, l, acch[l - 1], wave, lane);
  flush_own<MTO, CTH, NW>(part, dims, nh, acco, wave, lane);

  // loss partials: wave reduction, then the waves in order
  __shared__ double red[NW][2];
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
    for (int w = 0; w < NW; ++w) { ls += red[w][0]; ws += red[w][1]; }
    a.loss_partial[2 * blockIdx.x] = ls;
    a.loss_partial[2 * blockIdx.x + 1] = ws;
  }
}

int train_workgroups(int64_t B, int num_cus) {
  int64_t t = (B + kWGV - 1) / kWGV;
  int cap = num_cus < kMaxTrainWG ? num_cus : kMaxTrainWG;
  return (int)(t < cap ? (t < 1 ? 1 : t) : cap);
}

template <int H, int K, int PREC, int SEL>
static hipError_t launch_train_s(const TrainArgs& a, int n_wg, hipStream_t st) {
  typedef TrainCfg<H, K, PREC, SEL> C;
  const size_t stage = sizeof(typename C::S) * C::stage_elems();
  const size_t shmem = (size_t)a.lds_bytes + stage;
  auto kern = train_kernel<H, K, PREC, SEL>;
  // the largest footprint of this network shape (4 hidden layers)
  const NetDims d{H, C::NHMAX, K, SEL};
  const size_t wmax = PREC == 1 ? (size_t)Bf16Layout{d}.total_elems() * 2 : (size_t)F32Layout{d}.total_elems() * 4;
  hipError_t e = set_max_lds_once<train_kernel<H, K, PREC, SEL>>(wmax + stage);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(kern, dim3(n_wg), dim3(64 * C::NW), shmem, st, a);
  return hipGetLastError();
}

template <int H, int K, int PREC>
static hipError_t launch_train_t(const TrainArgs& a, int n_wg, hipStream_t st) {
  return a.sel ? launch_train_s<H, K, PREC, 1>(a, n_wg, st) : launch_train_s<H, K, PREC, 0>(a, n_wg, st);
}

hipError_t launch_train(const TrainArgs& a, int H, int K, int prec, int n_wg, hipStream_t st) {
#define NASG_CASE(h, k, p) \
  if (H == h && K == k && prec == p) return launch_train_t<h, k, p>(a, n_wg, st);
  NASG_FOR_EACH_NET(NASG_CASE)
#undef NASG_CASE
  return hipErrorInvalidValue;
}

// ---------------------------------------------------------------- reduce ----
// grad[i] = sum over workgroups of partial[wg][i] in FP32, in a fixed
// pairwise order: thread group q (of 16) of a block loads workgroups q, q+16,
// q+32, ... for four consecutive weights with 16-byte loads (all of them in
// flight) and adds them as a binary tree; the 16 group sums are then added
// as a binary tree too. Eight levels for 256 partials: the rounding error is
// at most 8 u times the sum of the partials' magnitudes, and the result is
// bitwise reproducible. Each block also writes its FP64 sum of grad^2 (the
// gradient norm of the non-finite check); block 0 totals the FP64 loss
// partials (strided per thread, then a fixed tree). n_weights is a multiple
// of 4 for every compiled network (checked on the host); at most 256
// workgroup partials, 512 loss partials.
constexpr int kRedW = 64;   // weights per block
constexpr int kRedQ = 16;   // workgroup groups per block
constexpr int kRedT = kMaxTrainWG / kRedQ;   // partial rows per group

__global__ __launch_bounds__(256) void reduce_kernel(ReduceArgs a) {
  const int j = threadIdx.x & 15, q = threadIdx.x >> 4;
  const int64_t i0 = (int64_t)blockIdx.x * kRedW + 4 * j;
  float4 x[kRedT];
#pragma unroll
  for (int t = 0; t < kRedT; ++t) x[t] = float4{0.0f, 0.0f, 0.0f, 0.0f};
  if (i0 < a.n_weights) {
    const float* p = a.partial + i0;
#pragma unroll
    for (int t = 0; t < kRedT; ++t) {
      const int wg = q + kRedQ * t;
      if (wg < a.n_wg) x[t] = *reinterpret_cast<const float4*>(p + (int64_t)wg * a.n_weights);
    }
  }
#pragma unroll
  for (int h = kRedT / 2; h >= 1; h >>= 1)
#pragma unroll
    for (int t = 0; t < h; ++t) {
      x[t].x += x[t + h].x;
      x[t].y += x[t + h].y;
      x[t].z += x[t + h].z;
      x[t].w += x[t + h].w;
    }
  __shared__ float part[kRedQ][kRedW];
  __shared__ double red[256];
  __shared__ double red_w[256];
  part[q][4 * j + 0] = x[0].x;
  part[q][4 * j + 1] = x[0].y;
  part[q][4 * j + 2] = x[0].z;
  part[q][4 * j + 3] = x[0].w;
  __syncthreads();
  if (threadIdx.x < kRedW) {
    const int64_t i = (int64_t)blockIdx.x * kRedW + threadIdx.x;
    float g[kRedQ];
#pragma unroll
    for (int k = 0; k < kRedQ; ++k) g[k] = part[k][threadIdx.x];
#pragma unroll
    for (int h = kRedQ / 2; h >= 1; h >>= 1)
#pragma unroll
      for (int k = 0; k < h; ++k) g[k] += g[k + h];
    const float gf = g[0];
    if (i < a.n_weights) a.grad[i] = gf;
    red[threadIdx.x] = i < a.n_weights ? (double)gf * (double)gf : 0.0;
  }
  __syncthreads();
  for (int k = kRedW / 2; k >= 1; k >>= 1) {
    if ((int)threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
    __syncthreads();
  }
  if (threadIdx.x == 0) a.norm_partial[blockIdx.x] = red[0];
  if (blockIdx.x == 0) {
    __syncthreads();
    double ls = 0.0, ws = 0.0;
    for (int wg = (int)threadIdx.x; wg < a.n_loss; wg += 256) {
      ls += a.loss_partial[2 * wg];
      ws += a.loss_partial[2 * wg + 1];
    }
    red[threadIdx.x] = ls;
    red_w[threadIdx.x] = ws;
    __syncthreads();
    for (int k = 128; k >= 1; k >>= 1) {
      if ((int)threadIdx.x < k) {
        red[threadIdx.x] += red[threadIdx.x + k];
        red_w[threadIdx.x] += red_w[threadIdx.x + k];
      }
      __syncthreads();
    }
    if (threadIdx.x == 0) {
      a.stats[0] = red[0] / (double)a.B;
      a.stats[1] = red_w[0];
      a.stats[3] = red[0];
      *a.step_snapshot = *a.step;
    }
  }
}

int reduce_blocks(int64_t n_weights) { return (int)((n_weights + kRedW - 1) / kRedW); }

hipError_t launch_reduce(const ReduceArgs& a, int n_blocks, hipStream_t st) {
  hipLaunchKernelGGL(reduce_kernel, dim3(n_blocks), dim3(256), 0, st, a);
  return hipGetLastError();
}

// ------------------------------------------------------------------ adam ----
__device__ __forceinline__ void locate(const NetDims& d, int64_t i, int& l, int& n, int& k) {
  l = 0;
  for (int t = 1; t <= d.NH; ++t)
    if (i >= d.canon_off(t)) l = t;
  const int64_t r = i - d.canon_off(l);
  n = (int)(r / d.cols(l));
  k = (int)(r % d.cols(l));
}

__device__ __forceinline__ void write_packed(const AdamArgs& a, const NetDims& d, int64_t i, float w) {
  int l, n, k;
  locate(d, i, l, n, k);
  if (a.prec == 1) {
    Bf16Layout Lt{d};
    __bf16* p = reinterpret_cast<__bf16*>(a.wpack);
    const __bf16 b = (__bf16)w;
    p[bf16_fwd_pos(Lt, l, n, k)] = b;
    if (l >= 1) p[bf16_bwd_pos(Lt, l, n, k)] = b;
  } else {
    F32Layout Lt{d};
    reinterpret_cast<float*>(a.wpack)[f32_pos(Lt, l, n, k)] = w;
  }
}

// Kingma and Ba's Adam, bias-corrected, no weight decay; skipped (weights,
// moments and step unchanged, flag bit 0 set) if the loss or the gradient norm
// is not finite. A thread's first element is loaded before the gradient norm
// is summed, so the two memory latencies overlap; the bias corrections are
// computed once per block, by two threads, during the norm sum.
__global__ __launch_bounds__(256) void adam_kernel(AdamArgs a) {
  __shared__ double red[256];
  __shared__ float corr[2];
  const int64_t i0 = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int64_t stride = (int64_t)gridDim.x * 256;
  float g0 = 0.0f, m0 = 0.0f, v0 = 0.0f, w0 = 0.0f;
  if (i0 < a.n_weights) {
    g0 = a.grad[i0];
    m0 = a.m[i0];
    v0 = a.v[i0];
    w0 = a.w[i0];
  }
  const int64_t t0 = *a.step_snapshot;
  // bias corrections of step t0 + 1 (used only if the step is taken),
  // computed while the other threads sum the norm partials
  if (threadIdx.x == 0) corr[0] = a.lr / (float)(1.0 - pow((double)a.beta1, (double)(t0 + 1)));   // lr / (1 - beta1^t)
  if (threadIdx.x == 64) corr[1] = (float)sqrt(1.0 - pow((double)a.beta2, (double)(t0 + 1)));     // sqrt(1 - beta2^t)
  double s = 0.0;
  for (int j = threadIdx.x; j < a.n_norm; j += 256) s += a.norm_partial[j];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int k = 128; k >= 1; k >>= 1) {
    if ((int)threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
    __syncthreads();
  }
  const double nsq = red[0];
  const double loss = a.stats[0];
  const bool skip = !isfinite(loss) || !isfinite(nsq);
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    a.stats[2] = sqrt(nsq);
    *a.flags = skip ? 1u : 0u;
    *a.step = skip ? t0 : t0 + 1;
  }
  if (skip) return;
  const float step_size = corr[0], bc2_sqrt = corr[1];
  const NetDims d{a.H, a.NH, a.K, a.S, a.E};
  for (int64_t i = i0; i < a.n_weights; i += stride) {
    if (i != i0) {
      g0 = a.grad[i];
      m0 = a.m[i];
      v0 = a.v[i];
      w0 = a.w[i];
    }
    const float m = fmaf(a.beta1, m0, (1.0f - a.beta1) * g0);
    const float v = fmaf(a.beta2, v0, (1.0f - a.beta2) * g0 * g0);
    const float denom = sqrtf(v) / bc2_sqrt + a.adam_eps;
    const float w = w0 - step_size * (m / denom);
    a.m[i] = m;
    a.v[i] = v;
    a.w[i] = w;
    write_packed(a, d, i, w);
  }
}

hipError_t launch_adam(const AdamArgs& a, hipStream_t st) {
  int grid = (int)((a.n_weights + 255) / 256);
  if (grid > 1024) grid = 1024;
  hipLaunchKernelGGL(adam_kernel, dim3(grid), dim3(256), 0, st, a);
  return hipGetLastError();
}

// ------------------------------------------------------------------ pack ----
__global__ __launch_bounds__(256) void pack_kernel(const float* __restrict__ w, void* wpack, NetDims d, int prec,
                                                   int64_t n_elems) {
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < n_elems; e += (int64_t)gridDim.x * 256) {
    int l, n, k;
    if (prec == 1) bf16_source(Bf16Layout{d}, e, l, n, k);
    else f32_source(F32Layout{d}, e, l, n, k);
    float x = k < 0 ? 0.0f : w[d.canon_off(l) + (int64_t)n * d.cols(l) + k];
    if (prec == 1) reinterpret_cast<__bf16*>(wpack)[e] = (__bf16)x;
    else reinterpret_cast<float*>(wpack)[e] = x;
  }
}

hipError_t launch_pack(const float* w, void* wpack, const NetDims& d, int prec, hipStream_t st) {
  int64_t n = prec == 1 ? Bf16Layout{d}.total_elems() : F32Layout{d}.total_elems();
  int grid = (int)((n + 255) / 256);
  if (grid > 1024) grid = 1024;
  hipLaunchKernelGGL(pack_kernel, dim3(grid), dim3(256), 0, st, w, wpack, d, prec, n);
  return hipGetLastError();
}

__global__ __launch_bounds__(256) void fill_kernel(uint32_t* p, int64_t n, uint32_t value) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) p[i] = value;
}

hipError_t launch_fill(void* p, int64_t n_words, uint32_t value, hipStream_t st) {
  if (n_words <= 0) return hipSuccess;
  int grid = (int)((n_words + 255) / 256);
  if (grid > 1024) grid = 1024;
  hipLaunchKernelGGL(fill_kernel, dim3(grid), dim3(256), 0, st, reinterpret_cast<uint32_t*>(p), n_words, value);
  return hipGetLastError();
}

}  // namespace nasg
