// Large networks (hidden 128, K = 32, BF16): query and training.
//
// The BF16 forward fragments of this network take 164 KiB and the backward
// ones another 160 KiB, more than one CU's 160 KiB of LDS, and its 83,200
// FP32 weight-gradient accumulators would need ~325 registers per lane in
// each of four waves. So:
// * weights stream through one 64 KiB LDS buffer a layer at a time (the
//   workgroup moves through the layers together, 64 vertices per tile);
// * training runs as three kernels over the batch: gradout_kernel does the
//   forward and the weighted-NLL / NASG backward (Sec. 4.2) and keeps only
//   dL/d(raw outputs) as BF16 (512 B per sample, the operand image the
//   backward reads); bwd_kernel<0> and bwd_kernel<1> each recompute the
//   forward, run dgrad and accumulate the weight gradient of one group of
//   layers (the output and last hidden layer; the rest) in registers.
//   Activations are recomputed, never stored.
#include <type_traits>

#include "epilogue.hpp"
#include "kernels.hpp"
#include "mlp.hpp"

namespace nasg {

constexpr int kLargeWGV = 64;   // vertices per workgroup tile

template <int H, int K>
struct LargeNet {
  typedef Mlp<H, K, 1> M;
  static constexpr int NH = 4;
  static constexpr int MTH = H / 16, MTO = K / 2, KQ = K / 4;
  static constexpr int KBO = K / 4;                         // 32-wide blocks over the 8K outputs
  static constexpr int BUF_ELEMS = (8 * K * H > H * H) ? 8 * K * H : H * H;   // largest layer
  static constexpr int SP = kLargeWGV + 8;                  // staging pitch (bf16)
  static constexpr int RMAX = 8 * K;

  // Replace the LDS weight buffer's contents (whole workgroup).
  __device__ static void wstage(__bf16* buf, const __bf16* src, int elems) {
    __syncthreads();
    block_copy_to_lds(buf, src, elems * 2);
    __syncthreads();
  }

  __device__ static void forward(const __bf16* wg, __bf16* buf, const typename M::Input& x,
                                 float (&h)[NH][MTH][4], float (&out)[MTO][4], int lane) {
    const Bf16Layout Lt{NetDims{H, NH, K}};
    wstage(buf, wg + Lt.fwd_off(0), H * 16);
    M::layer0(buf, x, h[0], lane);
#pragma unroll
    for (int l = 1; l < NH; ++l) {
      wstage(buf, wg + Lt.fwd_off(l), H * H);
      float y[MTH][4];
      M::template gemm<MTH>(buf, h[l - 1], y, lane);
#pragma unroll
      for (int mt = 0; mt < MTH; ++mt)
#pragma unroll
        for (int i = 0; i < 4; ++i) h[l][mt][i] = relu(y[mt][i]);
    }
    wstage(buf, wg + Lt.fwd_off(NH), 8 * K * H);
    M::template gemm<MTO>(buf, h[NH - 1], out, lane);
  }
};

// ---------------------------------------------------------------- query ----
template <int H, int K, int MODE>
__global__ __launch_bounds__(256) void large_query_kernel(QueryArgs a) {
  typedef LargeNet<H, K> N;
  typedef typename N::M M;
  constexpr int KQ = N::KQ;
  extern __shared__ __align__(16) unsigned char smem[];
  __bf16* buf = reinterpret_cast<__bf16*>(smem);
  const __bf16* wg = reinterpret_cast<const __bf16*>(a.wpack);
  const int lane = lane_id();
  const int g = lane >> 4, c = lane & 15;
  const int wave = threadIdx.x >> 6;
  const int64_t n_tiles = (a.B + kLargeWGV - 1) / kLargeWGV;
  for (int64_t tile = blockIdx.x; tile < n_tiles; tile += gridDim.x) {
    const int64_t v = tile * kLargeWGV + wave * 16 + c;
    const bool valid = v < a.B;
    typename M::Input x = M::load_input(a.feat, a.ld, v, valid, g);
    float h[N::NH][N::MTH][4];
    float out[N::MTO][4];
    N::forward(wg, buf, x, h, out, lane);
    if (MODE == 1) {
      if (valid) {
#pragma unroll
        for (int t = 0; t < 2 * K; ++t) {
          const int p = t / KQ, k = g * KQ + t % KQ;
          a.raw_out[(int64_t)(p * K + k) * a.ld + v] = out[t >> 2][t & 3];
        }
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
    const float logq = query_epilogue<KQ, N::MTO>(out, xi_sel, xi0, xi1, xi2, a.eps, g, c, lb, vx, vy, vz);
    if (valid && g == 0) {
      a.dir_out[v] = vx;
      a.dir_out[a.ld + v] = vy;
      a.dir_out[2 * a.ld + v] = vz;
      a.pdf_out[v] = fexp(logq);
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
template <int H, int K>
__global__ __launch_bounds__(256) void gradout_kernel(LargeTrainArgs a) {
  typedef LargeNet<H, K> N;
  typedef typename N::M M;
  constexpr int KQ = N::KQ, MTO = N::MTO, KBO = N::KBO;
  extern __shared__ __align__(16) unsigned char smem[];
  __bf16* buf = reinterpret_cast<__bf16*>(smem);
  const __bf16* wg = reinterpret_cast<const __bf16*>(a.wpack);
  const int lane = lane_id();
  const int g = lane >> 4, c = lane & 15;
  const int wave = threadIdx.x >> 6;
  const float inv_b = 1.0f / (float)a.B;
  double loss_sum = 0.0, w_sum = 0.0;
  const int64_t n_tiles = (a.B + kLargeWGV - 1) / kLargeWGV;
  for (int64_t tile = blockIdx.x; tile < n_tiles; tile += gridDim.x) {
    const int64_t v = tile * kLargeWGV + wave * 16 + c;
    const bool valid = v < a.B;
    typename M::Input x = M::load_input(a.feat, a.ld, v, valid, g);
    float h[N::NH][N::MTH][4];
    float out[MTO][4];
    N::forward(wg, buf, x, h, out, lane);
    float vx = 0.0f, vy = 0.0f, vz = 1.0f, wj = 0.0f;
    if (valid) {
      vx = a.dir[v]; vy = a.dir[a.ld + v]; vz = a.dir[2 * a.ld + v];
      wj = a.w[v];
      const float inv = frsq(fmaf(vx, vx, fmaf(vy, vy, vz * vz)));
      vx *= inv; vy *= inv; vz *= inv;
    }
    const float gs = valid ? -wj * inv_b : 0.0f;
    float dl[MTO][4];
    const float logq = train_epilogue<KQ, MTO>(out, vx, vy, vz, gs, valid, a.eps, dl);
    if (valid && g == 0) {
      loss_sum += (double)wj * (double)(-logq);
      w_sum += (double)wj;
    }
    // the output layer's dgrad B operands, one 16-byte slot per lane and block
    bf16x8* dst = reinterpret_cast<bf16x8*>(a.dout) + ((tile * 4 + wave) * KBO) * 64 + lane;
#pragma unroll
    for (int kb = 0; kb < KBO; ++kb) {
      bf16x8 b;
#pragma unroll
      for (int j = 0; j < 8; ++j) b[j] = (__bf16)dl[2 * kb + (j >> 2)][j & 3];
      dst[kb * 64] = b;
    }
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

// ------------------------------------------------------------- backward ----
// dgrad with W_l^T fragments in LDS (contraction over RT row tiles of layer l)
template <int H, int RT>
__device__ __forceinline__ void dgrad_bf16(const __bf16* wl, const float (&dl)[RT][4], float (&dp)[H / 16][4],
                                           int lane) {
  constexpr int KB = RT / 2;
  const bf16x8* frag = reinterpret_cast<const bf16x8*>(wl);
  bf16x8 b[KB];
#pragma unroll
  for (int kb = 0; kb < KB; ++kb)
#pragma unroll
    for (int j = 0; j < 8; ++j) b[kb][j] = (__bf16)dl[2 * kb + (j >> 2)][j & 3];
#pragma unroll
  for (int mt = 0; mt < H / 16; ++mt) {
    f32x4 acc = zero4();
#pragma unroll
    for (int kb = 0; kb < KB; ++kb) acc = mfma_bf16_32(frag[(mt * KB + kb) * 64 + lane], b[kb], acc);
#pragma unroll
    for (int i = 0; i < 4; ++i) dp[mt][i] = acc[i];
  }
}

template <int RT, int SP>
__device__ __forceinline__ void stage_bf16(__bf16* st, const float (&x)[RT][4], int wave, int lane) {
  const int g = lane >> 4, c = lane & 15;
#pragma unroll
  for (int mt = 0; mt < RT; ++mt)
#pragma unroll
    for (int i = 0; i < 4; ++i) st[(mt * 16 + 4 * g + i) * SP + wave * 16 + c] = (__bf16)x[mt][i];
}

// acc[r][ct] += D[row tile rt[r]][64 staged vertices] * Hs[col tile ct][...]^T
template <int SP, int NR, int NC>
__device__ __forceinline__ void wgrad_bf16(const __bf16* dst, const __bf16* hst, const int (&rt)[NR], int nrt,
                                           f32x4 (&acc)[NR][NC], int lane) {
  const int g = lane >> 4, c = lane & 15;
#pragma unroll
  for (int vb = 0; vb < kLargeWGV / 32; ++vb) {
    bf16x8 hb[NC];
#pragma unroll
    for (int ct = 0; ct < NC; ++ct)
      hb[ct] = *reinterpret_cast<const bf16x8*>(hst + (ct * 16 + c) * SP + vb * 32 + 8 * g);
#pragma unroll
    for (int r = 0; r < NR; ++r) {
      if (r < nrt) {
        const bf16x8 da = *reinterpret_cast<const bf16x8*>(dst + (rt[r] * 16 + c) * SP + vb * 32 + 8 * g);
#pragma unroll
        for (int ct = 0; ct < NC; ++ct) acc[r][ct] = mfma_bf16_32(da, hb[ct], acc[r][ct]);
      }
    }
  }
}

template <int NR, int NC>
__device__ __forceinline__ void flush_bf16(float* part, const NetDims& d, int l, const int (&rt)[NR], int nrt,
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
        part[off + (int64_t)n * cols + k] = acc[r][ct][i];
      }
    }
  }
}

// Hidden activations kept as bfloat16 pairs: the backward uses them only as
// BF16 staging operands and as ReLU masks (h > 0).
template <int MTH>
struct PackedAct {
  uint32_t p[MTH][2];
  __device__ void pack(const float (&h)[MTH][4]) {
#pragma unroll
    for (int mt = 0; mt < MTH; ++mt)
#pragma unroll
      for (int k = 0; k < 2; ++k) {
        const uint32_t lo = __builtin_bit_cast(unsigned short, (__bf16)h[mt][2 * k]);
        const uint32_t hi = __builtin_bit_cast(unsigned short, (__bf16)h[mt][2 * k + 1]);
        p[mt][k] = lo | (hi << 16);
      }
  }
  __device__ float get(int mt, int i) const {
    const uint32_t w = p[mt][i >> 1];
    return __uint_as_float((i & 1) ? (w & 0xffff0000u) : (w << 16));
  }
};

template <int MTH>
__device__ __forceinline__ void mask_relu(float (&d)[MTH][4], const PackedAct<MTH>& h) {
#pragma unroll
  for (int mt = 0; mt < MTH; ++mt)
#pragma unroll
    for (int i = 0; i < 4; ++i) d[mt][i] = h.get(mt, i) > 0.0f ? d[mt][i] : 0.0f;
}

template <int MTH, int SP>
__device__ __forceinline__ void stage_packed(__bf16* st, const PackedAct<MTH>& h, int wave, int lane) {
  const int g = lane >> 4, c = lane & 15;
#pragma unroll
  for (int mt = 0; mt < MTH; ++mt)
#pragma unroll
    for (int i = 0; i < 4; ++i) st[(mt * 16 + 4 * g + i) * SP + wave * 16 + c] = (__bf16)h.get(mt, i);
}

// GROUP 0: weight gradients of the output layer and the last hidden layer;
// GROUP 1: of hidden layers NH-2 .. 1 and layer 0.
template <int H, int K, int GROUP>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(1, 1)))
void bwd_kernel(LargeTrainArgs a) {
  typedef LargeNet<H, K> N;
  typedef typename N::M M;
  constexpr int NH = N::NH, MTH = N::MTH, MTO = N::MTO, KBO = N::KBO, SP = N::SP;
  constexpr int RTW_H = (MTH + 3) / 4, RTW_O = (MTO + 3) / 4, CTH = H / 16;
  extern __shared__ __align__(16) unsigned char smem[];
  __bf16* buf = reinterpret_cast<__bf16*>(smem);
  __bf16* dst = buf + N::BUF_ELEMS;
  __bf16* hst = dst + N::RMAX * SP;
  const __bf16* wg = reinterpret_cast<const __bf16*>(a.wpack);
  const Bf16Layout Lt{NetDims{H, NH, K}};
  const NetDims dims{H, NH, K};
  const int lane = lane_id();
  const int g = lane >> 4, c = lane & 15;
  const int wave = threadIdx.x >> 6;

  int rt_h[RTW_H], rt_o[RTW_O];
  int nrt_h = 0, nrt_o = 0;
#pragma unroll
  for (int r = 0; r < RTW_H; ++r) { rt_h[r] = wave + 4 * r; if (rt_h[r] < MTH) nrt_h = r + 1; }
#pragma unroll
  for (int r = 0; r < RTW_O; ++r) { rt_o[r] = wave + 4 * r; if (rt_o[r] < MTO) nrt_o = r + 1; }

  // GROUP 0: accA = output layer [RTW_O][CTH], accB = layer NH-1 [RTW_H][CTH]
  // GROUP 1: accA = layers NH-2..1 [NH-2][RTW_H][CTH], accB = layer 0 [RTW_H][1]
  f32x4 accO[GROUP == 0 ? RTW_O : 1][CTH];
  f32x4 accT[RTW_H][CTH];
  f32x4 accM[GROUP == 1 ? NH - 2 : 1][RTW_H][CTH];
  f32x4 acc0[RTW_H][1];
#pragma unroll
  for (int r = 0; r < RTW_H; ++r) {
    acc0[r][0] = zero4();
#pragma unroll
    for (int ct = 0; ct < CTH; ++ct) {
      accT[r][ct] = zero4();
#pragma unroll
      for (int l = 0; l < (GROUP == 1 ? NH - 2 : 1); ++l) accM[l][r][ct] = zero4();
    }
  }
#pragma unroll
  for (int r = 0; r < (GROUP == 0 ? RTW_O : 1); ++r)
#pragma unroll
    for (int ct = 0; ct < CTH; ++ct) accO[r][ct] = zero4();

  const int64_t n_tiles = (a.B + kLargeWGV - 1) / kLargeWGV;
  for (int64_t tile = blockIdx.x; tile < n_tiles; tile += gridDim.x) {
    const int64_t v = tile * kLargeWGV + wave * 16 + c;
    const bool valid = v < a.B;
    typename M::Input x = M::load_input(a.feat, a.ld, v, valid, g);
    PackedAct<MTH> hp[NH];
    {
      float h[NH][MTH][4];
      float out[MTO][4];
      N::forward(wg, buf, x, h, out, lane);
#pragma unroll
      for (int l = 0; l < NH; ++l) hp[l].pack(h[l]);
    }
    // dL/d(raw outputs) from gradout_kernel, back in accumulator layout
    float dl[MTO][4];
    {
      const bf16x8* src = reinterpret_cast<const bf16x8*>(a.dout) + ((tile * 4 + wave) * KBO) * 64 + lane;
#pragma unroll
      for (int kb = 0; kb < KBO; ++kb) {
        const bf16x8 b = src[kb * 64];
#pragma unroll
        for (int j = 0; j < 8; ++j) dl[2 * kb + (j >> 2)][j & 3] = (float)b[j];
      }
    }
    float dh[MTH][4];
    if constexpr (GROUP == 0) {
      stage_bf16<MTO, SP>(dst, dl, wave, lane);
      stage_packed<MTH, SP>(hst, hp[NH - 1], wave, lane);
      N::wstage(buf, wg + Lt.bwd_off(NH), 8 * K * H);   // also publishes the staging
      dgrad_bf16<H, MTO>(buf, dl, dh, lane);
      mask_relu<MTH>(dh, hp[NH - 1]);
      wgrad_bf16<SP, RTW_O, CTH>(dst, hst, rt_o, nrt_o, accO, lane);
      __syncthreads();
      stage_bf16<MTH, SP>(dst, dh, wave, lane);
      stage_packed<MTH, SP>(hst, hp[NH - 2], wave, lane);
      __syncthreads();
      wgrad_bf16<SP, RTW_H, CTH>(dst, hst, rt_h, nrt_h, accT, lane);
      __syncthreads();
    } else {
      N::wstage(buf, wg + Lt.bwd_off(NH), 8 * K * H);
      dgrad_bf16<H, MTO>(buf, dl, dh, lane);
      mask_relu<MTH>(dh, hp[NH - 1]);
      float d2[MTH][4];
      N::wstage(buf, wg + Lt.bwd_off(NH - 1), H * H);
      dgrad_bf16<H, MTH>(buf, dh, d2, lane);
      mask_relu<MTH>(d2, hp[NH - 2]);
#pragma unroll
      for (int l = NH - 2; l >= 1; --l) {
        stage_bf16<MTH, SP>(dst, d2, wave, lane);
        stage_packed<MTH, SP>(hst, hp[l - 1], wave, lane);
        N::wstage(buf, wg + Lt.bwd_off(l), H * H);
        float dn[MTH][4];
        dgrad_bf16<H, MTH>(buf, d2, dn, lane);
        mask_relu<MTH>(dn, hp[l - 1]);
        wgrad_bf16<SP, RTW_H, CTH>(dst, hst, rt_h, nrt_h, accM[l - 1], lane);
        __syncthreads();
#pragma unroll
        for (int mt = 0; mt < MTH; ++mt)
#pragma unroll
          for (int i = 0; i < 4; ++i) d2[mt][i] = dn[mt][i];
      }
      stage_bf16<MTH, SP>(dst, d2, wave, lane);
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int k = 4 * g + j;
        float xv = 0.0f;
        if (valid) {
          if (k < kInFeatures) xv = a.feat[(int64_t)k * a.ld + v];
          else if (k == kInFeatures) xv = 1.0f;
        }
        hst[k * SP + wave * 16 + c] = (__bf16)xv;
      }
      __syncthreads();
      wgrad_bf16<SP, RTW_H, 1>(dst, hst, rt_h, nrt_h, acc0, lane);
      __syncthreads();
    }
  }

  float* part = a.partial + (int64_t)blockIdx.x * a.n_weights;
  if constexpr (GROUP == 0) {
    flush_bf16<RTW_O, CTH>(part, dims, NH, rt_o, nrt_o, accO, lane);
    flush_bf16<RTW_H, CTH>(part, dims, NH - 1, rt_h, nrt_h, accT, lane);
  } else {
#pragma unroll
    for (int l = 1; l <= NH - 2; ++l) flush_bf16<RTW_H, CTH>(part, dims, l, rt_h, nrt_h, accM[l - 1], lane);
    flush_bf16<RTW_H, 1>(part, dims, 0, rt_h, nrt_h, acc0, lane);
  }
}

// ------------------------------------------------------------ launchers ----
template <typename Kern>
static hipError_t set_lds(Kern kern, size_t bytes) {
  return hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

template <int H, int K>
static hipError_t launch_large_query_t(const QueryArgs& a, int mode, hipStream_t st) {
  typedef LargeNet<H, K> N;
  const size_t shmem = (size_t)N::BUF_ELEMS * 2;
  auto kern = mode == 0 ? large_query_kernel<H, K, 0> : large_query_kernel<H, K, 1>;
  static bool attr[2] = {false, false};
  if (!attr[mode]) {
    hipError_t e = set_lds(kern, shmem);
    if (e != hipSuccess) return e;
    attr[mode] = true;
  }
  const int64_t n_tiles = (a.B + kLargeWGV - 1) / kLargeWGV;
  const int64_t cap = 2LL * a.num_cus;
  const int grid = (int)(n_tiles < cap ? (n_tiles < 1 ? 1 : n_tiles) : cap);
  hipLaunchKernelGGL(kern, dim3(grid), dim3(256), shmem, st, a);
  return hipGetLastError();
}

template <int H, int K>
static hipError_t launch_large_train_t(const LargeTrainArgs& a, int n_wg, hipStream_t st) {
  typedef LargeNet<H, K> N;
  const size_t sh_fwd = (size_t)N::BUF_ELEMS * 2;
  const size_t sh_bwd = sh_fwd + (size_t)(N::RMAX + H) * N::SP * 2;
  static bool attr = false;
  if (!attr) {
    auto k_grad = gradout_kernel<H, K>;
    auto k_bwd0 = bwd_kernel<H, K, 0>;
    auto k_bwd1 = bwd_kernel<H, K, 1>;
    hipError_t e = set_lds(k_grad, sh_fwd);
    if (e == hipSuccess) e = set_lds(k_bwd0, sh_bwd);
    if (e == hipSuccess) e = set_lds(k_bwd1, sh_bwd);
    if (e != hipSuccess) return e;
    attr = true;
  }
  auto k_grad = gradout_kernel<H, K>;
  auto k_bwd0 = bwd_kernel<H, K, 0>;
  auto k_bwd1 = bwd_kernel<H, K, 1>;
  hipLaunchKernelGGL(k_grad, dim3(n_wg), dim3(256), sh_fwd, st, a);
  hipLaunchKernelGGL(k_bwd0, dim3(n_wg), dim3(256), sh_bwd, st, a);
  hipLaunchKernelGGL(k_bwd1, dim3(n_wg), dim3(256), sh_bwd, st, a);
  return hipGetLastError();
}

hipError_t launch_large_query(const QueryArgs& a, int H, int K, int mode, hipStream_t st) {
  if (H == 128 && K == 32) return launch_large_query_t<128, 32>(a, mode, st);
  return hipErrorInvalidValue;
}

hipError_t launch_large_train(const LargeTrainArgs& a, int H, int K, int n_wg, hipStream_t st) {
  if (H == 128 && K == 32) return launch_large_train_t<128, 32>(a, n_wg, st);
  return hipErrorInvalidValue;
}

}  // namespace nasg
