// Fused guiding query: MLP forward on MFMA (weights LDS-resident), NASG
// decode, inverse-CDF lobe choice, direct sampling (App. C) and the mixture
// pdf at the sampled direction (Sec. 3.1), in 16-vertex blocks.
//
// Lane (g, c) of a wave owns vertex c of a 16-vertex block and lobes
// g*K/4 .. g*K/4 + K/4 - 1 of that vertex, so reductions over lobes are a
// within-lane loop plus two cross-lane steps (xor 16, xor 32). A wave takes
// one block per pass, four (one sample per lane: query_four_blocks) or two
// (the paper's network), with the multi-block passes' inputs staged in LDS
// one pass ahead.
#include <type_traits>

#include "epilogue.hpp"
#include "kernels.hpp"
#include "mlp.hpp"

namespace nasg {

// The hidden-64 BF16 networks' queries sample one vertex per lane (four
// blocks per wave pass; the four blocks' lobes take 144 registers, so two
// waves per SIMD). Their FP32 queries keep one block per pass and three
// waves per SIMD (the four blocks' lobes and the FP32 forward do not fit two
// waves' registers); the raw forwards run one wave per SIMD; the hidden-128
// network two, its 132 KiB of forward weights leaving room for one
// workgroup per CU.
constexpr bool query_four(int H, int K, int MODE, int PREC) { return H == 64 && K != 8 && MODE == 0 && PREC == 1; }
// dynamic LDS of a query launch: the weights, plus the four-block kernels'
// two input staging buffers per wave
constexpr size_t query_dynamic_lds(int weight_bytes, bool four, int nb, int nw) {
  return (size_t)weight_bytes +
         (four ? (size_t)nw * 2 * (kInFeatures + 4) * 64 * sizeof(float)
               : (nb == 2 ? (size_t)nw * 2 * (kInFeatures + 4) * 32 * sizeof(float) : 0));
}
constexpr int query_waves_per_eu(int H, int K, int MODE, int PREC) {
  return H == 64 ? (MODE == 0 ? (query_four(H, K, MODE, PREC) ? 2 : 3) : 1) : 2;
}

// Records of one 16-vertex block's lobes (optional output of a query).
template <int KQ>
__device__ __forceinline__ void store_records(const QueryArgs& a, const Lobe (&lb)[KQ], int64_t v, int g) {
  constexpr int K = 4 * KQ;
  float* base = a.rec_out + (v / kRecTile) * 9 * K * kRecTile + (v % kRecTile);
#pragma unroll
  for (int q = 0; q < KQ; ++q) {
    const int k = g * KQ + q;
    const float vals[9] = {lb[q].zx, lb[q].zy, lb[q].zz, lb[q].xx, lb[q].xy, lb[q].xz, lb[q].lam, lb[q].a, lb[q].logc};
#pragma unroll
    for (int p = 0; p < 9; ++p) base[(p * K + k) * kRecTile] = vals[p];
  }
}

// The rest of a query for one 16-vertex block from its raw outputs: decode,
// choose a lobe, sample, evaluate the pdf and store (MODE 0), or store the
// raw outputs in canonical row order (MODE 1).
template <int K, int MODE, int S, int MTO>
__device__ __forceinline__ void finish_block(const QueryArgs& a, const float (&out)[MTO][4], int64_t v, int g,
                                             int c, const float* xi, int64_t xi_ld, int64_t xi_col) {
  constexpr int KQ = K / 4;
  const bool valid = v < a.B;
  if (MODE == 1) {
    // accumulator t of lane group g is parameter t / KQ of lobe g*KQ + t % KQ
    if (valid) {
#pragma unroll
      for (int t = 0; t < 2 * K; ++t) {
        int p = t / KQ, k = g * KQ + t % KQ;
        a.raw_out[(int64_t)(p * K + k) * a.ld + v] = out[t >> 2][t & 3];
      }
      if (S == 1 && g == 0) a.raw_out[(int64_t)(8 * K) * a.ld + v] = out[MTO - 1][0];
    }
    return;
  }
  float xi_sel = 0.0f, xi0 = 0.0f, xi1 = 0.0f, xi2 = 0.0f;
  if (valid) {
    xi_sel = xi[xi_col];
    xi0 = xi[xi_ld + xi_col];
    xi1 = xi[2 * xi_ld + xi_col];
    xi2 = xi[3 * xi_ld + xi_col];
  }
  Lobe lb[KQ];
  float vx, vy, vz;
  const float logq = query_epilogue<KQ, MTO>(out, xi_sel, xi0, xi1, xi2, a.eps, g, c, lb, vx, vy, vz, a.amul);

  if (valid && g == 0) {
    a.dir_out[v] = vx;
    a.dir_out[a.ld + v] = vy;
    a.dir_out[2 * a.ld + v] = vz;
    a.pdf_out[v] = fexp(logq);
    // selection probability c = sigmoid(o[8K]) (Tab. "decoding")
    if (S == 1 && a.sel_out != nullptr) a.sel_out[v] = frcp(1.0f + fexp(-out[MTO - 1][0]));
  }
  if (a.rec_out != nullptr && valid) store_records<KQ>(a, lb, v, g);
}

// Inputs of one 64-vertex pass staged in LDS: the 9 feature rows and the 4
// uniform rows, 64 floats each (lane i of a row = vertex 64 tile + i).
constexpr int kPassRows = kInFeatures + 4;
constexpr int kPassStage = kPassRows * 64;   // floats per wave and buffer

// Direct-to-LDS copies of a pass's inputs (13 wave instructions, no
// registers). Lanes past the batch read vertex B - 1 instead (in bounds;
// their values are never used), so that every wave issues the same number of
// copies and s_waitcnt can count them.
__device__ __forceinline__ void stage_pass(const QueryArgs& a, int64_t tile, float* buf, int lane) {
  int64_t v = tile * (4 * kTileV) + lane;
  v = v < a.B ? v : a.B - 1;
#pragma unroll
  for (int k = 0; k < kInFeatures; ++k)
    __builtin_amdgcn_global_load_lds(a.feat + k * a.ld + v, (__attribute__((address_space(3))) void*)(buf + k * 64), 4,
                                     0, 0);
#pragma unroll
  for (int k = 0; k < 4; ++k)
    __builtin_amdgcn_global_load_lds(a.xi + k * a.ld + v,
                                     (__attribute__((address_space(3))) void*)(buf + (kInFeatures + k) * 64), 4, 0, 0);
}

// The same for a 32-vertex pass (two 16-vertex blocks): each copy moves two
// rows, lanes 0-31 the first and 32-63 the second (lanes past the last row
// copy nothing); the uniforms only for a query (XI). ceil(rows / 2) copies.
template <bool XI>
__device__ __forceinline__ void stage_pass32(const QueryArgs& a, int64_t tile, float* buf, int lane) {
  constexpr int rows = kInFeatures + (XI ? 4 : 0);
  int64_t v = tile * (2 * kTileV) + (lane & 31);
  v = v < a.B ? v : a.B - 1;
#pragma unroll
  for (int j = 0; j < (rows + 1) / 2; ++j) {
    const int r = 2 * j + (lane >> 5);
    if (r < rows) {
      const float* src = r < kInFeatures ? a.feat + r * a.ld + v : a.xi + (r - kInFeatures) * a.ld + v;
      __builtin_amdgcn_global_load_lds(src, (__attribute__((address_space(3))) void*)(buf + 2 * j * 32), 4, 0, 0);
    }
  }
}

// Layer 0's input of vertex `col` of a staged pass (as the Mlp's load_raw:
// features 4g .. 4g + 3 of the 9, then the constant one, then zeros)
__device__ __forceinline__ bf16x4 staged_input(const float* buf, int col, bool valid, int g) {
  float f[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int k = 4 * g + j;
    float x = 0.0f;
    if (valid) {
      if (k < kInFeatures) x = buf[k * 64 + col];
      else if (k == kInFeatures) x = 1.0f;
    }
    f[j] = x;
  }
  return bf16x4{(__bf16)f[0], (__bf16)f[1], (__bf16)f[2], (__bf16)f[3]};
}

// The query (MODE 0) of the hidden-64 networks, one sample per lane: a wave
// takes four 16-vertex blocks per pass. For each block it runs the forward,
// decodes the lobes (lane (g, c): vertex c, lobes g*K/4 ..), chooses a lobe
// per vertex and moves the chosen lobe to lane (block, c). Then every lane
// samples the vertex (block g, vertex c) once, instead of the four lanes of
// a vertex each repeating the sample; the directions go back to the lanes
// that hold each block's lobes for the pdf, and lane (g, c) stores the
// direction and pdf of vertex (g, c). Per vertex, the same operations in the
// same order as the one-block pass, so the same results bit for bit.
template <int H, int K, int PREC, int S, int E, int NW>
__device__ __forceinline__ void query_four_blocks(const QueryArgs& a, const typename Forward<H, K, PREC, 4, S, E>::W* wts,
                                                  int64_t tile, const float* in, int lane) {
  typedef Forward<H, K, PREC, 4, S, E> F;
  static_assert(E == 0, "staged raw features");
  constexpr int KQ = K / 4;
  constexpr int MTO = F::MTO;
  const int g = lane >> 4, c = lane & 15;
  Lobe lb[4][KQ];
  Lobe ch = {};
#pragma unroll
  for (int b = 0; b < 4; ++b) {
    const int64_t v = tile * (4 * kTileV) + b * kTileV + c;
    const bool valid = v < a.B;
    const bf16x4 x = staged_input(in, b * kTileV + c, valid, g);
    float out[MTO][4];
    F::run_query(wts, a.nh, x, out, lane);
    float A[KQ];
    query_decode<KQ, MTO>(out, a.eps, lb[b], A, a.amul);
    const float xs = valid ? in[kInFeatures * 64 + b * kTileV + c] : 0.0f;
    const int k = select_lobe<KQ>(A, xs, g, c);
    const Lobe r = broadcast_lobe<KQ>(lb[b], k, c);
    if (g == b) ch = r;
    // selection probability c = sigmoid(o[8K]) (Tab. "decoding")
    if (S == 1 && a.sel_out != nullptr && valid && g == 0) a.sel_out[v] = frcp(1.0f + fexp(-out[MTO - 1][0]));
    if (a.rec_out != nullptr && valid) store_records<KQ>(a, lb[b], v, g);
  }
  const int64_t vm = tile * (4 * kTileV) + lane;   // vertex (block g, c)
  const bool mine = vm < a.B;
  const float xi0 = mine ? in[(kInFeatures + 1) * 64 + lane] : 0.0f;
  const float xi1 = mine ? in[(kInFeatures + 2) * 64 + lane] : 0.0f;
  const float xi2 = mine ? in[(kInFeatures + 3) * 64 + lane] : 0.0f;
  float vx, vy, vz;
  sample_unit(ch, xi0, xi1, xi2, a.eps, vx, vy, vz);
  float logq = 0.0f;
#pragma unroll
  for (int b = 0; b < 4; ++b) {
    const int src = b * kTileV + c;
    const float bx = __shfl(vx, src), by = __shfl(vy, src), bz = __shfl(vz, src);
    const float lq = query_log_pdf<KQ>(lb[b], bx, by, bz, a.eps);
    if (g == b) logq = lq;
  }
  if (mine) {
    a.dir_out[vm] = vx;
    a.dir_out[a.ld + vm] = vy;
    a.dir_out[2 * a.ld + vm] = vz;
    a.pdf_out[vm] = fexp(logq);
  }
}

// MODE 0: query, 1: raw forward only; S = 1: the network has the selection
// output (row 8K, read by lane group 0 from the extra output tile); E = 1:
// the encoded input; NB: 16-vertex blocks per wave per pass (NB > 1 shares
// every weight fragment read among NB MFMAs); NW: waves per workgroup.
template <int H, int K, int PREC, int MODE, int S, int E, int NB, int NW>
__global__ __launch_bounds__(64 * NW) __attribute__((amdgpu_waves_per_eu(query_waves_per_eu(H, K, MODE, PREC))))
void query_kernel(QueryArgs a) {
  constexpr int NHMAX = 4;
  typedef Mlp<H, K, PREC, E> M;
  typedef Forward<H, K, PREC, NHMAX, S, E> F;
  typedef typename F::W W;
  static_assert(NB == 1 || PREC == 1, "multi-block passes are BF16 only");
  extern __shared__ __align__(16) unsigned char smem[];
  W* lds = reinterpret_cast<W*>(smem);
  // the forward weights by direct-to-LDS loads: every wave's copies are in
  // flight at once (a register round trip per 16 bytes waited on each load)
  lds_dma(lds, a.wpack, a.lds_bytes);
  lds_dma_wait();
  __syncthreads();
  const W* wts = lds;

  const int lane = lane_id();
  const int g = lane >> 4, c = lane & 15;
  const int wave = threadIdx.x >> 6;
  if constexpr (query_four(H, K, MODE, PREC)) {
    // each wave's two staging buffers follow the weights: the next pass's
    // inputs are copied while this pass runs, so no block waits for memory
    float* stage = reinterpret_cast<float*>(smem + a.lds_bytes) + wave * 2 * kPassStage;
    const int64_t n_tiles = (a.B + 4 * kTileV - 1) / (4 * kTileV);
    const int64_t stride = (int64_t)gridDim.x * NW;
    int64_t tile = (int64_t)blockIdx.x * NW + wave;
    if (tile < n_tiles) stage_pass(a, tile, stage, lane);
    for (int p = 0; tile < n_tiles; tile += stride, p ^= 1) {
      float* cur = stage + p * kPassStage;
      if (tile + stride < n_tiles) {
        stage_pass(a, tile + stride, stage + (p ^ 1) * kPassStage, lane);
        // the current pass's 13 copies and everything before them are done;
        // the 13 just issued may still be in flight
        __builtin_amdgcn_s_waitcnt(0x0F70 | 13);
      } else {
        lds_dma_wait();
      }
      query_four_blocks<H, K, PREC, S, E, NW>(a, wts, tile, cur, lane);
    }
    return;
  }
  constexpr int TV = kTileV * NB;   // vertices per wave pass
  const int64_t n_tiles = (a.B + TV - 1) / TV;
  const int64_t stride = (int64_t)gridDim.x * NW;
  if constexpr (NB == 1) {
    for (int64_t tile = (int64_t)blockIdx.x * NW + wave; tile < n_tiles; tile += stride) {
      const int64_t v = tile * kTileV + c;
      typename M::Input x = M::load_input(a.feat, a.ld, v, v < a.B, g);
      float out[F::MTO][4];
      F::run_query(wts, a.nh, x, out, lane);
      finish_block<K, MODE, S>(a, out, v, g, c, a.xi, a.ld, v);
    }
  } else {
    // two 16-vertex blocks per pass, their inputs staged in LDS one pass
    // ahead (as in query_four_blocks): the rows of a pass are [row][32]
    static_assert(NB == 2, "32-vertex passes");
    constexpr int ROWS = kInFeatures + (MODE == 0 ? 4 : 0);
    constexpr int COPIES = (ROWS + 1) / 2;
    float* stage = reinterpret_cast<float*>(smem + a.lds_bytes) + wave * 2 * (kPassRows * 32);
    int64_t tile = (int64_t)blockIdx.x * NW + wave;
    if (tile < n_tiles) stage_pass32<MODE == 0>(a, tile, stage, lane);
    for (int p = 0; tile < n_tiles; tile += stride, p ^= 1) {
      const float* cur = stage + p * (kPassRows * 32);
      if (tile + stride < n_tiles) {
        stage_pass32<MODE == 0>(a, tile + stride, stage + (p ^ 1) * (kPassRows * 32), lane);
        __builtin_amdgcn_s_waitcnt(0x0F70 | COPIES);
      } else {
        lds_dma_wait();
      }
      typename M::Input x[NB];
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) {
        const int64_t v = tile * TV + nb * kTileV + c;
        x[nb] = M::load_input(cur, 32, nb * kTileV + c, v < a.B, g);
      }
      float out[NB][F::MTO][4];
      F::template run_query_nb<NB, MODE == 0>(wts, a.nh, x, out, lane);
#pragma unroll
      for (int nb = 0; nb < NB; ++nb)
        finish_block<K, MODE, S>(a, out[nb], tile * TV + nb * kTileV + c, g, c, cur + kInFeatures * 32, 32,
                                 nb * kTileV + c);
    }
  }
}

template <int H, int K, int PREC, int S, int E, int NB, int NW>
static hipError_t launch_query_s(const QueryArgs& a, int mode, hipStream_t st) {
  auto kern = mode == 0 ? query_kernel<H, K, PREC, 0, S, E, NB, NW> : query_kernel<H, K, PREC, 1, S, E, NB, NW>;
  const bool four = query_four(H, K, mode, PREC);
  const int TV = kTileV * (four ? 4 : NB);   // vertices per wave pass
  const int64_t n_tiles = (a.B + TV - 1) / TV;
  const int64_t want = (n_tiles + NW - 1) / NW;
  const int64_t cap = (int64_t)(a.per_cu < 1 ? 1 : a.per_cu) * a.num_cus;
  int grid = (int)(want < cap ? want : cap);
  if (grid < 1) grid = 1;
  hipLaunchKernelGGL(kern, dim3(grid), dim3(64 * NW), query_dynamic_lds(a.lds_bytes, four, NB, NW), st, a);
  return hipGetLastError();
}

// The LDS limit is raised once to the footprint of the network shape's
// deepest variant (4 hidden layers); the occupancy is that of the caller's
// footprint.
template <int H, int K, int PREC, int S, int E, int NB, int NW>
static hipError_t occupancy_s(int mode, int lds_bytes, int* per_cu) {
  const NetDims dmax{H, 4, K, S, E};
  const int max_w = PREC == 1 ? (int)Bf16Layout{dmax}.fwd_elems() * 2 : (int)F32Layout{dmax}.total_elems() * 4;
  if (lds_bytes > max_w) return hipErrorInvalidValue;
  const bool four = query_four(H, K, mode, PREC);
  const int max_bytes = (int)query_dynamic_lds(max_w, four, NB, NW);
  lds_bytes = (int)query_dynamic_lds(lds_bytes, four, NB, NW);
  hipError_t e = mode == 0 ? set_max_lds_once<query_kernel<H, K, PREC, 0, S, E, NB, NW>>(max_bytes)
                           : set_max_lds_once<query_kernel<H, K, PREC, 1, S, E, NB, NW>>(max_bytes);
  if (e != hipSuccess) return e;
  auto kern = mode == 0 ? query_kernel<H, K, PREC, 0, S, E, NB, NW> : query_kernel<H, K, PREC, 1, S, E, NB, NW>;
  int n = 0;
  e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, kern, 64 * NW, lds_bytes);
  *per_cu = n < 1 ? 1 : n;
  return e;
}

template <int H, int K, int PREC>
static hipError_t launch_query_t(const QueryArgs& a, int mode, hipStream_t st) {
  return a.sel ? launch_query_s<H, K, PREC, 1, 0, 1, 4>(a, mode, st) : launch_query_s<H, K, PREC, 0, 0, 1, 4>(a, mode, st);
}

hipError_t launch_query(const QueryArgs& a, const NetDims& d, int prec, int mode, hipStream_t st) {
#define NASG_CASE(h, k, p) \
  if (d.H == h && d.K == k && prec == p && d.E == 0) return launch_query_t<h, k, p>(a, mode, st);
  NASG_FOR_EACH_NET(NASG_CASE)
#undef NASG_CASE
  // hidden-128 networks whose BF16 forward weights fit in LDS: two vertex
  // blocks per wave, eight waves per workgroup
#define NASG_CASE(h, k, p, s, e)                                          \
  if (d.H == h && d.K == k && prec == p && d.S == s && d.E == e) \
    return launch_query_s<h, k, p, s, e, 2, 8>(a, mode, st);
  NASG_FOR_EACH_RESIDENT_QUERY(NASG_CASE)
#undef NASG_CASE
  return hipErrorInvalidValue;
}

hipError_t query_workgroups_per_cu(const NetDims& d, int prec, int mode, int lds_bytes, int* per_cu) {
#define NASG_CASE(h, k, p)                                                        \
  if (d.H == h && d.K == k && prec == p && d.E == 0)                              \
    return d.S ? occupancy_s<h, k, p, 1, 0, 1, 4>(mode, lds_bytes, per_cu)       \
               : occupancy_s<h, k, p, 0, 0, 1, 4>(mode, lds_bytes, per_cu);
  NASG_FOR_EACH_NET(NASG_CASE)
#undef NASG_CASE
#define NASG_CASE(h, k, p, s, e)                                 \
  if (d.H == h && d.K == k && prec == p && d.S == s && d.E == e) \
    return occupancy_s<h, k, p, s, e, 2, 8>(mode, lds_bytes, per_cu);
  NASG_FOR_EACH_RESIDENT_QUERY(NASG_CASE)
#undef NASG_CASE
  return hipErrorInvalidValue;
}

bool query_is_resident(const NetDims& d, int prec) {
#define NASG_CASE(h, k, p) \
  if (d.H == h && d.K == k && prec == p && d.E == 0) return true;
  NASG_FOR_EACH_NET(NASG_CASE)
#undef NASG_CASE
#define NASG_CASE(h, k, p, s, e) \
  if (d.H == h && d.K == k && prec == p && d.S == s && d.E == e) return true;
  NASG_FOR_EACH_RESIDENT_QUERY(NASG_CASE)
#undef NASG_CASE
  return false;
}

}  // namespace nasg
