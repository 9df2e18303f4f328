// Kernel argument blocks, shared device helpers and launcher declarations.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "common.hpp"

// Network shapes with compiled kernels: (hidden width, lobes, precision).
#define NASG_FOR_EACH_NET(X) \
  X(64, 4, 0) X(64, 4, 1) X(64, 8, 0) X(64, 8, 1) X(64, 16, 0) X(64, 16, 1)
// Large networks (4 hidden layers): weights stream through LDS while the
// workgroup moves through the layers, and training runs as separate
// NASG-gradient and backward kernels. (hidden, lobes, precision, selection
// output, encoded input): K = 32 on the raw features, and the paper's default
// network (Sec. 4.1, Sec. 6).
// The two groups are compiled in translation units of their own.
#define NASG_FOR_EACH_LARGE_NET_K32(X) X(128, 32, 0, 0, 0) X(128, 32, 1, 0, 0)
#define NASG_FOR_EACH_LARGE_NET_PAPER(X) X(128, 8, 0, 1, 1) X(128, 8, 1, 1, 1)
#define NASG_FOR_EACH_LARGE_NET(X) NASG_FOR_EACH_LARGE_NET_K32(X) NASG_FOR_EACH_LARGE_NET_PAPER(X)
// Large networks whose BF16 forward weights fit in LDS (132 KiB): their
// queries run the LDS-resident query kernel; the others' queries stream
// their weights through the pipeline.
#define NASG_FOR_EACH_RESIDENT_QUERY(X) X(128, 8, 1, 1, 1)
#define NASG_FOR_EACH_STREAMED_QUERY_K32(X) X(128, 32, 0, 0, 0) X(128, 32, 1, 0, 0)
#define NASG_FOR_EACH_STREAMED_QUERY_PAPER(X) X(128, 8, 0, 1, 1)

namespace nasg {

struct QueryArgs {
  const void* wpack;
  int lds_bytes;
  int nh;
  float eps;
  const float* feat;
  const float* xi;
  int64_t ld, B;
  float* dir_out;
  float* pdf_out;
  float* rec_out;
  float* raw_out;
  float* sel_out;        // selection probability c per vertex (optional)
  int sel;               // 1: the network has the selection output (8K + 1 rows)
  float amul;            // 1: NASG lobes; 0: isotropic lobes (a = 0)
  int num_cus;
  int per_cu = 1;        // resident query kernel: workgroups per CU at this LDS footprint
};

struct RecArgs {
  const float* rec;
  const float* dir;   // pdf: directions to evaluate
  const float* xi;    // sample: uniforms
  int64_t ld, B;
  float eps;
  float* dir_out;
  float* pdf_out;
  float* grad_out;    // pdf_grad: [3][ld] gradient of log D on the sphere
};

struct TrainArgs {
  const void* wpack;
  int lds_bytes;
  int nh;
  float eps;
  const float* feat;
  const float* dir;
  const float* w;
  int64_t ld, B;
  float* partial;        // [n_wg][n_weights] dW partials, canonical layout
  double* loss_partial;  // [n_wg][2]: sum w*(-log terms), sum w
  int64_t n_weights;
  int num_cus;
  int sel;               // 1: selection output and the blended loss
  const float* bsdf_pdf; // [B] p_fs at each training direction (sel = 1)
  float mis_e;           // e of the blended loss (sel = 1)
  float amul;            // 1: NASG lobes; 0: isotropic lobes (a = 0)
};

struct LargeTrainArgs {
  const void* wpack;
  float eps;
  const float* feat;
  const float* dir;
  const float* w;
  const float* bsdf_pdf; // [B] p_fs at each training direction (selection output)
  float mis_e;           // e of the blended loss (selection output)
  int64_t ld, B;
  void* dout;            // dL/d(raw outputs) per 16 vertices: BF16 operand image (16 B x K/4 x 64,
                         // then 8 B x 64 for the selection tile) or FP32 accumulator image (16 B x K/2 x 64)
  float* partial;        // [n_wg][n_weights] (backward kernels' grid)
  double* loss_partial;  // [n_grad][2] (gradient kernel's grid)
  int64_t n_weights;
  float amul;            // 1: NASG lobes; 0: isotropic lobes (a = 0)
  int num_cus;
};

struct ReduceArgs {
  const float* partial;
  const double* loss_partial;
  int n_wg;              // dW partials
  int n_loss;            // loss partial pairs
  int64_t n_weights;
  int64_t B;
  float* grad;
  double* norm_partial;  // [n_blocks]
  double* stats;
  const int64_t* step;
  int64_t* step_snapshot;
};

struct AdamArgs {
  float* w;
  float* m;
  float* v;
  const float* grad;
  void* wpack;
  int64_t* step;
  const int64_t* step_snapshot;
  uint32_t* flags;
  double* stats;
  const double* norm_partial;
  int n_norm;
  int64_t n_weights;
  int H, NH, K, S, E, prec;
  float lr, beta1, beta2, adam_eps;
};

// Lobe choice by inverse CDF over k = g*KQ + q (this library's reading: the
// smallest k with xi_sel * sum(A) < A_0 + ... + A_k; the last lobe with
// A_k > 0 when rounding leaves none).
template <int KQ>
__device__ __forceinline__ int select_lobe(const float (&A)[KQ], float xi, int g, int c) {
  float cum[KQ];
  float run = 0.0f;
#pragma unroll
  for (int q = 0; q < KQ; ++q) { run += A[q]; cum[q] = run; }
  float t0 = __shfl(run, c), t1 = __shfl(run, c + 16), t2 = __shfl(run, c + 32), t3 = __shfl(run, c + 48);
  float p01 = t0 + t1, p012 = p01 + t2, total = p012 + t3;
  float P = g == 0 ? 0.0f : (g == 1 ? t0 : (g == 2 ? p01 : p012));
  float target = xi * total;
  int cand = 4 * KQ;
#pragma unroll
  for (int q = KQ - 1; q >= 0; --q)
    if (target < P + cum[q]) cand = g * KQ + q;
  int k = quad_min_i(cand);
  // The fallback: for xi_sel < 1 the target stays below the total, which the
  // last lane group's running sum equals bit for bit, so only xi_sel >= 1 or
  // a non-finite weight reaches it; evaluated when some lane of the wave
  // needs it (the quad reduction wants every lane).
  if (__any(k == 4 * KQ)) {
    int last = -1;
#pragma unroll
    for (int q = 0; q < KQ; ++q)
      if (A[q] > 0.0f) last = g * KQ + q;
    last = quad_max_i(last);
    if (k == 4 * KQ) k = last < 0 ? 0 : last;
  }
  return k;
}

// s ? a : b field by field (one select per field, no branch)
__device__ __forceinline__ Lobe select_lobe_fields(bool s, const Lobe& a, const Lobe& b) {
  Lobe r;
  r.zx = s ? a.zx : b.zx;
  r.zy = s ? a.zy : b.zy;
  r.zz = s ? a.zz : b.zz;
  r.xx = s ? a.xx : b.xx;
  r.xy = s ? a.xy : b.xy;
  r.xz = s ? a.xz : b.xz;
  r.lam = s ? a.lam : b.lam;
  r.a = s ? a.a : b.a;
  r.logc = s ? a.logc : b.logc;
  return r;
}

// The selected lobe's record, from the lane group that owns it.
template <int KQ>
__device__ __forceinline__ Lobe broadcast_lobe(const Lobe (&lb)[KQ], int k, int c) {
  const int gs = k / KQ, qs = k % KQ;
  Lobe mine = lb[0];
#pragma unroll
  for (int q = 1; q < KQ; ++q) mine = select_lobe_fields(q == qs, lb[q], mine);
  const int src = gs * 16 + c;
  Lobe r;
  r.zx = __shfl(mine.zx, src);
  r.zy = __shfl(mine.zy, src);
  r.zz = __shfl(mine.zz, src);
  r.xx = __shfl(mine.xx, src);
  r.xy = __shfl(mine.xy, src);
  r.xz = __shfl(mine.xz, src);
  r.lam = __shfl(mine.lam, src);
  r.a = __shfl(mine.a, src);
  r.logc = __shfl(mine.logc, src);
  return r;
}

// log sum_k exp(ell_k) over the lane's KQ lobes and the vertex's 4 lanes.
// XCHG: the cross-lane steps by lane swaps (xchg_max/xchg_sum) instead of
// LDS permutes.
template <int KQ, bool XCHG = false>
__device__ __forceinline__ float mixture_lse(const float (&ell)[KQ]) {
  float m = ell[0];
#pragma unroll
  for (int q = 1; q < KQ; ++q) m = fmaxf(m, ell[q]);
  m = XCHG ? xchg_max(m) : quad_max(m);
  float s = 0.0f;
#pragma unroll
  for (int q = 0; q < KQ; ++q) s += fexp_sub(ell[q], m);
  s = XCHG ? xchg_sum(s) : quad_sum(s);
  return m == -INFINITY ? -INFINITY : m + flog(s);
}

hipError_t launch_query(const QueryArgs& a, const NetDims& d, int prec, int mode, hipStream_t st);
// the network's queries run the LDS-resident query kernel
bool query_is_resident(const NetDims& d, int prec);
// workgroups per CU of the resident query kernel (mode 0 query, 1 raw
// forward) at `lds_bytes` of LDS; also raises the kernel's LDS limit
hipError_t query_workgroups_per_cu(const NetDims& d, int prec, int mode, int lds_bytes, int* per_cu);
hipError_t launch_pdf(const RecArgs& a, int K, hipStream_t st);
hipError_t launch_sample(const RecArgs& a, int K, hipStream_t st);
hipError_t launch_pdf_grad(const RecArgs& a, int K, hipStream_t st);
hipError_t launch_train(const TrainArgs& a, int H, int K, int prec, int n_wg, hipStream_t st);
hipError_t launch_large_query(const QueryArgs& a, const NetDims& d, int prec, int mode, hipStream_t st);
hipError_t launch_large_train(const LargeTrainArgs& a, const NetDims& d, int prec, int n_wg, int n_grad,
                              hipStream_t st);
// per translation unit: true when the network is one of its own
bool launch_large_query_k32(const QueryArgs& a, const NetDims& d, int prec, int mode, hipStream_t st, hipError_t* err);
bool launch_large_query_paper(const QueryArgs& a, const NetDims& d, int prec, int mode, hipStream_t st,
                              hipError_t* err);
bool launch_large_train_k32(const LargeTrainArgs& a, const NetDims& d, int prec, int n_wg, int n_grad, hipStream_t st,
                            hipError_t* err);
bool launch_large_train_paper(const LargeTrainArgs& a, const NetDims& d, int prec, int n_wg, int n_grad,
                              hipStream_t st, hipError_t* err);
hipError_t launch_reduce(const ReduceArgs& a, int n_blocks, hipStream_t st);
hipError_t launch_adam(const AdamArgs& a, hipStream_t st);
hipError_t launch_pack(const float* w, void* wpack, const NetDims& d, int prec, hipStream_t st);
hipError_t launch_fill(void* p, int64_t n_words, uint32_t value, hipStream_t st);

// Query / train kernel grid bounds (workgroups) for a batch of B vertices.
constexpr int kMaxTrainWG = 256;
int train_workgroups(int64_t B, int num_cus);
// the large network's training: its backward kernels' grid, the loss
// partials it writes (the workgroups of the kernel that evaluates the loss),
// and the bytes of its raw-output gradient images for up to B vertices
int large_train_workgroups(int64_t B, int num_cus, int prec);
int large_loss_workgroups(int64_t B, int num_cus, int prec);
size_t large_dout_bytes(int64_t B, int K, int S, int prec);
int reduce_blocks(int64_t n_weights);

}  // namespace nasg
