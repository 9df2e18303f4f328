// Hidden-128 networks: the backward-grid sizing, the workspace size of the
// stored raw-output gradient, and the launchers of the K = 32 networks; the
// paper's default network is instantiated in large_paper.hip (a translation
// unit of its own, so that its kernels do not change how the K = 32
// kernels are compiled). The kernels themselves are in large.hpp.
#include "large.hpp"

namespace nasg {

// BF16: the backward kernels' grid, one workgroup per 128-vertex tile up to
// one per CU; FP32: the backward kernels' 64-vertex tiles
int large_train_workgroups(int64_t B, int num_cus, int prec) {
  if (prec != 1) return train_workgroups(B, num_cus);
  const int64_t t = (B + kBwdV - 1) / kBwdV;
  const int64_t cap = num_cus < kMaxTrainWG ? num_cus : kMaxTrainWG;
  return (int)(t < cap ? (t < 1 ? 1 : t) : cap);
}

int large_loss_workgroups(int64_t B, int num_cus, int prec) {
  if (prec == 1) return large_train_workgroups(B, num_cus, prec);   // the fused backward kernel's grid
  const int64_t t = (B + kWGV - 1) / kWGV;                           // the FP32 gradient kernel: two per CU
  const int64_t cap = 2LL * (num_cus < kMaxTrainWG ? num_cus : kMaxTrainWG);
  return (int)(t < cap ? (t < 1 ? 1 : t) : cap);
}

// dL/d(raw outputs) images of a batch of up to B vertices, rounded up to
// whole backward tiles: out_rows values per vertex (BF16 or FP32)
size_t large_dout_bytes(int64_t B, int K, int S, int prec) {
  const int64_t v = (B + kBwdV - 1) / kBwdV * kBwdV;
  return (size_t)v * (size_t)(8 * K + 16 * S) * (prec == 1 ? 2 : 4);
}

NASG_LARGE_LAUNCHERS(k32, NASG_FOR_EACH_LARGE_NET_K32, NASG_FOR_EACH_STREAMED_QUERY_K32)

hipError_t launch_large_query(const QueryArgs& a, const NetDims& d, int prec, int mode, hipStream_t st) {
  hipError_t e = hipErrorInvalidValue;
  if (launch_large_query_k32(a, d, prec, mode, st, &e) || launch_large_query_paper(a, d, prec, mode, st, &e)) return e;
  return hipErrorInvalidValue;
}

hipError_t launch_large_train(const LargeTrainArgs& a, const NetDims& d, int prec, int n_wg, int n_grad,
                              hipStream_t st) {
  hipError_t e = hipErrorInvalidValue;
  if (launch_large_train_k32(a, d, prec, n_wg, n_grad, st, &e) ||
      launch_large_train_paper(a, d, prec, n_wg, n_grad, st, &e))
    return e;
  return hipErrorInvalidValue;
}

}  // namespace nasg
