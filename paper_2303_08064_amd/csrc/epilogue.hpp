// Per-vertex NASG epilogues on the MLP's output accumulators.
//
// `out[mt][i]` at lane (g, c) is raw output t = mt*4 + i of lobe
// g*KQ + t % KQ, parameter t / KQ (layout.hpp), for vertex c. Each lane
// handles KQ = K/4 lobes of one vertex; the four lanes c, c+16, c+32, c+48
// together hold the K lobes.
#pragma once

#include "kernels.hpp"

namespace nasg {

template <int KQ, int MTO>
__device__ __forceinline__ void lobe_raw(const float (&out)[MTO][4], int q, float o[8]) {
#pragma unroll
  for (int p = 0; p < 8; ++p) {
    const int t = p * KQ + q;
    o[p] = out[t >> 2][t & 3];
  }
}

// log-sum-exp of the K mixture logits (softmax of Tab. "decoding")
template <int KQ, int MTO>
__device__ __forceinline__ float logit_lse(const float (&out)[MTO][4]) {
  float alpha[KQ];
#pragma unroll
  for (int q = 0; q < KQ; ++q) {
    const int t = 7 * KQ + q;
    alpha[q] = out[t >> 2][t & 3];
  }
  float mx = alpha[0];
#pragma unroll
  for (int q = 1; q < KQ; ++q) mx = fmaxf(mx, alpha[q]);
  mx = quad_max(mx);
  float se = 0.0f;
#pragma unroll
  for (int q = 0; q < KQ; ++q) se += fexp_sub(alpha[q], mx);
  se = quad_sum(se);
  return mx + flog(se);
}

// Weighted NLL of one vertex and its gradient w.r.t. the raw outputs
// (Sec. 4.2): gs = dL/dlog q = -w/B (0 for padding lanes). Writes dl in the
// accumulator layout and returns the vertex's log term (log q; with the
// selection output, e log q_hat + (1 - e) log q).
//
// One pass over the lobes: each lobe is decoded and evaluated once, and its
// log-density's partials d ell_k / d o_p (p < 7) go straight into dl. They
// are linear in the upstream factor, which is only known once log q is:
// dL/d o_p = gq r_k d ell_k / d o_p with r_k = q_k / q, and for the logit
// dL/d o_7 = gq (r_k - A_k) (through the softmax). A second, cheap loop
// scales them.
//
// S = 1 (selection output, the blended loss of Sec. 4.2): with c the
// sigmoid of the selection logit (output row 8K, held by lane group 0) and
// q_hat = c q + (1 - c) p_fs, the loss term e log q_hat + (1 - e) log q has
// d/dlog q = e c q / q_hat + (1 - e), so gq = gs times that, and
// d/dz (z the selection logit) = e (q - p_fs) c (1 - c) / q_hat.
template <int KQ, int MTO, int S = 0>
__device__ __forceinline__ float train_epilogue(const float (&out)[MTO][4], float vx, float vy, float vz,
                                                float gs, bool valid, float eps, float (&dl)[MTO][4],
                                                float pdf_bsdf = 0.0f, float mis_e = 0.0f, float amul = 1.0f) {
  constexpr int TS = 2 * KQ;   // the selection tile (S = 1)
  static_assert(MTO == 2 * KQ + S, "output tiles: 8K rows plus the selection tile");
  // softmax of the K logits: A_k = e^{alpha_k - m} / sum, kept for the logit gradient
  float ea[KQ];
  float lse, inv_se;
  {
    float mx = -INFINITY;
#pragma unroll
    for (int q = 0; q < KQ; ++q) {
      const int t = 7 * KQ + q;
      mx = fmaxf(mx, out[t >> 2][t & 3]);
    }
    mx = xchg_max(mx);
    float se = 0.0f;
#pragma unroll
    for (int q = 0; q < KQ; ++q) {
      const int t = 7 * KQ + q;
      ea[q] = fexp_sub(out[t >> 2][t & 3], mx);
      se += ea[q];
    }
    se = xchg_sum(se);
    lse = mx + flog(se);
    inv_se = frcp(se);
  }
  float ell[KQ];
#pragma unroll
  for (int q = 0; q < KQ; ++q) {
    float o[8];
    lobe_raw<KQ, MTO>(out, q, o);
    Lobe L;
    LobeAux X;
    decode_lobe(o, eps, L, X, amul);
    L.logc = (o[7] - lse) - X.logK;
    const Eval e = eval_lobe(L, vx, vy, vz, eps);
    ell[q] = e.ell;
    float gq[8];
    backward_lobe(L, X, e, vx, vy, vz, eps, 1.0f, 0.0f, gq);
#pragma unroll
    for (int p = 0; p < 7; ++p) {
      const int t = p * KQ + q;
      dl[t >> 2][t & 3] = gq[p];
    }
  }
  const float logq = mixture_lse<KQ, true>(ell);
  float lterm = logq, gsq = gs;
  if constexpr (S == 1) {
    const int c = lane_id() & 15;
    const float z = __shfl(out[TS][0], c);   // lane (0, c) holds row 8K of vertex c
    const float cs = frcp(1.0f + fexp(-z));
    const float qv = fexp(logq);
    const float qh = fmaf(cs, qv - pdf_bsdf, pdf_bsdf);   // c q + (1 - c) p_fs
    const float iqh = frcp(qh);
    lterm = fmaf(mis_e, flog(qh), (1.0f - mis_e) * logq);
    gsq = gs * fmaf(mis_e * cs, qv * iqh, 1.0f - mis_e);
    const float gz = gs * mis_e * (qv - pdf_bsdf) * cs * (1.0f - cs) * iqh;
    const bool g0 = lane_id() < 16;
#pragma unroll
    for (int i = 0; i < 4; ++i) dl[TS][i] = (g0 && i == 0) ? gz : 0.0f;
  }
#pragma unroll
  for (int q = 0; q < KQ; ++q) {
    const int t7 = 7 * KQ + q;
    const float r = valid ? fexp_sub(ell[q], logq) : 0.0f;
    const float Aq = ea[q] * inv_se;
    const float sc = gsq * r;
#pragma unroll
    for (int p = 0; p < 7; ++p) {
      const int t = p * KQ + q;
      dl[t >> 2][t & 3] *= sc;
    }
    dl[t7 >> 2][t7 & 3] = gsq * (r - Aq);
  }
  // padding lanes (a branch taken only in a batch's last tile): zeroed
  // outright, so that no non-finite partial of their arbitrary lobes reaches
  // the weight gradient as 0 * inf
  if (!valid) {
#pragma unroll
    for (int mt = 0; mt < MTO; ++mt)
#pragma unroll
      for (int i = 0; i < 4; ++i) dl[mt][i] = 0.0f;
  }
  return lterm;
}

// A query's decode of one vertex's lobes (Tab. "decoding"): frames,
// lambda, a and log c = log(A_k / K_k) into lb, the mixture weights A_k
// (softmax of the K logits) into A.
template <int KQ, int MTO>
__device__ __forceinline__ void query_decode(const float (&out)[MTO][4], float eps, Lobe (&lb)[KQ], float (&A)[KQ],
                                             float amul) {
  float logK[KQ], alpha[KQ];
#pragma unroll
  for (int q = 0; q < KQ; ++q) {
    float o[8];
    lobe_raw<KQ, MTO>(out, q, o);
    logK[q] = decode_lobe_query(o, eps, lb[q], amul);
    alpha[q] = o[7];
  }
  // mixture weights: softmax over the K logits
  float mx = alpha[0];
#pragma unroll
  for (int q = 1; q < KQ; ++q) mx = fmaxf(mx, alpha[q]);
  mx = quad_max(mx);
  float ea[KQ];
  float se = 0.0f;
#pragma unroll
  for (int q = 0; q < KQ; ++q) {
    ea[q] = fexp_sub(alpha[q], mx);
    se += ea[q];
  }
  se = quad_sum(se);
  const float lse = mx + flog(se);
  const float inv_se = frcp(se);
#pragma unroll
  for (int q = 0; q < KQ; ++q) {
    lb[q].logc = (alpha[q] - lse) - logK[q];
    A[q] = ea[q] * inv_se;
  }
}

// One App. C sample from lobe s, normalised to unit length.
__device__ __forceinline__ void sample_unit(const Lobe& s, float xi0, float xi1, float xi2, float eps, float& vx,
                                            float& vy, float& vz) {
  sample_lobe(s, xi0, xi1, xi2, eps, vx, vy, vz);
  const float inv = frsq(fmaf(vx, vx, fmaf(vy, vy, vz * vz)));
  vx *= inv;
  vy *= inv;
  vz *= inv;
}

// log q at a unit direction: the lane's lobes, then the vertex's 4 lanes.
template <int KQ>
__device__ __forceinline__ float query_log_pdf(const Lobe (&lb)[KQ], float vx, float vy, float vz, float eps) {
  float ell[KQ];
#pragma unroll
  for (int q = 0; q < KQ; ++q) ell[q] = eval_lobe_ell(lb[q], vx, vy, vz, eps);
  return mixture_lse<KQ>(ell);
}

// Guiding query of one vertex: decode, inverse-CDF lobe choice, App. C
// sample, mixture pdf at the sample. Returns log q; v receives the unit
// direction; lb receives the decoded lobes (for the optional record store).
template <int KQ, int MTO>
__device__ __forceinline__ float query_epilogue(const float (&out)[MTO][4], float xi_sel, float xi0, float xi1,
                                                float xi2, float eps, int g, int c, Lobe (&lb)[KQ], float& vx,
                                                float& vy, float& vz, float amul = 1.0f) {
  float A[KQ];
  query_decode<KQ, MTO>(out, eps, lb, A, amul);
  const int ksel = select_lobe<KQ>(A, xi_sel, g, c);
  const Lobe s = broadcast_lobe<KQ>(lb, ksel, c);
  sample_unit(s, xi0, xi1, xi2, eps, vx, vy, vz);
  return query_log_pdf<KQ>(lb, vx, vy, vz, eps);
}

}  // namespace nasg
