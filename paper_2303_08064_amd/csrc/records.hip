// Mixture pdf and direct sampling from stored decoded records.
//
// One lane per vertex; the record tile [9][K][64] of a wave is read with one
// 256-byte contiguous load per (parameter, lobe), so the kernels stream the
// records from HBM once. Sec. 3.1 (mixture), eq. NASG, App. C (sampling).
#include "kernels.hpp"

namespace nasg {

// The record is read exactly once, so its loads are non-temporal (they do
// not displace other data in the caches). base: vertex v's first value in
// its tile, rec + (v / 64) 9 K 64 + v % 64.
template <int K>
__device__ __forceinline__ const float* record_base(const float* __restrict__ rec, int64_t v) {
  return rec + (v / kRecTile) * 9 * K * kRecTile + (v % kRecTile);
}
template <int K>
__device__ __forceinline__ Lobe load_record(const float* __restrict__ base, int k) {
  auto ld = [&](int p) { return __builtin_nontemporal_load(base + (p * K + k) * kRecTile); };
  Lobe L;
  L.zx = ld(0);
  L.zy = ld(1);
  L.zz = ld(2);
  L.xx = ld(3);
  L.xy = ld(4);
  L.xz = ld(5);
  L.lam = ld(6);
  L.a = ld(7);
  L.logc = ld(8);
  return L;
}
template <int K>
__device__ __forceinline__ void load_records(const float* __restrict__ rec, int64_t v, Lobe (&lb)[K]) {
  const float* base = record_base<K>(rec, v);
#pragma unroll
  for (int k = 0; k < K; ++k) lb[k] = load_record<K>(base, k);
}

template <int K>
__device__ __forceinline__ float log_mixture(const Lobe (&lb)[K], float vx, float vy, float vz, float eps) {
  float ell[K];
  float m = -INFINITY;
#pragma unroll
  for (int k = 0; k < K; ++k) {
    ell[k] = eval_lobe(lb[k], vx, vy, vz, eps).ell;
    m = fmaxf(m, ell[k]);
  }
  float s = 0.0f;
#pragma unroll
  for (int k = 0; k < K; ++k) s += fexp(ell[k] - m);
  return m == -INFINITY ? -INFINITY : m + flog(s);
}

template <int K>
__global__ __launch_bounds__(256) void pdf_kernel(RecArgs a) {
  const int64_t v = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (v >= a.B) return;
  float vx = a.dir[v], vy = a.dir[a.ld + v], vz = a.dir[2 * a.ld + v];
  float inv = frsq(fmaf(vx, vx, fmaf(vy, vy, vz * vz)));
  vx *= inv; vy *= inv; vz *= inv;
  Lobe lb[K];
  load_records<K>(a.rec, v, lb);
  a.pdf_out[v] = fexp(log_mixture<K>(lb, vx, vy, vz, a.eps));
}

template <int K>
__global__ __launch_bounds__(256) void sample_kernel(RecArgs a) {
  const int64_t v = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (v >= a.B) return;
  Lobe lb[K];
  load_records<K>(a.rec, v, lb);
  const float xi_sel = a.xi[v], xi0 = a.xi[a.ld + v], xi1 = a.xi[2 * a.ld + v], xi2 = a.xi[3 * a.ld + v];
  // mixture weights A_k = exp(log(A_k/K_k) + log K_k), K_k in closed form
  float A[K];
  float total = 0.0f;
#pragma unroll
  for (int k = 0; k < K; ++k) {
    float lk = log_normaliser(lb[k].lam, flog(lb[k].lam), lb[k].a, a.eps);
    A[k] = fexp(lb[k].logc + lk);
    total += A[k];
  }
  // inverse CDF over k in order (same rule as the query kernel)
  const float target = xi_sel * total;
  float run = 0.0f;
  int ksel = K, last = -1;
#pragma unroll
  for (int k = 0; k < K; ++k) {
    run += A[k];
    if (ksel == K && target < run) ksel = k;
    if (A[k] > 0.0f) last = k;
  }
  if (ksel == K) ksel = last < 0 ? 0 : last;
  Lobe s = lb[0];
#pragma unroll
  for (int k = 1; k < K; ++k)
    if (k == ksel) s = lb[k];
  float vx, vy, vz;
  sample_lobe(s, xi0, xi1, xi2, a.eps, vx, vy, vz);
  float inv = frsq(fmaf(vx, vx, fmaf(vy, vy, vz * vz)));
  vx *= inv; vy *= inv; vz *= inv;
  a.dir_out[v] = vx;
  a.dir_out[a.ld + v] = vy;
  a.dir_out[2 * a.ld + v] = vz;
  a.pdf_out[v] = fexp(log_mixture<K>(lb, vx, vy, vz, a.eps));
}

// Mixture pdf and the gradient of log D with respect to the direction on the
// sphere: sum_k r_k grad ell_k with r_k = D_k / D (each lobe's gradient is
// formed in the tangent plane of v). One pass over the lobes with one record
// in registers at a time: with m the running maximum of ell_k, the sum
// s = sum_k e^{ell_k - m} and the weighted gradient G = sum_k e^{ell_k - m}
// grad ell_k are rescaled by e^{m_old - m} whenever m rises, so that
// log D = m + log s and the gradient is G / s.
template <int K>
__global__ __launch_bounds__(256) void pdf_grad_kernel(RecArgs a) {
  const int64_t v = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (v >= a.B) return;
  float vx = a.dir[v], vy = a.dir[a.ld + v], vz = a.dir[2 * a.ld + v];
  float inv = frsq(fmaf(vx, vx, fmaf(vy, vy, vz * vz)));
  vx *= inv; vy *= inv; vz *= inv;
  const float* base = record_base<K>(a.rec, v);
  float m = -INFINITY, s = 0.0f, gx = 0.0f, gy = 0.0f, gz = 0.0f;
#pragma unroll 2
  for (int k = 0; k < K; ++k) {
    const Lobe L = load_record<K>(base, k);
    const Eval e = eval_lobe(L, vx, vy, vz, a.eps);
    float hx, hy, hz;
    dir_grad_lobe(L, e, vx, vy, vz, hx, hy, hz);
    const float mn = fmaxf(m, e.ell);
    // while every term so far is e^{-inf} = 0 there is nothing to rescale
    const bool none = mn == -INFINITY;
    const float sc = none ? 1.0f : fexp(m - mn);
    const float w = none ? 0.0f : fexp(e.ell - mn);
    s = fmaf(s, sc, w);
    gx = fmaf(gx, sc, w * hx);
    gy = fmaf(gy, sc, w * hy);
    gz = fmaf(gz, sc, w * hz);
    m = mn;
  }
  const float rs = frcp(s);
  a.pdf_out[v] = m == -INFINITY ? 0.0f : fexp(m + flog(s));
  a.grad_out[v] = gx * rs;
  a.grad_out[a.ld + v] = gy * rs;
  a.grad_out[2 * a.ld + v] = gz * rs;
}

template <int K>
static hipError_t launch_pdf_grad_t(const RecArgs& a, hipStream_t st) {
  int grid = (int)((a.B + 255) / 256);
  hipLaunchKernelGGL(pdf_grad_kernel<K>, dim3(grid), dim3(256), 0, st, a);
  return hipGetLastError();
}

hipError_t launch_pdf_grad(const RecArgs& a, int K, hipStream_t st) {
  switch (K) {
    case 4: return launch_pdf_grad_t<4>(a, st);
    case 8: return launch_pdf_grad_t<8>(a, st);
    case 16: return launch_pdf_grad_t<16>(a, st);
    case 32: return launch_pdf_grad_t<32>(a, st);
  }
  return hipErrorInvalidValue;
}

template <int K>
static hipError_t launch_pdf_t(const RecArgs& a, hipStream_t st) {
  int grid = (int)((a.B + 255) / 256);
  hipLaunchKernelGGL(pdf_kernel<K>, dim3(grid), dim3(256), 0, st, a);
  return hipGetLastError();
}

template <int K>
static hipError_t launch_sample_t(const RecArgs& a, hipStream_t st) {
  int grid = (int)((a.B + 255) / 256);
  hipLaunchKernelGGL(sample_kernel<K>, dim3(grid), dim3(256), 0, st, a);
  return hipGetLastError();
}

hipError_t launch_pdf(const RecArgs& a, int K, hipStream_t st) {
  switch (K) {
    case 4: return launch_pdf_t<4>(a, st);
    case 8: return launch_pdf_t<8>(a, st);
    case 16: return launch_pdf_t<16>(a, st);
    case 32: return launch_pdf_t<32>(a, st);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_sample(const RecArgs& a, int K, hipStream_t st) {
  switch (K) {
    case 4: return launch_sample_t<4>(a, st);
    case 8: return launch_sample_t<8>(a, st);
    case 16: return launch_sample_t<16>(a, st);
    case 32: return launch_sample_t<32>(a, st);
  }
  return hipErrorInvalidValue;
}

}  // namespace nasg
