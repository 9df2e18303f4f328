// Per-lobe NASG arithmetic in FP32 for gfx950: decode, normaliser, lobe
// evaluation, direct sampling and the closed-form backward.
//
// The formulas are the paper's (eq. NASG and App. A for the lobe, eq. "K for
// NASG" / App. B for the normaliser, App. C for the sampler, Tab. "decoding"
// and the Euler frame of Sec. 4.1), rewritten into forms that keep FP32
// accuracy near the lobe axis:
//   u = (v.z + 1)/2 = |v + z|^2 / 4,   1 - u = |v - z|^2 / 4,
//   c^2 = (v.x)^2 / (1 - (v.z)^2) = X^2 / (X^2 + Y^2) with X = v.x, Y = v.y,
//   log G = 2 lam (u^p - 1) + (p - 1) log u,  p = 1 + eps + a c^2,
// with log u and u^p - 1 = expm1(p log u) taken through minimax polynomials
// near u = 1.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace nasg {

constexpr float kLog2e = 1.44269504088896341f;
constexpr float kLn2 = 0.693147180559945309f;
constexpr float kLog2Pi = 1.83787706640934548f;   // log(2 pi)
constexpr float kLogClamp = 15.0f;                // log lambda, log a in [-15, 15]
// X^2 + Y^2 below the normal float range (v within ~1e-19 rad of the lobe
// axis): 1/(X^2 + Y^2) would overflow, so the anisotropy weight c^2 and its
// derivatives are taken as 0 there
constexpr float kMinNormal = 1.17549435e-38f;

__device__ __forceinline__ float fexp(float x) { return __builtin_amdgcn_exp2f(x * kLog2e); }
__device__ __forceinline__ float flog(float x) { return __builtin_amdgcn_logf(x) * kLn2; }
__device__ __forceinline__ float flog2(float x) { return __builtin_amdgcn_logf(x); }
// e^{a - b} as a log2(e) - b log2(e) in one FMA (the second product is shared
// across a loop over a with the same b) and one exp2
__device__ __forceinline__ float fexp_sub(float a, float b) {
  return __builtin_amdgcn_exp2f(fmaf(a, kLog2e, -(b * kLog2e)));
}
__device__ __forceinline__ float frcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ float frsq(float x) { return __builtin_amdgcn_rsqf(x); }
__device__ __forceinline__ float fsqrt(float x) { return __builtin_amdgcn_sqrtf(x); }
__device__ __forceinline__ float fsel(bool c, float a, float b) { return c ? a : b; }

// e^x - 1, accurate in relative terms: Taylor series to x^5 for |x| < 1/8
// (truncation below 5e-8 relative), exp(x) - 1 elsewhere.
__device__ __forceinline__ float expm1f_(float x) {
  float p = fmaf(x, 1.0f / 120.0f, 1.0f / 24.0f);
  p = fmaf(x, p, 1.0f / 6.0f);
  p = fmaf(x, p, 0.5f);
  p = fmaf(x, p, 1.0f);
  p = p * x;
  float e = fexp(x) - 1.0f;
  return fsel(fabsf(x) < 0.125f, p, e);
}

// e^x - 1 for x <= 0 (every caller but the sampler's e^{2 lam} - 1), the
// same function with one multiply-add fewer: for -1/8 < x <= 0 the
// polynomial x (1 + x (c0 + c1 x + c2 x^2)), whose coefficients are the
// minimax fit of relative error on [-1/8, 0] with the linear term held at x
// (Remez exchange; fit error 1.8e-8 relative, below FP32 rounding, where the
// Taylor series to x^5 leaves 4.4e-8); exp(x) - 1 elsewhere.
__device__ __forceinline__ float expm1_neg_poly(float x) {
  float q = fmaf(x, 0.0397158824f, 0.166526049f);
  q = fmaf(x, q, 0.499997109f);
  return x * fmaf(x, q, 1.0f);
}
__device__ __forceinline__ float expm1_neg(float x) {
  return fsel(x > -0.125f, expm1_neg_poly(x), fexp(x) - 1.0f);
}

// log(1 - w) for 0 <= w < 1/16: y (1 + y (d0 + d1 y + d2 y^2 + d3 y^3)) with
// y = -w, the minimax fit of relative error on [-1/16, 0] with the linear
// term held at y (Remez exchange; fit error 4e-10 relative).
__device__ __forceinline__ float log1m_poly(float w) {
  const float y = -w;
  float r = fmaf(y, 0.227763459f, -0.248499244f);
  r = fmaf(y, r, 0.333364844f);
  r = fmaf(y, r, -0.499999791f);
  return y * fmaf(y, r, 1.0f);
}

// log1m_poly(w4 / 4) from w4 = 4 w, with the same roundings: the
// polynomial's coefficients and variable are scaled by powers of 4, which is
// exact, so every intermediate is the same value times a power of 4.
__device__ __forceinline__ float log1m_poly4(float w4) {
  float r = fmaf(w4, 0.227763459f * (-1.0f / 1024.0f), -0.248499244f * (1.0f / 256.0f));
  r = fmaf(w4, r, 0.333364844f * (-1.0f / 64.0f));
  r = fmaf(w4, r, -0.499999791f * (1.0f / 16.0f));
  return w4 * fmaf(w4, r, -0.25f);
}

// log(1 + y) by its series to y^6 (truncation below 1e-8 relative for |y| < 1/16).
__device__ __forceinline__ float log1p_series(float y) {
  float p = fmaf(y, -1.0f / 6.0f, 1.0f / 5.0f);
  p = fmaf(y, p, -1.0f / 4.0f);
  p = fmaf(y, p, 1.0f / 3.0f);
  p = fmaf(y, p, -0.5f);
  p = fmaf(y, p, 1.0f);
  return p * y;
}

// log(1 + y) for y > -1, accurate in relative terms: the series for
// |y| < 1/16, log(1 + y) elsewhere.
__device__ __forceinline__ float log1pf_(float y) {
  return fsel(fabsf(y) < 0.0625f, log1p_series(y), flog(1.0f + y));
}

// Decoded lobe: orthonormal frame, sharpness, eccentricity, log normaliser.
struct Lobe {
  float zx, zy, zz, xx, xy, xz;
  float lam, a;
  float logc;   // log(A_k / K_k), filled once the mixture weights are known
};

// Euler-angle intermediates kept for the backward pass.
struct LobeAux {
  float ct, st, cp, sp, ctau, stau;
  float h1, h2, h3, h4;     // (1 - d_i^2)/2 = 2 e_i / (1 + e_i)^2 for the sin/cos pairs
  float inv_np, inv_nt;     // 1/|(d2,d1)|, 1/|(d4,d3)|
  float loglam, loga;       // clamped raw values
  bool lam_in, a_in;        // raw values inside the clamp range
  float logK;
  float omq;                // 1 - 2 lam / expm1(2 lam) = -d log K / d log lam
};

// A (cos, sin) pair divided by its norm; a zero pair becomes (1, 0).
__device__ __forceinline__ void unit_pair(float c, float s, float& cu, float& su, float& inv) {
  float n2 = fmaf(c, c, s * s);
  inv = frsq(n2);
  bool ok = n2 > 0.0f;
  cu = fsel(ok, c * inv, 1.0f);
  su = fsel(ok, s * inv, 0.0f);
  inv = fsel(ok, inv, 0.0f);
}

// log(2 pi) + log(one_m) - loglam - (1/2) log((1+eps)(1+eps+a)), the two
// logarithms taken in base 2 and scaled by ln 2 together.
__device__ __forceinline__ float log_normaliser_sum(float one_m, float loglam, float a, float eps) {
  const float l2 = fmaf(-0.5f, flog2((1.0f + eps) * (1.0f + eps + a)), flog2(one_m));
  return fmaf(l2, kLn2, kLog2Pi) - loglam;
}

// log K = log(2 pi) + log(1 - e^{-2 lam}) - log lam - (1/2) log((1+eps)(1+eps+a)).
__device__ __forceinline__ float log_normaliser(float lam, float loglam, float a, float eps) {
  float one_m = -expm1_neg(-2.0f * lam);
  return log_normaliser_sum(one_m, loglam, a, eps);
}

// The same, also returning omq = 1 - q with q = 2 lam / expm1(2 lam) =
// 2 lam e^{-2 lam} / (1 - e^{-2 lam}): d log K / d log lam = q - 1. As lam -> 0,
// q -> 1 and 1 - q ~ lam, so the difference is lost to cancellation (a
// relative error of u / lam); for t = 2 lam < 1/2 it comes instead from the
// series of t / expm1(t) in the Bernoulli numbers:
//   1 - q = t/2 - t^2/12 + t^4/720 - t^6/30240 + t^8/1209600 - ...,
// whose next term is below 1e-10 of the sum there.
__device__ __forceinline__ float log_normaliser(float lam, float loglam, float a, float eps, float& omq) {
  const float x = -2.0f * lam;
  const float ex = fexp(x);                           // e^{-2 lam}
  const float one_m = -fsel(x > -0.125f, expm1_neg_poly(x), ex - 1.0f);   // 1 - e^{-2 lam}
  const float t = -x;
  const float t2 = t * t;
  float ser = fmaf(t2, 1.0f / 1209600.0f, -1.0f / 30240.0f);
  ser = fmaf(t2, ser, 1.0f / 720.0f);
  ser = fmaf(t2 * t2, ser, t * fmaf(t, -1.0f / 12.0f, 0.5f));
  omq = fsel(t < 0.5f, ser, 1.0f - t * ex * frcp(one_m));   // -> 1 as e^{-2 lam} underflows
  return log_normaliser_sum(one_m, loglam, a, eps);
}

// Raw outputs o[0..7] of one lobe -> frame, lambda, a, log K (Tab. "decoding",
// Sec. 4.1 Euler frame). Pair normalisation and the clamp are this library's
// readings of the paper.
//
// cos(theta) = tanh(o0/2) needs absolute accuracy only; a sin/cos pair needs
// the ratio of its two tanh(o/2) = m/(2 - m) values (m = 1 - e^{-|o|}, kept
// accurate for small |o|), which the pair (m2 (2 - m1), m1 (2 - m2)) has
// without a division; one reciprocal R = 1/((2 - m1)(2 - m2)) per pair then
// gives the tanh' factors 2 e_i/(2 - m_i)^2 and the pair's norm.
__device__ __forceinline__ void decode_pair(float oc, float os, float& cu, float& su, float& inv_n, float& hc,
                                            float& hs) {
  const float mc = -expm1_neg(-fabsf(oc)), ms = -expm1_neg(-fabsf(os));
  const float tc = 2.0f - mc, ts = 2.0f - ms;
  const float R = frcp(tc * ts);
  float inv;
  unit_pair(copysignf(mc * ts, oc), copysignf(ms * tc, os), cu, su, inv);
  inv_n = tc * ts * inv;                             // 1/|(tanh(oc/2), tanh(os/2))|
  const float rc = ts * R, rs = tc * R;              // 1/(2 - mc), 1/(2 - ms)
  hc = 2.0f * (1.0f - mc) * rc * rc;
  hs = 2.0f * (1.0f - ms) * rs * rs;
}

// amul = 0 decodes isotropic lobes (a = 0: the normalised spherical
// Gaussian / von Mises-Fisher lobe; the anisotropy output then has zero
// gradient), 1 the NASG lobe.
__device__ __forceinline__ void decode_lobe(const float o[8], float eps, Lobe& L, LobeAux& X, float amul = 1.0f) {
  const float h0 = __builtin_amdgcn_exp2f(fabsf(o[0]) * (-0.5f * kLog2e));   // e^{-|o|/2}
  const float e0 = h0 * h0;
  const float r0 = frcp(1.0f + e0);
  X.ct = copysignf((1.0f - e0) * r0, o[0]);
  X.st = 2.0f * h0 * r0;                             // sech(o/2) = sqrt(1 - tanh^2)
  decode_pair(o[2], o[1], X.cp, X.sp, X.inv_np, X.h2, X.h1);
  decode_pair(o[4], o[3], X.ctau, X.stau, X.inv_nt, X.h4, X.h3);
  L.zx = X.cp * X.st;
  L.zy = X.sp * X.st;
  L.zz = X.ct;
  float ctc = X.ct * X.ctau;
  L.xx = fmaf(ctc, X.cp, -X.sp * X.stau);
  L.xy = fmaf(ctc, X.sp, X.cp * X.stau);
  L.xz = -X.st * X.ctau;
  X.lam_in = fabsf(o[5]) <= kLogClamp;
  X.a_in = fabsf(o[6]) <= kLogClamp;
  X.loglam = fminf(fmaxf(o[5], -kLogClamp), kLogClamp);
  X.loga = fminf(fmaxf(o[6], -kLogClamp), kLogClamp);
  L.lam = fexp(X.loglam);
  L.a = amul * fexp(X.loga);
  X.logK = log_normaliser(L.lam, X.loglam, L.a, eps, X.omq);
  L.logc = 0.0f;
}

// 1 - e^{-|o|}, accurate in relative terms (used where a pair of small raw
// outputs is normalised, so their ratio must survive).
__device__ __forceinline__ float one_minus_exp_neg(float ao) {
  return -expm1_neg(-ao);
}

// Forward-only decode for queries: the same function as decode_lobe, with
// the sin/cos pairs normalised without reciprocals (a pair of tanh(o/2) =
// m/(2 - m) values is scaled by (2 - m1)(2 - m2) > 0 before normalising) and
// log K folded into log c by the caller. Returns log K.
__device__ __forceinline__ float decode_lobe_query(const float o[8], float eps, Lobe& L, float amul = 1.0f) {
  // theta: cos = tanh(o0/2) (absolute accuracy suffices), sin = sech(o0/2)
  const float h0 = __builtin_amdgcn_exp2f(fabsf(o[0]) * (-0.5f * kLog2e));   // e^{-|o|/2}: sin without a square root
  const float e0 = h0 * h0;
  const float r0 = frcp(1.0f + e0);
  const float ct = copysignf((1.0f - e0) * r0, o[0]);
  const float st = 2.0f * h0 * r0;
  const float m1 = one_minus_exp_neg(fabsf(o[1])), m2 = one_minus_exp_neg(fabsf(o[2]));
  const float m3 = one_minus_exp_neg(fabsf(o[3])), m4 = one_minus_exp_neg(fabsf(o[4]));
  float cp, sp, ctau, stau, inv;
  unit_pair(copysignf(m2 * (2.0f - m1), o[2]), copysignf(m1 * (2.0f - m2), o[1]), cp, sp, inv);
  unit_pair(copysignf(m4 * (2.0f - m3), o[4]), copysignf(m3 * (2.0f - m4), o[3]), ctau, stau, inv);
  L.zx = cp * st;
  L.zy = sp * st;
  L.zz = ct;
  const float ctc = ct * ctau;
  L.xx = fmaf(ctc, cp, -sp * stau);
  L.xy = fmaf(ctc, sp, cp * stau);
  L.xz = -st * ctau;
  const float loglam = fminf(fmaxf(o[5], -kLogClamp), kLogClamp);
  const float loga = fminf(fmaxf(o[6], -kLogClamp), kLogClamp);
  L.lam = fexp(loglam);
  L.a = amul * fexp(loga);
  L.logc = 0.0f;
  return log_normaliser(L.lam, loglam, L.a, eps);
}

// Lobe value at a unit direction, with what the backward needs.
struct Eval {
  float ell;      // log c + log G(v)
  float L;        // log u
  float u;        // (v.z + 1)/2
  float w;        // 1 - u = |v - z|^2 / 4
  float E;        // expm1(p L) = u^p - 1 (accurate near u^p = 1)
  float epl;      // u^p = e^{p L} (accurate where it is tiny)
  float p, pm1;   // exponent p = 1 + eps + a c^2 and p - 1 = eps + a c^2
  float c2;       // anisotropy weight
  float X, Y, S;  // v.x, v.y, X^2 + Y^2
  float invS;     // 1 / S (used again by the derivatives)
};

__device__ __forceinline__ void cross(float ax, float ay, float az, float bx, float by, float bz,
                                      float& cx, float& cy, float& cz) {
  cx = fmaf(ay, bz, -az * by);
  cy = fmaf(az, bx, -ax * bz);
  cz = fmaf(ax, by, -ay * bx);
}

// log G(v) (eq. NASG; App. A with epsilon) for a unit v, plus log c.
__device__ __forceinline__ Eval eval_lobe(const Lobe& L, float vx, float vy, float vz, float eps) {
  Eval r;
  float yx, yy, yz;
  cross(L.zx, L.zy, L.zz, L.xx, L.xy, L.xz, yx, yy, yz);
  float dx = vx - L.zx, dy = vy - L.zy, dz = vz - L.zz;
  float sx = vx + L.zx, sy = vy + L.zy, sz = vz + L.zz;
  float w = 0.25f * fmaf(dx, dx, fmaf(dy, dy, dz * dz));   // 1 - u
  float u = 0.25f * fmaf(sx, sx, fmaf(sy, sy, sz * sz));   // u
  // log u: a polynomial in w for log(1 - w) near the axis, else the log of the
  // better-conditioned of 1 - w and u (one log either way)
  float lw = log1m_poly(w);
  float lu = flog(fsel(w <= 0.5f, 1.0f - w, u));
  r.L = fsel(w < 0.0625f, lw, lu);
  r.u = u;
  r.w = w;
  r.X = fmaf(vx, L.xx, fmaf(vy, L.xy, vz * L.xz));
  r.Y = fmaf(vx, yx, fmaf(vy, yy, vz * yz));
  r.S = fmaf(r.X, r.X, r.Y * r.Y);
  r.invS = frcp(r.S);
  r.c2 = fsel(r.S >= kMinNormal, r.X * r.X * r.invS, 0.0f);
  r.pm1 = fmaf(L.a, r.c2, eps);
  r.p = 1.0f + r.pm1;
  const float pl = r.p * r.L;
  r.E = expm1_neg(pl);                               // p L <= 0
  // u^p from the exponential expm1 already evaluates for p L <= -1/8: E + 1
  // would round a tiny u^p to 0
  r.epl = fsel(pl > -0.125f, r.E + 1.0f, fexp(pl));
  float lg = fmaf(2.0f * L.lam, r.E, r.pm1 * r.L);
  // G(-z) = 0: u == 0 only when v = -z exactly
  r.ell = fsel(u > 0.0f, L.logc + lg, -INFINITY);
  return r;
}

// log c + log G(v) alone (the query's mixture pdf): the same function as
// eval_lobe without the lobe's y axis. For a unit v and an orthonormal frame
// X^2 + Y^2 = 1 - (v.z)^2 = (1 - v.z)(1 + v.z) = 4 (1 - u) u, a product of the
// two cancellation-free terms already at hand; c^2 is capped at 1 against
// rounding (X^2 and 4 u (1 - u) come from different roundings).
__device__ __forceinline__ float eval_lobe_ell(const Lobe& L, float vx, float vy, float vz, float eps) {
  const float dx = vx - L.zx, dy = vy - L.zy, dz = vz - L.zz;
  const float sx = vx + L.zx, sy = vy + L.zy, sz = vz + L.zz;
  const float w4 = fmaf(dx, dx, fmaf(dy, dy, dz * dz));   // 4 (1 - u)
  const float u = 0.25f * fmaf(sx, sx, fmaf(sy, sy, sz * sz));
  // w = w4 / 4 exactly, so the tests on w4 and 1 - w = fma(w4, -1/4, 1) are
  // those on w, without forming it
  const float lw = log1m_poly4(w4);
  const float lu = flog(fsel(w4 <= 2.0f, fmaf(w4, -0.25f, 1.0f), u));
  const float Lu = fsel(w4 < 0.25f, lw, lu);
  const float X = fmaf(vx, L.xx, fmaf(vy, L.xy, vz * L.xz));
  const float S = w4 * u;
  const float c2 = fsel(S >= kMinNormal, fminf(X * X * frcp(S), 1.0f), 0.0f);
  const float pm1 = fmaf(L.a, c2, eps);                    // p - 1 without cancellation
  const float lg = fmaf(2.0f * L.lam, expm1_neg((1.0f + pm1) * Lu), pm1 * Lu);
  return fsel(u > 0.0f, L.logc + lg, -INFINITY);
}

// Gradient on the sphere of ell = log c + log G (eq. NASG; App. A) at a unit
// v, through v.z, X = v.x and Y = v.y (the same partials as backward_lobe):
// d ell/d(v.z) = (2 lam p u^p + p - 1) / (2u) and, with d ell/dp =
// log u (2 lam u^p + 1), the anisotropy c^2 = X^2 / (X^2 + Y^2) contributes
// a d ell/dp (2 X Y^2, -2 Y X^2) / (X^2 + Y^2)^2. Each partial multiplies the
// tangential part a - (v.a) v of its axis a, so the sum is tangential as it
// stands. Near the axis z - (v.z) v is formed without cancellation: as
// (v + z) - 2u v in the lobe's southern hemisphere and (z - v) + 2(1 - u) v
// in the northern one (exact identities, since 1 + v.z = 2u and 1 - v.z =
// 2(1 - u)); X/S and Y/S are formed before the products, so nothing
// overflows when v is within ~1e-10 rad of the axis. Zero where the lobe
// vanishes (v = -z).
__device__ __forceinline__ void dir_grad_lobe(const Lobe& L, const Eval& e, float vx, float vy, float vz,
                                              float& gx, float& gy, float& gz) {
  const bool live = e.u > 0.0f;
  const float epl = e.epl;   // u^p
  const float twolam = 2.0f * L.lam;
  const float GZ = fsel(live, fmaf(twolam * e.p, epl, e.pm1) * frcp(2.0f * e.u), 0.0f);
  const float Dp = e.L * fmaf(twolam, epl, 1.0f);
  const float coef = fsel(live && e.S >= kMinNormal, 2.0f * L.a * Dp, 0.0f);
  const float xs = e.X * e.invS, ys = e.Y * e.invS;
  const float GX = coef * xs * (e.Y * ys);
  const float GY = -coef * ys * (e.X * xs);
  float yx, yy, yz;
  cross(L.zx, L.zy, L.zz, L.xx, L.xy, L.xz, yx, yy, yz);
  const bool south = e.u <= 0.5f;
  const float sg = fsel(south, 1.0f, -1.0f);
  const float f = fsel(south, -2.0f * e.u, 2.0f * e.w);
  const float tzx = fmaf(f, vx, fmaf(sg, vx, L.zx));
  const float tzy = fmaf(f, vy, fmaf(sg, vy, L.zy));
  const float tzz = fmaf(f, vz, fmaf(sg, vz, L.zz));
  gx = fmaf(GZ, tzx, fmaf(GX, fmaf(-e.X, vx, L.xx), GY * fmaf(-e.Y, vx, yx)));
  gy = fmaf(GZ, tzy, fmaf(GX, fmaf(-e.X, vy, L.xy), GY * fmaf(-e.Y, vy, yy)));
  gz = fmaf(GZ, tzz, fmaf(GX, fmaf(-e.X, vz, L.xz), GY * fmaf(-e.Y, vz, yz)));
}

// One direction from a single lobe (App. C): (xi0, xi1) -> (s, rho) linearly,
// xi2 > 1/2 east. Stable form: (cos theta + 1)/2 = u with log u = log(1 + r)/p,
// r = log s / (2 lam) in [-1, 0], p = 1 + eps + a cos^2 phi, and (cos phi,
// sin phi) proportional to (cos rho, sqrt((1+eps+a)/(1+eps)) sin rho).
// log(1 + r) is taken two ways, each where it has no cancellation:
//  * r > -1/2: log1p(r), with log s = log(1 + (1 - xi0)(e^{-2 lam} - 1)) by
//    log1p (s > 1/2) or as the log of s itself;
//  * r <= -1/2 (s near its least value e^{-2 lam}, the lobe's far side):
//    1 + r = log(s e^{2 lam}) / (2 lam) = log1p(xi0 expm1(2 lam)) / (2 lam),
//    so xi0 = 0 gives exactly v = -z; beyond 2 lam = 88, where e^{-2 lam} is
//    below the normal float range, s = xi0 (to 1e-8 relative for xi0 >=
//    1e-30) and 1 + r = 1 + log(xi0) / (2 lam), 0 for xi0 = 0.
__device__ __forceinline__ void sample_lobe(const Lobe& L, float xi0, float xi1, float xi2,
                                            float eps, float& vx, float& vy, float& vz) {
  const float tl = 2.0f * L.lam;
  const float rtl = frcp(tl);
  float t = expm1_neg(-tl);                            // e^{-2 lam} - 1 in (-1, 0)
  float y0 = (1.0f - xi0) * t;                         // s - 1
  float ls_near = log1pf_(y0);
  float ls_far = flog(fmaf(1.0f - xi0, fexp(-tl), xi0));
  float ls = fsel(y0 > -0.5f, ls_near, ls_far);
  ls = fmaxf(ls, -tl);                                 // s >= e^{-2 lam}
  float rr = fmaxf(ls * rtl, -1.0f);                   // in [-1, 0]
  float opr_small = log1pf_(xi0 * expm1f_(fminf(tl, 88.0f))) * rtl;
  float opr_big = fsel(xi0 > 0.0f, fmaf(ls, rtl, 1.0f), 0.0f);
  float opr = fsel(tl <= 88.0f, opr_small, opr_big);  // 1 + r near 0
  float lopr = fsel(rr > -0.5f, log1pf_(rr), flog(opr));
  // cos(rho) = sin(pi xi1), sin(rho) = -cos(pi xi1); v_sin/v_cos take revolutions
  float crho = __builtin_amdgcn_sinf(0.5f * xi1);
  float srho = -__builtin_amdgcn_cosf(0.5f * xi1);
  float k = fsqrt((1.0f + eps + L.a) * frcp(1.0f + eps));
  float cphi, sphi, inv;
  unit_pair(crho, k * srho, cphi, sphi, inv);
  if (!(xi2 > 0.5f)) { cphi = -cphi; sphi = -sphi; }
  float p = fmaf(L.a, cphi * cphi, 1.0f + eps);
  float Lu = lopr * frcp(p);                           // log((cos theta + 1)/2)
  float u = fexp(Lu);
  float om = -expm1_neg(Lu);                           // 1 - u (Lu <= 0)
  float ct = 1.0f - 2.0f * om;
  float st = 2.0f * fsqrt(fmaxf(u * om, 0.0f));
  float yx, yy, yz;
  cross(L.zx, L.zy, L.zz, L.xx, L.xy, L.xz, yx, yy, yz);
  float ax = fmaf(cphi, L.xx, sphi * yx);
  float ay = fmaf(cphi, L.xy, sphi * yy);
  float az = fmaf(cphi, L.xz, sphi * yz);
  vx = fmaf(st, ax, ct * L.zx);
  vy = fmaf(st, ay, ct * L.zy);
  vz = fmaf(st, az, ct * L.zz);
}

// d(loss)/d(raw outputs) of one lobe. gk = dLoss/d ell_k (= g r_k with
// r_k the lobe's responsibility), galpha = dLoss/d logit_k (= g (r_k - A_k)).
// Derivation: ell = logA - logK + log G with
//   d(-logK)/d log lam = 1 - 2 lam / expm1(2 lam),  d(-logK)/d log a = a / (2 (1+eps+a)),
//   d logG/d log lam = 2 lam E,  d logG/d p = L (2 lam e^{pL} + 1),
//   d logG/d L = 2 lam p e^{pL} + p - 1,  dL/d(v.z) = 1/(2u),
//   d c^2/dX = 2 X Y^2 / S^2,  d c^2/dY = -2 Y X^2 / S^2,
// then through X = v.x, Y = v.y, v.z to the Euler sines/cosines, the pair
// normalisation and tanh(o/2)' = (1 - d^2)/2.
__device__ __forceinline__ void backward_lobe(const Lobe& L, const LobeAux& A, const Eval& e,
                                              float vx, float vy, float vz, float eps,
                                              float gk, float galpha, float g[8]) {
  bool live = e.u > 0.0f && gk != 0.0f;
  float epl = e.epl;
  float twolam = 2.0f * L.lam;
  // log lambda
  g[5] = fsel(A.lam_in && live, gk * fmaf(twolam, e.E, A.omq), 0.0f);
  // log a
  float Dp = e.L * fmaf(twolam, epl, 1.0f);
  float ga = L.a * fmaf(e.c2, Dp, 0.5f * frcp(1.0f + eps + L.a));
  g[6] = fsel(A.a_in && live, gk * ga, 0.0f);
  g[7] = galpha;
  // direction terms
  float DL = fmaf(twolam * e.p, epl, e.pm1);
  float gZ = fsel(live, gk * DL * frcp(2.0f * e.u), 0.0f);
  // X/S and Y/S first: (1/S)^2 alone would overflow within ~1e-10 rad of the axis
  float coef = fsel(live && e.S >= kMinNormal, gk * L.a * Dp * 2.0f, 0.0f);
  float xs = e.X * e.invS, ys = e.Y * e.invS;
  float gX = coef * xs * (e.Y * ys);
  float gY = -coef * ys * (e.X * xs);
  // X = ctau R + stau Q, Y = -stau R + ctau Q, Zc = st P + ct vz, R = ct P - st vz
  float P = fmaf(vx, A.cp, vy * A.sp);
  float Q = fmaf(-vx, A.sp, vy * A.cp);
  float R = fmaf(A.ct, P, -A.st * vz);
  float gR = fmaf(A.ctau, gX, -A.stau * gY);
  float gQ = fmaf(A.stau, gX, A.ctau * gY);
  float g_ctau = fmaf(R, gX, Q * gY);
  float g_stau = fmaf(Q, gX, -R * gY);
  float gP = fmaf(A.st, gZ, A.ct * gR);
  float g_ct = fmaf(vz, gZ, P * gR);
  float g_st = fmaf(P, gZ, -vz * gR);
  float g_cp = fmaf(vx, gP, vy * gQ);
  float g_sp = fmaf(vy, gP, -vx * gQ);
  // theta: ct = tanh(o0/2), st = sech(o0/2): dct/do0 = st^2/2, dst/do0 = -st ct/2
  g[0] = 0.5f * A.st * fmaf(A.st, g_ct, -A.ct * g_st);
  // (cp, sp) = (d2, d1)/n: d/d d1 = cp t, d/d d2 = -sp t with t = (cp g_sp - sp g_cp)/n
  float tp = fmaf(A.cp, g_sp, -A.sp * g_cp) * A.inv_np;
  float tt = fmaf(A.ctau, g_stau, -A.stau * g_ctau) * A.inv_nt;
  // tanh'(o/2) = (1 - d^2)/2
  g[1] = A.cp * tp * A.h1;
  g[2] = -A.sp * tp * A.h2;
  g[3] = A.ctau * tt * A.h3;
  g[4] = -A.stau * tt * A.h4;
}

}  // namespace nasg
