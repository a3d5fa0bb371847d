// Device math for the likelihood kernels: FP64 complex helpers, the Faddeeva
// function w(z) on the closed upper half plane, and erfcx on [0, inf).
//
// w(z) = e^{-z^2} erfc(-iz) enters through the Gaussian-resolution convolution
// of exponential decays (the paper's Faddeeva-function route and its large
// t/sigma limit).  Two published methods are combined:
//   * |z| >= 6 or Im z >= 3.4: Laplace's continued fraction for w in its even
//     contracted (Jacobi) form
//         w(z) = (i z / sqrt(pi)) / (z^2 - 1/2 - c_1/(z^2 - 5/2 - c_2/(z^2 - 9/2 - ...))),
//     c_k = (2k-1)(2k)/4, evaluated forward with the Wallis recurrences so that
//     only one complex division is needed; 10 levels give <= 2e-14 relative
//     error in this region.
//   * otherwise: Weideman's rational series with N = 40 (SIAM J. Numer. Anal.
//     31 (1994) 1497), <= 2e-14 relative for |z| < 6.
#pragma once

#include <hip/hip_runtime.h>

#include "cf_depth.h"
#include "minimax_coeffs.h"
#include "weideman_coeffs.h"

namespace ipx {

constexpr double kSqrtPi = 1.7724538509055160273;
constexpr double kInvSqrtPi = 0.56418958354775628695;
constexpr double kInvSqrt2Pi = 0.39894228040143267794;
constexpr double kSqrt2 = 1.4142135623730950488;
constexpr double kInvSqrt2 = 0.70710678118654752440;

struct cplx {
  double re, im;
};

// 1/x from the hardware reciprocal estimate and two Newton steps (relative
// error near 1 ulp, not correctly rounded; used where the exact IEEE quotient
// is not needed).  x must be finite and non-zero.
__device__ __forceinline__ double rcp(double x) {
  double r = __builtin_amdgcn_rcp(x);
  double e = fma(-x, r, 1.0);
  r = fma(e, r, r);
  e = fma(-x, r, 1.0);
  return fma(e, r, r);
}

__device__ __forceinline__ cplx cx(double re, double im) { return cplx{re, im}; }
__device__ __forceinline__ cplx cadd(cplx a, cplx b) { return cplx{a.re + b.re, a.im + b.im}; }
__device__ __forceinline__ cplx csub(cplx a, cplx b) { return cplx{a.re - b.re, a.im - b.im}; }
__device__ __forceinline__ cplx cscale(cplx a, double s) { return cplx{a.re * s, a.im * s}; }
__device__ __forceinline__ cplx cmul(cplx a, cplx b) {
  return cplx{a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
// Smith's scaled division (no overflow for |b| near the double range limits).
__device__ __forceinline__ cplx cdiv(cplx a, cplx b) {
  if (fabs(b.re) >= fabs(b.im)) {
    const double r = b.im * rcp(b.re);
    const double inv = rcp(b.re + b.im * r);
    return cplx{(a.re + a.im * r) * inv, (a.im - a.re * r) * inv};
  }
  const double r = b.re * rcp(b.im);
  const double inv = rcp(b.re * r + b.im);
  return cplx{(a.re * r + a.im) * inv, (a.im * r - a.re) * inv};
}

// ---------------------------------------------------------------------------
// Elementary functions of the event loops.  The library versions carry
// double-double steps and argument ranges the likelihood does not need; these
// take the textbook route (an additive reduction with the constant split in
// two, Cody and Waite's method, then a near-minimax polynomial on the reduced
// interval, with coefficients from gen_minimax.py) and are within about 2 ulp
// over their stated domains (measured against correctly rounded values by the
// math self-check entry point).
// ---------------------------------------------------------------------------
// Rare branches.  The functions below run their common path on every lane
// and then recompute, inside a wave vote, the lanes outside its domain: a
// wave where no lane needs the rare path pays one vote, not the exec-mask
// bookkeeping of a divergent if/else, and each lane's result is the one its
// own branch gives (the common path's values on such lanes are discarded).
__device__ __forceinline__ bool any_lane(bool c) { return __any(c) != 0; }

constexpr double kLn2Hi = 0x1.62e42fefa39efp-1;   // ln 2 rounded to double
constexpr double kLn2Lo = 0x1.abc9e3b39803fp-56;  // ln 2 - kLn2Hi
constexpr double kLog2E = 0x1.71547652b82fep+0;   // 1 / ln 2
constexpr double kPio2Hi = 0x1.921fb54442d18p+0;  // pi/2 rounded to double
constexpr double kPio2Lo = 0x1.1a62633145c07p-54; // pi/2 - kPio2Hi
constexpr double kTwoOverPi = 0x1.45f306dc9c883p-1;
constexpr double kSqrtHalf = 0x1.6a09e667f3bcdp-1;

// e^x for x in [-1100, 2^30] or NaN.  x = k ln2 + r with k = rint(x / ln2):
// x - k kLn2Hi is exact under the fused multiply-add (both are multiples of
// 2^-53 and the difference is below 1/2), so |r| <= ln2/2 up to rounding;
// e^r = 1 + r + r^2/2 + r^3 E(r) with the degree-8 near-minimax E of
// minimax_coeffs.h (approximation error below 4e-17 relative), then scaled by
// 2^k (0 below about -745, +inf above about 709.8: the scale saturates).
__device__ __forceinline__ double exp_core(double x) {
  const double k = rint(x * kLog2E);
  const double r = fma(-k, kLn2Lo, fma(-k, kLn2Hi, x));
  constexpr int n = sizeof(kExpPoly) / sizeof(double);
  double p = kExpPoly[n - 1];
#pragma unroll
  for (int i = n - 2; i >= 0; --i) p = fma(p, r, kExpPoly[i]);
  p = fma(p, r, 0.5);
  p = fma(p, r, 1.0);
  p = fma(p, r, 1.0);
  return ldexp(p, static_cast<int>(k));
}

// e^x for every x: arguments clamped to [-1100, 710] (results 0 and +inf
// beyond); NaN propagates.
__device__ __forceinline__ double exp_fast(double x) {
  const double y = exp_core(fmin(fmax(x, -1100.0), 710.0));
  return x == x ? y : x;
}

// e^x for x <= 2^30 (-inf and NaN included), the value exp_fast gives there,
// with one select instead of the two clamps and the NaN test: arguments below
// -1100 are raised to it (a comparison, so NaN passes through).  Above 2^30
// the value is unspecified (the scale 2^k leaves the int range; this hardware's
// conversion saturates, giving +inf).  The event loops use it where an
// argument exceeds 2^30 only for event values far outside any physical range
// (decay times beyond 10^9 ps, say).
__device__ __forceinline__ double exp_lo(double x) { return exp_core(x < -1100.0 ? -1100.0 : x); }

// ln x for x > 0 (positive normal or subnormal; other arguments go to the
// library log, so 0 gives -inf and negative x NaN).  x = 2^e m with m in
// [sqrt(1/2), sqrt 2), ln m = 2 atanh(s) = 2s + 2s s^2 L(s^2),
// s = (m - 1)/(m + 1), |s| <= 0.172, with the degree-6 near-minimax L of
// minimax_coeffs.h (approximation error below 5e-18 relative); ln x =
// e ln2 + ln m with the product e kLn2Hi exact inside the fused multiply-add.
__device__ __forceinline__ double log_fast(double x) {
  double m = __builtin_amdgcn_frexp_mant(x);  // [1/2, 1)
  int e = __builtin_amdgcn_frexp_exp(x);
  if (m < kSqrtHalf) {
    m *= 2.0;
    --e;
  }
  const double s = (m - 1.0) * rcp(m + 1.0);
  const double s2 = s * s;
  constexpr int n = sizeof(kLogPoly) / sizeof(double);
  double q = kLogPoly[n - 1];
#pragma unroll
  for (int i = n - 2; i >= 0; --i) q = fma(q, s2, kLogPoly[i]);
  const double s2x = 2.0 * s;
  const double lm = fma(s2x * s2, q, s2x);
  const double ef = static_cast<double>(e);
  double r = fma(ef, kLn2Hi, fma(ef, kLn2Lo, lm));
  const bool other = !__builtin_amdgcn_class(x, 0x180);  // not positive normal/subnormal
  if (any_lane(other)) {
    if (other) r = log(x);
  }
  return r;
}

// sin x and cos x for |x| <= 2^19 (the library sincos beyond): x = k pi/2 + r
// with x - k kPio2Hi exact under the fused multiply-add (|r| <= pi/4; absolute
// error of r below 2e-27), sin r = r - r^3 S(r^2) and cos r =
// 1 + r^2 (-1/2 + r^2 C(r^2)) with the degree-5 near-minimax S and C of
// minimax_coeffs.h (approximation errors below 3e-17 relative), then the
// quadrant k mod 4.
__device__ __forceinline__ void sincos_fast(double x, double* sn, double* cs) {
  const double k = rint(x * kTwoOverPi);
  const double r = fma(-k, kPio2Lo, fma(-k, kPio2Hi, x));
  const double r2 = r * r;
  constexpr int ns = sizeof(kSinPoly) / sizeof(double);
  double ps = kSinPoly[ns - 1];
#pragma unroll
  for (int i = ns - 2; i >= 0; --i) ps = fma(ps, r2, kSinPoly[i]);
  const double s = fma(-(r * r2), ps, r);
  constexpr int nc = sizeof(kCosPoly) / sizeof(double);
  double pc = kCosPoly[nc - 1];
#pragma unroll
  for (int i = nc - 2; i >= 0; --i) pc = fma(pc, r2, kCosPoly[i]);
  pc = fma(pc, r2, -0.5);
  const double c = fma(r2, pc, 1.0);
  const int q = static_cast<int>(k);
  const double a = (q & 1) ? c : s;   // sin of the quadrant's base
  const double b = (q & 1) ? s : c;
  double so = (q & 2) ? -a : a;
  double co = ((q + 1) & 2) ? -b : b;
  const bool big = fabs(x) > 0x1p19;
  if (any_lane(big)) {
    if (big) sincos(x, &so, &co);
  }
  *sn = so;
  *cs = co;
}

// e^x with a short Taylor polynomial when |x| <= 2^-9 (through x^5:
// truncation below 1e-19 relative), exp_fast otherwise.
__device__ __forceinline__ double exp_small(double x) {
  double r = 1.0 + x * (1.0 + x * (0.5 + x * (1.0 / 6.0 + x * (1.0 / 24.0 + x * (1.0 / 120.0)))));
  const bool large = fabs(x) > 0x1p-9;
  if (any_lane(large)) {
    if (large) r = exp_fast(x);
  }
  return r;
}

// sin and cos with Taylor polynomials when |x| <= 0.05 (sin through x^9, cos
// through x^8: truncation below 3e-20 relative), sincos_fast otherwise.
__device__ __forceinline__ void sincos_small(double x, double* s, double* c) {
  const double x2 = x * x;
  double so = x * (1.0 - x2 * (1.0 / 6.0 - x2 * (1.0 / 120.0 - x2 * (1.0 / 5040.0 - x2 * (1.0 / 362880.0)))));
  double co = 1.0 - x2 * (0.5 - x2 * (1.0 / 24.0 - x2 * (1.0 / 720.0 - x2 * (1.0 / 40320.0))));
  const bool large = fabs(x) > 0.05;
  if (any_lane(large)) {
    if (large) sincos_fast(x, &so, &co);
  }
  *s = so;
  *c = co;
}

// The depth thresholds of cf_depth.h are multiples of 1/8 in [1/8, 32): as
// integers 8 E_min[K] they pack into one 64-bit word (K = 1 .. 8) and one
// byte (K = 9), so that the depth search below reads no memory (a table in
// memory costs a dependent scalar load and its wait per search step).
constexpr unsigned long long cf_pack_thresholds() {
  unsigned long long v = 0;
  for (int i = 0; i < 8; ++i) v |= static_cast<unsigned long long>(kCfDepthE[i] * 8.0) << (8 * i);
  return v;
}
constexpr bool cf_thresholds_pack() {
  for (int i = 0; i < kCfMaxDepth - 1; ++i) {
    const double t = kCfDepthE[i] * 8.0;
    if (!(t >= 1.0 && t <= 255.0 && t == static_cast<double>(static_cast<int>(t)))) return false;
  }
  return true;
}
static_assert(kCfMaxDepth == 10 && cf_thresholds_pack(), "depth thresholds must be multiples of 1/8 in [1/8, 32)");
constexpr unsigned long long kCfTh8 = cf_pack_thresholds();
constexpr int kCfTh9 = static_cast<int>(kCfDepthE[8] * 8.0);

// Depth of the continued fraction for correction terms whose exponent
// E = (Im z)^2 - (Re z)^2 is at least the given value on every active lane of
// the wave (the table in cf_depth.h bounds the truncation error of a K-level
// fraction times the correction's size by 2^-57 of the main term).  The result
// is the same on all lanes: a binary search with wave votes on n = trunc(8 E),
// for which n < 8 E_min[K] exactly when E < E_min[K] (a NaN or negative E
// asks for the full depth).
__device__ __forceinline__ int cf_depth_wave(double E) {
  const int n = static_cast<int>(fmin(fmax(E * 8.0, -1.0), 1e9));
  int lo = 1, hi = kCfMaxDepth;
#pragma unroll
  for (int it = 0; it < 4; ++it) {
    const int mid = (lo + hi) >> 1;
    const int th = mid <= 8 ? static_cast<int>((kCfTh8 >> (8 * (mid - 1))) & 255u) : kCfTh9;
    if (__any(n < th)) lo = mid + 1;
    else hi = mid;
  }
  return hi;
}

// One level K of the Jacobi fraction's Wallis recurrences, in scaled form.
// The plain recurrence is P_K = (z^2 - a_K) P_{K-1} - c_K P_{K-2} with
// a_K = 2K + 1/2 and c_K = (2K - 1)(2K)/4, the same for Q.  Dividing by
// alpha_K = c_K alpha_{K-2} (alpha_{-1} = alpha_0 = 1) gives
// P'_K = d_K P'_{K-1} - P'_{K-2}, d_K = (z^2 - a_K) r_K, r_K = alpha_{K-1} /
// alpha_K, and the same for Q'; the fraction only needs Q/P = Q'/P', and the
// scaled level has no product with c_K (one fused operation per real
// component and step).  The constants are folded at compile time.  The two
// newest numerators live in p and pm and are updated in place, alternating
// (odd K writes pm, even K writes p), so that every early exit leaves them in
// the same registers.
constexpr double cf_c(int K) { return (2.0 * K - 1.0) * (2.0 * K) * 0.25; }
constexpr double cf_alpha(int K) { return K <= 0 ? 1.0 : cf_c(K) * cf_alpha(K - 2); }

// d a - b for complex d, a, b (two fused operations per component)
__device__ __forceinline__ cplx cmul_sub1(cplx d, cplx a, cplx b) {
  return cplx{fma(d.re, a.re, fma(-d.im, a.im, -b.re)), fma(d.re, a.im, fma(d.im, a.re, -b.im))};
}

template <int K>
__device__ __forceinline__ void cf_level(const cplx& z2, cplx& p, cplx& q, cplx& pm, cplx& qm) {
  constexpr double a = 2.0 * K + 0.5;
  constexpr double r = cf_alpha(K - 1) / cf_alpha(K);
  const cplx d{(z2.re - a) * r, z2.im * r};
  if constexpr (K % 2 == 1) {
    pm = cmul_sub1(d, p, pm);
    qm = cmul_sub1(d, q, qm);
  } else {
    p = cmul_sub1(d, pm, p);
    q = cmul_sub1(d, qm, q);
  }
}

template <int K>
__device__ __forceinline__ void cf_level(const double& z2, double& p, double& q, double& pm, double& qm) {
  constexpr double a = 2.0 * K + 0.5;
  constexpr double r = cf_alpha(K - 1) / cf_alpha(K);
  const double d = (z2 - a) * r;
  if constexpr (K % 2 == 1) {
    pm = fma(d, p, -pm);
    qm = fma(d, q, -qm);
  } else {
    p = fma(d, pm, -p);
    q = fma(d, qm, -q);
  }
}

// Levels 1 .. depth' with depth' = depth rounded up to odd, at most 10 (depth
// wave-uniform, 1 .. kCfMaxDepth): uniform branches around pairs of
// straight-line levels.  On return (p, q) hold the scaled numerators P', Q'
// of level depth'.
template <typename T>
__device__ __forceinline__ void cf_levels(const T& z2, T& p, T& q, T& pm, T& qm, int depth) {
  static_assert(kCfMaxDepth == 10, "the level calls below spell out 10 levels");
  cf_level<1>(z2, p, q, pm, qm);
  if (depth >= 2) {
    cf_level<2>(z2, p, q, pm, qm);
    cf_level<3>(z2, p, q, pm, qm);
    if (depth >= 4) {
      cf_level<4>(z2, p, q, pm, qm);
      cf_level<5>(z2, p, q, pm, qm);
      if (depth >= 6) {
        cf_level<6>(z2, p, q, pm, qm);
        cf_level<7>(z2, p, q, pm, qm);
        if (depth >= 8) {
          cf_level<8>(z2, p, q, pm, qm);
          cf_level<9>(z2, p, q, pm, qm);
          if (depth >= 10) cf_level<10>(z2, p, q, pm, qm);
        }
      }
    }
  }
  // an odd last level leaves the newest numerators in pm, qm
  if (depth < 10) {
    p = pm;
    q = qm;
  }
}

// Jacobi continued fraction with `depth` levels (1 .. 10, wave-uniform),
// forward Wallis recurrences.  Valid (and used) for Im z >= 3.4 or |z| >= 6
// with |z| <= 1e6; 10 levels give full precision there.
__device__ __forceinline__ cplx faddeeva_cf(cplx z, int depth) {
  const cplx z2 = cmul(z, z);
  cplx pm{1.0, 0.0}, qm{0.0, 0.0};          // P_{-1}, Q_{-1}
  cplx p{z2.re - 0.5, z2.im}, q{1.0, 0.0};  // P_0, Q_0
  cf_levels(z2, p, q, pm, qm, depth);
  // w = i z Q / (sqrt(pi) P) = i z Q conj(P) / (sqrt(pi) |P|^2) with the
  // scaled P', Q': for |z| <= 1e6 and at most 10 levels |P'|^2 stays far
  // inside the double range
  const cplx izq = cmul(cplx{-z.im, z.re}, q);
  const double inv = kInvSqrtPi * rcp(fma(p.re, p.re, p.im * p.im));
  return cplx{fma(izq.re, p.re, izq.im * p.im) * inv, fma(izq.im, p.re, -izq.re * p.im) * inv};
}

// Weideman N = 40 rational series, used for |z| < 6 and Im z < 3.4.
__device__ __noinline__ cplx faddeeva_series(cplx z) {
  const double L = IPX_WEID_L;
  const cplx lm{L + z.im, -z.re};  // L - i z
  const cplx lp{L - z.im, z.re};   // L + i z
  const cplx Z = cdiv(lp, lm);
  cplx p{ipx_weid_a[IPX_WEID_N - 1], 0.0};
  for (int n = IPX_WEID_N - 2; n >= 0; --n) {
    p = cmul(p, Z);
    p.re += ipx_weid_a[n];
  }
  const cplx r = cdiv(cplx{1.0, 0.0}, lm);
  return cadd(cscale(cmul(p, cmul(r, r)), 2.0), cscale(r, kInvSqrtPi));
}

// w(z) for Im z >= 0; depth as for faddeeva_cf (full precision by default).
__device__ __forceinline__ cplx faddeeva_upper(cplx z, int depth = kCfMaxDepth) {
  const double r2 = z.re * z.re + z.im * z.im;
  cplx w = faddeeva_cf(z, depth);
  const bool huge = r2 > 1e12;
  const bool inner = !(z.im >= 3.4 || r2 >= 36.0);  // (NaN included)
  if (any_lane(huge || inner)) {
    if (huge) {
      // asymptotic i/(sqrt(pi) z) (1 + 1/(2 z^2)); relative error < 1e-24 here
      const cplx iz = cdiv(cplx{0.0, kInvSqrtPi}, z);
      const cplx z2i = cdiv(cplx{0.5, 0.0}, cmul(z, z));
      w = cmul(iz, cplx{1.0 + z2i.re, z2i.im});
    } else if (inner) {
      w = faddeeva_series(z);
    }
  }
  return w;
}

// erfcx(y) = e^{y^2} erfc(y) = w(i y) for y >= 0: the continued fraction in
// real arithmetic (depth as for faddeeva_cf) for y >= 3.4, the (out-of-line)
// rational series otherwise.
__device__ __forceinline__ double erfcx_pos(double y, int depth = kCfMaxDepth) {
  const double z2 = -y * y;
  double pm = 1.0, qm = 0.0, p = z2 - 0.5, q = 1.0;
  cf_levels(z2, p, q, pm, qm, depth);
  double r = -y * q * kInvSqrtPi * rcp(p);
  const bool small = y < 3.4, huge = y > 1e6;
  if (any_lane(small || huge)) {
    if (small) r = faddeeva_series(cplx{0.0, y}).re;
    else if (huge) r = kInvSqrtPi / y * (1.0 - 0.5 / (y * y));
  }
  return r;
}

}  // namespace ipx
