// Ipatia signal shape (Example 1 of the paper: an Ipatia peak on an
// exponential background, the signal normalised numerically on a grid).
//
// Shape (Santos, Dupertuis, NIM A 764 (2014) 150), d = m - mu:
//   core   G(d) = q^{nu} K_{|nu|}(zeta q) e^{beta d},  nu = lambda - 1/2,
//          q = sqrt(1 + d^2 / (A^2 sigma^2)),  A^2 = zeta K_lambda(zeta) / K_{lambda+1}(zeta)
//          (zeta = 0: G = q^{2 lambda - 1} e^{beta d}, A^2 = -2 (lambda + 1));
//   tails  A_l (B_l - d)^{-n} below -a sigma, A_r (B_r + d)^{-n2} above a2 sigma,
//          matching G and dG/dd at the junctions (constants hoisted per call).
// Model: P(m) = f I(m - mu) / N_I + (1 - f) e^{-k (m - 5200)} / N_E, with
// N_I = dm sum_g I(m_g - mu) over 16384 grid midpoints (a device reduction in
// a fixed order, before the event pass), N_E analytic.
//
// K_mu and K_{mu+1} for |mu| <= 1/2 (the order reduced by an integer, then
// the upward recurrence K_{v+1} = K_{v-1} + (2v/x) K_v, stable for K):
//   x <= 2: Temme's series (J. Comput. Phys. 19 (1975) 324),
//           K_mu = sum_k c_k f_k,  K_{mu+1} = (2/x) sum_k c_k (p_k - k f_k),
//           c_k = (x^2/4)^k / k!, f_k = (k f_{k-1} + p_{k-1} + q_{k-1}) / (k^2 - mu^2),
//           p_k = p_{k-1} / (k - mu), q_k = q_{k-1} / (k + mu),
//           f_0 = mu pi / sin(mu pi) [cosh(s) G_1 + sinh(s)/s ln(2/x) G_2], s = mu ln(2/x),
//           p_0 = (x/2)^{-mu} Gamma(1 + mu) / 2, q_0 = (x/2)^{mu} Gamma(1 - mu) / 2,
//           with G_1, G_2, Gamma(1 +- mu) hoisted per call;
//   x > 2:  the trapezoidal rule (exponentially convergent for this analytic,
//           rapidly decaying integrand; Trefethen and Weideman, SIAM Rev. 56
//           (2014) 385) on K_v(x) = e^{-x} int_0^inf e^{-s^2} cosh(v t) 2 ds / sqrt(2x + s^2),
//           the substitution t = 2 asinh(s / sqrt(2x)) of the integral
//           int_0^inf e^{-x cosh t} cosh(v t) dt; step 0.35, 20 nodes
//           (relative error below 2e-14 for x >= 2, |v| <= 3/2).
#pragma once

#include <hip/hip_runtime.h>
#include <cmath>

#include "ipx_kernels.h"
#include "rgamma_coeffs.h"

namespace ipx {

constexpr int kIpatiaGrid = 1 << 14;
constexpr int kIpatiaGridWg = kIpatiaGrid / kThreads;   // 64 workgroups of grid points
constexpr int kTemmeTerms = 60;   // Temme's series: terms k = 1 .. kTemmeTerms - 1 at most
constexpr int kTrapNodes = 20;    // trapezoidal rule: nodes s_j = j h, j = 0 .. 19
constexpr double kTrapStep = 0.35;

struct IpatiaConst {
  double mu, beta;
  double a2s2;            // A^2 sigma^2
  double inv_a2s2;        // 1 / (A^2 sigma^2)
  double pw;              // exponent of q: lambda - 1/2 (zeta > 0) or 2 lambda - 1 (zeta = 0)
  double zeta;            // 0: the Student-like limit, no Bessel function
  // Bessel order |lambda - 1/2| = m + tmu, |tmu| <= 1/2, and Temme's constants
  double tmu, g1, g2, gp, gm, fact;
  double igp, igm;        // 1 / gp, 1 / gm
  int m;
  int pad;
  // the series' divisors as reciprocals, row k: 1/k, 1/(k - tmu), 1/(k + tmu),
  // 1/(k^2 - tmu^2) (row 0 unused)
  double rk[kTemmeTerms][4];
  // the trapezoidal rule's node weights (1/2 at j = 0) x 2 exp(-s_j^2) and s_j^2
  double tw[kTrapNodes], ts2[kTrapNodes];
  // tails
  double dl, Al, Bl, nl;  // junction -a sigma, A_l, B_l, n
  double dr, Ar, Br, nr;  // junction a2 sigma, A_r, B_r, n2
  // mixture
  double f, cB, k;        // f, (1 - f) / N_E, background slope
  double dm, lo;          // grid step and the range start
  const double* inv_norm; // device: 1 / N_I of this call (written by the grid pass)
};

// sinh(s) / s: its Taylor series through s^16 for |s| < 1/2 (truncation below
// 1e-19 relative), (e^s - e^-s) / (2 s) from the given exponentials above.
__device__ __forceinline__ double sinhc(double s, double es, double ies) {
  if (fabs(s) >= 0.5) return 0.5 * (es - ies) * rcp(s);
  const double t = s * s;
  double p = 1.0 / 355687428096000.0;        // 1/17!
  p = fma(p, t, 1.0 / 1307674368000.0);      // 1/15!
  p = fma(p, t, 1.0 / 6227020800.0);         // 1/13!
  p = fma(p, t, 1.0 / 39916800.0);           // 1/11!
  p = fma(p, t, 1.0 / 362880.0);             // 1/9!
  p = fma(p, t, 1.0 / 5040.0);
  p = fma(p, t, 1.0 / 120.0);
  p = fma(p, t, 1.0 / 6.0);
  return fma(p, t, 1.0);
}

// K_tmu(x), K_{tmu+1}(x), |tmu| <= 1/2, x > 0; ix = 1/x.  The divisions of
// both methods are products with reciprocals (the series' divisors hoisted
// per call, the rest through the hardware reciprocal), and the elementary
// functions are the event loops' own (ipx_math.h).
__device__ __forceinline__ void bessel_k_pair(const IpatiaConst& c, double x, double ix, double* k0, double* k1) {
  const double mu = c.tmu;
  if (x <= 2.0) {
    const double lx = log_fast(2.0 * ix);
    const double s = mu * lx;
    const double es = exp_fast(s);
    const double ies = rcp(es);
    const double ch = 0.5 * (es + ies);
    const double shs = sinhc(s, es, ies);
    double f = c.fact * (ch * c.g1 + shs * lx * c.g2);
    double p = 0.5 * es * c.igp;
    double q = 0.5 * ies * c.igm;
    double cc = 1.0;
    const double d = 0.25 * x * x;
    double s0 = f, s1 = p;
    for (int k = 1; k < kTemmeTerms; ++k) {
      const double dk = (double)k;
      const double* r = c.rk[k];
      f = (dk * f + p + q) * r[3];
      cc *= d * r[0];
      p *= r[1];
      q *= r[2];
      const double t0 = cc * f, t1 = cc * (p - dk * f);
      s0 += t0;
      s1 += t1;
      if (fabs(t0) < 1e-17 * fabs(s0) && fabs(t1) < 1e-17 * fabs(s1)) break;
    }
    *k0 = s0;
    *k1 = s1 * (2.0 * ix);
    return;
  }
  const double r2x = sqrt(2.0 * x), inv_r2x = rcp(r2x);
  double s0 = 0.0, s1 = 0.0;
#pragma unroll 4
  for (int j = 0; j < kTrapNodes; ++j) {
    const double sv = j * kTrapStep;
    const double y = sv * inv_r2x;
    const double r = sqrt(1.0 + y * y);
    const double em = exp_fast(2.0 * mu * log_fast(y + r));   // e^{mu t}
    const double iem = rcp(em);
    const double cm = 0.5 * (em + iem), sm = 0.5 * (em - iem);
    const double c1 = cm * (1.0 + 2.0 * y * y) + sm * (2.0 * y * r);   // cosh((mu + 1) t)
    const double wgt = c.tw[j] * rcp(sqrt(2.0 * x + c.ts2[j]));
    s0 += wgt * cm;
    s1 += wgt * c1;
  }
  const double ex = exp_fast(-x) * kTrapStep;
  *k0 = ex * s0;
  *k1 = ex * s1;
}

// K_{m + tmu}(x) by the upward recurrence.
__device__ __forceinline__ double bessel_k(const IpatiaConst& c, double x) {
  const double ix = rcp(x);
  double km, kp;
  bessel_k_pair(c, x, ix, &km, &kp);
  if (c.m == 0) return km;
  double v = c.tmu + 1.0;   // kp = K_v
  for (int j = 1; j < c.m; ++j) {
    const double kn = km + (2.0 * v * ix) * kp;
    km = kp;
    kp = kn;
    v += 1.0;
  }
  return kp;
}

// The shape: power-law tails, and the core q^pw e^{beta d} (one exponential
// of pw ln q + beta d) times the Bessel factor.
__device__ __forceinline__ double ipatia_shape(const IpatiaConst& c, double d) {
  if (d < c.dl) return c.Al * exp_fast(-c.nl * log_fast(c.Bl - d));
  if (d > c.dr) return c.Ar * exp_fast(-c.nr * log_fast(c.Br + d));
  const double q = sqrt(fma(d * d, c.inv_a2s2, 1.0));
  const double g = exp_fast(fma(c.pw, log_fast(q), c.beta * d));
  return c.zeta == 0.0 ? g : g * bessel_k(c, c.zeta * q);
}

// Grid pass: part[wg] = sum over the workgroup's grid points of I(m_g - mu).
__global__ __launch_bounds__(kThreads) void k_ipatia_grid(const IpatiaConst* __restrict__ kc,
                                                          double* __restrict__ part) {
  __shared__ double lds4[kThreads / 64];
  const IpatiaConst& c = *kc;
  const int g = blockIdx.x * kThreads + threadIdx.x;
  const double m = c.lo + ((double)g + 0.5) * c.dm;
  double v = ipatia_shape(c, m - c.mu);
  v = wave_sum(v);
  if ((threadIdx.x & 63) == 0) lds4[threadIdx.x >> 6] = v;
  __syncthreads();
  if (threadIdx.x == 0) part[blockIdx.x] = (lds4[0] + lds4[1]) + (lds4[2] + lds4[3]);
}

// inv[0] = 1 / (dm sum of the workgroup sums, in index order).
__global__ __launch_bounds__(kThreads) void k_ipatia_norm(const IpatiaConst* __restrict__ kc,
                                                          const double* __restrict__ part, double* __restrict__ inv) {
  const double t = reduce_component(part, kIpatiaGridWg);
  if (threadIdx.x == 0) inv[0] = 1.0 / (kc->dm * t);
}

// One event: acc[0] += w ln P.
__device__ __forceinline__ void event_ipatia(const IpatiaConst& c, double inv_norm, double m, double w,
                                             double* acc) {
  const double P = c.f * ipatia_shape(c, m - c.mu) * inv_norm + c.cB * exp_fast(-c.k * (m - kMLo));
  acc[0] += w * log_fast(P);
}

// Host: the per-call constants from theta = (f, mu, sigma, lambda, zeta,
// beta, a, n, a2, n2, k); false outside the domain (including a tail whose
// junction slope does not fall away from the core).
inline bool ipatia_valid_basic(const double* th) {
  for (int i = 0; i < 11; ++i)
    if (!std::isfinite(th[i])) return false;
  const double f = th[0], sigma = th[2], lam = th[3], zeta = th[4], a = th[6], n = th[7], a2 = th[8], n2 = th[9];
  if (!(f >= 0.0 && f <= 1.0 && sigma > 0.0 && zeta >= 0.0 && a > 0.0 && n > 0.0 && a2 > 0.0 && n2 > 0.0))
    return false;
  return zeta > 0.0 || lam < -1.0;
}

inline double host_rgamma(double z) {   // 1 / Gamma(1 + z) from its Taylor series (|z| <= 1/2)
  double s = 0.0;
  for (int k = kRGammaN - 1; k >= 0; --k) s = s * z + kRGamma[k];
  return s;
}

// host core and slope (std::cyl_bessel_k; K_{-v} = K_v)
inline double host_core(double d, double a2s2, double lam, double zeta, double beta, double* slope) {
  const double q = std::sqrt(1.0 + d * d / a2s2);
  const double e = std::exp(beta * d);
  const double dq = d / (a2s2 * q);
  if (zeta == 0.0) {
    const double p = 2.0 * lam - 1.0;
    const double g = std::pow(q, p);
    *slope = p * std::pow(q, p - 1.0) * dq * e + beta * g * e;
    return g * e;
  }
  const double nu = lam - 0.5;
  const double kn = std::cyl_bessel_k(std::fabs(nu), zeta * q);
  const double kn1 = std::cyl_bessel_k(std::fabs(nu - 1.0), zeta * q);
  const double g = std::pow(q, nu) * kn;
  *slope = -zeta * std::pow(q, nu) * kn1 * dq * e + beta * g * e;
  return g * e;
}

inline bool hoist_ipatia(const double* th, IpatiaConst& c) {
  if (!ipatia_valid_basic(th)) return false;
  const double f = th[0], mu = th[1], sigma = th[2], lam = th[3], zeta = th[4], beta = th[5];
  const double a = th[6], n = th[7], a2 = th[8], n2 = th[9], k = th[10];
  double A2;
  if (zeta == 0.0) {
    A2 = -2.0 * (lam + 1.0);
  } else {
    A2 = zeta * std::cyl_bessel_k(std::fabs(lam), zeta) / std::cyl_bessel_k(std::fabs(lam + 1.0), zeta);
  }
  if (!(A2 > 0.0) || !std::isfinite(A2)) return false;
  c.mu = mu;
  c.beta = beta;
  c.a2s2 = A2 * sigma * sigma;
  c.inv_a2s2 = 1.0 / c.a2s2;
  c.zeta = zeta;
  c.pw = zeta == 0.0 ? 2.0 * lam - 1.0 : lam - 0.5;
  const double nu = std::fabs(lam - 0.5);
  c.m = (int)std::floor(nu + 0.5);
  c.tmu = nu - c.m;
  const double gp = host_rgamma(c.tmu), gm = host_rgamma(-c.tmu);
  // Temme's Gamma_1 = (g(-mu) - g(mu)) / (2 mu) = -(g_1 + g_3 mu^2 + ...) and
  // Gamma_2 = (g(-mu) + g(mu)) / 2 = g_0 + g_2 mu^2 + ..., g(z) = 1 / Gamma(1 + z)
  double g1 = 0.0, g2 = 0.0, pe = 1.0, po = 1.0;
  for (int j = 0; j < kRGammaN; j += 2) {
    g2 += kRGamma[j] * pe;
    pe *= c.tmu * c.tmu;
  }
  for (int j = 1; j < kRGammaN; j += 2) {
    g1 -= kRGamma[j] * po;
    po *= c.tmu * c.tmu;
  }
  c.g1 = g1;
  c.g2 = g2;
  c.gp = gp;
  c.gm = gm;
  c.igp = 1.0 / gp;
  c.igm = 1.0 / gm;
  c.pad = 0;
  for (int j = 0; j < 4; ++j) c.rk[0][j] = 0.0;
  for (int kk = 1; kk < kTemmeTerms; ++kk) {
    const double dk = kk;
    c.rk[kk][0] = 1.0 / dk;
    c.rk[kk][1] = 1.0 / (dk - c.tmu);
    c.rk[kk][2] = 1.0 / (dk + c.tmu);
    c.rk[kk][3] = 1.0 / (dk * dk - c.tmu * c.tmu);
  }
  for (int j = 0; j < kTrapNodes; ++j) {
    const double sv = j * kTrapStep;
    c.ts2[j] = sv * sv;
    c.tw[j] = (j == 0 ? 0.5 : 1.0) * std::exp(-sv * sv) * 2.0;
  }
  c.fact = c.tmu == 0.0 ? 1.0 : M_PI * c.tmu / std::sin(M_PI * c.tmu);
  // tails
  double sl, sr;
  c.dl = -a * sigma;
  c.dr = a2 * sigma;
  const double gl = host_core(c.dl, c.a2s2, lam, zeta, beta, &sl);
  const double gr = host_core(c.dr, c.a2s2, lam, zeta, beta, &sr);
  if (!(sl > 0.0) || !(sr < 0.0) || !(gl > 0.0) || !(gr > 0.0)) return false;
  c.Bl = c.dl + n * gl / sl;
  c.Al = gl * std::pow(c.Bl - c.dl, n);
  c.Br = -c.dr - n2 * gr / sr;
  c.Ar = gr * std::pow(c.Br + c.dr, n2);
  c.nl = n;
  c.nr = n2;
  if (!std::isfinite(c.Al) || !std::isfinite(c.Ar) || !std::isfinite(c.Bl) || !std::isfinite(c.Br)) return false;
  // mixture
  const double L = kMHi - kMLo;
  const double NE = k == 0.0 ? L : -std::expm1(-k * L) / k;
  c.f = f;
  c.cB = (1.0 - f) / NE;
  c.k = k;
  c.dm = L / kIpatiaGrid;
  c.lo = kMLo;
  c.inv_norm = nullptr;
  return true;
}

}  // namespace ipx
