// Host-side hoisting: from theta to the per-call constants the kernels read,
// and the Jacobian that maps the kernels' adjoint sums back to dNLL/dtheta.
#pragma once

#include <cmath>

#include "ipx_models.h"

namespace ipx {

// ---------------------------------------------------------------------------
// Small forward-mode dual number on the host (value + N derivatives), used to
// differentiate the angular coefficient table with respect to its parameters.
// ---------------------------------------------------------------------------
template <int N>
struct HD {
  double v;
  double d[N];
  HD() : v(0.0) { for (int i = 0; i < N; ++i) d[i] = 0.0; }
  HD(double x) : v(x) { for (int i = 0; i < N; ++i) d[i] = 0.0; }  // NOLINT: constant
  static HD var(double x, int j) { HD r(x); r.d[j] = 1.0; return r; }
};
template <int N> inline HD<N> operator+(const HD<N>& a, const HD<N>& b) { HD<N> r; r.v = a.v + b.v; for (int i = 0; i < N; ++i) r.d[i] = a.d[i] + b.d[i]; return r; }
template <int N> inline HD<N> operator-(const HD<N>& a, const HD<N>& b) { HD<N> r; r.v = a.v - b.v; for (int i = 0; i < N; ++i) r.d[i] = a.d[i] - b.d[i]; return r; }
template <int N> inline HD<N> operator-(const HD<N>& a) { HD<N> r; r.v = -a.v; for (int i = 0; i < N; ++i) r.d[i] = -a.d[i]; return r; }
template <int N> inline HD<N> operator*(const HD<N>& a, const HD<N>& b) { HD<N> r; r.v = a.v * b.v; for (int i = 0; i < N; ++i) r.d[i] = a.d[i] * b.v + a.v * b.d[i]; return r; }
template <int N> inline HD<N> operator*(double s, const HD<N>& a) { HD<N> r; r.v = s * a.v; for (int i = 0; i < N; ++i) r.d[i] = s * a.d[i]; return r; }
template <int N> inline HD<N> hsin(const HD<N>& a) { HD<N> r; r.v = std::sin(a.v); const double c = std::cos(a.v); for (int i = 0; i < N; ++i) r.d[i] = c * a.d[i]; return r; }
template <int N> inline HD<N> hcos(const HD<N>& a) { HD<N> r; r.v = std::cos(a.v); const double s = -std::sin(a.v); for (int i = 0; i < N; ++i) r.d[i] = s * a.d[i]; return r; }
// sqrt; its slope is infinite at 0, where the gradient is not defined (the
// derivative table is built only inside theta_grad_valid's domain)
template <int N> inline HD<N> hsqrt(const HD<N>& a) { HD<N> r; r.v = std::sqrt(a.v); const double h = 0.5 / r.v; for (int i = 0; i < N; ++i) r.d[i] = h * a.d[i]; return r; }
// The same operations on plain values: code written for HD<N> computes, with
// double, exactly the values (.v) of its dual-number run.
inline double hsin(double a) { return std::sin(a); }
inline double hcos(double a) { return std::cos(a); }
inline double hsqrt(double a) { return std::sqrt(a); }
template <typename T> inline T hvar(double x, int j);
template <> inline double hvar<double>(double x, int) { return x; }
template <> inline HD<7> hvar<HD<7>>(double x, int j) { return HD<7>::var(x, j); }
inline double hval(double x) { return x; }
template <int N> inline double hval(const HD<N>& x) { return x.v; }

// ---------------------------------------------------------------------------
// Mass normalisations and their derivatives
// ---------------------------------------------------------------------------
struct GaussNorm {
  double N, dmu, dsig;  // N_G and its partial derivatives
};
inline GaussNorm gauss_norm(double mu, double sig) {
  const double r2s = std::sqrt(2.0) * sig;
  GaussNorm g;
  g.N = sig * std::sqrt(M_PI / 2.0) * (std::erfc((kMLo - mu) / r2s) - std::erfc((kMHi - mu) / r2s));
  const double za = (kMLo - mu) / sig, zb = (kMHi - mu) / sig;
  const double Ga = std::exp(-0.5 * za * za), Gb = std::exp(-0.5 * zb * zb);
  g.dmu = Ga - Gb;
  g.dsig = g.N / sig + za * Ga - zb * Gb;
  return g;
}

struct ExpNorm {
  double N, dlam;
};
inline ExpNorm exp_norm(double lam) {
  const double L = kMHi - kMLo;
  const double x = lam * L;
  ExpNorm e;
  if (std::fabs(x) < 1e-3) {
    // series of (1 - e^{-x})/x and its derivative, truncation < 1e-19 relative
    e.N = L * (1.0 - x / 2.0 + x * x / 6.0 - x * x * x / 24.0 + x * x * x * x / 120.0);
    e.dlam = L * L * (-0.5 + x / 3.0 - x * x / 8.0 + x * x * x / 30.0 - x * x * x * x / 144.0);
  } else {
    e.N = -std::expm1(-x) / lam;
    e.dlam = L * std::exp(-x) / lam - e.N / lam;
  }
  return e;
}

// ---------------------------------------------------------------------------
// Parameter domains
// ---------------------------------------------------------------------------
inline bool all_finite(const double* th, int n) {
  for (int i = 0; i < n; ++i)
    if (!std::isfinite(th[i])) return false;
  return true;
}
inline bool theta_valid(int model, const double* th) {
  if (model == 1) return all_finite(th, 4) && th[0] >= 0.0 && th[0] <= 1.0 && th[2] > 0.0;
  if (model == 2)
    return all_finite(th, 7) && th[0] >= 0.0 && th[0] <= 1.0 && th[2] > 0.0 && th[4] > 0.0 && th[5] > 0.0 &&
           th[6] > 0.0;
  if (model == 3 || model == 4)
    return all_finite(th, 12) && th[0] >= 0.0 && th[1] >= 0.0 && th[0] + th[1] <= 1.0 && th[2] >= 0.0 &&
           th[2] <= 1.0 && th[11] > 0.0 && th[6] - std::fabs(th[7]) / 2.0 > 0.0;
  return false;
}
// The gradient's domain.  The angular model's interference coefficients are
// linear in the amplitude moduli sqrt(|A_i|^2), whose slope is infinite where
// a squared modulus vanishes (Fs = 0 or 1, fL = 0, fperp = 0, fL + fperp = 1):
// there dNLL/dtheta does not exist.  The gradient is evaluated only where every
// squared modulus, computed as the hoisting computes it, is positive.
inline bool theta_grad_valid(int model, const double* th) {
  if (!theta_valid(model, th)) return false;
  if (model != 3 && model != 4) return true;
  const double fL = th[0], fpe = th[1], Fs = th[2];
  const double a0 = (1.0 - Fs) * fL, ape = (1.0 - Fs) * fpe, apa = (1.0 - Fs) * (1.0 - fL - fpe);
  return a0 > 0.0 && ape > 0.0 && apa > 0.0 && Fs > 0.0;
}

// ---------------------------------------------------------------------------
// Model 1
// ---------------------------------------------------------------------------
struct MassHoist {
  MassConst k;
  GaussNorm ng;
  ExpNorm ne;
};
inline MassHoist hoist_mass(const double* th) {
  MassHoist h;
  const double f = th[0], mu = th[1], sig = th[2], lam = th[3];
  h.ng = gauss_norm(mu, sig);
  h.ne = exp_norm(lam);
  h.k.cS = f / h.ng.N;
  h.k.cB = (1.0 - f) / h.ne.N;
  h.k.mu = mu;
  h.k.q = 1.0 / (2.0 * sig * sig);
  h.k.lam = lam;
  return h;
}
// a: adjoint sums (component 0 = sum w ln P); g: dNLL/dtheta
inline void grad_mass(const MassHoist& h, const double* th, const double* a, double* g) {
  const double f = th[0], sig = th[2];
  const double NG = h.ng.N, NE = h.ne.N;
  const double dl_f = a[1] / NG - a[2] / NE;
  const double dl_mu = a[3] - a[1] * f / (NG * NG) * h.ng.dmu;
  const double dl_sig = a[4] * (-1.0 / (sig * sig * sig)) - a[1] * f / (NG * NG) * h.ng.dsig;
  const double dl_lam = a[5] - a[2] * (1.0 - f) / (NE * NE) * h.ne.dlam;
  g[0] = -dl_f; g[1] = -dl_mu; g[2] = -dl_sig; g[3] = -dl_lam;
}

// ---------------------------------------------------------------------------
// Model 2
// ---------------------------------------------------------------------------
struct MassTimeHoist {
  MassTimeConst k;
  GaussNorm ng;
  ExpNorm ne;
};
inline MassTimeHoist hoist_masstime(const double* th) {
  MassTimeHoist h;
  const double f = th[0], mu = th[1], sig = th[2], lam = th[3], ts = th[4], tb = th[5], s = th[6];
  h.ng = gauss_norm(mu, sig);
  h.ne = exp_norm(lam);
  MassTimeConst& k = h.k;
  k.cS = f / h.ng.N;
  k.cB = (1.0 - f) / h.ne.N;
  k.mu = mu;
  k.q = 1.0 / (2.0 * sig * sig);
  k.lam = lam;
  k.s = s;
  k.gs = 1.0 / ts;
  k.gb = 1.0 / tb;
  k.hs2 = 0.5 * k.gs * k.gs;
  k.hb2 = 0.5 * k.gb * k.gb;
  k.gmax = k.gs > k.gb ? k.gs : k.gb;
  k.eAs = std::exp(-k.gs * kTLo);
  k.eBs = std::exp(-k.gs * kTHi);
  k.eAb = std::exp(-k.gb * kTLo);
  k.eBb = std::exp(-k.gb * kTHi);
  k.inv_gs = ts;
  k.inv_gb = tb;
  k.shA = k.gmax * kTLo;
  k.shB = k.gmax * kTHi;
  k.q2 = 2.0 * k.q;
  return h;
}
inline void grad_masstime(const MassTimeHoist& h, const double* th, const double* a, double* g) {
  const double f = th[0], sig = th[2], ts = th[4], tb = th[5];
  const double NG = h.ng.N, NE = h.ne.N;
  g[0] = -(a[1] / NG - a[2] / NE);
  g[1] = -(a[3] - a[1] * f / (NG * NG) * h.ng.dmu);
  g[2] = -(a[4] * (-1.0 / (sig * sig * sig)) - a[1] * f / (NG * NG) * h.ng.dsig);
  g[3] = -(a[5] - a[2] * (1.0 - f) / (NE * NE) * h.ne.dlam);
  g[4] = -(a[6] * (-1.0 / (ts * ts)));
  g[5] = -(a[7] * (-1.0 / (tb * tb)));
  g[6] = -a[8];
}

// ---------------------------------------------------------------------------
// Model 3
// ---------------------------------------------------------------------------
// Integrals of the ten angular functions over the full angular range.
constexpr double kXi[10] = {32.0 * M_PI / 9.0, 32.0 * M_PI / 9.0, 32.0 * M_PI / 9.0, 0.0, 0.0, 0.0,
                            32.0 * M_PI / 9.0, 0.0, 0.0, 0.0};

using HD7 = HD<7>;  // directions: fL, fperp, Fs, dpa, dpe, dS, phis

// Per-dataset constants of the angular models: the normalisation weights
// xi_k = integral eps(Omega) f_k dOmega of the angular efficiency eps (the
// analytic integrals for a flat efficiency) and the S-P interference factor
// C_SP of the sample's KK-mass bin (Example 2 fits one sample per bin).
struct AngSettings {
  double xi[10];
  double c_sp;
};
inline AngSettings ang_settings_default() {
  AngSettings a;
  for (int k = 0; k < 10; ++k) a.xi[k] = kXi[k];
  a.c_sp = 1.0;
  return a;
}

// C[k][j] = N_k (a_k, b_k, c_k, d_k), |lambda| = 1, delta_0 = 0, the S-P
// rows (k = 8, 9, 10) scaled by c_sp; T = double for the values, HD7 for
// values and derivatives.
template <typename T>
inline void angular_coefficients(const double* th, T C[10][4], double c_sp) {
  const T fL = hvar<T>(th[0], 0), fpe = hvar<T>(th[1], 1), Fs = hvar<T>(th[2], 2);
  const T dpa = hvar<T>(th[3], 3), dpe = hvar<T>(th[4], 4), dS = hvar<T>(th[5], 5);
  const T phis = hvar<T>(th[9], 6);
  const T one(1.0), zero(0.0);
  const T Cc = zero;            // (1 - |lambda|^2)/(1 + |lambda|^2)
  const T S = -hsin(phis);      // -2|lambda| sin(phis)/(1 + |lambda|^2)
  const T Dd = -hcos(phis);     // -2|lambda| cos(phis)/(1 + |lambda|^2)
  const T a0 = (one - Fs) * fL, ape = (one - Fs) * fpe, apa = (one - Fs) * (one - fL - fpe), aS = Fs;
  const T r0 = hsqrt(a0), rpe = hsqrt(ape), rpa = hsqrt(apa), rS = hsqrt(aS);
  const T d0 = zero;
  const T spp = hsin(dpe - dpa), cpp = hcos(dpe - dpa);
  const T cp0 = hcos(dpa - d0);
  const T se0 = hsin(dpe - d0), ce0 = hcos(dpe - d0);
  const T cpS = hcos(dpa - dS), spS = hsin(dpa - dS);
  const T seS = hsin(dpe - dS);
  const T c0S = hcos(d0 - dS), s0S = hsin(d0 - dS);
  const T csp(c_sp);
  const T N[10] = {a0, apa, ape, rpa * rpe, r0 * rpa, r0 * rpe, aS, csp * (rS * rpa), csp * (rS * rpe), csp * (rS * r0)};
  const T abcd[10][4] = {
      {one, Dd, Cc, -S},
      {one, Dd, Cc, -S},
      {one, -Dd, Cc, S},
      {Cc * spp, S * cpp, spp, Dd * cpp},
      {cp0, Dd * cp0, Cc * cp0, -(S * cp0)},
      {Cc * se0, S * ce0, se0, Dd * ce0},
      {one, -Dd, Cc, S},
      {Cc * cpS, S * spS, cpS, Dd * spS},
      {seS, -(Dd * seS), Cc * seS, S * seS},
      {Cc * c0S, S * s0S, c0S, Dd * s0S},
  };
  for (int k = 0; k < 10; ++k)
    for (int j = 0; j < 4; ++j) C[k][j] = N[k] * abcd[k][j];
}

struct AngTimeHoist {
  AngTimeConst k;
  HD7 C[10][4];   // the coefficient table with its derivatives (for the gradient only)
  GaussNorm ng;
  AngSettings set = ang_settings_default();  // the dataset's constants used by this hoist
};
// The kernel constants alone (what a launch needs); the derivative table can
// follow while the kernel runs (angtime_derivatives).
inline void hoist_angtime_values(const double* th, const AngSettings& set, AngTimeConst& k, GaussNorm& ng) {
  double Cv[10][4];
  angular_coefficients(th, Cv, set.c_sp);
  for (int j = 0; j < 4; ++j) {
    double s = 0.0;
    for (int kk = 0; kk < 10; ++kk) {
      k.C[kk][j] = Cv[kk][j];
      s += set.xi[kk] * Cv[kk][j];
    }
    k.D[j] = s;
  }
  const double G = th[6], DG = th[7], DM = th[8];
  k.gH = G - DG / 2.0;
  k.gL = G + DG / 2.0;
  k.g = G;
  k.dm = DM;
  k.gmax = std::fmax(std::fmax(k.gH, k.gL), G);
  k.hH2 = 0.5 * k.gH * k.gH;
  k.hL2 = 0.5 * k.gL * k.gL;
  k.hc2 = 0.5 * (G * G - DM * DM);
  k.gdm = G * DM;
  k.hdg = DG / 2.0;
  k.eAH = std::exp(-k.gH * kTLo); k.eBH = std::exp(-k.gH * kTHi);
  k.eAL = std::exp(-k.gL * kTLo); k.eBL = std::exp(-k.gL * kTHi);
  k.eAG = std::exp(-G * kTLo);    k.eBG = std::exp(-G * kTHi);
  k.cA = std::cos(DM * kTLo); k.sA = std::sin(DM * kTLo);
  k.cB = std::cos(DM * kTHi); k.sB = std::sin(DM * kTHi);
  k.inv_gH = 1.0 / k.gH;
  k.inv_gL = 1.0 / k.gL;
  const double den = G * G + DM * DM;  // 1/(G - i DM) = (G + i DM)/(G^2 + DM^2)
  k.izr = G / den;
  k.izi = DM / den;
  const double mu = th[10], sig = th[11];
  ng = gauss_norm(mu, sig);
  k.mu = mu;
  k.q = 1.0 / (2.0 * sig * sig);
  k.lnNG = std::log(ng.N);
  k.shA = k.gmax * kTLo;
  k.shB = k.gmax * kTHi;
  k.Dp = 0.5 * (k.D[0] + k.D[1]);
  k.Dm = 0.5 * (k.D[0] - k.D[1]);
  k.q2 = 2.0 * k.q;
}
// Fills h (kernel constants, mass normalisation, the settings used).
inline void hoist_angtime(const double* th, const AngSettings& set, AngTimeHoist& h) {
  h.set = set;
  hoist_angtime_values(th, set, h.k, h.ng);
}
inline void angtime_derivatives(const double* th, AngTimeHoist& h) { angular_coefficients(th, h.C, h.set.c_sp); }
inline void grad_angtime(const AngTimeHoist& h, const double* th, const double* a, double* g) {
  // total adjoint of C_kj: direct plus through D_j = sum_k xi_k C_kj
  // layout: a[0] l, a[1..4] dD_j, a[5..8] d(Gamma_H, Gamma_L, Re z, dm),
  // a[9] dmu, a[10] dq, a[11] sum w, a[12 + 4k + j] dC_kj
  double phys[7] = {0, 0, 0, 0, 0, 0, 0};
  for (int kk = 0; kk < 10; ++kk)
    for (int j = 0; j < 4; ++j) {
      const double adj = a[12 + 4 * kk + j] + h.set.xi[kk] * a[1 + j];
      for (int p = 0; p < 7; ++p) phys[p] += adj * h.C[kk][j].d[p];
    }
  const double dG = a[5] + a[6] + a[7];
  const double dDG = -0.5 * a[5] + 0.5 * a[6];
  const double dDM = a[8];
  const double sig = th[11];
  const double NG = h.ng.N;
  const double dmu = a[9] - a[11] * h.ng.dmu / NG;
  const double dsig = a[10] * (-1.0 / (sig * sig * sig)) - a[11] * h.ng.dsig / NG;
  const double dl[12] = {phys[0], phys[1], phys[2], phys[3], phys[4], phys[5], dG, dDG, dDM, phys[6], dmu, dsig};
  for (int i = 0; i < 12; ++i) g[i] = -dl[i];
}

}  // namespace ipx
