// Per-call hoisted constants of the three models (plain structs shared by the
// host code that fills them and the kernels that read them from kernel
// arguments, i.e. from scalar registers), and the reduction geometry.
#pragma once

#include <stdint.h>

namespace ipx {

// Observable ranges (mass in MeV, decay time in ps).
constexpr double kMLo = 5200.0, kMHi = 5500.0;
constexpr double kTLo = 0.3, kTHi = 15.0;

// Canonical tile: 256 lanes x 4 events.  Every reduction order is a function
// of the tile index only, so results do not depend on the launch size.
constexpr int kThreads = 256;
constexpr int kEventsPerLane = 4;
constexpr int kTile = kThreads * kEventsPerLane;

// Accumulator layout (component 0 is always sum_i w_i ln P_i).
constexpr int kAccMass = 6;       // l, dcS, dcB, dmu, dq, dlam
constexpr int kAccMassTime = 9;   // l, dcS, dcB, dmu, dq, dlam, dgs, dgb, ds
constexpr int kAccAngTime = 52;   // l, dD[4], dgH, dgL, dzr, ddm, dmu, dq, sum_w, dC[40]
constexpr int kAccMax = 52;

struct EventCols {
  const double* c[7];
  const double* w;  // nullptr: unit weights
  int64_t n;
};

struct MassConst {
  double cS;   // f / N_G
  double cB;   // (1 - f) / N_E
  double mu;
  double q;    // 1 / (2 sigma^2)
  double lam;
};

struct MassTimeConst {
  double cS, cB, mu, q, lam;
  double s;          // resolution scale
  double gs, gb;     // 1/tau_s, 1/tau_b
  double hs2, hb2;   // gs^2 / 2, gb^2 / 2
  double gmax;
  double eAs, eBs, eAb, eBb;  // exp(-gs T_LO), exp(-gs T_HI), exp(-gb T_LO), exp(-gb T_HI)
  double inv_gs, inv_gb;
  double shA, shB;   // gmax T_LO, gmax T_HI (per-call products of the event loop)
  double q2;         // 2 q
};

struct AngTimeConst {
  double C[10][4];   // N_k (a_k, b_k, c_k, d_k)
  double D[4];       // sum_k xi_k C_kj
  double gH, gL, g, dm;        // Gamma_H, Gamma_L, Gamma, Delta m
  double gmax;                 // max(Gamma_H, Gamma_L, Gamma)
  double hH2, hL2, hc2, gdm;   // Gamma_H^2/2, Gamma_L^2/2, (Gamma^2 - dm^2)/2, Gamma dm
  double hdg;                  // DeltaGamma / 2
  double eAH, eBH, eAL, eBL, eAG, eBG;  // exp(-rate * T_LO / T_HI)
  double cA, sA, cB, sB;       // cos, sin of dm T_LO and dm T_HI
  double inv_gH, inv_gL;
  double izr, izi;             // 1 / (Gamma - i dm)
  double mu, q, lnNG;          // signal mass: mean, 1/(2 sigma^2), ln N_G
  // per-call products the event loop would otherwise form on every event
  double shA, shB;             // gmax T_LO, gmax T_HI
  double Dp, Dm;               // (D_0 + D_1) / 2, (D_0 - D_1) / 2
  double q2;                   // 2 q
};

}  // namespace ipx
