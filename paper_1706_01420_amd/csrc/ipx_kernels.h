// Per-event likelihood code and the deterministic two-level FP64 reduction
// (the kernels that drive it are in ipx_batch.h).
//
// One lane evaluates kEventsPerLane events of a canonical tile (event index
// tile*kTile + e*256 + lane, so each load instruction of a wave reads 64
// consecutive doubles of a column), keeping the running sums of ln P and, for
// the gradient kernels, of the adjoints in registers.  At the end of a tile
// the sums are reduced across each wave through an LDS transpose (one lane per
// component adds the 64 lane values in a fixed order), across the four waves
// in wave order, and written as one partial per tile (component-major).  A
// second kernel sums the tile partials of each component in index order.
#pragma once

#include <hip/hip_runtime.h>

#include "ipx_math.h"
#include "ipx_models.h"

namespace ipx {

// ---------------------------------------------------------------------------
// Global-memory access.  Column pointers reach the kernels through structs in
// device memory, so the compiler sees generic pointers and would emit flat
// loads (which also wait on the LDS / scalar counters).  These helpers address
// the global segment explicitly: a wave-uniform base pointer plus a 32-bit lane
// offset, i.e. one scalar base register pair and one vector offset per access.
//
// COH = true makes every access device-coherent (relaxed atomics at agent
// scope: the L2 of each XCD is bypassed for stores and revalidated for loads).
// The persistent serving kernel uses it for everything that other workgroups
// of the same launch produce or consume (tile partials), and for
// the event columns (which may have been written after the launch started);
// the kernels of one-shot launches, ordered by kernel boundaries, use plain
// accesses.
// ---------------------------------------------------------------------------
typedef __attribute__((address_space(1))) const double gconst_double;
typedef __attribute__((address_space(1))) double gdouble;

template <bool COH = false>
__device__ __forceinline__ double ldg(const double* base, unsigned j) {
  if constexpr (COH) return __hip_atomic_load((gconst_double*)base + j, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  else return ((gconst_double*)base)[j];
}
template <bool COH = false>
__device__ __forceinline__ void stg(double* base, unsigned j, double v) {
  if constexpr (COH) __hip_atomic_store((gdouble*)base + j, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  else ((gdouble*)base)[j] = v;
}

// ---------------------------------------------------------------------------
// Reduction
// ---------------------------------------------------------------------------
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Tile reduction through LDS.  Each wave writes its lanes' sums column-wise
// into an LDS block (component-major rows of 64 lanes, padded to 65 doubles
// so that the row reads below spread over the banks); then lane c of the wave
// adds row c in a fixed order (four interleaved partial sums over the lanes,
// combined pairwise).  Components are done in chunks of at most CAP rows (the
// block the kernel provides: kThreads / 64 waves x CAP rows x kRedPitch).  The
// four wave totals are combined in wave order.  Every order is a function of
// the tile's lane layout only.  Components NACC .. NTOT - 1 arrive as wave
// totals that the caller has written to wsum (before the call) and are only
// combined across the waves.
constexpr int kRedPitch = 65;

template <int CAP>
struct alignas(16) RedBuf {
  double rows[kThreads / 64][CAP][kRedPitch];
  double wsum[kThreads / 64][kAccMax];
};

template <int NACC, bool COH, int CAP, int NTOT = NACC>
__device__ __forceinline__ void tile_store(const double (&acc)[NACC], double* __restrict__ partials,
                                           int64_t tile, int64_t n_tiles, RedBuf<CAP>& red) {
  static_assert(NTOT >= NACC && NTOT <= kAccMax, "wave totals live in wsum");
  constexpr int kChunk = NACC < CAP ? NACC : CAP;
  // the lane's LDS addresses are derived here, from an opaque copy of the
  // thread index: computed once at kernel entry they would stay live through
  // the caller's event loop (and the angular gradient kernel would spill them)
  int tid = (int)threadIdx.x;
  asm volatile("" : "+v"(tid));
  const int lane = tid & 63;
  const int wave = tid >> 6;
#pragma unroll
  for (int c0 = 0; c0 < NACC; c0 += kChunk) {
#pragma unroll
    for (int c = 0; c < kChunk; ++c)
      if (c0 + c < NACC) red.rows[wave][c][lane] = acc[c0 + c];
    __syncthreads();
    if (lane < kChunk && c0 + lane < NACC) {
      const double* row = red.rows[wave][lane];
      double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
#pragma unroll 4
      for (int r = 0; r < 64; r += 4) {
        s0 += row[r];
        s1 += row[r + 1];
        s2 += row[r + 2];
        s3 += row[r + 3];
      }
      red.wsum[wave][c0 + lane] = (s0 + s1) + (s2 + s3);
    }
    __syncthreads();
  }
  for (int c = threadIdx.x; c < NTOT; c += kThreads)
    stg<COH>(partials + (int64_t)c * n_tiles + tile, 0u,
             (red.wsum[0][c] + red.wsum[1][c]) + (red.wsum[2][c] + red.wsum[3][c]));
  __syncthreads();
}

// Sum of nt tile partials in a fixed order: lane-sequential over a stride of
// 256, wave butterfly, waves in order.  Used by every reduction of partials.
template <bool COH = false>
__device__ __forceinline__ double reduce_component(const double* __restrict__ p, int64_t nt) {
  double s = 0.0;
  // sixteen loads in flight per round (the ragged end masked), added in index
  // order: s = ((p[t] + p[t + 256]) + p[t + 512]) + ... for lane t
  constexpr int kFlight = 16;
  for (int64_t i0 = threadIdx.x; i0 < nt; i0 += kFlight * kThreads) {
    double v[kFlight];
#pragma unroll
    for (int u = 0; u < kFlight; ++u) v[u] = i0 + u * kThreads < nt ? ldg<COH>(p + i0 + u * kThreads, 0u) : 0.0;
#pragma unroll
    for (int u = 0; u < kFlight; ++u)
      if (i0 + u * kThreads < nt) s += v[u];
  }
  __shared__ double lds[kThreads / 64];
  s = wave_sum(s);
  if ((threadIdx.x & 63) == 0) lds[threadIdx.x >> 6] = s;
  __syncthreads();
  return (lds[0] + lds[1]) + (lds[2] + lds[3]);
}

// ---------------------------------------------------------------------------
// Model 1: mass
// ---------------------------------------------------------------------------
template <bool GRAD>
__device__ __forceinline__ void event_mass(const MassConst& k, double m, double w, double* acc) {
  const double d = m - k.mu;
  const double G = exp_lo(-d * d * k.q);
  const double E = exp_lo(-k.lam * (m - kMLo));
  const double P = k.cS * G + k.cB * E;
  acc[0] += w * log_fast(P);
  if constexpr (GRAD) {
    const double iw = w / P;
    const double ps = k.cS * G * iw;
    acc[1] += G * iw;
    acc[2] += E * iw;
    acc[3] += ps * 2.0 * k.q * d;
    acc[4] -= ps * d * d;
    acc[5] -= k.cB * E * iw * (m - kMLo);
  }
}

// ---------------------------------------------------------------------------
// Resolution-convolved exponentials
//   F(tau; z, s) = exp(z^2 s^2/2 - z tau) - 1/2 g w(-u)   (Im u < 0)
//               = 1/2 g w(u)                              (Im u >= 0)
//   u = i (z s^2 - tau)/(sqrt2 s),  g = exp(-tau^2/(2 s^2)).
// For a real rate, w on the imaginary axis is erfcx.
// ---------------------------------------------------------------------------
// A time point: whether its correction terms are needed, and the depth of the
// continued fraction that evaluates them.  The correction of rate r is
// exp(-E_r) w / 2 relative to the main term with E_r = (Im u_r)^2 - (Re u_r)^2;
// the smallest E over the rates is at the largest rate.  At the range ends
// the same decisions serve the Phi terms of the normalisation, whose size
// relative to the main term at T_LO is bounded with E lowered by gmax tau
// (e_shift).  The corrections are skipped when even their own size is below
// 2^-57 of the main term (E >= kCfSkipE); when Im u < 0 for some rate the
// correction is the whole value and takes the full depth.
struct TimePoint {
  double g;     // exp(-tau^2 / (2 s^2)), 0 when the correction is negligible
  bool need;    // correction evaluated
  int depth;    // continued-fraction levels (wave-uniform)
};

__device__ __forceinline__ TimePoint time_point(double tau, double gmax, double s2, double inv_r2s,
                                                double re_u2, double e_shift) {
  TimePoint p;
  const double x = (tau - gmax * s2) * inv_r2s;  // smallest |Im u| over the rates
  const double E = (x > 0.0 ? x * x - re_u2 : -1.0) - e_shift;
  p.need = !(E >= kCfSkipE);
  // the depth search (four wave votes) only where some lane needs it
  p.depth = __any(p.need) ? cf_depth_wave(p.need ? E : kCfSkipE) : 1;
  const double a = tau * inv_r2s;
  p.g = p.need ? exp_lo(-a * a) : 0.0;
  return p;
}

// F from its main term, where the time point needs the correction
__device__ __forceinline__ double conv_real_needed(double tau, double rate, double main, const TimePoint& p,
                                                   double s2, double inv_r2s) {
  const double y = (tau - rate * s2) * inv_r2s;  // -Im u
  const double c = 0.5 * p.g * erfcx_pos(fabs(y), p.depth);
  return y >= 0.0 ? main - c : c;
}

__device__ __forceinline__ double conv_real(double tau, double rate, double main, const TimePoint& p,
                                            double s2, double inv_r2s) {
  if (!p.need) return main;
  return conv_real_needed(tau, rate, main, p, s2, inv_r2s);
}

// complex rate Gamma - i dm; dmr = dm s / sqrt2 = Re u; where the time point
// needs the correction
__device__ __forceinline__ cplx conv_cplx_needed(double tau, double rate, double dmr, cplx main, const TimePoint& p,
                                                 double s2, double inv_r2s) {
  const double y = (tau - rate * s2) * inv_r2s;
  // w(-u) for y >= 0 (then F = main - g w(-u)/2), w(u) otherwise (F = g w(u)/2)
  const bool lower = y >= 0.0;
  const cplx c = cscale(faddeeva_upper(lower ? cplx{-dmr, y} : cplx{dmr, -y}, p.depth), 0.5 * p.g);
  return lower ? csub(main, c) : c;
}

// ---------------------------------------------------------------------------
// Model 2: mass x decay time, two real rates, per-event width s sigma_t
// ---------------------------------------------------------------------------
struct RateTerms {
  double F, I;      // F(t), integral over [T_LO, T_HI]
  double dlz, dls;  // d ln(F/I) / d rate, d ln(F/I) / d sigma
};

// One rate's F at t and at the range ends (main terms, corrected where the
// time point needs it), the two rates side by side so that each time point's
// corrections take one branch.
struct RatePair {
  double t[2], a[2], b[2];
  double phi_a, phi_b;  // the Phi terms 1/2 g erfcx(T / (sqrt2 s)) at the range ends, 0 where not needed
};

__device__ __forceinline__ RatePair rate_pair(double t, const MassTimeConst& k, double s2, double inv_r2s,
                                              const TimePoint& pt, const TimePoint& pa, const TimePoint& pb) {
  const double e2s = exp_lo(k.hs2 * s2), e2b = exp_lo(k.hb2 * s2);
  RatePair F{{e2s * exp_lo(-k.gs * t), e2b * exp_lo(-k.gb * t)}, {e2s * k.eAs, e2b * k.eAb}, {e2s * k.eBs, e2b * k.eBb},
             0.0, 0.0};
  if (pt.need) {
    F.t[0] = conv_real_needed(t, k.gs, F.t[0], pt, s2, inv_r2s);
    F.t[1] = conv_real_needed(t, k.gb, F.t[1], pt, s2, inv_r2s);
  }
  if (pa.need) {
    F.a[0] = conv_real_needed(kTLo, k.gs, F.a[0], pa, s2, inv_r2s);
    F.a[1] = conv_real_needed(kTLo, k.gb, F.a[1], pa, s2, inv_r2s);
    F.phi_a = 0.5 * pa.g * erfcx_pos(kTLo * inv_r2s, pa.depth);
  }
  if (pb.need) {
    F.b[0] = conv_real_needed(kTHi, k.gs, F.b[0], pb, s2, inv_r2s);
    F.b[1] = conv_real_needed(kTHi, k.gb, F.b[1], pb, s2, inv_r2s);
    F.phi_b = 0.5 * pb.g * erfcx_pos(kTHi * inv_r2s, pb.depth);
  }
  return F;
}

template <bool GRAD>
__device__ __forceinline__ RateTerms rate_terms(double t, double rate, double Ft, double Fa, double Fb,
                                                double inv_rate, double sig, double s2,
                                                const TimePoint& pt, const TimePoint& pa,
                                                const TimePoint& pb, double dphi) {
  RateTerms r;
  r.F = Ft;
  r.I = (dphi + Fa - Fb) * inv_rate;
  if constexpr (GRAD) {
    const double inv_sig = rcp(sig);
    const double Gt = pt.g * kInvSqrt2Pi * inv_sig;
    const double Ga = pa.g * kInvSqrt2Pi * inv_sig;
    const double Gb = pb.g * kInvSqrt2Pi * inv_sig;
    const double dzt = (s2 * rate - t) * Ft - s2 * Gt;
    const double dza = (s2 * rate - kTLo) * Fa - s2 * Ga;
    const double dzb = (s2 * rate - kTHi) * Fb - s2 * Gb;
    const double sr = sig * rate;
    const double dst = sr * rate * Ft - (sr + t * inv_sig) * Gt;
    const double dsa = sr * rate * Fa - (sr + kTLo * inv_sig) * Ga;
    const double dsb = sr * rate * Fb - (sr + kTHi * inv_sig) * Gb;
    // d Phi(x)/d sigma = -(x / sigma) G_t(x)
    const double dphis = -(kTHi * inv_sig) * Gb + (kTLo * inv_sig) * Ga;
    const double dIz = (-r.I + dza - dzb) * inv_rate;
    const double dIs = (dphis - dsb + dsa) * inv_rate;
    const double iF = rcp(Ft), iI = rcp(r.I);
    r.dlz = dzt * iF - dIz * iI;
    r.dls = dst * iF - dIs * iI;
  }
  return r;
}

template <bool GRAD>
__device__ __forceinline__ void event_masstime(const MassTimeConst& k, double m, double t, double sigt,
                                               double w, double* acc) {
  const double sig = k.s * sigt;
  const double s2 = sig * sig;
  const double inv_r2s = kInvSqrt2 * rcp(sig);
  const TimePoint pt = time_point(t, k.gmax, s2, inv_r2s, 0.0, 0.0);
  const TimePoint pa = time_point(kTLo, k.gmax, s2, inv_r2s, 0.0, k.shA);
  const TimePoint pb = time_point(kTHi, k.gmax, s2, inv_r2s, 0.0, k.shB);
  const RatePair F = rate_pair(t, k, s2, inv_r2s, pt, pa, pb);
  // Phi(T_HI) - Phi(T_LO) = 1/2 [g_a erfcx(T_LO/(sqrt2 s)) - g_b erfcx(T_HI/(sqrt2 s))]
  const double dphi = F.phi_a - F.phi_b;
  const RateTerms rs = rate_terms<GRAD>(t, k.gs, F.t[0], F.a[0], F.b[0], k.inv_gs, sig, s2, pt, pa, pb, dphi);
  const RateTerms rb = rate_terms<GRAD>(t, k.gb, F.t[1], F.a[1], F.b[1], k.inv_gb, sig, s2, pt, pa, pb, dphi);
  const double d = m - k.mu;
  const double G = exp_lo(-d * d * k.q);
  const double E = exp_lo(-k.lam * (m - kMLo));
  const double hs = rs.F * rcp(rs.I), hb = rb.F * rcp(rb.I);
  const double P = k.cS * G * hs + k.cB * E * hb;
  acc[0] += w * log_fast(P);
  if constexpr (GRAD) {
    const double iw = w * rcp(P);
    const double ps = k.cS * G * hs * iw;  // w x signal posterior
    const double pbk = k.cB * E * hb * iw;
    acc[1] += G * hs * iw;
    acc[2] += E * hb * iw;
    acc[3] += ps * k.q2 * d;
    acc[4] -= ps * d * d;
    acc[5] -= pbk * (m - kMLo);
    acc[6] += ps * rs.dlz;
    acc[7] += pbk * rb.dlz;
    acc[8] += sigt * (ps * rs.dls + pbk * rb.dls);
  }
}

// ---------------------------------------------------------------------------
// Model 3: angular x decay time x signal mass
// ---------------------------------------------------------------------------
struct Conv3 {
  double FH, FL;
  cplx Fc;
  double g;
  double phi;   // PHI: 1/2 g erfcx(tau / (sqrt2 s)) where needed, else 0
};

// The three convolved exponentials at one time point (and, at the range ends,
// the Phi term of the normalisation), their corrections in one branch.
template <bool PHI>
__device__ __forceinline__ Conv3 conv3(double tau, double mainH, double mainL, cplx mainC,
                                       const AngTimeConst& k, double s2, double inv_r2s, double dmr,
                                       double e_shift) {
  const TimePoint p = time_point(tau, k.gmax, s2, inv_r2s, dmr * dmr, e_shift);
  Conv3 r{mainH, mainL, mainC, p.g, 0.0};
  if (p.need) {
    r.FH = conv_real_needed(tau, k.gH, mainH, p, s2, inv_r2s);
    r.FL = conv_real_needed(tau, k.gL, mainL, p, s2, inv_r2s);
    r.Fc = conv_cplx_needed(tau, k.g, dmr, mainC, p, s2, inv_r2s);
    if constexpr (PHI) r.phi = 0.5 * p.g * erfcx_pos(tau * inv_r2s, p.depth);
  }
  return r;
}

// d F / d z = (s^2 z - tau) F - s^2 G_t(tau)
__device__ __forceinline__ double dconv_real(double tau, double rate, double F, double s2, double Gt) {
  return (s2 * rate - tau) * F - s2 * Gt;
}
__device__ __forceinline__ cplx dconv_cplx(double tau, const AngTimeConst& k, cplx F, double s2, double Gt) {
  const cplx a{s2 * k.g - tau, -s2 * k.dm};
  const cplx r = cmul(a, F);
  return cplx{r.re - s2 * Gt, r.im};
}

// The ten angular functions f_k(Omega) of the P + S wave decomposition.  The
// terms with sin(theta_K) and sin(theta_l) (through sin 2theta = 2 sin cos)
// need only the product sin(theta_K) sin(theta_l), one square root.
__device__ __forceinline__ void angular_functions(double ck, double cl, double ph, double* f) {
  const double sk2 = 1.0 - ck * ck, sl2 = 1.0 - cl * cl;
  const double v = cl * sqrt(sk2 * sl2);  // cos(theta_l) sin(theta_K) sin(theta_l)
  double sph, cph;
  sincos_fast(ph, &sph, &cph);
  constexpr double c5 = 4.0 * 0.70710678118654752440;  // 4 x sqrt2/2 (sin 2theta_K sin 2theta_l)
  constexpr double c8 = 2.0 * 0.81649658092772603273;  // 2 x sqrt6/3 (sin theta_K sin 2theta_l)
  constexpr double c10 = 2.3094010767585030580;        // 4 sqrt3/3
  const double ckv = ck * v;
  f[0] = 2.0 * ck * ck * sl2;
  f[1] = sk2 * (1.0 - sl2 * cph * cph);
  f[2] = sk2 * (1.0 - sl2 * sph * sph);
  f[3] = sk2 * sl2 * (2.0 * sph * cph);
  f[4] = -c5 * ckv * cph;
  f[5] = c5 * ckv * sph;
  f[6] = (2.0 / 3.0) * sl2;
  f[7] = -c8 * v * cph;
  f[8] = c8 * v * sph;
  f[9] = c10 * ck * sl2;
}

// Accumulator layout of the angular gradient: components 0 .. 11 are per-lane
// sums; the 40 coefficient adjoints (component kAngOuter0 + 4k + j, the sum
// over events of f_k tau_j) are formed per wave from the block below.
constexpr int kAngInner = 12;   // l, dD[4], dgH, dgL, dzr, ddm, dmu, dq, sum_w
constexpr int kAngOuter0 = 12;
constexpr int kAngOuter = 40;

// Per-wave LDS block of the angular gradient: row k < 10 holds f_k and row
// 10 + j holds tau_j of the wave's 64 current events, event (lane) e in column
// outer_col(e).  The block is read by lane 8b + g as the five f rows 5(b/4) ..
// 5(b/4) + 4 and the tau row b % 4, each over the eight events 8g .. 8g + 7 in
// pairs (16-byte reads): columns shifted by two after event 31 and a row pitch
// of 68 doubles put the 16 distinct f pairs of one read instruction in
// distinct banks.
constexpr int kOuterPitch = 68;
constexpr int kOuterRows = 14;
constexpr int kOuterWRow = 14;  // one more row: the events' weights until their last use
constexpr int kOuterQRow = 15;  // tagged model: the events' tag factors qd until their last use
constexpr int kOuterBlock = (kOuterRows + 1) * kOuterPitch;
constexpr int kOuterBlockTag = (kOuterRows + 2) * kOuterPitch;
__device__ __forceinline__ unsigned outer_col(unsigned e) { return e + ((e >> 5) << 1); }

// One event.  C is the coefficient table (row-major 10 x 4).  For the
// gradient, writes f_k and tau_j = w T_j / num into the wave's block at column
// ob, and takes the weight from the block's weight row (the caller puts it
// there when it loads the columns), not from w: read back only where it is
// first used, it holds no register through the event.
// TAG (tagged model): qd = q (1 - 2 omega) scales the cos and sin time terms
// and their integrals (the normalised mixture of the two flavours' PDFs for
// an event tagged q with mistag probability omega); untagged, qd is 1 and
// never read.  For the tagged gradient qd, like the weight, comes from the
// block (row kOuterQRow), read where it is used.
template <bool GRAD, bool COH = false, bool TAG = false>
__device__ __forceinline__ void event_angtime(const AngTimeConst& k, const double* __restrict__ C,
                                              double ck, double cl, double ph, double t, double sig,
                                              double m, double w, double* acc, double* ob, double qd = 1.0) {
  // time: per-event factors shared by t, T_LO and T_HI
  const double s2 = sig * sig;
  const double inv_sig = rcp(sig);
  const double inv_r2s = kInvSqrt2 * inv_sig;
  const double dmr = k.dm * sig * kInvSqrt2;
  const double eH2 = exp_small(k.hH2 * s2), eL2 = exp_small(k.hL2 * s2), ec2 = exp_lo(k.hc2 * s2);
  double sc, cc;
  sincos_small(k.gdm * s2, &sc, &cc);
  double st, ct;
  sincos_fast(k.dm * t, &st, &ct);
  // exp(z^2 s^2/2 - z tau) for z = Gamma - i dm has phase dm (tau - Gamma s^2);
  // e^{-Gamma_H t} = e^{-Gamma t} e^{DeltaGamma t/2}, e^{-Gamma_L t} = e^{-Gamma t} / e^{DeltaGamma t/2}
  const double eG = exp_lo(-k.g * t);
  const double eD = exp_lo(k.hdg * t);
  const double mt = ec2 * eG;
  const Conv3 Xt = conv3<false>(t, eH2 * (eG * eD), eL2 * (eG * rcp(eD)),
                         cplx{mt * (ct * cc + st * sc), mt * (st * cc - ct * sc)}, k, s2, inv_r2s, dmr, 0.0);
  const double ma = ec2 * k.eAG, mb = ec2 * k.eBG;
  const Conv3 Xa = conv3<true>(kTLo, eH2 * k.eAH, eL2 * k.eAL,
                         cplx{ma * (k.cA * cc + k.sA * sc), ma * (k.sA * cc - k.cA * sc)}, k, s2, inv_r2s, dmr,
                         k.shA);
  const Conv3 Xb = conv3<true>(kTHi, eH2 * k.eBH, eL2 * k.eBL,
                         cplx{mb * (k.cB * cc + k.sB * sc), mb * (k.sB * cc - k.cB * sc)}, k, s2, inv_r2s, dmr,
                         k.shB);
  // Phi(T_HI) - Phi(T_LO) = 1/2 [g_a erfcx(T_LO/(sqrt2 s)) - g_b erfcx(T_HI/(sqrt2 s))]
  const double dphi = Xa.phi - Xb.phi;
  const double IH = (dphi + Xa.FH - Xb.FH) * k.inv_gH;
  const double IL = (dphi + Xa.FL - Xb.FL) * k.inv_gL;
  const cplx Ic = cmul(cplx{dphi + Xa.Fc.re - Xb.Fc.re, Xa.Fc.im - Xb.Fc.im}, cplx{k.izr, k.izi});
  double T[4] = {0.5 * (Xt.FH + Xt.FL), 0.5 * (Xt.FH - Xt.FL), Xt.Fc.re, Xt.Fc.im};
  double I[4] = {0.5 * (IH + IL), 0.5 * (IH - IL), Ic.re, Ic.im};


  // angular part: A_j = sum_k f_k C_kj
  double f[10];
  angular_functions(ck, cl, ph, f);
  if constexpr (GRAD) {
    // to the block at once: f dies with the contraction below
#pragma unroll
    for (int kk = 0; kk < 10; ++kk) ob[kk * kOuterPitch] = f[kk];
  }
  double A[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int kk = 0; kk < 10; ++kk)
#pragma unroll
    for (int j = 0; j < 4; ++j) A[j] += f[kk] * C[4 * kk + j];
  double D2 = k.D[2], D3 = k.D[3];
  if constexpr (TAG) {
    // the tag factor multiplies the cos and sin terms: folded into their
    // angular sums and normalisation coefficients
    if constexpr (GRAD) {
      asm volatile("" ::: "memory");
      qd = ob[kOuterQRow * kOuterPitch];
    }
    A[2] *= qd;
    A[3] *= qd;
    D2 *= qd;
    D3 *= qd;
  }
  const double num = A[0] * T[0] + A[1] * T[1] + A[2] * T[2] + A[3] * T[3];
  const double den = k.D[0] * I[0] + k.D[1] * I[1] + D2 * I[2] + D3 * I[3];
  const double d = m - k.mu;
  if constexpr (GRAD) {
    asm volatile("" ::: "memory");
    w = ob[kOuterWRow * kOuterPitch];
  }
  acc[0] += w * (log_fast(num * rcp(den)) - d * d * k.q - k.lnNG);

  if constexpr (GRAD) {
    const double inum = w * rcp(num), iden = w * rcp(den);
    if constexpr (TAG) {
      // the derivatives with respect to the table's cos and sin columns and
      // their normalisation coefficients carry the tag factor
      const double inq = inum * qd, idq = iden * qd;
      ob[10 * kOuterPitch] = T[0] * inum;
      ob[11 * kOuterPitch] = T[1] * inum;
      ob[12 * kOuterPitch] = T[2] * inq;
      ob[13 * kOuterPitch] = T[3] * inq;
      acc[1] -= I[0] * iden;
      acc[2] -= I[1] * iden;
      acc[3] -= I[2] * idq;
      acc[4] -= I[3] * idq;
    } else {
#pragma unroll
      for (int j = 0; j < 4; ++j) ob[(10 + j) * kOuterPitch] = T[j] * inum;
#pragma unroll
      for (int j = 0; j < 4; ++j) acc[1 + j] -= I[j] * iden;
    }
    const double Gt = Xt.g * kInvSqrt2Pi * inv_sig;
    const double Ga = Xa.g * kInvSqrt2Pi * inv_sig;
    const double Gb = Xb.g * kInvSqrt2Pi * inv_sig;
    const double dFHt = dconv_real(t, k.gH, Xt.FH, s2, Gt);
    const double dFLt = dconv_real(t, k.gL, Xt.FL, s2, Gt);
    const cplx dFct = dconv_cplx(t, k, Xt.Fc, s2, Gt);
    const double dIH = (-IH + dconv_real(kTLo, k.gH, Xa.FH, s2, Ga) - dconv_real(kTHi, k.gH, Xb.FH, s2, Gb)) * k.inv_gH;
    const double dIL = (-IL + dconv_real(kTLo, k.gL, Xa.FL, s2, Ga) - dconv_real(kTHi, k.gL, Xb.FL, s2, Gb)) * k.inv_gL;
    const cplx dFca = dconv_cplx(kTLo, k, Xa.Fc, s2, Ga);
    const cplx dFcb = dconv_cplx(kTHi, k, Xb.Fc, s2, Gb);
    const cplx dIc = cmul(cplx{-Ic.re + dFca.re - dFcb.re, -Ic.im + dFca.im - dFcb.im}, cplx{k.izr, k.izi});
    acc[5] += 0.5 * (A[0] + A[1]) * dFHt * inum - k.Dp * dIH * iden;
    acc[6] += 0.5 * (A[0] - A[1]) * dFLt * inum - k.Dm * dIL * iden;
    acc[7] += (A[2] * dFct.re + A[3] * dFct.im) * inum - (D2 * dIc.re + D3 * dIc.im) * iden;
    acc[8] += (A[2] * dFct.im - A[3] * dFct.re) * inum - (D2 * dIc.im - D3 * dIc.re) * iden;
    acc[9] += w * k.q2 * d;
    acc[10] -= w * d * d;
    acc[11] += w;
  }
}

// ---------------------------------------------------------------------------
// Tile kernels
// ---------------------------------------------------------------------------
template <int MODEL>
struct ModelTraits;
template <>
struct ModelTraits<1> {
  using Const = MassConst;
  static constexpr int kAcc = kAccMass;
};
template <>
struct ModelTraits<2> {
  using Const = MassTimeConst;
  static constexpr int kAcc = kAccMassTime;
};

// Columns are addressed as (tile base pointer, 32-bit offset within the tile):
// the base is wave-uniform (scalar registers), so each load needs one 32-bit
// lane offset instead of a 64-bit address per column.
template <int MODEL, bool GRAD, bool COH = false>
__device__ __forceinline__ void event(const typename ModelTraits<MODEL>::Const& k, const EventCols& cols,
                                      int64_t base, unsigned j, double* acc) {
  const double w = cols.w ? ldg<COH>(cols.w + base, j) : 1.0;
  if constexpr (MODEL == 1) {
    event_mass<GRAD>(k, ldg<COH>(cols.c[0] + base, j), w, acc);
  } else {
    event_masstime<GRAD>(k, ldg<COH>(cols.c[0] + base, j), ldg<COH>(cols.c[1] + base, j),
                         ldg<COH>(cols.c[2] + base, j), w, acc);
  }
}

}  // namespace ipx
