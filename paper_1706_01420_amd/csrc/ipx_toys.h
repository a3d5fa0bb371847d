// Unbinned toy generation by accept-reject on the device (the paper's
// Example 5: pseudo-experiments generated on the GPU by accept-reject from a
// counter-based random stream; event counts fluctuated on the host).
//
// Stream: Philox4x64-10 (Salmon, Moraes, Dror, Shaw, SC'11), key
// (seed, toy_id), counter (c, b, model, 0) for candidate c and block b; each
// candidate uses a fixed number of blocks, so candidates are independent and
// can be evaluated in any order.  Uniforms u = ((word >> 12) + 0.5) 2^-52
// (exact).  Output: the first n accepted candidates in increasing c.
//
// Three passes per batch of candidates: k_gen_flags (one lane per candidate:
// proposal + acceptance test, flag per candidate), an exclusive prefix sum of
// the flags, and k_gen_write (accepted candidates re-derive their event from
// the same counters and write it at its rank).
//
// The arithmetic that turns uniforms into observables is written with
// contraction off, so the columns that depend on +, -, x only (m in the mass
// model, sigma_t in the time models, the angles) are bitwise reproducible on
// any IEEE implementation of the same recipe.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "ipx_kernels.h"

namespace ipx {

constexpr uint64_t kPhiloxM0 = 0xD2E7470EE14C6C93ull;
constexpr uint64_t kPhiloxM1 = 0xCA5A826395121157ull;
constexpr uint64_t kPhiloxW0 = 0x9E3779B97F4A7C15ull;
constexpr uint64_t kPhiloxW1 = 0xBB67AE8584CAA73Bull;
constexpr double kTwoPi = 6.283185307179586;   // 2 pi rounded to double
constexpr double kPi = 3.141592653589793;

struct Philox4 {
  uint64_t x[4];
};

__device__ __forceinline__ Philox4 philox4x64_10(uint64_t c0, uint64_t c1, uint64_t c2, uint64_t c3, uint64_t k0,
                                                 uint64_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint64_t hi0 = __umul64hi(kPhiloxM0, c0), lo0 = kPhiloxM0 * c0;
    const uint64_t hi1 = __umul64hi(kPhiloxM1, c2), lo1 = kPhiloxM1 * c2;
    c0 = hi1 ^ c1 ^ k0;
    c1 = lo1;
    c2 = hi0 ^ c3 ^ k1;
    c3 = lo0;
    k0 += kPhiloxW0;
    k1 += kPhiloxW1;
  }
  return Philox4{{c0, c1, c2, c3}};
}

__device__ __forceinline__ double u01(uint64_t x) { return ((double)(x >> 12) + 0.5) * 0x1p-52; }

template <int B>
__device__ __forceinline__ void candidate_uniforms(int model, uint64_t seed, uint64_t toy, uint64_t c, double* u) {
#pragma unroll
  for (int b = 0; b < B; ++b) {
    const Philox4 r = philox4x64_10(c, (uint64_t)b, (uint64_t)model, 0, seed, toy);
#pragma unroll
    for (int j = 0; j < 4; ++j) u[4 * b + j] = u01(r.x[j]);
  }
}

// Per-call generator constants (host-hoisted).
struct GenConst {
  uint64_t seed, toy;
  double M;            // acceptance bound
  // model 1 / 2 mass shape
  double f, mu, sig_m, lam, cS, cB, L_e;  // L_e = -expm1(-lam L) (background inverse CDF)
  // model 2
  double tau_s, tau_b, s, rs_num;         // rs_num = sig_m sqrt(2 pi) / N_G
  MassTimeConst mt;                       // rates for the per-event normalisation
  // model 3
  double gmin, G, DG, DM, mu3, sig3;
};

struct Candidate {
  bool accept;
  bool violation;
  double col[6];
  double w;
};

// Integral of F(t; rate, sigma) over [T_LO, T_HI] (real rate).
__device__ __forceinline__ double conv_integral_real(double rate, double h2, double eA, double eB, double inv_rate,
                                                     double gmax, double sig) {
  const double s2 = sig * sig;
  const double inv_r2s = kInvSqrt2 * rcp(sig);
  // the generator keeps the full continued-fraction depth (its accept
  // decisions follow the full-precision density)
  TimePoint pa = time_point(kTLo, gmax, s2, inv_r2s, 0.0, 0.0);
  TimePoint pb = time_point(kTHi, gmax, s2, inv_r2s, 0.0, 0.0);
  pa.depth = pb.depth = kCfMaxDepth;
  double dphi = 0.0;
  if (pa.need) dphi += 0.5 * pa.g * erfcx_pos(kTLo * inv_r2s);
  if (pb.need) dphi -= 0.5 * pb.g * erfcx_pos(kTHi * inv_r2s);
  const double e2 = exp(h2 * s2);
  const double Fa = conv_real(kTLo, rate, e2 * eA, pa, s2, inv_r2s);
  const double Fb = conv_real(kTHi, rate, e2 * eB, pb, s2, inv_r2s);
  return (dphi + Fa - Fb) * inv_rate;
}

#pragma clang fp contract(off)

template <int MODEL>
__device__ __forceinline__ Candidate gen_candidate(const GenConst& g, const double* __restrict__ C, uint64_t c) {
  Candidate r;
  r.w = 1.0;
  if constexpr (MODEL == 1) {
    double u[4];
    candidate_uniforms<1>(1, g.seed, g.toy, c, u);
    const double m = kMLo + (kMHi - kMLo) * u[0];
    const double d = m - g.mu;
    const double P = g.cS * exp(-(d * d) / (2.0 * g.sig_m * g.sig_m)) + g.cB * exp(-g.lam * (m - kMLo));
    const double lhs = u[1] * g.M;
    r.accept = lhs < P;
    r.violation = P > g.M;
    r.col[0] = m;
  } else if constexpr (MODEL == 2) {
    double u[8];
    candidate_uniforms<2>(2, g.seed, g.toy, c, u);
    const double st = 0.03 + 0.03 * u[0];
    const bool is_sig = u[1] < g.f;
    const double rr = sqrt(-2.0 * log(u[2]));
    double sb, cb;
    sincos(kTwoPi * u[3], &sb, &cb);
    const double g1 = rr * cb, g2 = rr * sb;
    double mb;
    if (g.lam == 0.0) mb = kMLo + (kMHi - kMLo) * u[4];
    else mb = kMLo - log1p(-u[4] * g.L_e) / g.lam;
    const double m = is_sig ? g.mu + g.sig_m * g1 : mb;
    const double t = -(is_sig ? g.tau_s : g.tau_b) * log(u[5]) + g.s * st * g2;
    const bool inr = m >= kMLo && m <= kMHi && t >= kTLo && t <= kTHi;
    const double sig = g.s * st;
    const MassTimeConst& k = g.mt;
    double R;
    if (is_sig) R = g.rs_num / (k.gs * conv_integral_real(k.gs, k.hs2, k.eAs, k.eBs, k.inv_gs, k.gmax, sig));
    else R = 1.0 / (k.gb * conv_integral_real(k.gb, k.hb2, k.eAb, k.eBb, k.inv_gb, k.gmax, sig));
    const double lhs = u[6] * g.M;
    r.accept = inr && lhs < R;
    r.violation = R > g.M;
    r.col[0] = m;
    r.col[1] = t;
    r.col[2] = st;
  } else {
    double u[12];
    candidate_uniforms<3>(3, g.seed, g.toy, c, u);
    const double st = 0.03 + 0.03 * u[0];
    const double t0 = -log(u[1]) / g.gmin;
    const double ck = 2.0 * u[2] - 1.0, cl = 2.0 * u[3] - 1.0, ph = kPi * (2.0 * u[4] - 1.0);
    double f[10];
    angular_functions(ck, cl, ph, f);
    const double e = exp((g.gmin - g.G) * t0);
    const double x = g.DG * t0 / 2.0;
    const double ex = exp(x), emx = exp(-x);
    double sd, cd;
    sincos(g.DM * t0, &sd, &cd);
    const double h[4] = {e * ((ex + emx) / 2.0), e * ((ex - emx) / 2.0), e * cd, e * sd};
    double R = 0.0;
#pragma unroll
    for (int kk = 0; kk < 10; ++kk) {
      double s = 0.0;
#pragma unroll
      for (int j = 0; j < 4; ++j) s += C[4 * kk + j] * h[j];
      R += f[kk] * s;
    }
    const double lhs = u[5] * g.M;
    const double rr = sqrt(-2.0 * log(u[6]));
    double sb, cb;
    sincos(kTwoPi * u[7], &sb, &cb);
    const double t = t0 + st * (rr * cb);
    const double m = g.mu3 + g.sig3 * (rr * sb);
    const bool inr = t >= kTLo && t <= kTHi && m >= kMLo && m <= kMHi;
    r.accept = inr && lhs < R;
    r.violation = R > g.M;
    r.col[0] = ck;
    r.col[1] = cl;
    r.col[2] = ph;
    r.col[3] = t;
    r.col[4] = st;
    r.col[5] = m;
    r.w = 0.8 + 0.2 * u[8];
  }
  return r;
}

#pragma clang fp contract(fast)

// Pass 1: flag[c - c0] = accepted; violations counted.
template <int MODEL>
__global__ __launch_bounds__(256) void k_gen_flags(GenConst g, const double* __restrict__ Cg, uint64_t c0,
                                                   int64_t count, int* __restrict__ flags,
                                                   unsigned long long* __restrict__ violations) {
  __shared__ double sC[40];
  if (MODEL == 3 && threadIdx.x < 40) sC[threadIdx.x] = Cg[threadIdx.x];
  __syncthreads();
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count) return;
  const Candidate r = gen_candidate<MODEL>(g, sC, c0 + (uint64_t)i);
  flags[i] = r.accept ? 1 : 0;
  if (r.violation) atomicAdd(violations, 1ull);
}

// Pass 3: accepted candidates write their event at out_base + rank while the
// rank is below `need`; the candidate giving the last needed event records
// its index + 1 in *last.
template <int MODEL>
__global__ __launch_bounds__(256) void k_gen_write(GenConst g, const double* __restrict__ Cg, uint64_t c0,
                                                   int64_t count, const int* __restrict__ flags,
                                                   const int* __restrict__ rank, int64_t out_base, int64_t need,
                                                   double* const* __restrict__ cols_ptr, double* __restrict__ wout,
                                                   unsigned long long* __restrict__ last) {
  __shared__ double sC[40];
  if (MODEL == 3 && threadIdx.x < 40) sC[threadIdx.x] = Cg[threadIdx.x];
  __syncthreads();
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count || !flags[i]) return;
  const int64_t rk = rank[i];
  if (rk >= need) return;
  const Candidate r = gen_candidate<MODEL>(g, sC, c0 + (uint64_t)i);
  const int64_t o = out_base + rk;
  constexpr int ncols = MODEL == 1 ? 1 : MODEL == 2 ? 3 : 6;
#pragma unroll
  for (int c = 0; c < ncols; ++c) cols_ptr[c][o] = r.col[c];
  if (MODEL == 3 && wout) wout[o] = r.w;
  if (rk == need - 1) *last = (unsigned long long)(c0 + (uint64_t)i) + 1ull;
}

// ---------------------------------------------------------------------------
// Batched generation: the candidates of many toys in one launch.  Segment j
// covers global positions [start, start + count) and maps position i to
// candidate c0 + (i - start) of toy j; each toy keeps its own key, candidate
// order and output, so its events are those a single-toy generation gives.
// ---------------------------------------------------------------------------
struct GenSeg {
  uint64_t toy;        // Philox key word 1
  uint64_t c0;         // first candidate of this round
  int64_t start;       // first global position
  int64_t count;       // candidates of this round
  int64_t out_base;    // events already written
  int64_t need;        // events still needed
  double* cols[6];
  double* w;           // nullptr: no weight column
};

__device__ __forceinline__ int gen_find_seg(const GenSeg* __restrict__ segs, int nseg, int64_t i) {
  int lo = 0, hi = nseg - 1;   // the last segment with start <= i
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (segs[mid].start <= i) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

template <int MODEL>
__global__ __launch_bounds__(256) void k_gen_flags_batch(GenConst g, const double* __restrict__ Cg,
                                                         const GenSeg* __restrict__ segs, int nseg, int64_t total,
                                                         int* __restrict__ flags,
                                                         unsigned long long* __restrict__ violations) {
  __shared__ double sC[40];
  if (MODEL == 3 && threadIdx.x < 40) sC[threadIdx.x] = Cg[threadIdx.x];
  __syncthreads();
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= total) return;
  const int j = gen_find_seg(segs, nseg, i);
  GenConst gj = g;
  gj.toy = segs[j].toy;
  const Candidate r = gen_candidate<MODEL>(gj, sC, segs[j].c0 + (uint64_t)(i - segs[j].start));
  flags[i] = r.accept ? 1 : 0;
  if (r.violation) atomicAdd(&violations[j], 1ull);
}

template <int MODEL>
__global__ __launch_bounds__(256) void k_gen_write_batch(GenConst g, const double* __restrict__ Cg,
                                                         const GenSeg* __restrict__ segs, int nseg, int64_t total,
                                                         const int* __restrict__ flags, const int* __restrict__ rank,
                                                         unsigned long long* __restrict__ last) {
  __shared__ double sC[40];
  if (MODEL == 3 && threadIdx.x < 40) sC[threadIdx.x] = Cg[threadIdx.x];
  __syncthreads();
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= total || !flags[i]) return;
  const int j = gen_find_seg(segs, nseg, i);
  const GenSeg& sg = segs[j];
  const int64_t rk = (int64_t)rank[i] - (int64_t)rank[sg.start];
  if (rk >= sg.need) return;
  GenConst gj = g;
  gj.toy = sg.toy;
  const uint64_t c = sg.c0 + (uint64_t)(i - sg.start);
  const Candidate r = gen_candidate<MODEL>(gj, sC, c);
  const int64_t o = sg.out_base + rk;
  constexpr int ncols = MODEL == 1 ? 1 : MODEL == 2 ? 3 : 6;
#pragma unroll
  for (int cc = 0; cc < ncols; ++cc) sg.cols[cc][o] = r.col[cc];
  if (MODEL == 3 && sg.w) sg.w[o] = r.w;
  if (rk == sg.need - 1) last[j] = (unsigned long long)c + 1ull;
}

// accepted[j] = candidates of segment j accepted in this round
__global__ void k_gen_counts(const GenSeg* __restrict__ segs, int nseg, const int* __restrict__ flags,
                             const int* __restrict__ rank, int64_t* __restrict__ accepted) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= nseg) return;
  const int64_t a = segs[j].start, b = a + segs[j].count - 1;
  accepted[j] = (int64_t)rank[b] + flags[b] - (int64_t)rank[a];
}

}  // namespace ipx
