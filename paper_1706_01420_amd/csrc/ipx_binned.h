// Binned path (the paper's Examples 3-5 on the binned side): a signal shape
// filled per bin and smeared by a Gaussian, an exponential background per
// bin, the binned Poisson likelihood of observed counts, binned Poisson toys
// and the CL_s construction from their test statistic.
//
// Conventions (equal bins of width dx on [lo, hi), centres x_b = lo + (b + 1/2) dx):
//   smearing     S_b = sum_j h_j g(x_b - x_j) dx, g the unit Gaussian density
//                (the rectangle rule of the convolution integral, no
//                wrap-around at the ends); a Toeplitz product, tiled over
//                outputs and input chunks through LDS (k_smear_part).
//   background   e_b = exp(-k (x_b - x_0)) / Z, Z = sum_b exp(-k b dx) in
//                closed form (a geometric sum).
//   likelihood   NLL = sum_b [nu_b - n_b ln nu_b], nu_b = ns s_b + nb e_b.
//   toys         n_b = the smallest k with u <= F(k), F summed from k = 0
//                (p_0 = e^{-nu}, p_k = p_{k-1} nu / k, F(k) = F(k-1) + p_k, in
//                that order, with IEEE division and no contraction), u from
//                Philox4x64-10, key (seed, 0xB1), counter (b >> 2, toy,
//                hypothesis, 0), word b & 3; the search stops at
//                k_max = floor(nu + 30 sqrt(nu + 1) + 30).
//   statistic    q = 2 (sum_b s_b - sum_b n_b ln(1 + s_b / b_b)) for signal
//                s_b = ns S_b and background b_b = nb e_b.
// Every reduction has a fixed order (lane-strided sums, wave butterfly, waves
// in order, workgroups in index order).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "ipx_kernels.h"
#include "ipx_toys.h"

namespace ipx {

constexpr uint64_t kBinnedKey = 0xB1;
constexpr int kBinnedAcc = 5;   // NLL, sum r s, sum r e^, sum r e^ y, sum e^ y

// Sum of v over the workgroup in a fixed order (wave butterfly, waves in
// order); the result is valid in thread 0.
__device__ __forceinline__ double block_sum(double v, double* lds4) {
  v = wave_sum(v);
  if ((threadIdx.x & 63) == 0) lds4[threadIdx.x >> 6] = v;
  __syncthreads();
  const double t = (lds4[0] + lds4[1]) + (lds4[2] + lds4[3]);
  __syncthreads();
  return t;
}

// kern[i] = g((i - (n - 1)) dx) dx, i = 0 .. 2n - 2.
__global__ __launch_bounds__(kThreads) void k_smear_kernel(double* __restrict__ kern, int n, double dx,
                                                           double sigma) {
  const int i = blockIdx.x * kThreads + threadIdx.x;
  if (i >= 2 * n - 1) return;
  const double d = (double)(i - (n - 1)) * dx;
  kern[i] = exp(-d * d / (2.0 * sigma * sigma)) / (2.5066282746310005024 * sigma) * dx;
}

// Smearing as a Toeplitz product out[b] = sum_j h[j] kern[b - j + n - 1],
// tiled over outputs and inputs: workgroup (bx, by) takes the 1024 outputs
// from 1024 bx and the inputs of chunk by (kSmearChunk x steps inputs from
// jA = by x steps x kSmearChunk) and writes its partial sums to
// part[by n + b]; k_smear_sum adds the chunks in order.  Lane t holds the
// four outputs 1024 bx + 4t + r.  Per step of 256 inputs the workgroup stages
// the 1279 kernel values the tile touches and the 256 inputs in LDS; per
// eight inputs a lane reads the eleven kernel values its 4 x 8 products use
// (output r and input q take value r - q + 7 of the window) and eight inputs
// as four broadcast pairs, then does 32 fused multiply-adds.  The kernel
// values are stored skewed (position i + i / 4) so that the lanes' windows,
// four values apart, spread over the banks.  Each output's products are
// added in increasing input order.
constexpr int kSmearOut = 1024;       // outputs per workgroup (4 per lane)
constexpr int kSmearChunk = 256;      // inputs staged per step
constexpr int kSmearWin = kSmearOut + kSmearChunk - 1;
__device__ __forceinline__ int smear_pos(int i) { return i + (i >> 2); }

__global__ __launch_bounds__(kThreads) void k_smear_part(const double* __restrict__ h, const double* __restrict__ kern,
                                                         double* __restrict__ part, int n, int steps) {
  __shared__ double sk[kSmearWin + kSmearWin / 4 + 4];
  __shared__ __attribute__((aligned(16))) double sh[kSmearChunk];
  const int t = threadIdx.x;
  const int b0 = blockIdx.x * kSmearOut;
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  for (int st = 0; st < steps; ++st) {
    const int jA = (blockIdx.y * steps + st) * kSmearChunk;
    if (jA >= n) break;
    // kernel index of window entry i: b0 - jA + n - kSmearChunk + i
    const int kb = b0 - jA + n - kSmearChunk;
    __syncthreads();  // the previous step's reads are done
    for (int i = t; i < kSmearWin; i += kThreads) {
      const int g = kb + i;
      sk[smear_pos(i)] = (g >= 0 && g < 2 * n - 1) ? kern[g] : 0.0;
    }
    sh[t] = jA + t < n ? h[jA + t] : 0.0;
    __syncthreads();
#pragma unroll 2
    for (int jb = 0; jb < kSmearChunk; jb += 8) {
      // window entry base + s, base = 4t - jb + kSmearChunk - 8 (a multiple of 4)
      const int u = t - (jb >> 2) + (kSmearChunk >> 2) - 2;
      double w[11];
#pragma unroll
      for (int s = 0; s < 11; ++s) w[s] = sk[5 * u + s + (s >> 2)];
      const double2* hp = reinterpret_cast<const double2*>(sh + jb);
      double hv[8];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const double2 v = hp[q];
        hv[2 * q] = v.x;
        hv[2 * q + 1] = v.y;
      }
#pragma unroll
      for (int q = 0; q < 8; ++q)
#pragma unroll
        for (int r = 0; r < 4; ++r) acc[r] = fma(hv[q], w[r - q + 7], acc[r]);
    }
  }
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int b = b0 + 4 * t + r;
    if (b < n) part[(size_t)blockIdx.y * n + b] = acc[r];
  }
}

// out[b] = sum over c < nc of part[c n + b], c in increasing order.
__global__ __launch_bounds__(kThreads) void k_smear_sum(const double* __restrict__ part, double* __restrict__ out,
                                                        int n, int nc) {
  const int b = blockIdx.x * kThreads + threadIdx.x;
  if (b >= n) return;
  // eight loads in flight, added in chunk order
  double s = 0.0;
  for (int c0 = 0; c0 < nc; c0 += 8) {
    double v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) v[u] = c0 + u < nc ? part[(size_t)(c0 + u) * n + b] : 0.0;
#pragma unroll
    for (int u = 0; u < 8; ++u)
      if (c0 + u < nc) s += v[u];
  }
  out[b] = s;
}

// Input chunks of a smearing launch: enough workgroups to fill the chip, the
// partials held to 2^23 doubles (64 MiB) where n allows.
inline void smear_grid(int n, int* chunks, int* steps) {
  const int nstep = (n + kSmearChunk - 1) / kSmearChunk;
  const int nout = (n + kSmearOut - 1) / kSmearOut;
  int c = (2048 + nout - 1) / nout;                       // ~2048 workgroups
  const long long cap = (1ll << 23) / (n > 0 ? n : 1);
  if (c > cap) c = (int)cap;
  if (c > nstep) c = nstep;
  if (c < 1) c = 1;
  *steps = (nstep + c - 1) / c;
  *chunks = (nstep + *steps - 1) / *steps;
}

// core[b] = exp(-(x_b - mu)^2 / (2 sigma^2)).
__global__ __launch_bounds__(kThreads) void k_gauss_core(double* __restrict__ core, int n, double lo, double dx,
                                                         double mu, double sigma) {
  const int b = blockIdx.x * kThreads + threadIdx.x;
  if (b >= n) return;
  const double x = lo + ((double)b + 0.5) * dx;
  core[b] = exp(-(x - mu) * (x - mu) / (2.0 * sigma * sigma));
}

// v[b] *= scale.
__global__ __launch_bounds__(kThreads) void k_scale(double* __restrict__ v, int n, double scale) {
  const int b = blockIdx.x * kThreads + threadIdx.x;
  if (b < n) v[b] *= scale;
}

// One workgroup: out[0] = sum of v[0 .. n) (lane-strided, then block_sum).
__global__ __launch_bounds__(kThreads) void k_sum(const double* __restrict__ v, int n, double* __restrict__ out) {
  __shared__ double lds4[kThreads / 64];
  double s = 0.0;
  for (int b = threadIdx.x; b < n; b += kThreads) s += v[b];
  const double t = block_sum(s, lds4);
  if (threadIdx.x == 0) out[0] = t;
}

struct BinnedConst {
  double ns, nb, k, invZ;   // yields, background slope, 1 / sum_b exp(-k b dx)
  double lo, dx;
  int n;
};

// Per-workgroup partials of the binned NLL and its adjoints:
// part[c * nwg + wg] for c < kBinnedAcc.
__global__ __launch_bounds__(kThreads) void k_binned_nll(BinnedConst c, const double* __restrict__ sig,
                                                         const double* __restrict__ cnt, double* __restrict__ part) {
  __shared__ double lds4[kThreads / 64];
  const int b = blockIdx.x * kThreads + threadIdx.x;
  double a[kBinnedAcc] = {0.0, 0.0, 0.0, 0.0, 0.0};
  if (b < c.n) {
    const double y = (double)b * c.dx;           // x_b - x_0
    const double eh = exp(-c.k * y);
    const double s = sig[b];
    const double nu = c.ns * s + c.nb * eh * c.invZ;
    const double nb_ = cnt[b];
    a[0] = nu - (nb_ > 0.0 ? nb_ * log(nu) : 0.0);
    const double r = 1.0 - nb_ / nu;
    a[1] = r * s;
    a[2] = r * eh;
    a[3] = r * eh * y;
    a[4] = eh * y;
  }
  const int nwg = gridDim.x;
#pragma unroll
  for (int k = 0; k < kBinnedAcc; ++k) {
    const double t = block_sum(a[k], lds4);
    if (threadIdx.x == 0) part[k * nwg + blockIdx.x] = t;
  }
}

// Per bin and hypothesis h (0: background only, 1: signal + background):
// nu, e^{-nu}, k_max; L_b = ln(1 + s_b / b_b); and the first kCdf steps of
// the inversion's recurrence, F(0) .. F(kCdf - 1) and p_{kCdf - 1}, computed
// once per call with the same operations as the search itself (every toy
// of a bin walks the same sequence; only u differs).
constexpr int kCdf = 16;
constexpr int kCdfStride = kCdf + 2;   // F(0 .. kCdf - 1), p_{kCdf - 1}, pad (16-byte rows)
struct ToyTables {
  double* nu;     // [2][n]
  double* em;     // [2][n]
  double* kmax;   // [2][n]
  double* L;      // [n]
  double* cdf;    // [2][n][kCdfStride]
};

// Poisson inversion in the order of the conventions above.
#pragma clang fp contract(off)
// The first kCdf states (F(k), and p at the last) of the recurrence above.
__device__ __forceinline__ void poisson_cdf_head(double nu, double em, double* __restrict__ row) {
  double k = 0.0, p = em, F = em;
  row[0] = F;
  for (int i = 1; i < kCdf; ++i) {
    k += 1.0;
    p = p * nu / k;
    F = F + p;
    row[i] = F;
  }
  row[kCdf] = p;
  row[kCdf + 1] = 0.0;
}

// The inversion: the smallest k with u <= F(k), stepping p_k = p_{k-1} nu / k,
// F(k) = F(k-1) + p_k from p_0 = F(0) = e^{-nu}, stopping at k_max.  Its
// first kCdf steps are read from the table row (k_max >= 60 > kCdf, so the
// cap cannot stop the search there); past the row the recurrence continues
// from (kCdf - 1, p_{kCdf - 1}, F(kCdf - 1)), the state it would have
// reached, so the result is that of the plain recurrence from k = 0.
__device__ __forceinline__ double poisson_inverse_cached(double u, double nu, double kmax,
                                                         const double* __restrict__ row) {
  // F is non-decreasing, so the steps with u > F(k) are a prefix of the row
  // and their count is the first k with u <= F(k): the whole row is loaded
  // at once and counted without branches
  const double2* r2 = reinterpret_cast<const double2*>(row);
  double2 f[kCdf / 2];
#pragma unroll
  for (int i = 0; i < kCdf / 2; ++i) f[i] = r2[i];
  int c = 0;
#pragma unroll
  for (int i = 0; i < kCdf / 2; ++i) c += (u > f[i].x) + (u > f[i].y);
  if (c < kCdf) return (double)c;
  double k = (double)(kCdf - 1), p = row[kCdf], F = f[kCdf / 2 - 1].y;
  while (u > F && k < kmax) {
    k += 1.0;
    p = p * nu / k;
    F = F + p;
  }
  return k;
}
#pragma clang fp contract(on)

__global__ __launch_bounds__(kThreads) void k_toy_tables(BinnedConst c, const double* __restrict__ sig,
                                                         ToyTables tb) {
  const int b = blockIdx.x * kThreads + threadIdx.x;
  if (b >= c.n) return;
  const double s = c.ns * sig[b];
  const double bk = c.nb * exp(-c.k * ((double)b * c.dx)) * c.invZ;
  const double nus[2] = {bk, s + bk};
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const double nu = nus[h];
    const double em = exp(-nu);
    tb.nu[h * c.n + b] = nu;
    tb.em[h * c.n + b] = em;
    tb.kmax[h * c.n + b] = floor(nu + 30.0 * sqrt(nu + 1.0) + 30.0);
    poisson_cdf_head(nu, em, tb.cdf + ((size_t)h * c.n + b) * kCdfStride);
  }
  tb.L[b] = log1p(s / bk);
}


// Counts of one toy of hypothesis h: the lane that handles bins 4i .. 4i + 3
// draws them from one Philox block.
__device__ __forceinline__ void toy_block(const ToyTables& tb, int n, int h, uint64_t seed, uint64_t toy, int i,
                                          double cnt[4]) {
  const Philox4 r = philox4x64_10((uint64_t)i, toy, (uint64_t)h, 0, seed, kBinnedKey);
#pragma unroll
  for (int w = 0; w < 4; ++w) {
    const int b = 4 * i + w;
    cnt[w] = b < n ? poisson_inverse_cached(u01(r.x[w]), tb.nu[h * n + b], tb.kmax[h * n + b],
                                            tb.cdf + ((size_t)h * n + b) * kCdfStride)
                   : 0.0;
  }
}

// CL_s toys, blocked by bins.  Workgroup (x, y, h) takes bin block x (quads
// 64 x .. 64 x + 63, four bins each) for the toys kClsToys y .. of
// hypothesis h: it stages the block's CDF heads in LDS as T[w][k][quad] (w
// the bin within its quad), so that the lanes, one quad each, read
// consecutive addresses at every k (35 KB: four workgroups per compute
// unit); each wave takes one toy at a time (wave i the toys i, i + 4, ...).
// Per toy a lane adds n_b L_b over its four bins in order, the wave adds its
// lanes (butterfly), and the block's sum goes to part[(h nblk + x) ntoys +
// toy].  k_cls_q adds the blocks in order.  With obs != nullptr the counts
// are obs[b] instead of a toy's (grid (nblk, 1, 1), one "toy"), which gives
// q_obs in the same order.
constexpr int kClsQuads = 64;
constexpr int kClsToys = 256;
constexpr int kClsRows = kCdf + 1;   // F(0 .. kCdf - 1), then p_{kCdf - 1}

#pragma clang fp contract(off)
__device__ __forceinline__ double poisson_inverse_lds(double u, const double (*Tw)[kClsQuads], int qi,
                                                      const ToyTables& tb, int h, int n, int b) {
  int c = 0;
#pragma unroll
  for (int k = 0; k < kCdf; ++k) c += (u > Tw[k][qi]);
  if (c < kCdf) return (double)c;
  double k = (double)(kCdf - 1), p = Tw[kCdf][qi], F = Tw[kCdf - 1][qi];
  const double nu = tb.nu[h * n + b], kmax = tb.kmax[h * n + b];
  while (u > F && k < kmax) {
    k += 1.0;
    p = p * nu / k;
    F = F + p;
  }
  return k;
}
#pragma clang fp contract(on)

__global__ __launch_bounds__(kThreads) void k_cls_block(ToyTables tb, int n, uint64_t seed, int ntoys,
                                                        const double* __restrict__ obs, double* __restrict__ part) {
  static_assert(kClsQuads == 64, "one wave per toy");
  __shared__ double T[4][kClsRows][kClsQuads];
  const int h = blockIdx.z;
  const int nq = (n + 3) / 4, nblk = gridDim.x;
  const int q0 = blockIdx.x * kClsQuads;
  const int qi = threadIdx.x % kClsQuads, slot = threadIdx.x / kClsQuads;   // slot: the wave
  const int q = q0 + qi;
  if (!obs) {
    for (int e = threadIdx.x; e < 4 * kClsRows * kClsQuads; e += kThreads) {
      const int qq = e % kClsQuads, k = (e / kClsQuads) % kClsRows, w = e / (kClsQuads * kClsRows);
      const int b = 4 * (q0 + qq) + w;
      T[w][k][qq] = b < n ? tb.cdf[((size_t)h * n + b) * kCdfStride + k] : 0.0;
    }
  }
  double L[4];
#pragma unroll
  for (int w = 0; w < 4; ++w) L[w] = (q < nq && 4 * q + w < n) ? tb.L[4 * q + w] : 0.0;
  __syncthreads();
  const int lane = threadIdx.x & 63;
  const int tend = obs ? 1 : kClsToys;
  for (int tt = 0; tt < tend; tt += kThreads / kClsQuads) {
    const int toy = blockIdx.y * kClsToys + tt + slot;
    double v = 0.0;
    if (q < nq && (obs ? toy == 0 : toy < ntoys)) {
      double cnt[4];
      if (obs) {
#pragma unroll
        for (int w = 0; w < 4; ++w) cnt[w] = 4 * q + w < n ? obs[4 * q + w] : 0.0;
      } else {
        const Philox4 r = philox4x64_10((uint64_t)q, (uint64_t)toy, (uint64_t)h, 0, seed, kBinnedKey);
#pragma unroll
        for (int w = 0; w < 4; ++w)
          cnt[w] = 4 * q + w < n ? poisson_inverse_lds(u01(r.x[w]), T[w], qi, tb, h, n, 4 * q + w) : 0.0;
      }
#pragma unroll
      for (int w = 0; w < 4; ++w) v += cnt[w] * L[w];
    }
    v = wave_sum(v);
    if (lane == 0 && (obs ? toy == 0 : toy < ntoys)) part[((size_t)h * nblk + blockIdx.x) * (obs ? 1 : ntoys) + toy] = v;
  }
}

// q[h ntoys + toy] = 2 (S - sum over the bin blocks, in order, of part);
// grid (ceil(ntoys / kThreads), hypotheses).
__global__ __launch_bounds__(kThreads) void k_cls_q(const double* __restrict__ part, int nblk, int ntoys, double S,
                                                    double* __restrict__ q) {
  const int toy = blockIdx.x * kThreads + threadIdx.x;
  const int h = blockIdx.y;
  if (toy >= ntoys) return;
  double s = 0.0;
  for (int x = 0; x < nblk; ++x) s += part[((size_t)h * nblk + x) * ntoys + toy];
  q[(size_t)h * ntoys + toy] = 2.0 * (S - s);
}

// ge[h] = number of toys of hypothesis h with q >= q_obs (integer counts).
__global__ __launch_bounds__(kThreads) void k_count_ge(const double* __restrict__ q, int ntoys,
                                                       const double* __restrict__ q_obs,
                                                       unsigned long long* __restrict__ ge) {
  const int i = blockIdx.x * kThreads + threadIdx.x;
  const int h = blockIdx.y;
  const bool hit = i < ntoys && q[(int64_t)h * ntoys + i] >= q_obs[0];
  const unsigned long long m = __ballot(hit);
  if ((threadIdx.x & 63) == 0 && m) atomicAdd(&ge[h], (unsigned long long)__popcll(m));
}

// The counts of one toy (for inspection): cnt[b], b < n.
__global__ __launch_bounds__(kThreads) void k_toy_counts(ToyTables tb, int n, int h, uint64_t seed, uint64_t toy,
                                                         double* __restrict__ cnt) {
  const int i = blockIdx.x * kThreads + threadIdx.x;
  if (4 * i >= n) return;
  double c[4];
  toy_block(tb, n, h, seed, toy, i, c);
#pragma unroll
  for (int w = 0; w < 4; ++w)
    if (4 * i + w < n) cnt[4 * i + w] = c[w];
}

}  // namespace ipx
