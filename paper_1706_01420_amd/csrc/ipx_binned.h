// Binned path (the paper's Examples 3-5 on the binned side): a signal shape
// filled per bin and smeared by a Gaussian, an exponential background per
// bin, the binned Poisson likelihood of observed counts, binned Poisson toys
// and the CL_s construction from their test statistic.
//
// Conventions (equal bins of width dx on [lo, hi), centres x_b = lo + (b + 1/2) dx):
//   smearing     S_b = sum_j h_j g(x_b - x_j) dx, g the unit Gaussian density
//                (the rectangle rule of the convolution integral, no
//                wrap-around at the ends); a banded Toeplitz product, tiled
//                through LDS: 256 outputs per workgroup, 256 inputs per step.
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

// out[b] = sum_j h[j] kern[b - j + n - 1].
__global__ __launch_bounds__(kThreads) void k_smear(const double* __restrict__ h, const double* __restrict__ kern,
                                                    double* __restrict__ out, int n) {
  __shared__ double sh[kThreads];
  __shared__ double sk[2 * kThreads];
  const int b0 = blockIdx.x * kThreads;
  const int t = threadIdx.x;
  double acc = 0.0;
  for (int j0 = 0; j0 < n; j0 += kThreads) {
    sh[t] = j0 + t < n ? h[j0 + t] : 0.0;
    // kernel indices b - j + n - 1 for b in [b0, b0 + 255], j in [j0, j0 + 255]
    const int base = b0 - j0 - (kThreads - 1) + n - 1;
    for (int s = t; s < 2 * kThreads; s += kThreads) {
      const int i = base + s;
      sk[s] = (i >= 0 && i < 2 * n - 1) ? kern[i] : 0.0;
    }
    __syncthreads();
#pragma unroll 8
    for (int jj = 0; jj < kThreads; ++jj) acc = fma(sh[jj], sk[t - jj + kThreads - 1], acc);
    __syncthreads();
  }
  if (b0 + t < n) out[b0 + t] = acc;
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
// nu, e^{-nu}, k_max; and L_b = ln(1 + s_b / b_b).
struct ToyTables {
  double* nu;     // [2][n]
  double* em;     // [2][n]
  double* kmax;   // [2][n]
  double* L;      // [n]
};

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
    tb.nu[h * c.n + b] = nu;
    tb.em[h * c.n + b] = exp(-nu);
    tb.kmax[h * c.n + b] = floor(nu + 30.0 * sqrt(nu + 1.0) + 30.0);
  }
  tb.L[b] = log1p(s / bk);
}

// Poisson inversion in the order of the conventions above.
#pragma clang fp contract(off)
__device__ __forceinline__ double poisson_inverse(double u, double nu, double em, double kmax) {
  double k = 0.0, p = em, F = em;
  while (u > F && k < kmax) {
    k += 1.0;
    p = p * nu / k;
    F = F + p;
  }
  return k;
}
#pragma clang fp contract(on)

// Counts of one toy of hypothesis h: the lane that handles bins 4i .. 4i + 3
// draws them from one Philox block.
__device__ __forceinline__ void toy_block(const ToyTables& tb, int n, int h, uint64_t seed, uint64_t toy, int i,
                                          double cnt[4]) {
  const Philox4 r = philox4x64_10((uint64_t)i, toy, (uint64_t)h, 0, seed, kBinnedKey);
#pragma unroll
  for (int w = 0; w < 4; ++w) {
    const int b = 4 * i + w;
    cnt[w] = b < n ? poisson_inverse(u01(r.x[w]), tb.nu[h * n + b], tb.em[h * n + b], tb.kmax[h * n + b]) : 0.0;
  }
}

// q of each toy: grid (toys, 2 hypotheses), one workgroup per toy.  The sum
// of n_b L_b runs over the lane's bin blocks i = t, t + 256, ... in
// increasing order, then block_sum; q = 2 (S - sum).
__global__ __launch_bounds__(kThreads) void k_cls_toys(ToyTables tb, int n, double S, uint64_t seed,
                                                       uint64_t toy0, int ntoys, double* __restrict__ q) {
  __shared__ double lds4[kThreads / 64];
  const int h = blockIdx.y;
  const uint64_t toy = toy0 + blockIdx.x;
  const int nblk = (n + 3) / 4;
  double sum = 0.0;
  for (int i = threadIdx.x; i < nblk; i += kThreads) {
    double cnt[4];
    toy_block(tb, n, h, seed, toy, i, cnt);
#pragma unroll
    for (int w = 0; w < 4; ++w)
      if (4 * i + w < n) sum += cnt[w] * tb.L[4 * i + w];
  }
  const double t = block_sum(sum, lds4);
  if (threadIdx.x == 0) q[(int64_t)h * ntoys + blockIdx.x] = 2.0 * (S - t);
}

// q of given counts, in the order of k_cls_toys (one workgroup).
__global__ __launch_bounds__(kThreads) void k_q_counts(const double* __restrict__ cnt, const double* __restrict__ L,
                                                       int n, double S, double* __restrict__ q) {
  __shared__ double lds4[kThreads / 64];
  const int nblk = (n + 3) / 4;
  double sum = 0.0;
  for (int i = threadIdx.x; i < nblk; i += kThreads) {
#pragma unroll
    for (int w = 0; w < 4; ++w)
      if (4 * i + w < n) sum += cnt[4 * i + w] * L[4 * i + w];
  }
  const double t = block_sum(sum, lds4);
  if (threadIdx.x == 0) q[0] = 2.0 * (S - t);
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
