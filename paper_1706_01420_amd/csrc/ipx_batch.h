// Batched evaluation: one launch evaluates many datasets of one model, each at
// its own parameter vector (the paper's Examples 4-5: hundreds of
// pseudo-experiments generated and fitted; here their likelihood calls are
// fused).  Every dataset keeps its own canonical tiles and partial buffers,
// and each tile runs the same per-event code as the single-dataset kernels,
// so a dataset's result does not depend on what else is in the batch.
//
// Work decomposition: a table of (segment, local tile) pairs covers the
// active datasets; workgroups stride over it.  Per-segment constants live in
// device memory (read with uniform addresses, i.e. scalar loads).
#pragma once

#include "ipx_kernels.h"

namespace ipx {

struct SegInfo {
  EventCols cols;
  double* partials;      // n_tiles x kAccMax, component-major
  double* tau;           // angular gradient scratch (4 x tau_stride)
  int64_t tau_stride;
  int64_t n_tiles;
  int64_t n_tiles_outer;
};

struct TileRef {
  int seg;
  int tile;
};

// ---------------------------------------------------------------------------
// Tile bodies (shared by the batch kernels and the persistent server kernel).
// k may live in device memory, kernel arguments or LDS: the arithmetic is the
// same, so a tile's partials do not depend on which kernel computed them.
// ---------------------------------------------------------------------------
template <int MODEL, bool GRAD, bool COH, int CAP>
__device__ __forceinline__ void tile_nll(const SegInfo& S, const typename ModelTraits<MODEL>::Const& k,
                                         int64_t tile, RedBuf<CAP>& red) {
  constexpr int NACC = GRAD ? ModelTraits<MODEL>::kAcc : 1;
  double acc[NACC];
#pragma unroll
  for (int c = 0; c < NACC; ++c) acc[c] = 0.0;
  const int64_t base = tile * kTile;
#pragma unroll 1
  for (int e = 0; e < kEventsPerLane; ++e) {
    const unsigned j = threadIdx.x + (unsigned)e * kThreads;
    if (base + j < S.cols.n) event<MODEL, GRAD, COH>(k, S.cols, base, j, acc);
  }
  tile_store<NACC, COH>(acc, S.partials, tile, S.n_tiles, red);
}

// Angular model; C is the coefficient table in LDS.
template <bool GRAD, bool COH, int CAP>
__device__ __forceinline__ void tile_angtime(const SegInfo& S, const AngTimeConst& k, const double* C,
                                             int64_t tile, RedBuf<CAP>& red) {
  constexpr int NACC = GRAD ? kAngInner : 1;
  double acc[NACC];
#pragma unroll
  for (int c = 0; c < NACC; ++c) acc[c] = 0.0;
  const int64_t base = tile * kTile;
#pragma unroll 1
  for (int e = 0; e < kEventsPerLane; ++e) {
    const unsigned j = threadIdx.x + (unsigned)e * kThreads;
    // keeps the LDS table reads inside the loop (re-read per event rather
    // than pinned in 80 registers)
    asm volatile("" ::: "memory");
    if (base + j < S.cols.n) {
      const EventCols& cl = S.cols;
      const double w = cl.w ? ldg<COH>(cl.w + base, j) : 1.0;
      event_angtime<GRAD, COH>(k, C, ldg<COH>(cl.c[0] + base, j), ldg<COH>(cl.c[1] + base, j),
                               ldg<COH>(cl.c[2] + base, j), ldg<COH>(cl.c[3] + base, j), ldg<COH>(cl.c[4] + base, j),
                               ldg<COH>(cl.c[5] + base, j), w, acc, S.tau + base, S.tau_stride, j);
    }
  }
  tile_store<NACC, COH>(acc, S.partials, tile, S.n_tiles, red);
}

// Angular gradient: coefficient adjoints over one outer tile.
template <bool COH, int CAP>
__device__ __forceinline__ void tile_angtime_outer(const SegInfo& S, int64_t tile, RedBuf<CAP>& red) {
  double acc[kAngOuter];
#pragma unroll
  for (int c = 0; c < kAngOuter; ++c) acc[c] = 0.0;
  const int64_t base = tile * kOuterTile;
#pragma unroll 1
  for (int e = 0; e < kOuterEventsPerLane; ++e) {
    const unsigned j = threadIdx.x + (unsigned)e * kThreads;
    if (base + j < S.cols.n) {
      double f[10];
      angular_functions(ldg<COH>(S.cols.c[0] + base, j), ldg<COH>(S.cols.c[1] + base, j),
                        ldg<COH>(S.cols.c[2] + base, j), f);
      const double* tau = S.tau + base;
      const int64_t ts = S.tau_stride;
      const double t0 = ldg<COH>(tau, j), t1 = ldg<COH>(tau + ts, j), t2 = ldg<COH>(tau + 2 * ts, j),
                   t3 = ldg<COH>(tau + 3 * ts, j);
#pragma unroll
      for (int kk = 0; kk < 10; ++kk) {
        acc[4 * kk + 0] += f[kk] * t0;
        acc[4 * kk + 1] += f[kk] * t1;
        acc[4 * kk + 2] += f[kk] * t2;
        acc[4 * kk + 3] += f[kk] * t3;
      }
    }
  }
  tile_store<kAngOuter, COH>(acc, S.partials + kAngOuter0 * S.n_tiles, tile, S.n_tiles, red);
}

// ---------------------------------------------------------------------------
// Batch kernels
// ---------------------------------------------------------------------------
// Models 1 and 2.
template <int MODEL, bool GRAD>
__global__ __launch_bounds__(kThreads) void k_nll_batch(const SegInfo* __restrict__ segs,
                                                        const TileRef* __restrict__ tiles, int64_t n_tiles,
                                                        const typename ModelTraits<MODEL>::Const* __restrict__ consts,
                                                        const unsigned char* __restrict__ active) {
  constexpr int kCap = GRAD ? ModelTraits<MODEL>::kAcc : 1;
  __shared__ RedBuf<kCap> red;
  for (int64_t g = blockIdx.x; g < n_tiles; g += gridDim.x) {
    const TileRef tr = tiles[g];
    if (!active[tr.seg]) continue;
    const typename ModelTraits<MODEL>::Const k = consts[tr.seg];
    tile_nll<MODEL, GRAD, false>(segs[tr.seg], k, tr.tile, red);
  }
}

// Angular model: per-event kernel.
// The gradient instance is held to 128 VGPRs (4 waves/SIMD; its natural
// allocation is 129, i.e. 3 waves, and the extra wave shortens the tail of the
// launch more than the few spilled registers cost).
template <bool GRAD>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(GRAD ? 4 : 1))) void k_angtime_batch(const SegInfo* __restrict__ segs,
                                                            const TileRef* __restrict__ tiles, int64_t n_tiles,
                                                            const AngTimeConst* __restrict__ consts,
                                                            const unsigned char* __restrict__ active) {
  __shared__ double sC[40];
  __shared__ RedBuf<GRAD ? kAngInner : 1> red;
  for (int64_t g = blockIdx.x; g < n_tiles; g += gridDim.x) {
    const TileRef tr = tiles[g];
    if (!active[tr.seg]) continue;
    const AngTimeConst& k = consts[tr.seg];
    if (threadIdx.x < 40) sC[threadIdx.x] = (&k.C[0][0])[threadIdx.x];
    __syncthreads();
    tile_angtime<GRAD, false>(segs[tr.seg], k, sC, tr.tile, red);
  }
}

// Angular model: coefficient adjoints over the outer tiles of each segment.
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(4))) void k_angtime_outer_batch(const SegInfo* __restrict__ segs,
                                                                  const TileRef* __restrict__ tiles,
                                                                  int64_t n_tiles,
                                                                  const unsigned char* __restrict__ active) {
  __shared__ RedBuf<kAngOuter / 4> red;   // 4 passes of 10 components: 22 KB, 4 workgroups per CU
  for (int64_t g = blockIdx.x; g < n_tiles; g += gridDim.x) {
    const TileRef tr = tiles[g];
    if (!active[tr.seg]) continue;
    tile_angtime_outer<false>(segs[tr.seg], tr.tile, red);
  }
}

// out[seg * kAccMax + c] = sum of the segment's tile partials of component c;
// grid (nacc, n_segments).  Components >= split use the outer tile count.
__global__ __launch_bounds__(kThreads) void k_reduce_batch(const SegInfo* __restrict__ segs,
                                                           const unsigned char* __restrict__ active, int split,
                                                           double* __restrict__ out) {
  const int seg = blockIdx.y;
  if (!active[seg]) return;
  const int c = blockIdx.x;
  const SegInfo& S = segs[seg];
  const int64_t nt = c < split ? S.n_tiles : S.n_tiles_outer;
  const double total = reduce_component(S.partials + (int64_t)c * S.n_tiles, nt);
  if (threadIdx.x == 0) out[(int64_t)seg * kAccMax + c] = total;
}

}  // namespace ipx
