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
  int64_t n_tiles;
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

// Make a wave's LDS writes visible to its other lanes and keep the compiler
// from moving LDS accesses across (a wave's LDS operations complete in issue
// order, so no wait instruction is needed).
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Reduction rows that hold a wave's adjoint block: whole 16-byte units per
// wave, so that every wave's block starts 16-byte aligned.
constexpr int kOuterCap = ((kOuterBlock + kRedPitch - 1) / kRedPitch + 1) & ~1;
constexpr int kOuterCapTag = ((kOuterBlockTag + kRedPitch - 1) / kRedPitch + 1) & ~1;

// Angular model; C is the coefficient table (device memory read with uniform
// addresses, or LDS).  For the gradient, after
// each round of 64 events a wave forms the 40 coefficient adjoints of those
// events from its LDS block, so the per-event factors never leave the chip:
// lane 8b + g (b = 4h + j) sums f_k tau_j over the events 8g .. 8g + 7 for
// the five k = 5h .. 5h + 4 (one tau read serves five products), and lane
// 8b + g, g < 5, adds sum g of the eight lanes of b (through the block) to
// its running total of coefficient (5h + g, j).  Lanes
// without an event write zeros to the block.  The block is the wave's part of
// the reduction buffer, which the tile reduction reuses afterwards.
template <bool GRAD, bool COH, int CAP, bool TAG = false>
__device__ __forceinline__ void tile_angtime(const SegInfo& S, const AngTimeConst& k, const double* C,
                                             int64_t tile, RedBuf<CAP>& red) {
  static_assert(!GRAD || (CAP >= (TAG ? kOuterCapTag : kOuterCap) && CAP % 2 == 0),
                "the adjoint block lives in the reduction buffer");
  constexpr int NACC = GRAD ? kAngInner : 1;
  double acc[NACC];
#pragma unroll
  for (int c = 0; c < NACC; ++c) acc[c] = 0.0;
  double outer = 0.0;
  const unsigned lane = threadIdx.x & 63u;
  double* blk = &red.rows[threadIdx.x >> 6][0][0];
  const int64_t base = tile * kTile;
#pragma unroll 1
  for (int e = 0; e < kEventsPerLane; ++e) {
    const unsigned j = threadIdx.x + (unsigned)e * kThreads;
    // keeps the table reads inside the loop (re-read per event rather than
    // pinned in 80 registers)
    asm volatile("" ::: "memory");
    if (base + j < S.cols.n) {
      const EventCols& cl = S.cols;
      double w = cl.w ? ldg<COH>(cl.w + base, j) : 1.0;
      if constexpr (GRAD) {
        blk[kOuterWRow * kOuterPitch + outer_col(lane)] = w;
        w = 0.0;  // the event reads its weight back from the block
      }
      double qd = TAG ? ldg<COH>(cl.c[6] + base, j) : 1.0;
      if constexpr (GRAD && TAG) {
        blk[kOuterQRow * kOuterPitch + outer_col(lane)] = qd;
        qd = 0.0;  // read back from the block where it is used
      }
      event_angtime<GRAD, COH, TAG>(k, C, ldg<COH>(cl.c[0] + base, j), ldg<COH>(cl.c[1] + base, j),
                                    ldg<COH>(cl.c[2] + base, j), ldg<COH>(cl.c[3] + base, j),
                                    ldg<COH>(cl.c[4] + base, j), ldg<COH>(cl.c[5] + base, j), w, acc,
                                    blk + outer_col(lane), qd);
    } else if constexpr (GRAD) {
#pragma unroll
      for (int r = 0; r < kOuterRows; ++r) blk[r * kOuterPitch + outer_col(lane)] = 0.0;
    }
    if constexpr (GRAD) {
      wave_lds_sync();
      const unsigned g = lane & 7u, b = lane >> 3;
      const double* fr = blk + 5 * (b >> 2) * kOuterPitch;
      const double* tr = blk + (10 + (b & 3u)) * kOuterPitch;
      double a[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (unsigned i = 0; i < 8; ++i) {
        const unsigned c = outer_col(8 * g + i);
        const double t = tr[c];
#pragma unroll
        for (int r = 0; r < 5; ++r) a[r] = fma(fr[r * kOuterPitch + c], t, a[r]);
      }
      wave_lds_sync();
      // the eight lanes of b add their sums through the block: each lane
      // puts its five in rows 0 .. 4 (column = lane), and lane 8b + g, g < 5,
      // adds row g over the lanes 8b .. 8b + 7 pairwise, in the order of an
      // xor butterfly
#pragma unroll
      for (int r = 0; r < 5; ++r) blk[r * kOuterPitch + lane] = a[r];
      wave_lds_sync();
      if (g < 5) {
        const double2* q = reinterpret_cast<const double2*>(blk + g * kOuterPitch + 8 * b);
        const double2 c01 = q[0], c23 = q[1], c45 = q[2], c67 = q[3];
        outer += ((c01.x + c01.y) + (c23.x + c23.y)) + ((c45.x + c45.y) + (c67.x + c67.y));
      }
      wave_lds_sync();
    }
  }
  if constexpr (GRAD) {
    unsigned tid = threadIdx.x;
    asm volatile("" : "+v"(tid));  // the address is derived here, not kept live through the loop
    const unsigned g = tid & 7u, b = (tid & 63u) >> 3;
    if (g < 5) red.wsum[tid >> 6][kAngOuter0 + 4 * (5 * (b >> 2) + g) + (b & 3u)] = outer;
    tile_store<NACC, COH, CAP, kAccAngTime>(acc, S.partials, tile, S.n_tiles, red);
  } else {
    tile_store<NACC, COH, CAP>(acc, S.partials, tile, S.n_tiles, red);
  }
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

// Angular model.
// The gradient instance is held to 128 VGPRs (4 waves/SIMD; the extra wave
// shortens the tail of the launch more than the few spilled registers cost);
// its LDS (adjoint blocks sharing the reduction buffer, ~35 KB) allows 4
// workgroups per compute unit.  WPE > 0 builds a variant for another
// waves-per-SIMD target (a launch-schedule choice: the arithmetic, and so
// every result, is the same).
template <bool GRAD, bool TAG = false, int WPE = 0>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(WPE > 0 ? WPE : (GRAD ? 4 : 1)))) void k_angtime_batch(const SegInfo* __restrict__ segs,
                                                            const TileRef* __restrict__ tiles, int64_t n_tiles,
                                                            const AngTimeConst* __restrict__ consts,
                                                            const unsigned char* __restrict__ active) {
  constexpr int kCap = GRAD ? (TAG ? kOuterCapTag : kOuterCap) : 1;
  __shared__ RedBuf<kCap> red;
  for (int64_t g = blockIdx.x; g < n_tiles; g += gridDim.x) {
    const TileRef tr = tiles[g];
    if (!active[tr.seg]) continue;
    // the coefficient table is read where it is used, with uniform addresses
    // (scalar loads: the contraction's operands come straight from scalar
    // registers)
    const AngTimeConst& k = consts[tr.seg];
    tile_angtime<GRAD, false, kCap, TAG>(segs[tr.seg], k, &k.C[0][0], tr.tile, red);
  }
}

// out[seg * kAccMax + c] = sum of the segment's tile partials of component c;
// grid (nacc, n_segments).
__global__ __launch_bounds__(kThreads) void k_reduce_batch(const SegInfo* __restrict__ segs,
                                                           const unsigned char* __restrict__ active,
                                                           double* __restrict__ out) {
  const int seg = blockIdx.y;
  if (!active[seg]) return;
  const int c = blockIdx.x;
  const SegInfo& S = segs[seg];
  const double total = reduce_component(S.partials + (int64_t)c * S.n_tiles, S.n_tiles);
  if (threadIdx.x == 0) out[(int64_t)seg * kAccMax + c] = total;
}

}  // namespace ipx
