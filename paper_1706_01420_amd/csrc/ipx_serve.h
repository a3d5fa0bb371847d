// Served likelihood: a persistent kernel that takes NLL / gradient requests
// from a host-visible mailbox while it runs (continuous batching: requests
// that arrive while others are being evaluated join the same launch).
//
// Protocol (S slots; workgroup 0 is the poller, the others are workers):
//   host    writes the request descriptor desc[s] into fine-grained host
//           memory, then mail[s] = seq and bumps gen (in that order).
//   poller  the only workgroup that reads host memory.  When gen changes it
//           reads every mail word; for each slot with a new sequence number it
//           copies desc[s] into device memory, clears the slot's completion
//           counters, writes lim[s] = (seq << 32) | claims, then publishes
//           claim[s] = seq << 32 and sets the slot's bit in the claimable-slot
//           mask.  A claim is a run of serve_chunk(items, workers) consecutive
//           tiles (one tile for requests smaller than twice the workers).
//   workers take one claim at a time with one atomic add on claim[s] of a
//           slot in the mask: each workgroup from its own starting slot
//           (policy 0, requests spread over the workers), the oldest opened
//           request first (policy 1: the first wave reads the open stamps of
//           the claimable slots and picks the smallest), or the request with
//           the fewest unclaimed claims first (policy 2: the first wave reads
//           the claim and limit words of the claimable slots); the returned
//           word names the request (high half) and the claim (low half).  The
//           claim is valid if lim[s] names the same request and the claim is
//           below its count; any other increment is a late claim on a
//           finished request and is dropped, so no request can lose a tile.
//           The worker that takes a slot's last claim clears its mask bit.
//           After a claim's tiles, done[s] += 1; the worker that completes a
//           request's last claim sums every component's tile partials in
//           index order (the order of the other entry points), writes out[s],
//           then fin[s] = seq.
//   exit    the poller counts its polls that find neither a new request nor
//           a claimable item; after `idle_limit` of them in a row it sets quit
//           and opens no more requests.  Workers leave on quit or stop (after
//           finishing the claim they hold) and count themselves out of `live`;
//           the poller leaves when no worker is left, or at once on stop.
//           Workers never leave on their own, so a loop that is running has
//           all its workgroups (a request arriving after quit waits for the
//           host to relaunch the loop).
//
// Memory ordering without cache-wide fences.  On this GPU every XCD has its
// own L2, and an agent-scope release or acquire fence writes back or
// invalidates that whole cache; with hundreds of workgroups fencing per item
// the fences cost more than the tiles.  Instead, every location that one
// workgroup writes and another reads during the launch (descriptors, lim,
// claim, counters, tile partials; also the event columns,
// which may have been written after the launch) is accessed with relaxed
// device-coherent atomics, and a writer waits for its stores to complete
// (s_waitcnt, then the workgroup barrier) before the atomic that publishes
// them.  A reader issues its loads only after it has observed that atomic,
// and coherent loads see every completed coherent store.  Host memory is read
// and written with system-coherent atomics in the same way.
//
// No workgroup waits on another's work, and every scan is bounded, so the
// grid always drains.
#pragma once

#include "ipx_batch.h"

namespace ipx {

constexpr int kServeMaxSlots = 64;

struct ServeDesc {
  unsigned long long seq;  // the request's sequence number in its slot
  int model;
  int grad;
  int items;         // tiles of the dataset
  int nacc;          // reduced components
  SegInfo seg;       // columns of the dataset + this request's scratch
  union {
    MassConst m1;
    MassTimeConst m2;
    AngTimeConst m3;
  } k;
};
static_assert(sizeof(ServeDesc) % 8 == 0, "descriptor is copied in 8-byte words");

struct ServeSlot {                 // device memory, touched by the GPU only
  unsigned long long claim;        // (seq << 32) | next item
  unsigned long long lim;          // (seq << 32) | items of the request in the slot
  unsigned long long open;         // last seq opened by the poller
  unsigned long long stamp;        // opening order of the request in the slot (ServeCtl::opened)
  unsigned int done;               // completed items
  unsigned int pad;
};

struct ServeCtl {                  // device memory
  unsigned long long mask;         // slots that may have unclaimed items
  unsigned long long stop;         // mirror of the host's stop
  unsigned long long opened;       // requests opened so far (written by the poller only)
  unsigned int live;               // worker workgroups still running (set by the host at launch)
  unsigned int quit;               // set by the poller after idle_limit idle polls (0 at launch)
};

// Claim policies of the workers.
enum : int { kServeSpread = 0, kServeOldestFirst = 1, kServeFewestFirst = 2 };

// Tiles per claim of a request of `items` tiles with `workers` worker
// workgroups: about two claims per worker for large requests (each claim is
// one atomic on the slot's claim word and one on its done count, and every
// worker of the loop would otherwise contend for them once per tile), one
// tile per claim for requests smaller than twice the workers, at most 16.
__host__ __device__ __forceinline__ unsigned serve_chunk(unsigned items, unsigned workers) {
  const unsigned w2 = 2u * (workers > 0u ? workers : 1u);
  const unsigned k = (items + w2 - 1u) / w2;
  return k < 1u ? 1u : (k > 16u ? 16u : k);
}
__host__ __device__ __forceinline__ unsigned serve_claims(unsigned items, unsigned workers) {
  const unsigned k = serve_chunk(items, workers);
  return (items + k - 1u) / k;
}

struct ServeShared {               // fine-grained host memory
  unsigned long long gen;          // bumped by the host after each publication
  unsigned long long stop;
  unsigned long long mail[kServeMaxSlots];
  unsigned long long fin[kServeMaxSlots];
  double out[kServeMaxSlots][kAccMax];
  ServeDesc desc[kServeMaxSlots];
};

template <typename T>
__device__ __forceinline__ T load_sys(const T* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
}
template <typename T>
__device__ __forceinline__ void store_sys(T* p, T v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
}
template <typename T>
__device__ __forceinline__ T load_dev(const T* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <typename T>
__device__ __forceinline__ void store_dev(T* p, T v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Wait until every memory access this lane has issued has completed; also a
// compiler barrier for memory operations.
__device__ __forceinline__ void wait_mem() { asm volatile("s_waitcnt vmcnt(0) lgkmcnt(0)" ::: "memory"); }

// Copy n 8-byte words with the workgroup's lanes: host (system-coherent) to
// device (device-coherent), or device (device-coherent) to LDS.
__device__ __forceinline__ void copy_host_to_dev(unsigned long long* dst, const unsigned long long* src, int n) {
  for (int i = threadIdx.x; i < n; i += kThreads) store_dev(dst + i, load_sys(src + i));
}
__device__ __forceinline__ void copy_dev_to_lds(unsigned long long* dst, const unsigned long long* src, int n) {
  for (int i = threadIdx.x; i < n; i += kThreads) dst[i] = load_dev(src + i);
}

enum : int { kCmdIdle = 0, kCmdWork = 1, kCmdExit = 2, kCmdScan = 3 };

// Poller: opens slot s for request seq (whole workgroup).
__device__ __forceinline__ void serve_open(ServeShared* hs, ServeCtl* ctl, ServeDesc* __restrict__ dd,
                                           ServeSlot* __restrict__ st, int s, unsigned long long seq) {
  constexpr int kWords = (int)(sizeof(ServeDesc) / sizeof(unsigned long long));
  copy_host_to_dev((unsigned long long*)&dd[s], (const unsigned long long*)&hs->desc[s], kWords);
  wait_mem();
  __syncthreads();
  if (threadIdx.x == 0) {
    const unsigned claims = serve_claims((unsigned)load_dev(&dd[s].items), gridDim.x - 1u);
    const unsigned long long stamp = load_dev(&ctl->opened) + 1ull;
    store_dev(&ctl->opened, stamp);
    store_dev(&st[s].stamp, stamp);
    store_dev(&st[s].open, seq);
    store_dev(&st[s].done, 0u);
    store_dev(&st[s].lim, (seq << 32) | (unsigned long long)claims);
    wait_mem();
    store_dev(&st[s].claim, seq << 32);
    wait_mem();
    __hip_atomic_fetch_or(&ctl->mask, 1ull << s, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  __syncthreads();
}

__device__ __forceinline__ void serve_poll(ServeShared* hs, ServeCtl* ctl, ServeDesc* __restrict__ dd,
                                           ServeSlot* __restrict__ st, int nslots, int idle_limit) {
  __shared__ int pcmd;
  __shared__ unsigned long long pseq[kServeMaxSlots];
  unsigned long long seen = 0;  // last host generation scanned (thread 0)
  int idle = 0;                 // consecutive idle polls (thread 0)
  for (;;) {
    if (threadIdx.x == 0) {
      const unsigned long long g = load_sys(&hs->gen);
      if (load_sys(&hs->stop)) {
        pcmd = kCmdExit;
        store_dev(&ctl->stop, 1ull);
      } else if (load_dev(&ctl->quit)) {
        // draining: no new request is opened; leave with the last worker
        pcmd = load_dev(&ctl->live) == 0u ? kCmdExit : kCmdIdle;
      } else if (g != seen) {
        // set before the scan: a publication during the scan bumps gen again
        seen = g;
        idle = 0;
        pcmd = kCmdScan;
      } else if (load_dev(&ctl->mask) != 0ull) {
        idle = 0;
        pcmd = kCmdIdle;
      } else {
        if (++idle > idle_limit) store_dev(&ctl->quit, 1u);
        pcmd = kCmdIdle;
      }
      wait_mem();  // the mail words below are read after gen
    }
    __syncthreads();
    const int c = pcmd;
    if (c == kCmdExit) return;
    if (c == kCmdScan) {
      for (int s = threadIdx.x; s < nslots; s += kThreads) {
        const unsigned long long m = load_sys(&hs->mail[s]);
        pseq[s] = m > load_dev(&st[s].open) ? m : 0ull;
      }
      wait_mem();  // descriptors are read after their mail word
      __syncthreads();
      for (int s = 0; s < nslots; ++s)
        if (pseq[s]) serve_open(hs, ctl, dd, st, s, pseq[s]);
    } else {
      __builtin_amdgcn_s_sleep(8);
    }
    __syncthreads();
  }
}

// Thread 0: one claim on slot s; true (and the item in cslot/citem) if the
// claim names the request in the slot and an item below its count.
__device__ __forceinline__ bool serve_claim(ServeCtl* ctl, ServeSlot* __restrict__ st, int s, int* cslot,
                                            int* citem) {
  const unsigned long long old =
      __hip_atomic_fetch_add(&st[s].claim, 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  wait_mem();  // lim is read after the claim word it validates
  const unsigned long long lim = load_dev(&st[s].lim);
  const unsigned item = (unsigned)(old & 0xffffffffull);
  const unsigned n = (unsigned)(lim & 0xffffffffull);
  if ((lim >> 32) != (old >> 32) || item >= n) return false;
  *cslot = s;
  *citem = (int)item;
  if (item == n - 1u)
    __hip_atomic_fetch_and(&ctl->mask, ~(1ull << s), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  return true;
}

// The totals of components c0 .. c0 + 7 (those below nacc) of a request's
// tile partials (component-major, nt per component), each added in exactly
// the order of reduce_component: thread t sums tiles t, t + 256, ... in
// index order, the wave adds its lanes by the xor butterfly, the four wave
// totals are added as (w0 + w1) + (w2 + w3).  The eight components share the
// memory round trips (the partials' loads of one stride step are in flight
// together) instead of taking one reduction each.  Result in tot (LDS).
constexpr int kServeReduceGroup = 8;
__device__ __forceinline__ void serve_reduce_group(const double* __restrict__ partials, int64_t nt, int c0, int nacc,
                                                   double* tot) {
  __shared__ double wl[kServeReduceGroup][kThreads / 64];
  double sum[kServeReduceGroup];
#pragma unroll
  for (int k = 0; k < kServeReduceGroup; ++k) sum[k] = 0.0;
  for (int64_t i = threadIdx.x; i < nt; i += kThreads) {
    double v[kServeReduceGroup];
#pragma unroll
    for (int k = 0; k < kServeReduceGroup; ++k)
      v[k] = c0 + k < nacc ? ldg<true>(partials + (int64_t)(c0 + k) * nt + i, 0u) : 0.0;
#pragma unroll
    for (int k = 0; k < kServeReduceGroup; ++k) sum[k] += v[k];
  }
#pragma unroll
  for (int k = 0; k < kServeReduceGroup; ++k) sum[k] = wave_sum(sum[k]);
  if ((threadIdx.x & 63) == 0)
#pragma unroll
    for (int k = 0; k < kServeReduceGroup; ++k) wl[k][threadIdx.x >> 6] = sum[k];
  __syncthreads();
  if (threadIdx.x < kServeReduceGroup) {
    const int k = threadIdx.x;
    tot[k] = (wl[k][0] + wl[k][1]) + (wl[k][2] + wl[k][3]);
  }
  __syncthreads();
}

__device__ __forceinline__ void serve_work(ServeShared* hs, ServeCtl* ctl, ServeDesc* __restrict__ dd,
                                           ServeSlot* __restrict__ st, int policy) {
  __shared__ ServeDesc sd;          // the current item's request
  __shared__ RedBuf<kOuterCapTag> red;
  __shared__ int cmd, cslot, citem;
  __shared__ int last;
  __shared__ double red_totals[kServeReduceGroup];
  const unsigned rot = blockIdx.x & 63u;  // spreads the workers' first choice over the slots
  for (;;) {
    if (policy != kServeSpread) {
      // the first wave picks the claimable slot with the smallest key (lane s
      // reads slot s's open stamp, or its unclaimed items); thread 0 claims,
      // and on a refusal (the slot ran out of items meanwhile) the next
      // smallest is tried
      if (threadIdx.x < 64) {
        const unsigned lane = threadIdx.x;
        int ex = 0;
        unsigned long long m = 0ull;
        if (lane == 0) {  // the three control words in one round trip
          const unsigned long long stop = load_dev(&ctl->stop);
          const unsigned int quit = load_dev(&ctl->quit);
          const unsigned long long mask = load_dev(&ctl->mask);
          ex = stop || quit;
          if (!ex) m = mask;
        }
        ex = __shfl(ex, 0, 64);
        m = __shfl(m, 0, 64);
        int got = 0;
        if (lane == 0) cmd = ex ? kCmdExit : kCmdIdle;
        if (!ex && m != 0ull) {
          unsigned long long stamp = ~0ull;
          if ((m >> lane) & 1ull) {
            if (policy == kServeOldestFirst) {
              stamp = load_dev(&st[lane].stamp);
            } else {
              // unclaimed items of the request the claim word names (a
              // claim word of another request, or none left: last)
              const unsigned long long c = load_dev(&st[lane].claim), l = load_dev(&st[lane].lim);
              const unsigned next = (unsigned)(c & 0xffffffffull), n = (unsigned)(l & 0xffffffffull);
              stamp = ((c >> 32) == (l >> 32) && next < n) ? (unsigned long long)(n - next) : (1ull << 40);
            }
          }
          while (m != 0ull && !got) {
            unsigned long long key = ((m >> lane) & 1ull) ? ((stamp << 6) | lane) : ~0ull;
#pragma unroll
            for (int off = 32; off >= 1; off >>= 1) {
              const unsigned long long o = __shfl_xor(key, off, 64);
              key = o < key ? o : key;
            }
            const int s = (int)(key & 63ull);
            if (lane == 0 && serve_claim(ctl, st, s, &cslot, &citem)) {
              cmd = kCmdWork;
              got = 1;
            }
            got = __shfl(got, 0, 64);
            m &= ~(1ull << s);
          }
        }
        if (lane == 0) wait_mem();  // the descriptor is read after the claim
      }
    } else if (threadIdx.x == 0) {
      cmd = kCmdIdle;
      // the three control words in one round trip
      const unsigned long long stop = load_dev(&ctl->stop);
      const unsigned int quit = load_dev(&ctl->quit);
      unsigned long long m = load_dev(&ctl->mask);
      if (stop || quit) {
        cmd = kCmdExit;
      } else {
        m = rot ? (m >> rot) | (m << (64u - rot)) : m;
        while (m != 0ull && cmd == kCmdIdle) {
          const int s = (int)((__builtin_ctzll(m) + rot) & 63u);
          m &= m - 1ull;
          if (serve_claim(ctl, st, s, &cslot, &citem)) cmd = kCmdWork;
        }
      }
      wait_mem();  // the descriptor is read after the claim
    }
    __syncthreads();
    const int c = cmd;
    if (c == kCmdExit) {
      if (threadIdx.x == 0)
        __hip_atomic_fetch_sub(&ctl->live, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      return;
    }
    if (c == kCmdIdle) {
      __builtin_amdgcn_s_sleep(32);
      __syncthreads();
      continue;
    }
    const int s = cslot;
    // the request's descriptor into LDS
    copy_dev_to_lds((unsigned long long*)&sd, (const unsigned long long*)&dd[s],
                    (int)(sizeof(ServeDesc) / sizeof(unsigned long long)));
    __syncthreads();
    // claim citem covers the tiles chunk x citem .. (the request's last tile)
    const unsigned chunk = serve_chunk((unsigned)sd.items, gridDim.x - 1u);
    const int t0 = citem * (int)chunk;
    const int t1 = min(t0 + (int)chunk, sd.items);
    for (int tile = t0; tile < t1; ++tile) {
      if (sd.model == 1) {
        if (sd.grad) tile_nll<1, true, true>(sd.seg, sd.k.m1, tile, red);
        else tile_nll<1, false, true>(sd.seg, sd.k.m1, tile, red);
      } else if (sd.model == 2) {
        if (sd.grad) tile_nll<2, true, true>(sd.seg, sd.k.m2, tile, red);
        else tile_nll<2, false, true>(sd.seg, sd.k.m2, tile, red);
      } else if (sd.model == 3) {
        if (sd.grad) tile_angtime<true, true, kOuterCapTag>(sd.seg, sd.k.m3, &sd.k.m3.C[0][0], tile, red);
        else tile_angtime<false, true, kOuterCapTag>(sd.seg, sd.k.m3, &sd.k.m3.C[0][0], tile, red);
      } else {
        if (sd.grad) tile_angtime<true, true, kOuterCapTag, true>(sd.seg, sd.k.m3, &sd.k.m3.C[0][0], tile, red);
        else tile_angtime<false, true, kOuterCapTag, true>(sd.seg, sd.k.m3, &sd.k.m3.C[0][0], tile, red);
      }
    }
    // every lane's stores of this claim's tiles (their partials) complete
    // before the claim is counted as done
    wait_mem();
    __syncthreads();
    if (threadIdx.x == 0) {
      const unsigned int prev = __hip_atomic_fetch_add(&st[s].done, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      last = prev + 1 == serve_claims((unsigned)sd.items, gridDim.x - 1u) ? 1 : 0;
      wait_mem();  // the partials are read after the count
    }
    __syncthreads();
    if (last) {
      // every item of the request is complete: fixed-order reduction, eight
      // components at a time
      for (int c0 = 0; c0 < sd.nacc; c0 += kServeReduceGroup) {
        serve_reduce_group(sd.seg.partials, sd.seg.n_tiles, c0, sd.nacc, red_totals);
        if (threadIdx.x < kServeReduceGroup && c0 + (int)threadIdx.x < sd.nacc)
          store_sys(&hs->out[s][c0 + threadIdx.x], red_totals[threadIdx.x]);
        __syncthreads();
      }
      if (threadIdx.x == 0) {
        wait_mem();  // the results reach host memory before fin
        store_sys(&hs->fin[s], sd.seq);
      }
    }
    __syncthreads();
  }
}

// Workgroup 0 polls the host, the others evaluate; grid >= 2 workgroups.
// Held to 168 VGPRs (3 waves per SIMD): the one kernel carries every model's
// tile body, and at 128 it would spill ~50 registers.
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(3))) void k_serve(
    ServeShared* hs, ServeCtl* ctl, ServeDesc* __restrict__ dd, ServeSlot* __restrict__ st, int nslots,
    int idle_limit, int policy) {
  if (blockIdx.x == 0) serve_poll(hs, ctl, dd, st, nslots, idle_limit);
  else serve_work(hs, ctl, dd, st, policy);
}

}  // namespace ipx
