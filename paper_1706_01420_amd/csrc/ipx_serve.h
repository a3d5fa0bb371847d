// Served likelihood: a persistent kernel that takes NLL / gradient requests
// from a host-visible mailbox while it runs (continuous batching: requests
// that arrive while others are being evaluated join the same launch).
//
// Protocol (S slots):
//   host   writes the request descriptor desc[s] into fine-grained host memory,
//          then mail[s] = seq (release) and bumps gen.
//   device one workgroup "opens" the request (CAS on open[s]): it copies
//          desc[s] into device memory with vector loads, clears the slot's
//          completion counters and publishes claim[s] = seq << 32 (release).
//          Workgroups claim items with atomicAdd on claim[s]; the high word
//          tells which request the item belongs to, so a late claim on a
//          finished request is recognised and ignored.
//          Items: the request's canonical tiles (A), then for the angular
//          gradient its coefficient-adjoint tiles (B, which start once all A
//          tiles are done).  The workgroup that completes the last item sums
//          every component's tile partials in index order (the same order as
//          the other entry points) and writes out[s], then fin[s] = seq
//          (system-scope release).
//   exit   every workgroup leaves after `idle_limit` consecutive empty scans or
//          when the host sets stop; waits for phase A are capped by
//          `spin_limit` (a request that hits it is finished with status 1).
//
// All waits are bounded, so the grid always drains.  No workgroup waits on
// work that has not been claimed by a running workgroup.
#pragma once

#include "ipx_batch.h"

namespace ipx {

constexpr int kServeMaxSlots = 64;

struct ServeDesc {
  int model;
  int grad;
  int nA, nB;        // items: per-event tiles, coefficient-adjoint tiles
  int nacc, split;   // reduced components; components >= split use the outer tiles
  int pad[2];
  SegInfo seg;       // columns of the dataset + this request's scratch
  union {
    MassConst m1;
    MassTimeConst m2;
    AngTimeConst m3;
  } k;
};

struct ServeSlot {                 // device memory, touched by the GPU only
  unsigned long long claim;        // (seq << 32) | next item
  unsigned long long open;         // seq opened by the device
  unsigned int doneA;              // completed A items
  unsigned int done;               // completed items
  unsigned long long pad;
};

struct ServeCtl {                  // device memory: mirror of the host's gen / stop
  unsigned long long gen;
  unsigned long long stop;
};

constexpr int kServePollers = 4;   // workgroups that read the host's gen / stop

struct ServeShared {               // fine-grained host memory
  unsigned long long gen;          // bumped by the host after each publication
  unsigned long long stop;
  unsigned long long mail[kServeMaxSlots];
  unsigned long long fin[kServeMaxSlots];
  int status[kServeMaxSlots];
  double out[kServeMaxSlots][kAccMax];
  ServeDesc desc[kServeMaxSlots];
};

__device__ __forceinline__ unsigned long long load_sys(const unsigned long long* p) {
  return __hip_atomic_load(p, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_SYSTEM);
}
__device__ __forceinline__ void store_sys(unsigned long long* p, unsigned long long v) {
  __hip_atomic_store(p, v, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
}
__device__ __forceinline__ unsigned long long load_dev(const unsigned long long* p) {
  return __hip_atomic_load(p, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ unsigned int load_dev32(const unsigned int* p) {
  return __hip_atomic_load(p, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
}

// Copy n 8-byte words with the workgroup's lanes (vector loads and stores).
__device__ __forceinline__ void wg_copy(unsigned long long* __restrict__ dst, const unsigned long long* src, int n) {
  for (int i = threadIdx.x; i < n; i += kThreads) dst[i] = __hip_atomic_load(src + i, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
}

enum : int { kCmdIdle = 0, kCmdOpen = 1, kCmdWork = 2, kCmdExit = 3 };

__global__ __launch_bounds__(kThreads) void k_serve(ServeShared* hs, ServeCtl* __restrict__ ctl,
                                                    ServeDesc* __restrict__ dd, ServeSlot* __restrict__ st,
                                                    int nslots, int idle_limit, int spin_limit) {
  __shared__ ServeDesc sd;          // the current item's request
  __shared__ int cmd, cslot, citem;
  __shared__ unsigned long long cseq;
  __shared__ int last;
  int idle = 0;
  unsigned long long seen_gen = 0;  // host publications already scanned (thread 0)
  for (;;) {
    if (threadIdx.x == 0) {
      cmd = kCmdIdle;
      if (blockIdx.x < kServePollers) {
        // a few workgroups mirror the host's counters into device memory
        atomicMax(&ctl->gen, load_sys(&hs->gen));
        if (load_sys(&hs->stop)) atomicMax(&ctl->stop, 1ull);
      }
      const unsigned long long gen = load_dev(&ctl->gen);
      const bool rescan = gen != seen_gen;
      if (load_dev(&ctl->stop)) {
        cmd = kCmdExit;
      } else {
        bool scanned_all = true;
        for (int i = 0; i < nslots && cmd == kCmdIdle; ++i) {
          const int s = (int)((blockIdx.x + (unsigned)i) % (unsigned)nslots);
          const unsigned long long opened = load_dev(&st[s].open);
          if (rescan) {
            const unsigned long long seq = load_sys(&hs->mail[s]);
            if (seq > opened) {
              if (atomicCAS(&st[s].open, opened, seq) == opened) {
                cmd = kCmdOpen;
                cslot = s;
                cseq = seq;
                scanned_all = i == nslots - 1;
              }
              continue;
            }
          }
          if (opened == 0) continue;
          // claimable?  (the claim word carries the sequence number it counts for)
          const unsigned long long c = load_dev(&st[s].claim);
          const unsigned long long seq = c >> 32;
          if (seq != opened) continue;
          const int total = __hip_atomic_load(&dd[s].nA, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) +
                            __hip_atomic_load(&dd[s].nB, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          if ((int)(c & 0xffffffffull) >= total) continue;
          const unsigned long long old = atomicAdd(&st[s].claim, 1ull);
          if ((old >> 32) == seq && (int)(old & 0xffffffffull) < total) {
            cmd = kCmdWork;
            cslot = s;
            cseq = seq;
            citem = (int)(old & 0xffffffffull);
            scanned_all = false;
          }
        }
        if (rescan && scanned_all && cmd != kCmdOpen) seen_gen = gen;
      }
    }
    __syncthreads();
    const int c = cmd;
    if (c == kCmdExit) return;
    if (c == kCmdIdle) {
      if (++idle > idle_limit) return;
      __builtin_amdgcn_s_sleep(32);
      __syncthreads();
      continue;
    }
    idle = 0;
    const int s = cslot;
    const unsigned long long seq = cseq;
    if (c == kCmdOpen) {
      // device copy of the descriptor, counters cleared, then claims open
      wg_copy((unsigned long long*)&dd[s], (const unsigned long long*)&hs->desc[s],
              (int)(sizeof(ServeDesc) / sizeof(unsigned long long)));
      __threadfence();
      __syncthreads();
      if (threadIdx.x == 0) {
        __hip_atomic_store(&st[s].doneA, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_store(&st[s].done, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __threadfence();
        atomicExch(&st[s].claim, seq << 32);
      }
      __syncthreads();
      continue;
    }
    // work item: the request's descriptor into LDS (vector loads)
    __threadfence();
    wg_copy((unsigned long long*)&sd, (const unsigned long long*)&dd[s],
            (int)(sizeof(ServeDesc) / sizeof(unsigned long long)));
    __syncthreads();
    const int item = citem;
    const bool isA = item < sd.nA;
    bool ok = true;
    if (isA) {
      if (sd.model == 1) {
        if (sd.grad) tile_nll<1, true>(sd.seg, sd.k.m1, item);
        else tile_nll<1, false>(sd.seg, sd.k.m1, item);
      } else if (sd.model == 2) {
        if (sd.grad) tile_nll<2, true>(sd.seg, sd.k.m2, item);
        else tile_nll<2, false>(sd.seg, sd.k.m2, item);
      } else {
        if (sd.grad) tile_angtime<true>(sd.seg, sd.k.m3, &sd.k.m3.C[0][0], item);
        else tile_angtime<false>(sd.seg, sd.k.m3, &sd.k.m3.C[0][0], item);
      }
    } else {
      // phase B needs every A tile (their per-event factors); all A items were
      // claimed before any B item, so they are held by running workgroups
      if (threadIdx.x == 0) {
        int spins = 0;
        while (load_dev32(&st[s].doneA) < (unsigned)sd.nA && spins < spin_limit) {
          __builtin_amdgcn_s_sleep(2);
          ++spins;
        }
        last = spins < spin_limit ? 1 : 0;
      }
      __syncthreads();
      ok = last != 0;
      __threadfence();
      if (ok) tile_angtime_outer(sd.seg, item - sd.nA);
    }
    // every lane's stores of this item (tile partials, per-event factors) must
    // be visible device-wide before the item is counted as done
    __threadfence();
    __syncthreads();
    if (threadIdx.x == 0) {
      if (!ok) hs->status[s] = 1;
      __threadfence();
      if (isA) atomicAdd(&st[s].doneA, 1u);
      const unsigned int prev = atomicAdd(&st[s].done, 1u);
      last = prev + 1 == (unsigned)(sd.nA + sd.nB) ? 1 : 0;
    }
    __syncthreads();
    if (last) {
      // every item of the request is complete: fixed-order reduction
      __threadfence();
      for (int comp = 0; comp < sd.nacc; ++comp) {
        const int64_t nt = comp < sd.split ? sd.seg.n_tiles : sd.seg.n_tiles_outer;
        const double total = reduce_component(sd.seg.partials + (int64_t)comp * sd.seg.n_tiles, nt);
        if (threadIdx.x == 0) hs->out[s][comp] = total;
        __syncthreads();
      }
      if (threadIdx.x == 0) {
        __threadfence_system();
        store_sys(&hs->fin[s], seq);
      }
    }
    __syncthreads();
  }
}

}  // namespace ipx
