// Prefix sums and a stable radix sort, for the steps around the likelihood:
// the ordered compaction of accepted toy candidates (an exclusive scan of
// their flags) and the resolution-band ordering of a dataset's events (a
// stable sort of 64-bit keys carrying the event index).
//
// Scan: three launches.  Tiles of kScanTile items: each tile's total
// (k_scan_reduce), an exclusive scan of the tile totals in one workgroup
// (k_scan_sums), then each tile scanned with its offset (k_scan_apply).  Items
// are 32-bit counts whose total fits in an int.
//
// Sort: least-significant digit first, 8-bit digits, eight passes over the
// 64-bit keys, for one array or several at once (segments, each sorted on
// its own).  A pass counts the digits of each tile of kScanTile keys
// (k_radix_hist, digit-major counts per segment), scans the counts (the
// segment's base, the digit's base within it, then the tile's base within
// the digit), and moves every key and value to its place (k_radix_scatter).  Within a
// tile the keys go in index order: 16 rounds of 256 keys; in a round each
// wave finds the lanes that share a lane's digit (eight ballots) and the
// lane's rank among them, and the waves take their places in wave order.
// Every pass is therefore stable, and so is the sort.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ipx {

constexpr int kScanThreads = 256;
constexpr int kScanItems = 16;
constexpr int kScanTile = kScanThreads * kScanItems;

// Exclusive prefix of v over the workgroup in thread order; *total gets the
// workgroup's sum.  lds holds one int per wave.  Every thread must call it.
__device__ __forceinline__ int block_exclusive_scan(int v, int* lds, int* total) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  int x = v;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const int y = __shfl_up(x, off, 64);
    if (lane >= off) x += y;
  }
  if (lane == 63) lds[wave] = x;
  __syncthreads();
  int wbase = 0, tot = 0;
#pragma unroll
  for (int w = 0; w < kScanThreads / 64; ++w) {
    const int s = lds[w];
    if (w < wave) wbase += s;
    tot += s;
  }
  __syncthreads();
  *total = tot;
  return wbase + x - v;
}

__global__ __launch_bounds__(kScanThreads) void k_scan_reduce(const int* __restrict__ in, int n,
                                                              int* __restrict__ sums) {
  __shared__ int lds[kScanThreads / 64];
  const int64_t base = (int64_t)blockIdx.x * kScanTile;
  int s = 0;
#pragma unroll
  for (int i = 0; i < kScanItems; ++i) {
    const int64_t j = base + (int64_t)i * kScanThreads + threadIdx.x;
    if (j < n) s += in[j];
  }
  int tot;
  (void)block_exclusive_scan(s, lds, &tot);
  if (threadIdx.x == 0) sums[blockIdx.x] = tot;
}

// One workgroup: sums[0 .. nb) replaced by their exclusive prefix sums.
__global__ __launch_bounds__(kScanThreads) void k_scan_sums(int* __restrict__ sums, int nb) {
  __shared__ int lds[kScanThreads / 64];
  int carry = 0;
  for (int c0 = 0; c0 < nb; c0 += kScanThreads) {
    const int i = c0 + (int)threadIdx.x;
    const int v = i < nb ? sums[i] : 0;
    int tot;
    const int ex = block_exclusive_scan(v, lds, &tot);
    if (i < nb) sums[i] = carry + ex;
    carry += tot;
  }
}

// out[j] = offset of the tile + the exclusive prefix of in within the tile;
// thread t takes the tile's items 16t .. 16t + 15.  out may be in.
__global__ __launch_bounds__(kScanThreads) void k_scan_apply(const int* in, int* out, int n,
                                                             const int* __restrict__ sums) {
  __shared__ int lds[kScanThreads / 64];
  const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
  int v[kScanItems];
  int s = 0;
#pragma unroll
  for (int i = 0; i < kScanItems; ++i) {
    v[i] = base + i < n ? in[base + i] : 0;
    s += v[i];
  }
  int tot;
  int ex = block_exclusive_scan(s, lds, &tot) + sums[blockIdx.x];
#pragma unroll
  for (int i = 0; i < kScanItems; ++i) {
    if (base + i < n) out[base + i] = ex;
    ex += v[i];
  }
}

// Ints of temporary storage scan_exclusive needs for n items.
inline size_t scan_temp_ints(int64_t n) { return (size_t)((n + kScanTile - 1) / kScanTile) + 1; }

// out[j] = in[0] + ... + in[j - 1] for j < n (n >= 0); tmp holds
// scan_temp_ints(n) ints.  Stream-ordered, no synchronisation.
inline hipError_t scan_exclusive(const int* in, int* out, int64_t n, int* tmp, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const unsigned nb = (unsigned)((n + kScanTile - 1) / kScanTile);
  hipLaunchKernelGGL(k_scan_reduce, dim3(nb), dim3(kScanThreads), 0, s, in, (int)n, tmp);
  hipLaunchKernelGGL(k_scan_sums, dim3(1), dim3(kScanThreads), 0, s, tmp, (int)nb);
  hipLaunchKernelGGL(k_scan_apply, dim3(nb), dim3(kScanThreads), 0, s, in, out, (int)n, (const int*)tmp);
  return hipGetLastError();
}

// A tile of the sort: up to kScanTile consecutive keys [start, start +
// count) of one segment; its count of digit d goes to hist[hidx + d hstride].
// Segments (several arrays sorted at once, each on its own) are laid out
// end to end, each with its own digit-major block of counts, hidx = the
// segment's block + the tile's index within the segment, hstride = the
// segment's tile count; the scan of all counts then gives every key its
// place in the concatenation (the segment's start + its place within it).
struct RadixTile {
  int64_t start;
  int count;
  int seg;
  int hidx;
  int hstride;
};

__global__ __launch_bounds__(kScanThreads) void k_radix_hist(const unsigned long long* __restrict__ keys,
                                                             const RadixTile* __restrict__ tiles, int shift,
                                                             int* __restrict__ hist) {
  __shared__ int cnt[256];
  const RadixTile tl = tiles[blockIdx.x];
  cnt[threadIdx.x] = 0;
  __syncthreads();
#pragma unroll 4
  for (int r = 0; r < kScanItems; ++r) {
    const int i = r * kScanThreads + (int)threadIdx.x;
    if (i < tl.count) atomicAdd(&cnt[(int)((keys[tl.start + i] >> shift) & 255ull)], 1);
  }
  __syncthreads();
  hist[(size_t)tl.hidx + (size_t)threadIdx.x * tl.hstride] = cnt[threadIdx.x];
}

// Moves the tile's keys and values to offs[hidx + d hstride] + their rank
// among the tile's keys of digit d (in index order).
__global__ __launch_bounds__(kScanThreads) void k_radix_scatter(const unsigned long long* __restrict__ kin,
                                                                const int* __restrict__ vin,
                                                                unsigned long long* __restrict__ kout,
                                                                int* __restrict__ vout, int64_t total,
                                                                const RadixTile* __restrict__ tiles, int shift,
                                                                const int* __restrict__ offs) {
  __shared__ int base[256];
  __shared__ int wcnt[kScanThreads / 64][256];
  const RadixTile tl = tiles[blockIdx.x];
  const int t = (int)threadIdx.x, lane = t & 63, wave = t >> 6;
  base[t] = offs[(size_t)tl.hidx + (size_t)t * tl.hstride];
#pragma unroll
  for (int w = 0; w < kScanThreads / 64; ++w) wcnt[w][t] = 0;
  __syncthreads();
  const unsigned long long below = (1ull << lane) - 1ull;
  for (int r = 0; r < kScanItems; ++r) {
    const int i = r * kScanThreads + t;
    const bool valid = i < tl.count;
    const unsigned long long key = valid ? kin[tl.start + i] : 0ull;
    const int val = valid ? vin[tl.start + i] : 0;
    const int d = (int)((key >> shift) & 255ull);
    unsigned long long peers = __ballot(valid);
#pragma unroll
    for (int b = 0; b < 8; ++b) {
      const int bit = (d >> b) & 1;
      const unsigned long long m = __ballot(bit);
      peers &= bit ? m : ~m;
    }
    const int rank = __popcll(peers & below);
    if (valid && rank == 0) wcnt[wave][d] = __popcll(peers);
    __syncthreads();
    {  // digit t: the waves' bases in wave order
      int p = base[t];
#pragma unroll
      for (int w = 0; w < kScanThreads / 64; ++w) {
        const int c = wcnt[w][t];
        wcnt[w][t] = p;
        p += c;
      }
      base[t] = p;
    }
    __syncthreads();
    const int64_t pos = (int64_t)wcnt[wave][d] + rank;
    if (valid && pos >= 0 && pos < total) {   // (always, with correct offsets)
      kout[pos] = key;
      vout[pos] = val;
    }
    __syncthreads();
#pragma unroll
    for (int w = 0; w < kScanThreads / 64; ++w) wcnt[w][t] = 0;
    __syncthreads();
  }
}

// Stable sort of (keys[i], vals[i]) within every segment of the tile table
// (ntiles tiles, nhist digit counts in all), by key; keys_tmp / vals_tmp are
// ping-pong buffers of total entries, tmp holds nhist + scan_temp_ints(nhist)
// ints.  The result is in keys / vals (eight passes).  Stream-ordered.
inline hipError_t radix_sort_pairs(unsigned long long* keys, int* vals, unsigned long long* keys_tmp, int* vals_tmp,
                                   int64_t total, const RadixTile* tiles, int ntiles, int64_t nhist, int* tmp,
                                   hipStream_t s) {
  if (total <= 1 || ntiles <= 0) return hipSuccess;
  int* hist = tmp;
  int* stmp = tmp + nhist;
  unsigned long long *ka = keys, *kb = keys_tmp;
  int *va = vals, *vb = vals_tmp;
  for (int pass = 0; pass < 8; ++pass) {
    const int shift = 8 * pass;
    hipLaunchKernelGGL(k_radix_hist, dim3(ntiles), dim3(kScanThreads), 0, s, (const unsigned long long*)ka, tiles,
                       shift, hist);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) e = scan_exclusive(hist, hist, nhist, stmp, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_radix_scatter, dim3(ntiles), dim3(kScanThreads), 0, s, (const unsigned long long*)ka,
                       (const int*)va, kb, vb, total, tiles, shift, (const int*)hist);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    unsigned long long* kt = ka;
    ka = kb;
    kb = kt;
    int* vt = va;
    va = vb;
    vb = vt;
  }
  return hipSuccess;
}

}  // namespace ipx
