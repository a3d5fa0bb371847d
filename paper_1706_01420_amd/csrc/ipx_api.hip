// libipx: C ABI (include/ipx.h) over the gfx950 likelihood kernels.
//
// A call of nll_eval / nll_grad:
//   1. validates theta and hoists every parameter-dependent constant on the
//      host (normalisations, decay constants, the 10 x 4 coefficient table);
//      the constants travel as kernel arguments, so the kernel reads them from
//      scalar registers;
//   2. launches the per-event tile kernel (events -> one partial per tile);
//   3. launches the tile reduction (partials -> one double per component);
//   4. copies the (1 + K) sums to pinned host memory and synchronises;
//   5. for the gradient, applies the Jacobian of step 1 on the host.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <limits>
#include <string>
#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <mutex>
#include <thread>
#include <vector>

#include "../../include/ipx.h"
#include "ipx_hoist.h"
#include "ipx_kernels.h"
#include "ipx_toys.h"
#include "ipx_batch.h"
#include "ipx_serve.h"
#include "ipx_binned.h"
#include "ipx_scan.h"
#include "ipx_ipatia.h"

using namespace ipx;

// ---------------------------------------------------------------------------
// Errors
// ---------------------------------------------------------------------------
static thread_local std::string g_last_error;

static ipx_status fail(ipx_status s, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
static ipx_status fail(ipx_status s, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return s;
}

#define HIP_TRY(expr)                                                                    \
  do {                                                                                   \
    hipError_t e_ = (expr);                                                              \
    if (e_ != hipSuccess)                                                                \
      return fail(IPX_EDEVICE, "%s failed: %s", #expr, hipGetErrorString(e_));           \
  } while (0)

// ---------------------------------------------------------------------------
// Handles
// ---------------------------------------------------------------------------
struct ipx_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  int n_cu = 0;
  bool timing = false;
  hipEvent_t ev_pool[2][64];
  int ev_used = 0;
  double timing_ms = 0.0;
  int64_t timing_launches = 0;
  std::mutex ws_mu;                // guards the smearing workspace
  double* smear_ws = nullptr;      // kernel table and chunk partials of ipx_smear (grows, kept)
  size_t smear_ws_doubles = 0;
};

struct ipx_dataset {
  int model = 0;
  int64_t n = 0;
  int64_t n_pad = 0;
  int ncols = 0;
  double* base = nullptr;          // owned column storage (nullptr when borrowed)
  const double* cols[7] = {};
  const double* w = nullptr;
  int64_t n_tiles = 0;
  bool sorted = false;             // events stored in resolution-band order
  double* partials = nullptr;      // n_tiles x kAccMax
  double* out_dev = nullptr;       // kAccMax
  double* out_host = nullptr;      // kAccMax, pinned
  size_t bytes = 0;
  struct ipx_plan* self = nullptr; // one-dataset plan used by nll_eval / nll_grad
  int plan_refs = 0;               // user plans that reference this dataset
  AngSettings ang = ang_settings_default();  // angular models: efficiency weights, C_SP
  double* aux = nullptr;           // Ipatia model: constants, grid partials, 1/N_I, tile partials, total
};

static const int kNParams[6] = {-1, 4, 7, 12, 12, 11};
static const int kNCols[6] = {-1, 1, 3, 6, 7, 1};
static bool angular_model(int model) { return model == 3 || model == 4; }
static bool time_model(int model) { return model >= 2 && model <= 4; }
constexpr int kModelIpatia = 5;

// ---------------------------------------------------------------------------
// Event-store ordering for the models with a decay time: by the band of
// t / sigma_t (width 1/2, the last band open above t / sigma_t = 10), then by
// decreasing sigma_t within a band.  The resolution correction at t and the
// depth of its continued fraction depend on t / sigma_t; those at the range
// ends and the normalisation on sigma_t alone; so the waves of this order need
// the same corrections at about the same depth.  Tiles run in storage order:
// the low bands (correction at t) and the wide resolutions (deep corrections
// at the range ends) come first and the cheapest tiles last, which keeps the
// tail of a launch short.  The NLL is a sum over events: the order only
// changes the rounding of the sum.
// ---------------------------------------------------------------------------
constexpr int kBands = 21;   // bands 0 .. 20 of 2 t / sigma_t (5 bits)

// key = band << 58 | (2^63 - 1 - bits of sigma_t) >> 6; sigma_t > 0, so its
// bit pattern orders as its value (decreasing here)
__device__ __forceinline__ unsigned long long band_key(double t, double sig) {
  const double r = 2.0 * t / sig;
  const double b = r > 0.0 ? fmin(floor(r), (double)kBands - 1.0) : 0.0;  // NaN -> 0
  return ((unsigned long long)b << 58) | ((0x7fffffffffffffffull - (unsigned long long)__double_as_longlong(sig)) >> 6);
}

// One dataset of a joint ordering: its ordering columns and every column to
// permute (the observables, then the weights), its first key in the
// concatenation of all keys.
struct SortSeg {
  const double* t;
  const double* sig;
  double* cols[8];
  int ncols;
  int64_t off;
};

__global__ __launch_bounds__(kScanThreads) void k_seg_keys(const RadixTile* __restrict__ tiles,
                                                           const SortSeg* __restrict__ segs,
                                                           unsigned long long* __restrict__ keys, int* __restrict__ vals) {
  const RadixTile tl = tiles[blockIdx.x];
  const SortSeg& sg = segs[tl.seg];
  for (int i = (int)threadIdx.x; i < tl.count; i += kScanThreads) {
    const int64_t g = tl.start + i;
    const int64_t k = g - sg.off;
    keys[g] = band_key(sg.t[k], sg.sig[k]);
    vals[g] = (int)k;
  }
}

// tmp[g] = column c of the key's dataset at the sorted index vals[g].
__global__ __launch_bounds__(kScanThreads) void k_seg_gather(const RadixTile* __restrict__ tiles,
                                                             const SortSeg* __restrict__ segs,
                                                             const int* __restrict__ vals, int c,
                                                             double* __restrict__ tmp) {
  const RadixTile tl = tiles[blockIdx.x];
  const SortSeg& sg = segs[tl.seg];
  if (c >= sg.ncols) return;
  const double* __restrict__ src = sg.cols[c];
  for (int i = (int)threadIdx.x; i < tl.count; i += kScanThreads) tmp[tl.start + i] = src[vals[tl.start + i]];
}

__global__ __launch_bounds__(kScanThreads) void k_seg_put(const RadixTile* __restrict__ tiles,
                                                          const SortSeg* __restrict__ segs, int c,
                                                          const double* __restrict__ tmp) {
  const RadixTile tl = tiles[blockIdx.x];
  const SortSeg& sg = segs[tl.seg];
  if (c >= sg.ncols) return;
  double* __restrict__ dst = sg.cols[c];
  for (int i = (int)threadIdx.x; i < tl.count; i += kScanThreads) dst[tl.start + i - sg.off] = tmp[tl.start + i];
}

// Puts the events of every dataset of ds (models with a decay time) in
// resolution-band order, all datasets in one set of launches.
static ipx_status sort_events(ipx_dataset* const* ds, int nds, hipStream_t s) {
  std::vector<SortSeg> segs;
  std::vector<RadixTile> tiles;
  int64_t total = 0, nhist = 0;
  int maxcols = 0;
  for (int j = 0; j < nds; ++j) {
    ipx_dataset* d = ds[j];
    if (!d || d->n < 2) continue;
    const int tcol = d->model == 2 ? 1 : 3;
    const int scol = d->model == 2 ? 2 : 4;
    SortSeg sg{};
    sg.t = d->cols[tcol];
    sg.sig = d->cols[scol];
    sg.ncols = d->ncols + (d->w ? 1 : 0);
    for (int c = 0; c < sg.ncols; ++c) sg.cols[c] = const_cast<double*>(c < d->ncols ? d->cols[c] : d->w);
    sg.off = total;
    maxcols = std::max(maxcols, sg.ncols);
    const int nt = (int)((d->n + kScanTile - 1) / kScanTile);
    for (int lt = 0; lt < nt; ++lt)
      tiles.push_back(RadixTile{total + (int64_t)lt * kScanTile,
                                (int)std::min<int64_t>(kScanTile, d->n - (int64_t)lt * kScanTile), (int)segs.size(),
                                (int)(nhist + lt), nt});
    nhist += 256 * (int64_t)nt;
    total += d->n;
    segs.push_back(sg);
  }
  if (segs.empty()) return IPX_OK;
  if (nhist + (int64_t)scan_temp_ints(nhist) > 0x7fffffff)
    return fail(IPX_EINVAL, "ordering the events: too many tiles (%lld)", (long long)tiles.size());
  unsigned long long* keys = nullptr;
  unsigned long long* keys_tmp = nullptr;
  double* tmp = nullptr;
  int* perm = nullptr;
  int* perm_tmp = nullptr;
  int* scratch = nullptr;
  RadixTile* d_tiles = nullptr;
  SortSeg* d_segs = nullptr;
  hipError_t e = hipMalloc(&keys, (size_t)total * sizeof(unsigned long long));
  if (e == hipSuccess) e = hipMalloc(&keys_tmp, (size_t)total * sizeof(unsigned long long));
  if (e == hipSuccess) e = hipMalloc(&tmp, (size_t)total * sizeof(double));
  if (e == hipSuccess) e = hipMalloc(&perm, (size_t)total * sizeof(int));
  if (e == hipSuccess) e = hipMalloc(&perm_tmp, (size_t)total * sizeof(int));
  if (e == hipSuccess) e = hipMalloc(&scratch, ((size_t)nhist + scan_temp_ints(nhist)) * sizeof(int));
  if (e == hipSuccess) e = hipMalloc(&d_tiles, tiles.size() * sizeof(RadixTile));
  if (e == hipSuccess) e = hipMalloc(&d_segs, segs.size() * sizeof(SortSeg));
  if (e == hipSuccess) e = hipMemcpyAsync(d_tiles, tiles.data(), tiles.size() * sizeof(RadixTile), hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipMemcpyAsync(d_segs, segs.data(), segs.size() * sizeof(SortSeg), hipMemcpyHostToDevice, s);
  const unsigned nt = (unsigned)tiles.size();
  if (e == hipSuccess) {
    hipLaunchKernelGGL(k_seg_keys, dim3(nt), dim3(kScanThreads), 0, s, (const RadixTile*)d_tiles,
                       (const SortSeg*)d_segs, keys, perm);
    e = hipGetLastError();
  }
  if (e == hipSuccess)
    e = radix_sort_pairs(keys, perm, keys_tmp, perm_tmp, total, d_tiles, (int)nt, nhist, scratch, s);
  for (int c = 0; c < maxcols && e == hipSuccess; ++c) {
    hipLaunchKernelGGL(k_seg_gather, dim3(nt), dim3(kScanThreads), 0, s, (const RadixTile*)d_tiles,
                       (const SortSeg*)d_segs, (const int*)perm, c, tmp);
    hipLaunchKernelGGL(k_seg_put, dim3(nt), dim3(kScanThreads), 0, s, (const RadixTile*)d_tiles,
                       (const SortSeg*)d_segs, c, (const double*)tmp);
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  (void)hipFree(keys);
  (void)hipFree(keys_tmp);
  (void)hipFree(tmp);
  (void)hipFree(perm);
  (void)hipFree(perm_tmp);
  (void)hipFree(scratch);
  (void)hipFree(d_tiles);
  (void)hipFree(d_segs);
  if (e != hipSuccess) return fail(IPX_EDEVICE, "ordering the events failed: %s", hipGetErrorString(e));
  for (int j = 0; j < nds; ++j)
    if (ds[j] && ds[j]->n >= 2) ds[j]->sorted = true;
  return IPX_OK;
}

extern "C" {

const char* ipx_last_error(void) { return g_last_error.c_str(); }

static ipx_status noalloc_setup(int device);

int ipx_model_nparams(int model) { return (model >= 1 && model <= 5) ? kNParams[model] : -1; }
int ipx_model_ncols(int model) { return (model >= 1 && model <= 5) ? kNCols[model] : -1; }

ipx_status ipx_create(int device, ipx_ctx** out) {
  if (!out) return fail(IPX_EINVAL, "ipx_create: out is NULL");
  *out = nullptr;
  int count = 0;
  HIP_TRY(hipGetDeviceCount(&count));
  if (device < 0 || device >= count) return fail(IPX_EINVAL, "ipx_create: device %d of %d", device, count);
  HIP_TRY(hipSetDevice(device));
  {
    // the allocation-free entry point's scratch address on this device
    ipx_status st = noalloc_setup(device);
    if (st != IPX_OK) return st;
  }
  ipx_ctx* c = new (std::nothrow) ipx_ctx();
  if (!c) return fail(IPX_ENOMEM, "ipx_create: host allocation failed");
  c->device = device;
  hipError_t e = hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking);
  if (e != hipSuccess) {
    delete c;
    return fail(IPX_EDEVICE, "hipStreamCreate: %s", hipGetErrorString(e));
  }
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, device) == hipSuccess) c->n_cu = prop.multiProcessorCount;
  for (int i = 0; i < 64; ++i) {
    if (hipEventCreate(&c->ev_pool[0][i]) != hipSuccess || hipEventCreate(&c->ev_pool[1][i]) != hipSuccess) {
      (void)hipStreamDestroy(c->stream);
      delete c;
      return fail(IPX_EDEVICE, "hipEventCreate failed");
    }
  }
  *out = c;
  return IPX_OK;
}

void ipx_destroy(ipx_ctx* c) {
  if (!c) return;
  (void)hipSetDevice(c->device);
  (void)hipStreamSynchronize(c->stream);
  for (int i = 0; i < 64; ++i) {
    (void)hipEventDestroy(c->ev_pool[0][i]);
    (void)hipEventDestroy(c->ev_pool[1][i]);
  }
  (void)hipStreamDestroy(c->stream);
  if (c->smear_ws) (void)hipFree(c->smear_ws);
  delete c;
}

static void free_plan(struct ipx_plan* p);
static void free_dataset(ipx_dataset* d) {
  if (d->self) free_plan(d->self);
  if (d->base) (void)hipFree(d->base);
  if (d->partials) (void)hipFree(d->partials);
  if (d->out_dev) (void)hipFree(d->out_dev);
  if (d->out_host) (void)hipHostFree(d->out_host);
  if (d->aux) (void)hipFree(d->aux);
  delete d;
}

ipx_status ipx_dataset_create(ipx_ctx* ctx, int model, int64_t n, const double* const* cols, int ncols,
                              const double* w, unsigned flags, ipx_dataset** out) {
  if (!ctx || !out) return fail(IPX_EINVAL, "ipx_dataset_create: NULL ctx/out");
  *out = nullptr;
  if (model < 1 || model > 5) return fail(IPX_EINVAL, "ipx_dataset_create: unknown model %d", model);
  if (ncols != kNCols[model])
    return fail(IPX_EINVAL, "ipx_dataset_create: model %d takes %d columns, got %d", model, kNCols[model], ncols);
  if (n < 0) return fail(IPX_EINVAL, "ipx_dataset_create: negative size");
  if (n > 0 && !cols) return fail(IPX_EINVAL, "ipx_dataset_create: NULL cols");
  for (int c = 0; c < ncols && n > 0; ++c)
    if (!cols[c]) return fail(IPX_EINVAL, "ipx_dataset_create: column %d is NULL", c);
  const unsigned kind = flags & 3u;
  if (kind > IPX_BORROW_DEVICE || (flags & ~(3u | IPX_KEEP_ORDER)) != 0)
    return fail(IPX_EINVAL, "ipx_dataset_create: bad flags %u", flags);
  HIP_TRY(hipSetDevice(ctx->device));
  ipx_dataset* d = new (std::nothrow) ipx_dataset();
  if (!d) return fail(IPX_ENOMEM, "ipx_dataset_create: host allocation failed");
  d->model = model;
  d->n = n;
  d->ncols = ncols;
  d->n_pad = (n + 31) / 32 * 32;  // 256-byte aligned columns
  d->n_tiles = (n + kTile - 1) / kTile;
  const int64_t tiles_alloc = d->n_tiles > 0 ? d->n_tiles : 1;
  hipError_t e = hipSuccess;
  if (kind == IPX_BORROW_DEVICE) {
    for (int c = 0; c < ncols; ++c) d->cols[c] = cols ? cols[c] : nullptr;
    d->w = w;
  } else {
    const int nstore = ncols + (w ? 1 : 0);
    const size_t bytes = (size_t)nstore * (size_t)(d->n_pad > 0 ? d->n_pad : 32) * sizeof(double);
    e = hipMalloc(&d->base, bytes);
    if (e != hipSuccess) {
      free_dataset(d);
      return fail(IPX_ENOMEM, "ipx_dataset_create: hipMalloc(%zu) failed: %s", bytes, hipGetErrorString(e));
    }
    d->bytes += bytes;
    const hipMemcpyKind ckind = kind == IPX_COPY_HOST ? hipMemcpyHostToDevice : hipMemcpyDeviceToDevice;
    for (int c = 0; c < nstore; ++c) {
      double* dst = d->base + (size_t)c * d->n_pad;
      const double* src = c < ncols ? cols[c] : w;
      if (n > 0) e = hipMemcpyAsync(dst, src, (size_t)n * sizeof(double), ckind, ctx->stream);
      if (e != hipSuccess) break;
      if (c < ncols) d->cols[c] = dst; else d->w = dst;
    }
    if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
    if (e != hipSuccess) {
      free_dataset(d);
      return fail(IPX_EDEVICE, "ipx_dataset_create: copy failed: %s", hipGetErrorString(e));
    }
    if (time_model(model) && !(flags & IPX_KEEP_ORDER) && n >= 2 && n <= 0x7fffffff) {
      ipx_status st = sort_events(&d, 1, ctx->stream);
      if (st != IPX_OK) {
        free_dataset(d);
        return st;
      }
    }
  }
  const size_t pbytes = (size_t)tiles_alloc * kAccMax * sizeof(double);
  if ((e = hipMalloc(&d->partials, pbytes)) != hipSuccess || (e = hipMalloc(&d->out_dev, kAccMax * sizeof(double))) != hipSuccess ||
      (e = hipHostMalloc(&d->out_host, kAccMax * sizeof(double), hipHostMallocDefault)) != hipSuccess) {
    free_dataset(d);
    return fail(IPX_ENOMEM, "ipx_dataset_create: scratch allocation failed: %s", hipGetErrorString(e));
  }
  d->bytes += pbytes + kAccMax * sizeof(double);
  *out = d;
  return IPX_OK;
}

ipx_status ipx_dataset_destroy(ipx_ctx* ctx, ipx_dataset* d) {
  if (!ctx || !d) return fail(IPX_EINVAL, "ipx_dataset_destroy: NULL argument");
  if (d->plan_refs > 0)
    return fail(IPX_EBUSY, "ipx_dataset_destroy: dataset is used by %d plan(s); destroy them first", d->plan_refs);
  HIP_TRY(hipSetDevice(ctx->device));
  HIP_TRY(hipStreamSynchronize(ctx->stream));
  free_dataset(d);
  return IPX_OK;
}

size_t ipx_dataset_bytes(const ipx_dataset* d) { return d ? d->bytes : 0; }
int64_t ipx_dataset_size(const ipx_dataset* d) { return d ? d->n : -1; }
int ipx_dataset_model(const ipx_dataset* d) { return d ? d->model : -1; }

ipx_status ipx_dataset_set_angular(ipx_ctx* ctx, ipx_dataset* d, const double* xi, double c_sp) {
  if (!ctx || !d) return fail(IPX_EINVAL, "ipx_dataset_set_angular: NULL argument");
  if (!angular_model(d->model))
    return fail(IPX_EINVAL, "ipx_dataset_set_angular: model %d has no angular constants", d->model);
  AngSettings a = ang_settings_default();
  if (xi)
    for (int k = 0; k < 10; ++k) a.xi[k] = xi[k];
  a.c_sp = c_sp;
  for (int k = 0; k < 10; ++k)
    if (!std::isfinite(a.xi[k])) return fail(IPX_EINVAL, "ipx_dataset_set_angular: xi[%d] is not finite", k);
  if (!std::isfinite(c_sp)) return fail(IPX_EINVAL, "ipx_dataset_set_angular: c_sp is not finite");
  d->ang = a;
  return IPX_OK;
}

ipx_status ipx_dataset_column(const ipx_dataset* d, int col, const double** p) {
  if (!d || !p) return fail(IPX_EINVAL, "ipx_dataset_column: NULL argument");
  if (col < 0 || col > d->ncols) return fail(IPX_EINVAL, "ipx_dataset_column: column %d out of range", col);
  *p = col < d->ncols ? d->cols[col] : d->w;
  return IPX_OK;
}

ipx_status ipx_dataset_read(ipx_ctx* ctx, const ipx_dataset* d, int col, int64_t offset, int64_t count,
                            double* host) {
  if (!ctx || !d || (!host && count > 0)) return fail(IPX_EINVAL, "ipx_dataset_read: NULL argument");
  if (col < 0 || col > d->ncols || (col == d->ncols && !d->w))
    return fail(IPX_EINVAL, "ipx_dataset_read: column %d not present", col);
  if (offset < 0 || count < 0 || offset + count > d->n)
    return fail(IPX_EINVAL, "ipx_dataset_read: range [%lld, %lld) outside [0, %lld)", (long long)offset,
                (long long)(offset + count), (long long)d->n);
  if (count == 0) return IPX_OK;
  const double* src = (col < d->ncols ? d->cols[col] : d->w) + offset;
  HIP_TRY(hipSetDevice(ctx->device));
  HIP_TRY(hipMemcpyAsync(host, src, (size_t)count * sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
  HIP_TRY(hipStreamSynchronize(ctx->stream));
  return IPX_OK;
}

ipx_status ipx_timing_enable(ipx_ctx* ctx, int enable) {
  if (!ctx) return fail(IPX_EINVAL, "ipx_timing_enable: NULL ctx");
  ctx->timing = enable != 0;
  return IPX_OK;
}

static ipx_status timing_drain(ipx_ctx* ctx) {
  for (int i = 0; i < ctx->ev_used; ++i) {
    HIP_TRY(hipEventSynchronize(ctx->ev_pool[1][i]));
    float ms = 0.f;
    HIP_TRY(hipEventElapsedTime(&ms, ctx->ev_pool[0][i], ctx->ev_pool[1][i]));
    ctx->timing_ms += ms;
    ctx->timing_launches += 1;
  }
  ctx->ev_used = 0;
  return IPX_OK;
}

ipx_status ipx_timing_read(ipx_ctx* ctx, double* total_ms, int64_t* launches, int reset) {
  if (!ctx) return fail(IPX_EINVAL, "ipx_timing_read: NULL ctx");
  ipx_status s = timing_drain(ctx);
  if (s != IPX_OK) return s;
  if (total_ms) *total_ms = ctx->timing_ms;
  if (launches) *launches = ctx->timing_launches;
  if (reset) {
    ctx->timing_ms = 0.0;
    ctx->timing_launches = 0;
  }
  return IPX_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// FP64 ceiling of the device: every lane runs eight independent fused
// multiply-add chains; each workgroup records its shader-clock cycles
// (s_memtime) and wall-clock ticks (s_memrealtime) over the loop.
// ---------------------------------------------------------------------------
// (The factor is a literal, built in scalar registers, and the addend 0.5 an
// inline constant, so the loop is the multiply-adds and a few scalar
// instructions; a factor passed as an argument is reloaded from the argument
// block in every iteration, as the device code is built without machine
// loop-invariant code motion.)
__global__ void k_fp64_probe(double* __restrict__ out, long long* __restrict__ cyc, long long* __restrict__ wall,
                             int iters) {
  constexpr double b = 1.0000001;
  double x[8];
#pragma unroll
  for (int u = 0; u < 8; ++u) x[u] = threadIdx.x * 1e-3 + u;
  const long long t0 = clock64();
  const long long w0 = wall_clock64();
  for (int i = 0; i < iters; ++i) {
#pragma unroll
    for (int u = 0; u < 8; ++u) x[u] = fma(x[u], b, 0.5);
  }
  const long long t1 = clock64();
  const long long w1 = wall_clock64();
  double s = 0.0;
#pragma unroll
  for (int u = 0; u < 8; ++u) s += x[u];
  out[(size_t)blockIdx.x * blockDim.x + threadIdx.x] = s;
  if (threadIdx.x == 0) {
    cyc[blockIdx.x] = t1 - t0;
    wall[blockIdx.x] = w1 - w0;
  }
}

extern "C" ipx_status ipx_fp64_peak_probe(ipx_ctx* ctx, double* tflops, double* clock_ghz) {
  if (!ctx || !tflops || !clock_ghz) return fail(IPX_EINVAL, "ipx_fp64_peak_probe: NULL argument");
  HIP_TRY(hipSetDevice(ctx->device));
  int wrate = 0;
  HIP_TRY(hipDeviceGetAttribute(&wrate, hipDeviceAttributeWallClockRate, ctx->device));
  if (wrate <= 0) return fail(IPX_EDEVICE, "ipx_fp64_peak_probe: no wall-clock rate");
  const int blocks = 8 * std::max(1, ctx->n_cu), threads = 256, iters = 200000;
  char* buf = nullptr;
  const size_t nout = (size_t)blocks * threads;
  HIP_TRY(hipMalloc(&buf, nout * sizeof(double) + 2 * (size_t)blocks * sizeof(long long)));
  double* out = (double*)buf;
  long long* cyc = (long long*)(out + nout);
  long long* wall = cyc + blocks;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  hipError_t e = hipEventCreate(&e0);
  if (e == hipSuccess) e = hipEventCreate(&e1);
  double best = 0.0, best_ghz = 0.0;
  std::vector<long long> c(blocks), w(blocks);
  for (int rep = 0; rep < 3 && e == hipSuccess; ++rep) {
    e = hipEventRecord(e0, ctx->stream);
    if (e == hipSuccess) {
      hipLaunchKernelGGL(k_fp64_probe, dim3(blocks), dim3(threads), 0, ctx->stream, out, cyc, wall, iters);
      e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipEventRecord(e1, ctx->stream);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    float ms = 0.f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
    if (e == hipSuccess) e = hipMemcpy(c.data(), cyc, blocks * sizeof(long long), hipMemcpyDeviceToHost);
    if (e == hipSuccess) e = hipMemcpy(w.data(), wall, blocks * sizeof(long long), hipMemcpyDeviceToHost);
    if (e != hipSuccess || ms <= 0.f) break;
    std::vector<double> f(blocks);
    for (int i = 0; i < blocks; ++i) f[i] = (double)c[i] * (wrate * 1e3) / std::max<double>(1.0, (double)w[i]) / 1e9;
    std::sort(f.begin(), f.end());
    const double tf = 2.0 * 8.0 * iters * (double)nout / (ms * 1e-3) / 1e12;
    if (tf > best) {
      best = tf;
      best_ghz = f[blocks / 2];
    }
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  const hipError_t ef = hipFree(buf);
  if (e != hipSuccess) return fail(IPX_EDEVICE, "ipx_fp64_peak_probe: %s", hipGetErrorString(e));
  if (ef != hipSuccess) return fail(IPX_EDEVICE, "ipx_fp64_peak_probe: hipFree: %s", hipGetErrorString(ef));
  *tflops = best;
  *clock_ghz = best_ghz;
  return IPX_OK;
}

// ---------------------------------------------------------------------------
// Self-check of the device elementary functions (the same inline functions the
// event kernels use), element by element.
// ---------------------------------------------------------------------------
__global__ void k_math_eval(int fn, int64_t n, const double* __restrict__ x, const double* __restrict__ x2,
                            double* __restrict__ y, double* __restrict__ y2) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double a = x[i];
  switch (fn) {
    case IPX_FN_EXP: y[i] = ipx::exp_fast(a); break;
    case IPX_FN_LOG: y[i] = ipx::log_fast(a); break;
    case IPX_FN_SINCOS: {
      double s, c;
      ipx::sincos_fast(a, &s, &c);
      y[i] = s;
      y2[i] = c;
      break;
    }
    case IPX_FN_ERFCX: y[i] = ipx::erfcx_pos(a); break;
    case IPX_FN_FADDEEVA: {
      const ipx::cplx w = ipx::faddeeva_upper(ipx::cplx{a, x2[i]});
      y[i] = w.re;
      y2[i] = w.im;
      break;
    }
    default: break;
  }
}

extern "C" ipx_status ipx_math_eval(ipx_ctx* ctx, int fn, int64_t n, const double* x, const double* x2, double* y,
                                    double* y2) {
  if (!ctx) return fail(IPX_EINVAL, "ipx_math_eval: NULL ctx");
  if (fn < IPX_FN_EXP || fn > IPX_FN_FADDEEVA) return fail(IPX_EINVAL, "ipx_math_eval: unknown function %d", fn);
  if (n < 0 || n > (int64_t(1) << 28)) return fail(IPX_EINVAL, "ipx_math_eval: n = %lld out of [0, 2^28]", (long long)n);
  const bool two_in = fn == IPX_FN_FADDEEVA, two_out = fn == IPX_FN_SINCOS || fn == IPX_FN_FADDEEVA;
  if (n > 0 && (!x || !y || (two_in && !x2) || (two_out && !y2)))
    return fail(IPX_EINVAL, "ipx_math_eval: NULL buffer");
  if (n == 0) return IPX_OK;
  HIP_TRY(hipSetDevice(ctx->device));
  const size_t b = (size_t)n * sizeof(double);
  double* d = nullptr;
  HIP_TRY(hipMalloc(&d, 4 * b));
  double *dx = d, *dx2 = d + n, *dy = d + 2 * n, *dy2 = d + 3 * n;
  hipError_t e = hipMemcpyAsync(dx, x, b, hipMemcpyHostToDevice, ctx->stream);
  if (e == hipSuccess && two_in) e = hipMemcpyAsync(dx2, x2, b, hipMemcpyHostToDevice, ctx->stream);
  if (e == hipSuccess) {
    const unsigned blocks = (unsigned)((n + 255) / 256);
    hipLaunchKernelGGL(k_math_eval, dim3(blocks), dim3(256), 0, ctx->stream, fn, n, dx, dx2, dy, dy2);
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = hipMemcpyAsync(y, dy, b, hipMemcpyDeviceToHost, ctx->stream);
  if (e == hipSuccess && two_out) e = hipMemcpyAsync(y2, dy2, b, hipMemcpyDeviceToHost, ctx->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
  const hipError_t ef = hipFree(d);
  if (e != hipSuccess) return fail(IPX_EDEVICE, "ipx_math_eval: %s", hipGetErrorString(e));
  if (ef != hipSuccess) return fail(IPX_EDEVICE, "ipx_math_eval: hipFree: %s", hipGetErrorString(ef));
  return IPX_OK;
}

// ---------------------------------------------------------------------------
// Launch helpers
// ---------------------------------------------------------------------------
static EventCols cols_of(const ipx_dataset* d) {
  EventCols c;
  for (int i = 0; i < 7; ++i) c.c[i] = d->cols[i];
  c.w = d->w;
  c.n = d->n;
  return c;
}

// ---------------------------------------------------------------------------
// Toy generation
// ---------------------------------------------------------------------------
// Integral of the resolution-convolved exponential over [T_LO, T_HI] on the
// host (bounds only): (1/G)[Phi(b) - Phi(a) - F(b) + F(a)].
static double host_conv_integral(double G, double sig) {
  const double r2s = std::sqrt(2.0) * sig;
  auto F = [&](double t) { return 0.5 * std::exp(0.5 * G * G * sig * sig - G * t) * std::erfc((G * sig * sig - t) / r2s); };
  const double dphi = 0.5 * (std::erfc(kTLo / r2s) - std::erfc(kTHi / r2s));
  return (dphi - F(kTHi) + F(kTLo)) / G;
}

static double g_DG_sign(double dg) { return dg < 0.0 ? -1.0 : 1.0; }
static const double kAngMax[10] = {2.0, 1.0, 1.0, 1.0, 0.70710678118654752440, 0.70710678118654752440,
                                   2.0 / 3.0, 0.81649658092772603273, 0.81649658092772603273,
                                   2.3094010767585030580};

struct GenSetup {
  GenConst g;
  double C[40];
};

static void gen_setup(int model, const double* th, uint64_t seed, uint64_t toy, GenSetup& h) {
  std::memset(&h, 0, sizeof h);
  GenConst& g = h.g;
  g.seed = seed;
  g.toy = toy;
  if (model == 1) {
    const MassHoist m = hoist_mass(th);
    g.f = th[0]; g.mu = th[1]; g.sig_m = th[2]; g.lam = th[3];
    g.cS = m.k.cS; g.cB = m.k.cB;
    const double emax = g.lam >= 0.0 ? 1.0 : std::exp(-g.lam * (kMHi - kMLo));
    g.M = g.cS + g.cB * emax;
  } else if (model == 2) {
    const MassTimeHoist m = hoist_masstime(th);
    g.f = th[0]; g.mu = th[1]; g.sig_m = th[2]; g.lam = th[3];
    g.tau_s = th[4]; g.tau_b = th[5]; g.s = th[6];
    g.L_e = -std::expm1(-g.lam * (kMHi - kMLo));
    g.rs_num = g.sig_m * std::sqrt(2.0 * M_PI) / m.ng.N;
    g.mt = m.k;
    double M = 0.0;
    for (int i = 0; i < 64; ++i) {
      const double sig = g.s * (0.03 + 0.03 * i / 63.0);
      const double rs = g.rs_num / (m.k.gs * host_conv_integral(m.k.gs, sig));
      const double rb = 1.0 / (m.k.gb * host_conv_integral(m.k.gb, sig));
      M = std::fmax(M, std::fmax(rs, rb));
    }
    g.M = (1.0 + 1e-3) * M;
  } else {
    AngTimeHoist a;
    hoist_angtime(th, ang_settings_default(), a);
    // M3 = (1 + 1e-12) [max(S0, S1 / 2) + S2]: with x = e^{-|DeltaGamma| t0},
    // e^{Gamma_min t0} times the time functions are (1 + x)/2, s (1 - x)/2
    // (s the sign of DeltaGamma) and a pair of length sqrt(x) <= 1; the
    // cosh / sinh part is linear in x, largest at x = 0 or 1; S0, S1, S2
    // bound |A_0|, |A_0 + s A_1| and |(A_2, A_3)| (A_j = sum_k f_k C_kj) by
    // triangle inequalities with m_k = max|f_k|; the factor covers rounding
    const double sg = g_DG_sign(th[7]);
    double S0 = 0.0, S1 = 0.0, S2 = 0.0;
    for (int k = 0; k < 10; ++k) {
      for (int j = 0; j < 4; ++j) h.C[4 * k + j] = a.k.C[k][j];
      const double c0 = a.k.C[k][0], c1 = a.k.C[k][1], c2 = a.k.C[k][2], c3 = a.k.C[k][3];
      S0 += kAngMax[k] * std::fabs(c0);
      S1 += kAngMax[k] * std::fabs(c0 + sg * c1);
      S2 += kAngMax[k] * std::sqrt(c2 * c2 + c3 * c3);
    }
    g.M = (1.0 + 1e-12) * (std::fmax(S0, 0.5 * S1) + S2);
    g.G = th[6]; g.DG = th[7]; g.DM = th[8];
    g.gmin = g.G - std::fabs(g.DG) / 2.0;
    g.mu3 = th[10]; g.sig3 = th[11];
  }
}

struct GenScratch {
  int* flags = nullptr;
  int* rank = nullptr;
  void* scan = nullptr;
  size_t scan_bytes = 0;
  unsigned long long* counters = nullptr;  // [0] violations, [1] last candidate + 1
  double* C = nullptr;
  double** colp = nullptr;
  int* tail = nullptr;                     // last rank, last flag
  ~GenScratch() {
    (void)hipFree(flags); (void)hipFree(rank); (void)hipFree(scan); (void)hipFree(counters);
    (void)hipFree(C); (void)hipFree(colp); (void)hipFree(tail);
  }
};

static const double kGenEfficiency[4] = {0.0, 0.25, 0.5, 0.1};  // first-batch guesses
static const int64_t kGenMaxBatch = 1 << 24;

template <int MODEL>
static ipx_status gen_batch(const GenConst& g, GenScratch& sc, uint64_t c0, int64_t count, int64_t got, int64_t need,
                            double* wout, hipStream_t s, int64_t* accepted) {
  const unsigned blocks = (unsigned)((count + 255) / 256);
  hipLaunchKernelGGL((k_gen_flags<MODEL>), dim3(blocks), dim3(256), 0, s, g, (const double*)sc.C, c0, count,
                     sc.flags, sc.counters);
  HIP_TRY(hipGetLastError());
  HIP_TRY(scan_exclusive(sc.flags, sc.rank, count, (int*)sc.scan, s));
  hipLaunchKernelGGL((k_gen_write<MODEL>), dim3(blocks), dim3(256), 0, s, g, (const double*)sc.C, c0, count,
                     (const int*)sc.flags, (const int*)sc.rank, got, need, (double* const*)sc.colp, wout,
                     sc.counters + 1);
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipMemcpyAsync(sc.tail, sc.rank + count - 1, sizeof(int), hipMemcpyDeviceToDevice, s));
  HIP_TRY(hipMemcpyAsync(sc.tail + 1, sc.flags + count - 1, sizeof(int), hipMemcpyDeviceToDevice, s));
  int tail[2];
  HIP_TRY(hipMemcpyAsync(tail, sc.tail, 2 * sizeof(int), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  *accepted = (int64_t)tail[0] + tail[1];
  return IPX_OK;
}

// A dataset of n events for the generator to fill: one allocation of the
// columns (and weights), the reduction partials, the result buffers.
static hipError_t alloc_toy_dataset(int model, int64_t n, bool weighted, ipx_dataset** out) {
  *out = nullptr;
  const int ncols = kNCols[model];
  ipx_dataset* d = new (std::nothrow) ipx_dataset();
  if (!d) return hipErrorOutOfMemory;
  d->model = model;
  d->n = n;
  d->ncols = ncols;
  d->n_pad = (n + 31) / 32 * 32;
  d->n_tiles = (n + kTile - 1) / kTile;
  const int nstore = ncols + (weighted ? 1 : 0);
  const size_t bytes = (size_t)nstore * (size_t)(d->n_pad > 0 ? d->n_pad : 32) * sizeof(double);
  hipError_t e = hipMalloc(&d->base, bytes);
  const int64_t tiles_alloc = d->n_tiles > 0 ? d->n_tiles : 1;
  if (e == hipSuccess) e = hipMalloc(&d->partials, (size_t)tiles_alloc * kAccMax * sizeof(double));
  if (e == hipSuccess) e = hipMalloc(&d->out_dev, kAccMax * sizeof(double));
  if (e == hipSuccess) e = hipHostMalloc(&d->out_host, kAccMax * sizeof(double), hipHostMallocDefault);
  if (e != hipSuccess) {
    free_dataset(d);
    return e;
  }
  d->bytes = bytes + (size_t)tiles_alloc * kAccMax * sizeof(double) + kAccMax * sizeof(double);
  for (int c = 0; c < ncols; ++c) d->cols[c] = d->base + (size_t)c * d->n_pad;
  if (weighted) d->w = d->base + (size_t)ncols * d->n_pad;
  *out = d;
  return hipSuccess;
}

extern "C" ipx_status toy_generate(ipx_ctx* ctx, int model, const double* theta, int np, uint64_t seed,
                                   uint64_t toy_id, int64_t n, unsigned flags, ipx_dataset** out,
                                   ipx_toy_stats* stats) {
  if (!ctx || !theta || !out) return fail(IPX_EINVAL, "toy_generate: NULL argument");
  *out = nullptr;
  if (model < 1 || model > 3) return fail(IPX_EINVAL, "toy_generate: unknown model %d", model);
  if (np != kNParams[model]) return fail(IPX_EINVAL, "toy_generate: model %d takes %d parameters", model, kNParams[model]);
  if (n < 0 || n > 0x7fffffff) return fail(IPX_EINVAL, "toy_generate: n = %lld out of range", (long long)n);
  if (flags & ~(IPX_KEEP_ORDER | IPX_NO_WEIGHTS)) return fail(IPX_EINVAL, "toy_generate: bad flags %u", flags);
  if (!theta_valid(model, theta)) return fail(IPX_EDOMAIN, "toy_generate: parameters outside the domain");
  HIP_TRY(hipSetDevice(ctx->device));
  hipStream_t s = ctx->stream;
  GenSetup h;
  gen_setup(model, theta, seed, toy_id, h);
  if (!(h.g.M > 0.0) || !std::isfinite(h.g.M)) return fail(IPX_EDOMAIN, "toy_generate: no finite acceptance bound");

  // output dataset, columns written in candidate order
  const int ncols = kNCols[model];
  const bool weighted = model == 3 && !(flags & IPX_NO_WEIGHTS);
  ipx_dataset* d = nullptr;
  hipError_t e = alloc_toy_dataset(model, n, weighted, &d);
  if (e != hipSuccess) return fail(IPX_ENOMEM, "toy_generate: allocation failed: %s", hipGetErrorString(e));
  double* colp_host[6] = {};
  for (int c = 0; c < ncols; ++c) colp_host[c] = const_cast<double*>(d->cols[c]);
  double* wout = const_cast<double*>(d->w);

  uint64_t candidates = 0, violations = 0;
  if (n > 0) {
    GenScratch sc;
    const int64_t cap = std::min<int64_t>(kGenMaxBatch, std::max<int64_t>(65536, (int64_t)(n / kGenEfficiency[model] * 1.05)));
    e = hipMalloc(&sc.flags, (size_t)cap * sizeof(int));
    if (e == hipSuccess) e = hipMalloc(&sc.rank, (size_t)cap * sizeof(int));
    if (e == hipSuccess) e = hipMalloc(&sc.counters, 2 * sizeof(unsigned long long));
    if (e == hipSuccess) e = hipMalloc(&sc.C, 40 * sizeof(double));
    if (e == hipSuccess) e = hipMalloc(&sc.colp, 6 * sizeof(double*));
    if (e == hipSuccess) e = hipMalloc(&sc.tail, 2 * sizeof(int));
    sc.scan_bytes = scan_temp_ints(cap) * sizeof(int);
    if (e == hipSuccess) e = hipMalloc(&sc.scan, sc.scan_bytes);
    unsigned long long zero2[2] = {0ull, 0ull};
    if (e == hipSuccess) e = hipMemcpyAsync(sc.counters, zero2, sizeof zero2, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipMemcpyAsync(sc.C, h.C, sizeof h.C, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipMemcpyAsync(sc.colp, colp_host, sizeof colp_host, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) {
      free_dataset(d);
      return fail(IPX_ENOMEM, "toy_generate: scratch allocation failed: %s", hipGetErrorString(e));
    }
    int64_t got = 0;
    uint64_t c0 = 0;
    double eff = kGenEfficiency[model];
    while (got < n) {
      const int64_t want = (int64_t)((n - got) / eff * 1.05) + 4096;
      const int64_t count = std::min<int64_t>(cap, std::max<int64_t>(65536, want));
      int64_t acc = 0;
      ipx_status st = model == 1 ? gen_batch<1>(h.g, sc, c0, count, got, n - got, wout, s, &acc)
                    : model == 2 ? gen_batch<2>(h.g, sc, c0, count, got, n - got, wout, s, &acc)
                                 : gen_batch<3>(h.g, sc, c0, count, got, n - got, wout, s, &acc);
      if (st != IPX_OK) {
        free_dataset(d);
        return st;
      }
      if (acc > 0) eff = std::max(1e-4, (double)acc / (double)count);
      got += std::min<int64_t>(acc, n - got);
      c0 += (uint64_t)count;
      if (c0 > (1ull << 48)) {
        free_dataset(d);
        return fail(IPX_EDOMAIN, "toy_generate: acceptance too low (%lld of %lld after 2^48 candidates)",
                    (long long)got, (long long)n);
      }
    }
    unsigned long long cnt[2];
    e = hipMemcpy(cnt, sc.counters, sizeof cnt, hipMemcpyDeviceToHost);
    if (e != hipSuccess) {
      free_dataset(d);
      return fail(IPX_EDEVICE, "toy_generate: readback failed: %s", hipGetErrorString(e));
    }
    violations = cnt[0];
    candidates = cnt[1];
  }
  if (model >= 2 && !(flags & IPX_KEEP_ORDER) && n >= 2) {
    ipx_status st = sort_events(&d, 1, s);
    if (st != IPX_OK) {
      free_dataset(d);
      return st;
    }
  }
  if (stats) {
    stats->n_candidates = candidates;
    stats->n_violations = violations;
  }
  *out = d;
  return IPX_OK;
}

// Batched generation: every toy's candidates of a round in one flags launch,
// one prefix sum and one write launch; rounds repeat for the toys still short
// of events.  Each toy's events, candidates and order are those of
// toy_generate with the same arguments.
struct GenBatchScratch {
  GenSeg* segs = nullptr;
  int* flags = nullptr;
  int* rank = nullptr;
  void* scan = nullptr;
  size_t scan_bytes = 0;
  double* C = nullptr;
  unsigned long long* viol = nullptr;
  unsigned long long* last = nullptr;
  int64_t* acc = nullptr;
  ~GenBatchScratch() {
    (void)hipFree(segs); (void)hipFree(flags); (void)hipFree(rank); (void)hipFree(scan); (void)hipFree(C);
    (void)hipFree(viol); (void)hipFree(last); (void)hipFree(acc);
  }
};

template <int MODEL>
static ipx_status gen_round(const GenConst& g, GenBatchScratch& sc, int nseg, int64_t total, hipStream_t s) {
  const unsigned blocks = (unsigned)((total + 255) / 256);
  hipLaunchKernelGGL((k_gen_flags_batch<MODEL>), dim3(blocks), dim3(256), 0, s, g, (const double*)sc.C,
                     (const GenSeg*)sc.segs, nseg, total, sc.flags, sc.viol);
  HIP_TRY(hipGetLastError());
  HIP_TRY(scan_exclusive(sc.flags, sc.rank, total, (int*)sc.scan, s));
  hipLaunchKernelGGL((k_gen_write_batch<MODEL>), dim3(blocks), dim3(256), 0, s, g, (const double*)sc.C,
                     (const GenSeg*)sc.segs, nseg, total, (const int*)sc.flags, (const int*)sc.rank, sc.last);
  HIP_TRY(hipGetLastError());
  hipLaunchKernelGGL(k_gen_counts, dim3((unsigned)((nseg + 255) / 256)), dim3(256), 0, s, (const GenSeg*)sc.segs,
                     nseg, (const int*)sc.flags, (const int*)sc.rank, sc.acc);
  HIP_TRY(hipGetLastError());
  return IPX_OK;
}

static const int64_t kGenBatchCap = (int64_t)1 << 26;   // candidates per round

extern "C" ipx_status toy_generate_batch(ipx_ctx* ctx, int model, const double* theta, int np, uint64_t seed,
                                         int ntoys, const uint64_t* toy_ids, const int64_t* n, unsigned flags,
                                         ipx_dataset** out, ipx_toy_stats* stats) {
  if (!ctx || !theta || !out || (ntoys > 0 && (!toy_ids || !n)))
    return fail(IPX_EINVAL, "toy_generate_batch: NULL argument");
  if (ntoys < 0) return fail(IPX_EINVAL, "toy_generate_batch: ntoys = %d", ntoys);
  for (int j = 0; j < ntoys; ++j) out[j] = nullptr;
  if (model < 1 || model > 3) return fail(IPX_EINVAL, "toy_generate_batch: unknown model %d", model);
  if (np != kNParams[model])
    return fail(IPX_EINVAL, "toy_generate_batch: model %d takes %d parameters", model, kNParams[model]);
  for (int j = 0; j < ntoys; ++j)
    if (n[j] < 0 || n[j] > 0x7fffffff)
      return fail(IPX_EINVAL, "toy_generate_batch: n[%d] = %lld out of range", j, (long long)n[j]);
  if (flags & ~(IPX_KEEP_ORDER | IPX_NO_WEIGHTS)) return fail(IPX_EINVAL, "toy_generate_batch: bad flags %u", flags);
  if (!theta_valid(model, theta)) return fail(IPX_EDOMAIN, "toy_generate_batch: parameters outside the domain");
  HIP_TRY(hipSetDevice(ctx->device));
  hipStream_t s = ctx->stream;
  GenSetup h;
  gen_setup(model, theta, seed, 0, h);
  if (!(h.g.M > 0.0) || !std::isfinite(h.g.M))
    return fail(IPX_EDOMAIN, "toy_generate_batch: no finite acceptance bound");
  const bool weighted = model == 3 && !(flags & IPX_NO_WEIGHTS);
  auto release = [&]() {
    for (int j = 0; j < ntoys; ++j) {
      if (out[j]) free_dataset(out[j]);
      out[j] = nullptr;
    }
  };
  for (int j = 0; j < ntoys; ++j) {
    hipError_t e = alloc_toy_dataset(model, n[j], weighted, &out[j]);
    if (e != hipSuccess) {
      release();
      return fail(IPX_ENOMEM, "toy_generate_batch: allocation failed: %s", hipGetErrorString(e));
    }
  }
  std::vector<int64_t> got(ntoys, 0);
  std::vector<uint64_t> c0(ntoys, 0);
  std::vector<unsigned long long> viol(ntoys, 0), last(ntoys, 0);
  int64_t total_need = 0;
  for (int j = 0; j < ntoys; ++j) total_need += n[j];
  if (total_need > 0) {
    GenBatchScratch sc;
    const int64_t cap = std::min<int64_t>(kGenBatchCap, std::max<int64_t>(65536, (int64_t)(total_need / kGenEfficiency[model] * 1.1)
                                                                         + (int64_t)ntoys * 4096));
    hipError_t e = hipMalloc(&sc.segs, (size_t)std::max(ntoys, 1) * sizeof(GenSeg));
    if (e == hipSuccess) e = hipMalloc(&sc.flags, (size_t)cap * sizeof(int));
    if (e == hipSuccess) e = hipMalloc(&sc.rank, (size_t)cap * sizeof(int));
    if (e == hipSuccess) e = hipMalloc(&sc.C, 40 * sizeof(double));
    if (e == hipSuccess) e = hipMalloc(&sc.viol, (size_t)ntoys * sizeof(unsigned long long));
    if (e == hipSuccess) e = hipMalloc(&sc.last, (size_t)ntoys * sizeof(unsigned long long));
    if (e == hipSuccess) e = hipMalloc(&sc.acc, (size_t)ntoys * sizeof(int64_t));
    sc.scan_bytes = scan_temp_ints(cap) * sizeof(int);
    if (e == hipSuccess) e = hipMalloc(&sc.scan, sc.scan_bytes);
    if (e == hipSuccess) e = hipMemcpyAsync(sc.C, h.C, sizeof h.C, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipMemcpyAsync(sc.viol, viol.data(), viol.size() * sizeof(unsigned long long), hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipMemcpyAsync(sc.last, last.data(), last.size() * sizeof(unsigned long long), hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) {
      release();
      return fail(IPX_ENOMEM, "toy_generate_batch: scratch allocation failed: %s", hipGetErrorString(e));
    }
    double eff = kGenEfficiency[model];
    std::vector<GenSeg> segs;
    std::vector<int> seg_toy;
    std::vector<int64_t> acc;
    int next = 0;   // round-robin start over the toys still short of events
    for (;;) {
      segs.clear();
      seg_toy.clear();
      int64_t total = 0;
      for (int k = 0; k < ntoys; ++k) {
        const int j = (next + k) % ntoys;
        const int64_t need = n[j] - got[j];
        if (need <= 0) continue;
        const int64_t count = std::max<int64_t>(4096, (int64_t)(need / eff * 1.05) + 4096);
        if (total + count > cap && !segs.empty()) break;
        const int64_t cnt = std::min<int64_t>(count, cap - total);
        GenSeg g{};
        g.toy = toy_ids[j];
        g.c0 = c0[j];
        g.start = total;
        g.count = cnt;
        g.out_base = got[j];
        g.need = need;
        for (int c = 0; c < kNCols[model]; ++c) g.cols[c] = const_cast<double*>(out[j]->cols[c]);
        g.w = const_cast<double*>(out[j]->w);
        segs.push_back(g);
        seg_toy.push_back(j);
        total += cnt;
        if (total >= cap) break;
      }
      if (segs.empty()) break;
      next = (seg_toy.back() + 1) % ntoys;
      const int nseg = (int)segs.size();
      // per-segment counters live at the segment's index: reset them
      std::vector<unsigned long long> zeros(nseg, 0ull);
      hipError_t e2 = hipMemcpyAsync(sc.segs, segs.data(), nseg * sizeof(GenSeg), hipMemcpyHostToDevice, s);
      if (e2 == hipSuccess) e2 = hipMemcpyAsync(sc.viol, zeros.data(), nseg * sizeof(unsigned long long), hipMemcpyHostToDevice, s);
      if (e2 == hipSuccess) e2 = hipMemcpyAsync(sc.last, zeros.data(), nseg * sizeof(unsigned long long), hipMemcpyHostToDevice, s);
      if (e2 != hipSuccess) {
        release();
        return fail(IPX_EDEVICE, "toy_generate_batch: upload failed: %s", hipGetErrorString(e2));
      }
      ipx_status st = model == 1 ? gen_round<1>(h.g, sc, nseg, total, s)
                    : model == 2 ? gen_round<2>(h.g, sc, nseg, total, s)
                                 : gen_round<3>(h.g, sc, nseg, total, s);
      if (st != IPX_OK) {
        release();
        return st;
      }
      acc.assign(nseg, 0);
      std::vector<unsigned long long> v(nseg), l(nseg);
      e2 = hipMemcpyAsync(acc.data(), sc.acc, nseg * sizeof(int64_t), hipMemcpyDeviceToHost, s);
      if (e2 == hipSuccess) e2 = hipMemcpyAsync(v.data(), sc.viol, nseg * sizeof(unsigned long long), hipMemcpyDeviceToHost, s);
      if (e2 == hipSuccess) e2 = hipMemcpyAsync(l.data(), sc.last, nseg * sizeof(unsigned long long), hipMemcpyDeviceToHost, s);
      if (e2 == hipSuccess) e2 = hipStreamSynchronize(s);
      if (e2 != hipSuccess) {
        release();
        return fail(IPX_EDEVICE, "toy_generate_batch: readback failed: %s", hipGetErrorString(e2));
      }
      int64_t acc_sum = 0, cnt_sum = 0;
      for (int k = 0; k < nseg; ++k) {
        const int j = seg_toy[k];
        viol[j] += v[k];
        if (l[k]) last[j] = l[k];
        got[j] += std::min<int64_t>(acc[k], n[j] - got[j]);
        c0[j] += (uint64_t)segs[k].count;
        acc_sum += acc[k];
        cnt_sum += segs[k].count;
        if (c0[j] > (1ull << 48)) {
          release();
          return fail(IPX_EDOMAIN, "toy_generate_batch: acceptance too low in toy %d", j);
        }
      }
      if (acc_sum > 0) eff = std::max(1e-4, (double)acc_sum / (double)cnt_sum);
    }
  }
  if (model >= 2 && !(flags & IPX_KEEP_ORDER)) {
    // every toy in one joint ordering (each toy's events among themselves)
    ipx_status st = sort_events(out, ntoys, s);
    if (st != IPX_OK) {
      release();
      return st;
    }
  }
  if (stats)
    for (int j = 0; j < ntoys; ++j) {
      stats[j].n_candidates = last[j];
      stats[j].n_violations = viol[j];
    }
  return IPX_OK;
}

// ---------------------------------------------------------------------------
// Batched evaluation plans
// ---------------------------------------------------------------------------
struct ipx_plan {
  ipx_ctx* ctx = nullptr;
  int model = 0;
  int nb = 0;
  std::vector<ipx_dataset*> ds;
  size_t const_size = 0;
  SegInfo* d_segs = nullptr;
  TileRef* d_tiles = nullptr;
  int64_t n_tiles = 0;
  ipx_schedule sched{0, 0, 1, 0};  // launch schedule (results do not depend on it)
  void* h_consts = nullptr;        // pinned [constants | active flags], written by the host
  unsigned char* h_active = nullptr;
  void* d_consts = nullptr;        // the same block's device address (read by the kernels)
  unsigned char* d_active = nullptr;
  size_t stage_bytes = 0;
  double* h_out = nullptr;         // pinned results, written by the reduction kernel
  double* h_out_dev = nullptr;     // its device address
  hipGraphExec_t exec[2] = {nullptr, nullptr};  // [eval, grad]
  bool counted = false;            // holds a reference on each dataset
  hipStream_t exec_stream[2] = {nullptr, nullptr};
  std::vector<AngTimeHoist> h3;    // angular model: per-dataset hoists, kept between calls
};

static void free_plan(struct ipx_plan* p) {
  if (p->counted)
    for (ipx_dataset* d : p->ds) d->plan_refs--;
  for (int i = 0; i < 2; ++i)
    if (p->exec[i]) (void)hipGraphExecDestroy(p->exec[i]);
  (void)hipFree(p->d_segs); (void)hipFree(p->d_tiles);
  if (p->h_consts) (void)hipHostFree(p->h_consts);
  if (p->h_out) (void)hipHostFree(p->h_out);
  delete p;
}

// The plan's table of (segment, local tile) pairs in the order the kernels
// take them: segment by segment (order 0), or interleaved by local tile index
// (order 1: the first tile of every segment, then the second, ...; within a
// segment the tiles run in storage order, the expensive ones first).  A tile's
// partials, and so every result, do not depend on the order.
static std::vector<TileRef> tile_table(const ipx_plan* p, int order) {
  std::vector<TileRef> tiles;
  int64_t most = 0;
  for (const ipx_dataset* d : p->ds) most = std::max(most, d->n_tiles);
  if (order == 0) {
    for (int j = 0; j < p->nb; ++j)
      for (int64_t t = 0; t < p->ds[j]->n_tiles; ++t) tiles.push_back(TileRef{j, (int)t});
  } else {
    for (int64_t t = 0; t < most; ++t)
      for (int j = 0; j < p->nb; ++j)
        if (t < p->ds[j]->n_tiles) tiles.push_back(TileRef{j, (int)t});
  }
  return tiles;
}

static size_t const_size_of(int model) {
  return model == 1 ? sizeof(MassConst) : model == 2 ? sizeof(MassTimeConst) : sizeof(AngTimeConst);
}
static int nacc_of(int model, bool grad) {
  return !grad ? 1 : model == 1 ? kAccMass : model == 2 ? kAccMassTime : kAccAngTime;
}

static ipx_status plan_create(ipx_ctx* ctx, int nb, ipx_dataset* const* ds, ipx_plan** out, bool counted);
extern "C" ipx_status ipx_plan_create(ipx_ctx* ctx, int nb, ipx_dataset* const* ds, ipx_plan** out) {
  return plan_create(ctx, nb, ds, out, true);
}
static ipx_status plan_create(ipx_ctx* ctx, int nb, ipx_dataset* const* ds, ipx_plan** out, bool counted) {
  if (!ctx || !out || (nb > 0 && !ds)) return fail(IPX_EINVAL, "ipx_plan_create: NULL argument");
  *out = nullptr;
  if (nb <= 0) return fail(IPX_EINVAL, "ipx_plan_create: empty batch");
  const int model = ds[0] ? ds[0]->model : 0;
  if (model == kModelIpatia)
    return fail(IPX_EINVAL, "ipx_plan_create: the Ipatia model is evaluated by nll_eval only");
  for (int j = 0; j < nb; ++j) {
    if (!ds[j]) return fail(IPX_EINVAL, "ipx_plan_create: dataset %d is NULL", j);
    if (ds[j]->model != model) return fail(IPX_EINVAL, "ipx_plan_create: datasets of different models");
    for (int i = 0; i < j; ++i)
      if (ds[i] == ds[j]) return fail(IPX_EINVAL, "ipx_plan_create: dataset %d repeated", j);
  }
  HIP_TRY(hipSetDevice(ctx->device));
  ipx_plan* p = new (std::nothrow) ipx_plan();
  if (!p) return fail(IPX_ENOMEM, "ipx_plan_create: host allocation failed");
  p->ctx = ctx;
  p->model = model;
  p->nb = nb;
  p->ds.assign(ds, ds + nb);
  p->const_size = const_size_of(model);
  std::vector<SegInfo> segs(nb);
  hipError_t e = hipSuccess;
  for (int j = 0; j < nb; ++j) {
    ipx_dataset* d = ds[j];
    SegInfo& S = segs[j];
    S.cols = cols_of(d);
    S.partials = d->partials;
    S.n_tiles = d->n_tiles;
  }
  const std::vector<TileRef> tiles = tile_table(p, 0);
  p->n_tiles = (int64_t)tiles.size();
  if (e == hipSuccess) e = hipMalloc(&p->d_segs, nb * sizeof(SegInfo));
  if (e == hipSuccess) e = hipMalloc(&p->d_tiles, std::max<size_t>(1, tiles.size()) * sizeof(TileRef));
  const size_t cbytes = (nb * p->const_size + 255) / 256 * 256;
  p->stage_bytes = cbytes + (size_t)nb;
  if (e == hipSuccess) e = hipHostMalloc(&p->h_consts, p->stage_bytes, hipHostMallocDefault);
  if (e == hipSuccess) e = hipHostGetDevicePointer(&p->d_consts, p->h_consts, 0);
  if (e == hipSuccess) {
    p->d_active = (unsigned char*)p->d_consts + cbytes;
    p->h_active = (unsigned char*)p->h_consts + cbytes;
  }
  if (e == hipSuccess) e = hipHostMalloc((void**)&p->h_out, (size_t)nb * kAccMax * sizeof(double), hipHostMallocDefault);
  if (e == hipSuccess) e = hipHostGetDevicePointer((void**)&p->h_out_dev, p->h_out, 0);
  if (e == hipSuccess) e = hipMemcpy(p->d_segs, segs.data(), nb * sizeof(SegInfo), hipMemcpyHostToDevice);
  if (e == hipSuccess && !tiles.empty())
    e = hipMemcpy(p->d_tiles, tiles.data(), tiles.size() * sizeof(TileRef), hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    free_plan(p);
    return fail(IPX_ENOMEM, "ipx_plan_create: allocation failed: %s", hipGetErrorString(e));
  }
  if (counted) {
    for (ipx_dataset* d : p->ds) d->plan_refs++;
    p->counted = true;
  }
  *out = p;
  return IPX_OK;
}

extern "C" void ipx_plan_destroy(ipx_plan* p) {
  if (!p) return;
  (void)hipSetDevice(p->ctx->device);
  (void)hipStreamSynchronize(p->ctx->stream);
  free_plan(p);
}

// ---------------------------------------------------------------------------
// Simultaneous fit over categories: a plan over the categories' datasets,
// evaluated in one batched launch; the categories' NLLs are added in
// category order and their 12-parameter gradients are added at the positions
// their parameters take in the simultaneous vector.
// ---------------------------------------------------------------------------
constexpr int kSimShared = 10;   // fL, fperp, dpa, dpe, Gamma, DeltaGamma, Dm, phis, mu_m, sigma_m
struct ipx_sim {
  ipx_ctx* ctx = nullptr;
  ipx_plan* plan = nullptr;
  int ncat = 0, nbins = 0;
  std::vector<int> bin;
  std::vector<double> th, f, g;   // per-category parameters, NLLs, gradients
};

// Position in the simultaneous vector of parameter j (model order) of bin b.
static int sim_index(int j, int b) {
  static const int kMap[12] = {0, 1, -1, 2, 3, -2, 4, 5, 6, 7, 8, 9};
  const int m = kMap[j];
  return m == -1 ? kSimShared + 2 * b : m == -2 ? kSimShared + 2 * b + 1 : m;
}

extern "C" ipx_status ipx_sim_create(ipx_ctx* ctx, int ncat, ipx_dataset* const* ds, const int* bin, int nbins,
                                     ipx_sim** out) {
  if (!ctx || !ds || !bin || !out) return fail(IPX_EINVAL, "ipx_sim_create: NULL argument");
  *out = nullptr;
  if (ncat <= 0 || nbins <= 0 || nbins > (1 << 20)) return fail(IPX_EINVAL, "ipx_sim_create: ncat %d, nbins %d", ncat, nbins);
  for (int c = 0; c < ncat; ++c) {
    if (!ds[c]) return fail(IPX_EINVAL, "ipx_sim_create: dataset %d is NULL", c);
    if (!angular_model(ds[c]->model)) return fail(IPX_EINVAL, "ipx_sim_create: dataset %d is not of an angular model", c);
    if (bin[c] < 0 || bin[c] >= nbins) return fail(IPX_EINVAL, "ipx_sim_create: bin %d of category %d", bin[c], c);
  }
  ipx_plan* p = nullptr;
  ipx_status st = plan_create(ctx, ncat, ds, &p, true);
  if (st != IPX_OK) return st;
  ipx_sim* S = new (std::nothrow) ipx_sim();
  if (!S) {
    ipx_plan_destroy(p);
    return fail(IPX_ENOMEM, "ipx_sim_create: host allocation failed");
  }
  S->ctx = ctx;
  S->plan = p;
  S->ncat = ncat;
  S->nbins = nbins;
  S->bin.assign(bin, bin + ncat);
  S->th.resize((size_t)ncat * 12);
  S->f.resize(ncat);
  S->g.resize((size_t)ncat * 12);
  *out = S;
  return IPX_OK;
}

extern "C" void ipx_sim_destroy(ipx_sim* S) {
  if (!S) return;
  ipx_plan_destroy(S->plan);
  delete S;
}

extern "C" int ipx_sim_nparams(const ipx_sim* S) { return S ? kSimShared + 2 * S->nbins : -1; }

extern "C" ipx_status nll_sim(ipx_ctx* ctx, ipx_sim* S, const double* theta, int np, double* nll, double* grad,
                              void* stream) {
  if (!ctx || !S || !theta || !nll) return fail(IPX_EINVAL, "nll_sim: NULL argument");
  if (S->ctx != ctx) return fail(IPX_EINVAL, "nll_sim: set belongs to another context");
  if (np != kSimShared + 2 * S->nbins)
    return fail(IPX_EINVAL, "nll_sim: the set takes %d parameters, got %d", kSimShared + 2 * S->nbins, np);
  for (int c = 0; c < S->ncat; ++c)
    for (int j = 0; j < 12; ++j) S->th[(size_t)c * 12 + j] = theta[sim_index(j, S->bin[c])];
  const ipx_status st = nll_eval_batch(ctx, S->plan, S->th.data(), nullptr, S->f.data(),
                                       grad ? S->g.data() : nullptr, stream);
  if (st == IPX_EDOMAIN) {
    *nll = std::numeric_limits<double>::infinity();
    if (grad)
      for (int i = 0; i < np; ++i) grad[i] = std::numeric_limits<double>::quiet_NaN();
    return fail(IPX_EDOMAIN, "nll_sim: a category is outside its domain or has a non-finite likelihood");
  }
  if (st != IPX_OK) return st;
  double tot = 0.0;
  for (int c = 0; c < S->ncat; ++c) tot += S->f[c];
  *nll = tot;
  if (grad) {
    for (int i = 0; i < np; ++i) grad[i] = 0.0;
    for (int c = 0; c < S->ncat; ++c)
      for (int j = 0; j < 12; ++j) grad[sim_index(j, S->bin[c])] += S->g[(size_t)c * 12 + j];
  }
  return IPX_OK;
}

// The body of one batched evaluation, as stream operations (captured once
// into a graph per plan and mode).
static ipx_status timing_begin(ipx_ctx* ctx, hipStream_t s) {
  if (!ctx || !ctx->timing) return IPX_OK;
  if (ctx->ev_used == 64) {
    ipx_status st = timing_drain(ctx);
    if (st != IPX_OK) return st;
  }
  HIP_TRY(hipEventRecord(ctx->ev_pool[0][ctx->ev_used], s));
  return IPX_OK;
}
static ipx_status timing_end(ipx_ctx* ctx, hipStream_t s) {
  if (!ctx || !ctx->timing) return IPX_OK;
  HIP_TRY(hipEventRecord(ctx->ev_pool[1][ctx->ev_used], s));
  ctx->ev_used++;
  return IPX_OK;
}

// The per-event kernel over a tile table (timed through `timer` when given),
// then the per-segment reductions writing nacc totals per segment to `out`.
// Shared by plans and the allocation-free entry point, so a dataset's tiles
// run the same instructions whichever way it is evaluated.
// Waves-per-SIMD targets of the angular kernel variants (schedule.variant = 1).
constexpr int kAltWavesGrad = 3, kAltWavesNll = 6;

static ipx_status launch_eval(int model, bool grad, unsigned grid, const SegInfo* segs, const TileRef* tiles,
                              int64_t n_tiles, const void* consts, const unsigned char* active, int nb, double* out,
                              hipStream_t s, ipx_ctx* timer, int variant = 0) {
  int nacc = 1;
  {
    ipx_status st = timing_begin(timer, s);
    if (st != IPX_OK) return st;
  }
  if (model == 1) {
    nacc = grad ? kAccMass : 1;
    if (grad) hipLaunchKernelGGL((k_nll_batch<1, true>), dim3(grid), dim3(kThreads), 0, s, segs, tiles, n_tiles, (const MassConst*)consts, active);
    else hipLaunchKernelGGL((k_nll_batch<1, false>), dim3(grid), dim3(kThreads), 0, s, segs, tiles, n_tiles, (const MassConst*)consts, active);
  } else if (model == 2) {
    nacc = grad ? kAccMassTime : 1;
    if (grad) hipLaunchKernelGGL((k_nll_batch<2, true>), dim3(grid), dim3(kThreads), 0, s, segs, tiles, n_tiles, (const MassTimeConst*)consts, active);
    else hipLaunchKernelGGL((k_nll_batch<2, false>), dim3(grid), dim3(kThreads), 0, s, segs, tiles, n_tiles, (const MassTimeConst*)consts, active);
  } else if (model == 3) {
    nacc = grad ? kAccAngTime : 1;
    const AngTimeConst* k3 = (const AngTimeConst*)consts;
    if (grad && variant == 1) hipLaunchKernelGGL((k_angtime_batch<true, false, kAltWavesGrad>), dim3(grid), dim3(kThreads), 0, s, segs, tiles, n_tiles, k3, active);
    else if (grad) hipLaunchKernelGGL((k_angtime_batch<true>), dim3(grid), dim3(kThreads), 0, s, segs, tiles, n_tiles, k3, active);
    else if (variant == 1) hipLaunchKernelGGL((k_angtime_batch<false, false, kAltWavesNll>), dim3(grid), dim3(kThreads), 0, s, segs, tiles, n_tiles, k3, active);
    else hipLaunchKernelGGL((k_angtime_batch<false>), dim3(grid), dim3(kThreads), 0, s, segs, tiles, n_tiles, k3, active);
  } else {
    nacc = grad ? kAccAngTime : 1;
    if (grad) hipLaunchKernelGGL((k_angtime_batch<true, true>), dim3(grid), dim3(kThreads), 0, s, segs, tiles, n_tiles, (const AngTimeConst*)consts, active);
    else hipLaunchKernelGGL((k_angtime_batch<false, true>), dim3(grid), dim3(kThreads), 0, s, segs, tiles, n_tiles, (const AngTimeConst*)consts, active);
  }
  HIP_TRY(hipGetLastError());
  {
    ipx_status st = timing_end(timer, s);
    if (st != IPX_OK) return st;
  }
  hipLaunchKernelGGL(k_reduce_batch, dim3(nacc, nb), dim3(kThreads), 0, s, segs, active, out);
  HIP_TRY(hipGetLastError());
  return IPX_OK;
}

// Stream operations of one (batched) evaluation.  The kernels read the
// hoisted constants and active flags from pinned host memory (written by the
// host before the launch; the few hundred bytes are cached on the device after
// the first workgroup's read) and the reductions write the results into pinned
// host memory (visible once the stream has synchronised), so an evaluation
// needs no copies.
static ipx_status enqueue_batch(ipx_plan* p, bool grad, hipStream_t s, ipx_ctx* timer) {
  const int64_t wg = p->sched.workgroups > 0 ? std::min<int64_t>(p->sched.workgroups, p->n_tiles) : p->n_tiles;
  const unsigned grid = (unsigned)std::max<int64_t>(1, wg);
  return launch_eval(p->model, grad, grid, p->d_segs, p->d_tiles, p->n_tiles, p->d_consts, p->d_active, p->nb,
                     p->h_out_dev, s, timer, p->sched.variant);
}

extern "C" ipx_status nll_eval_batch(ipx_ctx* ctx, ipx_plan* p, const double* theta, const unsigned char* active,
                                     double* nll, double* grad, void* stream) {
  if (!ctx || !p || !theta || !nll) return fail(IPX_EINVAL, "nll_eval_batch: NULL argument");
  if (p->ctx != ctx) return fail(IPX_EINVAL, "nll_eval_batch: plan belongs to another context");
  HIP_TRY(hipSetDevice(ctx->device));
  const int model = p->model, nb = p->nb, np = kNParams[model];
  std::vector<MassHoist> h1;
  std::vector<MassTimeHoist> h2;
  if (model == 1) h1.resize(nb);
  else if (model == 2) h2.resize(nb);
  else if ((int)p->h3.size() != nb) p->h3.resize(nb);
  std::vector<AngTimeHoist>& h3 = p->h3;
  int n_active = 0;
  for (int j = 0; j < nb; ++j) {
    const double* th = theta + (size_t)j * np;
    bool on = active ? active[j] != 0 : true;
    if (on && (!theta_valid(model, th) || (grad && !theta_grad_valid(model, th)))) {
      on = false;
      nll[j] = std::numeric_limits<double>::infinity();
      if (grad)
        for (int i = 0; i < np; ++i) grad[(size_t)j * np + i] = std::numeric_limits<double>::quiet_NaN();
    }
    p->h_active[j] = on ? 1 : 0;
    if (!on) continue;
    ++n_active;
    char* dst = (char*)p->h_consts + (size_t)j * p->const_size;
    if (model == 1) { h1[j] = hoist_mass(th); std::memcpy(dst, &h1[j].k, sizeof(MassConst)); }
    else if (model == 2) { h2[j] = hoist_masstime(th); std::memcpy(dst, &h2[j].k, sizeof(MassTimeConst)); }
    else { hoist_angtime(th, p->ds[j]->ang, h3[j]); std::memcpy(dst, &h3[j].k, sizeof(AngTimeConst)); }
  }
  if (n_active > 0) {
    hipStream_t s = stream ? (hipStream_t)stream : ctx->stream;
    const int mode = grad ? 1 : 0;
    if (!p->sched.graph) {
      ipx_status st = enqueue_batch(p, grad != nullptr, s, nullptr);
      if (st != IPX_OK) return st;
    } else if (!p->exec[mode]) {
      hipGraph_t g = nullptr;
      HIP_TRY(hipStreamBeginCapture(ctx->stream, hipStreamCaptureModeThreadLocal));
      ipx_status st = enqueue_batch(p, grad != nullptr, ctx->stream, nullptr);
      hipError_t e = hipStreamEndCapture(ctx->stream, &g);
      if (st != IPX_OK) {
        if (g) (void)hipGraphDestroy(g);
        return st;
      }
      if (e != hipSuccess) return fail(IPX_EDEVICE, "nll_eval_batch: graph capture failed: %s", hipGetErrorString(e));
      e = hipGraphInstantiate(&p->exec[mode], g, nullptr, nullptr, 0);
      (void)hipGraphDestroy(g);
      if (e != hipSuccess) {
        p->exec[mode] = nullptr;
        return fail(IPX_EDEVICE, "nll_eval_batch: graph instantiation failed: %s", hipGetErrorString(e));
      }
    }
    if (p->sched.graph) HIP_TRY(hipGraphLaunch(p->exec[mode], s));
    // the derivative tables of the angular coefficients serve only the
    // gradient's Jacobian: computed while the kernels run
    if (angular_model(model) && grad)
      for (int j = 0; j < nb; ++j)
        if (p->h_active[j]) angtime_derivatives(theta + (size_t)j * np, h3[j]);
    HIP_TRY(hipStreamSynchronize(s));
  }
  ipx_status result = IPX_OK;
  for (int j = 0; j < nb; ++j) {
    if (!p->h_active[j]) {
      if (!(active ? active[j] != 0 : true)) continue;
      result = IPX_EDOMAIN;
      continue;
    }
    const double* a = p->h_out + (size_t)j * kAccMax;
    double* g = grad ? grad + (size_t)j * np : nullptr;
    if (!std::isfinite(a[0])) {
      nll[j] = std::numeric_limits<double>::infinity();
      if (g)
        for (int i = 0; i < np; ++i) g[i] = std::numeric_limits<double>::quiet_NaN();
      result = IPX_EDOMAIN;
      continue;
    }
    nll[j] = -a[0];
    if (g) {
      const double* th = theta + (size_t)j * np;
      if (model == 1) grad_mass(h1[j], th, a, g);
      else if (model == 2) grad_masstime(h2[j], th, a, g);
      else grad_angtime(h3[j], th, a, g);
    }
  }
  if (result != IPX_OK) return fail(result, "nll_eval_batch: some entries are outside the domain or non-finite");
  return IPX_OK;
}

extern "C" ipx_status ipx_plan_set_schedule(ipx_plan* p, const ipx_schedule* sc) {
  if (!p || !sc) return fail(IPX_EINVAL, "ipx_plan_set_schedule: NULL argument");
  if (sc->workgroups < 0) return fail(IPX_EINVAL, "ipx_plan_set_schedule: workgroups %d < 0", sc->workgroups);
  if (sc->order < 0 || sc->order > 1) return fail(IPX_EINVAL, "ipx_plan_set_schedule: unknown order %d", sc->order);
  if (sc->graph < 0 || sc->graph > 1) return fail(IPX_EINVAL, "ipx_plan_set_schedule: graph must be 0 or 1");
  if (sc->variant < 0 || sc->variant > (p->model == 3 ? 1 : 0))
    return fail(IPX_EINVAL, "ipx_plan_set_schedule: kernel variant %d for model %d", sc->variant, p->model);
  HIP_TRY(hipSetDevice(p->ctx->device));
  HIP_TRY(hipStreamSynchronize(p->ctx->stream));
  if (sc->order != p->sched.order) {
    const std::vector<TileRef> tiles = tile_table(p, sc->order);
    if (!tiles.empty())
      HIP_TRY(hipMemcpy(p->d_tiles, tiles.data(), tiles.size() * sizeof(TileRef), hipMemcpyHostToDevice));
  }
  p->sched = *sc;
  // the captured graphs hold the old launch dimensions
  for (int m = 0; m < 2; ++m)
    if (p->exec[m]) {
      (void)hipGraphExecDestroy(p->exec[m]);
      p->exec[m] = nullptr;
    }
  return IPX_OK;
}

extern "C" ipx_status ipx_plan_get_schedule(const ipx_plan* p, ipx_schedule* out) {
  if (!p || !out) return fail(IPX_EINVAL, "ipx_plan_get_schedule: NULL argument");
  *out = p->sched;
  return IPX_OK;
}

extern "C" ipx_status ipx_plan_autotune(ipx_ctx* ctx, ipx_plan* p, const double* theta, int grad, int reps,
                                        ipx_schedule* best, double* best_us, ipx_tune_entry* table, int* ntable) {
  if (!ctx || !p || !theta || !best) return fail(IPX_EINVAL, "ipx_plan_autotune: NULL argument");
  if (p->ctx != ctx) return fail(IPX_EINVAL, "ipx_plan_autotune: plan belongs to another context");
  if (reps < 1) return fail(IPX_EINVAL, "ipx_plan_autotune: reps %d < 1", reps);
  const int np = kNParams[p->model];
  // candidates: one workgroup per tile, or a grid of 8 / 16 workgroups per
  // compute unit striding over the tiles; tiles by segment or interleaved;
  // replayed as a graph or launched directly
  const int cu = std::max(1, ctx->n_cu);
  std::vector<ipx_schedule> cand;
  for (int variant = 0; variant <= (p->model == 3 ? 1 : 0); ++variant)
    for (int graph = 1; graph >= 0; --graph)
      for (int order = 0; order <= (p->nb > 1 ? 1 : 0); ++order)
        for (int wg : {0, 16 * cu, 8 * cu}) cand.push_back(ipx_schedule{wg, order, graph, variant});
  std::vector<double> nll(p->nb), g(grad ? (size_t)p->nb * np : 0);
  // rounds over all candidates (so that clock drift does not favour one):
  // in each, a candidate is set, evaluated once untimed (graph capture, first
  // touch) and once timed; a candidate's time is its median over the rounds
  std::vector<std::vector<double>> times(cand.size());
  for (int r = 0; r < reps; ++r)
    for (size_t c = 0; c < cand.size(); ++c) {
      ipx_status st = ipx_plan_set_schedule(p, &cand[c]);
      if (st != IPX_OK) return st;
      for (int k = 0; k < 2; ++k) {
        const auto t0 = std::chrono::steady_clock::now();
        st = nll_eval_batch(ctx, p, theta, nullptr, nll.data(), grad ? g.data() : nullptr, nullptr);
        const auto t1 = std::chrono::steady_clock::now();
        if (st != IPX_OK && st != IPX_EDOMAIN) return st;
        if (k == 1) times[c].push_back(std::chrono::duration<double, std::micro>(t1 - t0).count());
      }
    }
  double best_t = std::numeric_limits<double>::infinity();
  ipx_schedule best_s = p->sched;
  int filled = 0;
  for (size_t c = 0; c < cand.size(); ++c) {
    std::sort(times[c].begin(), times[c].end());
    const double med = times[c][times[c].size() / 2];
    if (table && ntable && filled < *ntable) table[filled++] = ipx_tune_entry{cand[c], med};
    if (med < best_t) {
      best_t = med;
      best_s = cand[c];
    }
  }
  if (ntable) *ntable = filled;
  ipx_status st = ipx_plan_set_schedule(p, &best_s);
  if (st != IPX_OK) return st;
  *best = best_s;
  if (best_us) *best_us = best_t;
  return IPX_OK;
}

// ---------------------------------------------------------------------------
// Served likelihood (persistent kernel + host-visible mailbox)
// ---------------------------------------------------------------------------
struct ServeReq {
  uint64_t ticket = 0;
  ipx_dataset* ds = nullptr;
  int model = 0, grad = 0, np = 0;
  double theta[12];
  MassHoist h1;
  MassTimeHoist h2;
  AngTimeHoist h3;
  int slot = -1;
  uint64_t seq = 0;
  size_t off = 0, bytes = 0;
  std::chrono::steady_clock::time_point t_submit, t_done;
  bool done = false;
  ipx_result res;
};

struct ipx_server {
  ipx_ctx* ctx = nullptr;
  ipx_server_cfg cfg;
  hipStream_t stream = nullptr;
  hipEvent_t kernel_done = nullptr;
  bool kernel_launched = false;
  ServeShared* hs = nullptr;     // fine-grained host memory
  ServeShared* hs_dev = nullptr; // its device-side address
  ServeCtl* ctl = nullptr;
  ServeDesc* dd = nullptr;
  ServeSlot* st = nullptr;
  char* pool = nullptr;
  std::map<size_t, size_t> free_list;  // offset -> size
  std::mutex mu;
  std::condition_variable cv;
  std::thread worker;
  bool stopping = false;
  std::string worker_error;
  uint64_t next_ticket = 1;
  std::vector<uint64_t> slot_seq;      // last sequence number per slot
  std::vector<ServeReq*> slot_req;     // request in the slot (nullptr = free)
  std::deque<ServeReq*> pending;
  std::atomic<int> n_pending{0};       // pending.size(), readable without mu
  std::map<uint64_t, ServeReq*> reqs;
  ipx_server_stats stats{};
  int draining = 0;                    // ipx_server_drain calls in progress (submissions refused)
  bool closed = false;                 // ipx_server_stop has drained: waiters return, nothing new starts
  std::atomic<int> users{0};           // client calls inside the server (stop frees it only at 0)
};

// Counts a client call as inside the server for its whole duration, so that
// ipx_server_stop frees the server only after such calls have returned.
struct ServerUse {
  ipx_server* S;
  explicit ServerUse(ipx_server* s) : S(s) { S->users.fetch_add(1, std::memory_order_acq_rel); }
  ~ServerUse() { S->users.fetch_sub(1, std::memory_order_acq_rel); }
};

static bool pool_alloc(ipx_server* S, size_t bytes, size_t* off) {
  for (auto it = S->free_list.begin(); it != S->free_list.end(); ++it) {
    if (it->second >= bytes) {
      *off = it->first;
      const size_t rest = it->second - bytes;
      const size_t roff = it->first + bytes;
      S->free_list.erase(it);
      if (rest) S->free_list[roff] = rest;
      return true;
    }
  }
  return false;
}

static void pool_free(ipx_server* S, size_t off, size_t bytes) {
  auto it = S->free_list.emplace(off, bytes).first;
  auto nx = std::next(it);
  if (nx != S->free_list.end() && it->first + it->second == nx->first) {
    it->second += nx->second;
    S->free_list.erase(nx);
  }
  if (it != S->free_list.begin()) {
    auto pv = std::prev(it);
    if (pv->first + pv->second == it->first) {
      pv->second += it->second;
      S->free_list.erase(it);
    }
  }
}

static size_t align256(size_t b) { return (b + 255) / 256 * 256; }

static int serve_nacc(int model, int grad) { return nacc_of(model, grad != 0); }

static size_t request_bytes(const ipx_dataset* d, int grad) {
  return align256((size_t)std::max<int64_t>(1, d->n_tiles) * serve_nacc(d->model, grad) * sizeof(double));
}

// Fill the descriptor of a request in its slot and publish it.
static void serve_publish(ipx_server* S, ServeReq* r) {
  ServeDesc& D = S->hs->desc[r->slot];
  std::memset(&D, 0, sizeof D);
  const ipx_dataset* d = r->ds;
  D.model = r->model;
  D.grad = r->grad;
  D.items = (int)d->n_tiles;
  D.nacc = serve_nacc(r->model, r->grad);
  D.seg.cols = cols_of(d);
  D.seg.partials = (double*)(S->pool + r->off);
  D.seg.n_tiles = d->n_tiles;
  if (r->model == 1) D.k.m1 = r->h1.k;
  else if (r->model == 2) D.k.m2 = r->h2.k;
  else D.k.m3 = r->h3.k;
  r->seq = ++S->slot_seq[r->slot];
  D.seq = r->seq;
  __atomic_store_n(&S->hs->mail[r->slot], (unsigned long long)r->seq, __ATOMIC_RELEASE);
  __atomic_fetch_add(&S->hs->gen, 1ull, __ATOMIC_RELEASE);
}

static void serve_finish(ipx_server* S, ServeReq* r, int status, const double* a) {
  r->t_done = std::chrono::steady_clock::now();
  r->res.latency_us = std::chrono::duration<double, std::micro>(r->t_done - r->t_submit).count();
  r->res.np = r->np;
  r->res.status = status;
  r->res.nll = std::numeric_limits<double>::quiet_NaN();
  if (status == IPX_OK) {
    if (!std::isfinite(a[0])) {
      r->res.status = IPX_EDOMAIN;
      r->res.nll = std::numeric_limits<double>::infinity();
      for (int i = 0; i < r->np; ++i) r->res.grad[i] = std::numeric_limits<double>::quiet_NaN();
    } else {
      r->res.nll = -a[0];
      if (r->grad) {
        if (r->model == 1) grad_mass(r->h1, r->theta, a, r->res.grad);
        else if (r->model == 2) grad_masstime(r->h2, r->theta, a, r->res.grad);
        else grad_angtime(r->h3, r->theta, a, r->res.grad);
      }
    }
  }
  r->done = true;
}

static bool serve_kernel_live(ipx_server* S) {
  if (!S->kernel_launched) return false;
  return hipEventQuery(S->kernel_done) == hipErrorNotReady;
}

// The host side of the server.  Only this thread writes slot_req, so it reads
// it without the lock: while requests are in flight it polls their completion
// words lock-free and takes the lock only when a request has completed, one
// is waiting for a slot, or every 50 us (kernel liveness, stop); clients
// submitting or waiting are never held off by the polling.
static void serve_worker(ipx_server* S) {
  (void)hipSetDevice(S->ctx->device);
  const int nslots = S->cfg.slots;
  std::unique_lock<std::mutex> lk(S->mu);
  auto last_progress = std::chrono::steady_clock::now();
  auto last_pass = last_progress;
  for (;;) {
    last_pass = std::chrono::steady_clock::now();
    bool progress = false;
    int busy = 0;
    for (int s = 0; s < nslots; ++s) {
      ServeReq* r = S->slot_req[s];
      if (!r) continue;
      if (__atomic_load_n(&S->hs->fin[s], __ATOMIC_ACQUIRE) == r->seq) {
        serve_finish(S, r, IPX_OK, S->hs->out[s]);
        ++S->stats.completed;
        pool_free(S, r->off, r->bytes);
        S->slot_req[s] = nullptr;
        progress = true;
      } else {
        ++busy;
      }
    }
    while (!S->pending.empty()) {
      ServeReq* r = S->pending.front();
      int slot = -1;
      for (int s = 0; s < nslots; ++s)
        if (!S->slot_req[s]) {
          slot = s;
          break;
        }
      if (slot < 0) break;
      size_t off = 0;
      if (!pool_alloc(S, r->bytes, &off)) break;  // admission by footprint: wait for memory
      S->pending.pop_front();
      S->n_pending.fetch_sub(1, std::memory_order_relaxed);
      ++S->stats.published;
      r->slot = slot;
      r->off = off;
      S->slot_req[slot] = r;
      serve_publish(S, r);
      ++busy;
      progress = true;
    }
    if (busy > 0 && !serve_kernel_live(S)) {
      // workgroup 0 polls, the others work: the poller leaves once `live` is 0
      hipError_t e = hipMemsetD32Async((hipDeviceptr_t)&S->ctl->live, S->cfg.workgroups - 1, 1, S->stream);
      if (e == hipSuccess) e = hipMemsetD32Async((hipDeviceptr_t)&S->ctl->quit, 0, 1, S->stream);
      if (e == hipSuccess) {
        hipLaunchKernelGGL(k_serve, dim3((unsigned)S->cfg.workgroups), dim3(kThreads), 0, S->stream, S->hs_dev,
                           S->ctl, S->dd, S->st, nslots, S->cfg.idle_iterations, S->cfg.policy);
        e = hipGetLastError();
      }
      if (e == hipSuccess) e = hipEventRecord(S->kernel_done, S->stream);
      S->kernel_launched = true;
      ++S->stats.launches;
      if (e != hipSuccess) {
        // the device loop cannot run: every request ends with a device error
        S->worker_error = hipGetErrorString(e);
        for (int s = 0; s < nslots; ++s)
          if (S->slot_req[s]) {
            serve_finish(S, S->slot_req[s], IPX_EDEVICE, nullptr);
            pool_free(S, S->slot_req[s]->off, S->slot_req[s]->bytes);
            S->slot_req[s] = nullptr;
          }
        for (ServeReq* r : S->pending) serve_finish(S, r, IPX_EDEVICE, nullptr);
        S->pending.clear();
        S->n_pending.store(0, std::memory_order_relaxed);
        S->kernel_launched = false;
        busy = 0;
        progress = true;
      }
    }
    const auto now = std::chrono::steady_clock::now();
    if (progress) {
      S->cv.notify_all();
      last_progress = now;
    }
    if (S->stopping && busy == 0 && S->pending.empty()) break;
    if (S->stopping && now - last_progress > std::chrono::seconds(10)) {
      // nothing has completed for 10 s while stopping: give the rest up
      for (int s = 0; s < nslots; ++s)
        if (S->slot_req[s]) {
          serve_finish(S, S->slot_req[s], IPX_ETIMEOUT, nullptr);
          S->slot_req[s] = nullptr;
        }
      for (ServeReq* r : S->pending) serve_finish(S, r, IPX_ETIMEOUT, nullptr);
      S->pending.clear();
      S->n_pending.store(0, std::memory_order_relaxed);
      break;
    }
    if (busy == 0 && S->pending.empty()) {
      S->cv.wait_for(lk, std::chrono::milliseconds(1));  // idle: ipx_submit notifies
    } else {
      // requests in flight: poll the completion words, without the lock and
      // without a timed sleep (a timed wait rounds up to the scheduler's timer
      // slack, tens of us), until something needs the locked pass
      lk.unlock();
      for (;;) {
        std::this_thread::yield();
        bool done = false;
        int used = 0;
        for (int s = 0; s < nslots && !done; ++s) {
          const ServeReq* r = S->slot_req[s];
          if (!r) continue;
          ++used;
          done = __atomic_load_n(&S->hs->fin[s], __ATOMIC_ACQUIRE) == r->seq;
        }
        if (done || (S->n_pending.load(std::memory_order_relaxed) > 0 && used < nslots) ||
            std::chrono::steady_clock::now() - last_pass > std::chrono::microseconds(50))
          break;
      }
      lk.lock();
    }
  }
  S->cv.notify_all();
}

extern "C" ipx_status ipx_server_start(ipx_ctx* ctx, const ipx_server_cfg* cfg, ipx_server** out) {
  if (!ctx || !out) return fail(IPX_EINVAL, "ipx_server_start: NULL argument");
  *out = nullptr;
  ipx_server_cfg c{};
  if (cfg) c = *cfg;
  if (c.slots <= 0) c.slots = 32;
  if (c.slots > kServeMaxSlots) return fail(IPX_EINVAL, "ipx_server_start: at most %d slots", kServeMaxSlots);
  if (c.scratch_bytes == 0) c.scratch_bytes = (size_t)1 << 31;
  if (c.workgroups == 0) c.workgroups = 3 * std::max(1, ctx->n_cu);
  if (c.policy != kServeOldestFirst && c.policy != kServeSpread && c.policy != kServeFewestFirst)
    return fail(IPX_EINVAL, "ipx_server_start: unknown claim policy %d", c.policy);
  if (c.workgroups < 2) return fail(IPX_EINVAL, "ipx_server_start: at least 2 workgroups (one polls the host)");
  if (c.idle_iterations <= 0) c.idle_iterations = 20000;
  HIP_TRY(hipSetDevice(ctx->device));
  ipx_server* S = new (std::nothrow) ipx_server();
  if (!S) return fail(IPX_ENOMEM, "ipx_server_start: host allocation failed");
  S->ctx = ctx;
  S->cfg = c;
  S->slot_seq.assign(c.slots, 0);
  S->slot_req.assign(c.slots, nullptr);
  hipError_t e = hipStreamCreateWithFlags(&S->stream, hipStreamNonBlocking);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&S->kernel_done, hipEventDisableTiming);
  if (e == hipSuccess) e = hipHostMalloc((void**)&S->hs, sizeof(ServeShared), hipHostMallocCoherent | hipHostMallocMapped);
  if (e == hipSuccess) e = hipMalloc(&S->dd, kServeMaxSlots * sizeof(ServeDesc));
  if (e == hipSuccess) e = hipMalloc(&S->st, kServeMaxSlots * sizeof(ServeSlot));
  if (e == hipSuccess) e = hipMalloc(&S->ctl, sizeof(ServeCtl));
  if (e == hipSuccess) e = hipMemset(S->ctl, 0, sizeof(ServeCtl));
  if (e == hipSuccess) e = hipHostGetDevicePointer((void**)&S->hs_dev, S->hs, 0);
  if (e == hipSuccess) e = hipMalloc(&S->pool, c.scratch_bytes);
  if (e == hipSuccess) e = hipMemset(S->st, 0, kServeMaxSlots * sizeof(ServeSlot));
  if (e == hipSuccess) e = hipDeviceSynchronize();
  if (e != hipSuccess) {
    if (S->pool) (void)hipFree(S->pool);
    if (S->st) (void)hipFree(S->st);
    if (S->ctl) (void)hipFree(S->ctl);
    if (S->dd) (void)hipFree(S->dd);
    if (S->hs) (void)hipHostFree(S->hs);
    if (S->kernel_done) (void)hipEventDestroy(S->kernel_done);
    if (S->stream) (void)hipStreamDestroy(S->stream);
    delete S;
    return fail(IPX_ENOMEM, "ipx_server_start: allocation failed: %s", hipGetErrorString(e));
  }
  std::memset(S->hs, 0, sizeof(ServeShared));
  S->free_list[0] = c.scratch_bytes;
  S->worker = std::thread(serve_worker, S);
  *out = S;
  return IPX_OK;
}

extern "C" ipx_status ipx_submit(ipx_server* S, const ipx_request* q, uint64_t* ticket) {
  if (!S || !q || !ticket || !q->ds || !q->theta) return fail(IPX_EINVAL, "ipx_submit: NULL argument");
  ServerUse use(S);
  ipx_dataset* d = const_cast<ipx_dataset*>(q->ds);
  const int model = d->model, np = kNParams[model];
  if (model == kModelIpatia) return fail(IPX_EINVAL, "ipx_submit: the Ipatia model is evaluated by nll_eval only");
  if (q->np != np) return fail(IPX_EINVAL, "ipx_submit: model %d takes %d parameters", model, np);
  ServeReq* r = new (std::nothrow) ServeReq();
  if (!r) return fail(IPX_ENOMEM, "ipx_submit: host allocation failed");
  r->ds = d;
  r->model = model;
  r->grad = q->want_grad ? 1 : 0;
  r->np = np;
  std::memcpy(r->theta, q->theta, np * sizeof(double));
  r->t_submit = std::chrono::steady_clock::now();
  r->bytes = request_bytes(d, r->grad);
  // hoisting outside the server's lock (the derivative table only for a
  // gradient request)
  const bool valid = theta_valid(model, r->theta) && (!r->grad || theta_grad_valid(model, r->theta));
  if (valid) {
    if (model == 1) r->h1 = hoist_mass(r->theta);
    else if (model == 2) r->h2 = hoist_masstime(r->theta);
    else {
      hoist_angtime(r->theta, d->ang, r->h3);
      if (r->grad) angtime_derivatives(r->theta, r->h3);
    }
  }
  std::lock_guard<std::mutex> lk(S->mu);
  if (S->stopping || S->closed) {
    delete r;
    return fail(IPX_EBUSY, "ipx_submit: server is stopping");
  }
  if (S->draining > 0) {
    delete r;
    return fail(IPX_EBUSY, "ipx_submit: server is draining");
  }
  if (r->bytes > S->cfg.scratch_bytes) {
    delete r;
    return fail(IPX_ENOMEM, "ipx_submit: request needs %zu scratch bytes, budget %zu", r->bytes, S->cfg.scratch_bytes);
  }
  if (S->cfg.max_pending > 0 && (int)S->pending.size() >= S->cfg.max_pending) {
    delete r;
    return fail(IPX_EBUSY, "ipx_submit: queue full");
  }
  r->ticket = S->next_ticket++;
  S->reqs[r->ticket] = r;
  *ticket = r->ticket;
  if (!valid) {
    serve_finish(S, r, IPX_EDOMAIN, nullptr);
    r->res.nll = std::numeric_limits<double>::infinity();
    for (int i = 0; i < np; ++i) r->res.grad[i] = std::numeric_limits<double>::quiet_NaN();
    S->cv.notify_all();
    return IPX_OK;
  }
  if (d->n == 0) {  // nothing to evaluate: the empty sum
    double zeros[kAccMax] = {};
    serve_finish(S, r, IPX_OK, zeros);
    S->cv.notify_all();
    return IPX_OK;
  }
  S->pending.push_back(r);
  S->n_pending.fetch_add(1, std::memory_order_relaxed);
  S->cv.notify_all();
  return IPX_OK;
}

static ipx_status take_result(ipx_server* S, std::map<uint64_t, ServeReq*>::iterator it, ipx_result* out) {
  ServeReq* r = it->second;
  if (out) *out = r->res;
  S->reqs.erase(it);
  const int st = r->res.status;
  delete r;
  return st == IPX_OK ? IPX_OK : fail((ipx_status)st, "request finished with status %d", st);
}

extern "C" ipx_status ipx_poll(ipx_server* S, uint64_t ticket, ipx_result* out) {
  if (!S) return fail(IPX_EINVAL, "ipx_poll: NULL server");
  ServerUse use(S);
  std::lock_guard<std::mutex> lk(S->mu);
  auto it = S->reqs.find(ticket);
  if (it == S->reqs.end()) return fail(IPX_ENOTFOUND, "ipx_poll: unknown ticket %llu", (unsigned long long)ticket);
  if (!it->second->done) return IPX_EBUSY;
  return take_result(S, it, out);
}

extern "C" ipx_status ipx_wait(ipx_server* S, uint64_t ticket, int64_t timeout_ns, ipx_result* out) {
  if (!S) return fail(IPX_EINVAL, "ipx_wait: NULL server");
  ServerUse use(S);
  std::unique_lock<std::mutex> lk(S->mu);
  auto it = S->reqs.find(ticket);
  if (it == S->reqs.end()) return fail(IPX_ENOTFOUND, "ipx_wait: unknown ticket %llu", (unsigned long long)ticket);
  ServeReq* r = it->second;
  const auto deadline = std::chrono::steady_clock::now() + std::chrono::nanoseconds(timeout_ns < 0 ? (int64_t)1 << 62 : timeout_ns);
  while (!r->done) {
    if (S->closed) return fail(IPX_ENOTFOUND, "ipx_wait: server stopped before ticket %llu finished", (unsigned long long)ticket);
    if (S->cv.wait_until(lk, deadline) == std::cv_status::timeout && !r->done)
      return fail(IPX_ETIMEOUT, "ipx_wait: ticket %llu not done", (unsigned long long)ticket);
  }
  return take_result(S, S->reqs.find(ticket), out);
}

extern "C" ipx_status ipx_cancel(ipx_server* S, uint64_t ticket) {
  if (!S) return fail(IPX_EINVAL, "ipx_cancel: NULL server");
  ServerUse use(S);
  std::lock_guard<std::mutex> lk(S->mu);
  auto it = S->reqs.find(ticket);
  if (it == S->reqs.end()) return fail(IPX_ENOTFOUND, "ipx_cancel: unknown ticket %llu", (unsigned long long)ticket);
  ServeReq* r = it->second;
  auto p = std::find(S->pending.begin(), S->pending.end(), r);
  if (r->done || p == S->pending.end())
    return fail(IPX_EBUSY, "ipx_cancel: ticket %llu is %s", (unsigned long long)ticket,
                r->done ? "finished" : "on the device");
  // still waiting: it holds no slot and no scratch
  S->pending.erase(p);
  S->n_pending.store((int)S->pending.size(), std::memory_order_relaxed);
  r->res.status = IPX_ECANCELED;
  r->res.np = r->np;
  r->res.nll = std::numeric_limits<double>::infinity();
  r->t_done = std::chrono::steady_clock::now();
  r->res.latency_us = std::chrono::duration<double, std::micro>(r->t_done - r->t_submit).count();
  r->done = true;
  ++S->stats.cancelled;
  S->cv.notify_all();
  return IPX_OK;
}

extern "C" ipx_status ipx_server_stats_read(ipx_server* S, ipx_server_stats* out) {
  if (!S || !out) return fail(IPX_EINVAL, "ipx_server_stats_read: NULL argument");
  ServerUse use(S);
  std::lock_guard<std::mutex> lk(S->mu);
  *out = S->stats;
  out->pending = S->pending.size();
  out->in_flight = 0;
  for (ServeReq* r : S->slot_req) out->in_flight += r != nullptr;
  return IPX_OK;
}

// True when no request is waiting for a slot or in a device slot (S->mu held;
// slot_req is written only under the lock).
static bool server_idle(const ipx_server* S) {
  if (!S->pending.empty()) return false;
  for (const ServeReq* r : S->slot_req)
    if (r) return false;
  return true;
}

extern "C" ipx_status ipx_server_drain(ipx_server* S) {
  if (!S) return fail(IPX_EINVAL, "ipx_server_drain: NULL server");
  ServerUse use(S);
  std::unique_lock<std::mutex> lk(S->mu);
  if (S->stopping || S->closed) return fail(IPX_EBUSY, "ipx_server_drain: server is stopping");
  ++S->draining;
  // the host worker notifies after every completion and admission
  while (!server_idle(S)) S->cv.wait_for(lk, std::chrono::milliseconds(1));
  --S->draining;
  return IPX_OK;
}

extern "C" ipx_status ipx_server_stop(ipx_server* S) {
  if (!S) return fail(IPX_EINVAL, "ipx_server_stop: NULL server");
  {
    std::lock_guard<std::mutex> lk(S->mu);
    S->stopping = true;
    S->cv.notify_all();
  }
  if (S->worker.joinable()) S->worker.join();   // drains in-flight and pending requests
  __atomic_store_n(&S->hs->stop, 1ull, __ATOMIC_RELEASE);
  (void)hipSetDevice(S->ctx->device);
  hipError_t e = hipStreamSynchronize(S->stream);
  {
    // every request has finished: wake the clients blocked in ipx_wait (they
    // take their results) and let the calls inside the server return before
    // it is freed
    std::lock_guard<std::mutex> lk(S->mu);
    S->closed = true;
    S->cv.notify_all();
  }
  while (S->users.load(std::memory_order_acquire) > 0) {
    {
      std::lock_guard<std::mutex> lk(S->mu);
      S->cv.notify_all();
    }
    std::this_thread::yield();
  }
  for (auto& kv : S->reqs) delete kv.second;
  (void)hipFree(S->pool);
  (void)hipFree(S->st);
  (void)hipFree(S->ctl);
  (void)hipFree(S->dd);
  (void)hipHostFree(S->hs);
  (void)hipEventDestroy(S->kernel_done);
  (void)hipStreamDestroy(S->stream);
  const std::string werr = S->worker_error;
  delete S;
  if (e != hipSuccess) return fail(IPX_EDEVICE, "ipx_server_stop: %s", hipGetErrorString(e));
  if (!werr.empty()) return fail(IPX_EDEVICE, "ipx_server_stop: kernel launch failed: %s", werr.c_str());
  return IPX_OK;
}

// Per-call host state of one evaluation: the hoisted constants of the model
// in use and, for the angular gradient, the derivative table of the hoisting.
struct EvalHoist {
  MassHoist h1;
  MassTimeHoist h2;
  AngTimeHoist h3;
  const void* consts = nullptr;
  size_t bytes = 0;
};

// Domain check shared by the evaluation entry points: outside the model's
// domain (or the gradient's) the outputs are +inf / NaN and nothing runs.
static ipx_status check_theta(int model, const double* theta, int np, double* nll, double* grad) {
  if (theta_valid(model, theta) && (!grad || theta_grad_valid(model, theta))) return IPX_OK;
  *nll = std::numeric_limits<double>::infinity();
  if (grad)
    for (int i = 0; i < np; ++i) grad[i] = std::numeric_limits<double>::quiet_NaN();
  return fail(IPX_EDOMAIN, grad ? "parameters outside the gradient's domain of model %d"
                                : "parameters outside the domain of model %d", model);
}

static void hoist_eval(int model, const double* theta, const AngSettings& set, EvalHoist& h) {
  if (model == 1) { h.h1 = hoist_mass(theta); h.consts = &h.h1.k; h.bytes = sizeof h.h1.k; }
  else if (model == 2) { h.h2 = hoist_masstime(theta); h.consts = &h.h2.k; h.bytes = sizeof h.h2.k; }
  else { hoist_angtime(theta, set, h.h3); h.consts = &h.h3.k; h.bytes = sizeof h.h3.k; }
}

// NLL and gradient from the reduced totals a[] (a[0] = sum of w ln P).
static ipx_status finish_eval(int model, const EvalHoist& h, const double* theta, int np, const double* a,
                              double* nll, double* grad) {
  if (!std::isfinite(a[0])) {
    *nll = std::numeric_limits<double>::infinity();
    if (grad)
      for (int i = 0; i < np; ++i) grad[i] = std::numeric_limits<double>::quiet_NaN();
    return fail(IPX_EDOMAIN, "non-finite likelihood (an event has P <= 0 or a non-finite term)");
  }
  *nll = -a[0];
  if (grad) {
    if (model == 1) grad_mass(h.h1, theta, a, grad);
    else if (model == 2) grad_masstime(h.h2, theta, a, grad);
    else grad_angtime(h.h3, theta, a, grad);
  }
  return IPX_OK;
}

// out[c] = sum of part[c * nwg .. c * nwg + nwg) in the fixed order of
// reduce_component; grid (components).
static __global__ __launch_bounds__(kThreads) void k_reduce_parts(const double* __restrict__ part, int nwg,
                                                                  double* __restrict__ out) {
  const double t = reduce_component(part + (int64_t)blockIdx.x * nwg, nwg);
  if (threadIdx.x == 0) out[blockIdx.x] = t;
}

// ---------------------------------------------------------------------------
// Ipatia model (nll_eval only): grid pass -> 1/N_I, tile pass, tile reduction.
// The dataset's aux buffer: [constants | grid partials (64) | 1/N_I | total |
// tile partials (n_tiles)].
// ---------------------------------------------------------------------------
constexpr size_t kIpaConstBytes = (sizeof(IpatiaConst) + 255) / 256 * 256;
static double* ipa_part(ipx_dataset* d) { return (double*)((char*)d->aux + kIpaConstBytes); }
static double* ipa_inv(ipx_dataset* d) { return ipa_part(d) + kIpatiaGridWg; }
static double* ipa_total(ipx_dataset* d) { return ipa_inv(d) + 1; }
static double* ipa_tiles(ipx_dataset* d) { return ipa_inv(d) + 2; }

// Events per lane of the Ipatia event pass: one up to 2^19 events (four times
// the workgroups: a 10^5-event sample fills 391 of them instead of 98), the
// canonical four above (fewer tile partials; at 10^7 events one per lane was
// 9 % slower).
static int ipa_epl(const ipx_dataset* d) { return d->n <= (int64_t)1 << 19 ? 1 : kEventsPerLane; }
static int64_t ipa_ntiles(const ipx_dataset* d) {
  const int64_t t = (int64_t)kThreads * ipa_epl(d);
  return std::max<int64_t>(1, (d->n + t - 1) / t);
}

static __global__ __launch_bounds__(kThreads) void k_ipatia_tiles(EventCols cols, const IpatiaConst* __restrict__ kc,
                                                                  double* __restrict__ partials, int64_t n_tiles,
                                                                  int epl) {
  __shared__ RedBuf<1> red;
  const IpatiaConst& c = *kc;
  const double inv = *c.inv_norm;
  const int64_t tile = blockIdx.x;
  const int64_t base = tile * kThreads * epl;
  double acc[1] = {0.0};
#pragma unroll 1
  for (int e = 0; e < epl; ++e) {
    const unsigned j = threadIdx.x + (unsigned)e * kThreads;
    if (base + j < cols.n) {
      const double w = cols.w ? ldg(cols.w + base, j) : 1.0;
      event_ipatia(c, inv, ldg(cols.c[0] + base, j), w, acc);
    }
  }
  tile_store<1, false, 1>(acc, partials, tile, n_tiles, red);
}

static __global__ __launch_bounds__(kThreads) void k_event_logp_ipatia(EventCols cols,
                                                                       const IpatiaConst* __restrict__ kc,
                                                                       double* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (i >= cols.n) return;
  const IpatiaConst& c = *kc;
  double acc[1] = {0.0};
  event_ipatia(c, *c.inv_norm, cols.c[0][i], cols.w ? cols.w[i] : 1.0, acc);
  out[i] = acc[0];
}

// Hoists theta into the dataset's aux buffer and enqueues the grid passes.
static ipx_status ipatia_prepare(ipx_ctx* ctx, ipx_dataset* d, const double* theta, hipStream_t s) {
  IpatiaConst c;
  if (!hoist_ipatia(theta, c)) return fail(IPX_EDOMAIN, "parameters outside the domain of the Ipatia model");
  if (!d->aux) {
    const size_t bytes = kIpaConstBytes + (kIpatiaGridWg + 2 + (size_t)ipa_ntiles(d)) * sizeof(double);
    HIP_TRY(hipMalloc(&d->aux, bytes));
  }
  c.inv_norm = ipa_inv(d);
  HIP_TRY(hipMemcpyAsync(d->aux, &c, sizeof c, hipMemcpyHostToDevice, s));
  hipLaunchKernelGGL(k_ipatia_grid, dim3(kIpatiaGridWg), dim3(kThreads), 0, s, (const IpatiaConst*)d->aux, ipa_part(d));
  hipLaunchKernelGGL(k_ipatia_norm, dim3(1), dim3(kThreads), 0, s, (const IpatiaConst*)d->aux, ipa_part(d), ipa_inv(d));
  HIP_TRY(hipGetLastError());
  return IPX_OK;
}

static ipx_status run_ipatia(ipx_ctx* ctx, ipx_dataset* d, const double* theta, double* nll, double* grad,
                             void* stream) {
  if (grad) return fail(IPX_EINVAL, "the Ipatia model has no analytic gradient (nll_eval only)");
  HIP_TRY(hipSetDevice(ctx->device));
  hipStream_t s = stream ? (hipStream_t)stream : ctx->stream;
  ipx_status st = ipatia_prepare(ctx, d, theta, s);
  if (st != IPX_OK) {
    *nll = std::numeric_limits<double>::infinity();
    return st;
  }
  const int64_t nt = ipa_ntiles(d);
  st = timing_begin(ctx, s);
  if (st != IPX_OK) return st;
  hipLaunchKernelGGL(k_ipatia_tiles, dim3((unsigned)nt), dim3(kThreads), 0, s, cols_of(d), (const IpatiaConst*)d->aux,
                     ipa_tiles(d), nt, ipa_epl(d));
  HIP_TRY(hipGetLastError());
  st = timing_end(ctx, s);
  if (st != IPX_OK) return st;
  hipLaunchKernelGGL(k_reduce_parts, dim3(1), dim3(kThreads), 0, s, ipa_tiles(d), (int)nt, ipa_total(d));
  HIP_TRY(hipGetLastError());
  double a = 0.0;
  HIP_TRY(hipMemcpyAsync(&a, ipa_total(d), sizeof a, hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  if (!std::isfinite(a)) {
    *nll = std::numeric_limits<double>::infinity();
    return fail(IPX_EDOMAIN, "non-finite likelihood (an event has P <= 0 or a non-finite term)");
  }
  *nll = -a;
  return IPX_OK;
}

static ipx_status run(ipx_ctx* ctx, const ipx_dataset* dc, const double* theta, int np, double* nll,
                      double* grad, void* stream) {
  if (!ctx || !dc || !theta || !nll) return fail(IPX_EINVAL, "NULL argument");
  ipx_dataset* d = const_cast<ipx_dataset*>(dc);  // lazily created plan and scratch only
  const int model = d->model;
  if (np != kNParams[model]) return fail(IPX_EINVAL, "model %d takes %d parameters, got %d", model, kNParams[model], np);
  if (model == kModelIpatia) return run_ipatia(ctx, d, theta, nll, grad, stream);
  {
    ipx_status st = check_theta(model, theta, np, nll, grad);
    if (st != IPX_OK) return st;
  }
  HIP_TRY(hipSetDevice(ctx->device));
  if (!d->self) {
    ipx_dataset* one[1] = {d};
    ipx_status st = plan_create(ctx, 1, one, &d->self, false);
    if (st != IPX_OK) return st;
  }
  ipx_plan* p = d->self;
  hipStream_t s = stream ? (hipStream_t)stream : ctx->stream;
  EvalHoist h;
  hoist_eval(model, theta, d->ang, h);
  std::memcpy(p->h_consts, h.consts, h.bytes);
  p->h_active[0] = 1;
  ipx_status st = enqueue_batch(p, grad != nullptr, s, ctx);
  if (st != IPX_OK) return st;
  if (angular_model(model) && grad) angtime_derivatives(theta, h.h3);  // while the kernels run
  HIP_TRY(hipStreamSynchronize(s));
  return finish_eval(model, h, theta, np, p->h_out, nll, grad);
}

// ---------------------------------------------------------------------------
// Allocation-free evaluation (nll_eval_noalloc).  Its per-call scratch -- the
// one-segment record, the hoisted constants, the active flag, the reduced
// totals, the tile table and the tile partials -- lives in `scratch`, a
// file-scope device array of fixed size: every device the library runs on
// holds its own copy until the process ends.  Host code never names the array
// itself (on the host its name is not a device address): its device address is
// taken once per device, with that device current, when the first context is
// created there, and only that address is passed to copies and kernels.
// ---------------------------------------------------------------------------
constexpr int64_t kNoAllocMaxEvents = (int64_t)1 << 24;           // 16,777,216 events
constexpr int64_t kNoAllocMaxTiles = kNoAllocMaxEvents / kTile;   // 16,384 tiles
constexpr size_t kNaSeg = 0;                                      // SegInfo
constexpr size_t kNaConst = 256;                                  // constant block (<= 2 KiB)
constexpr size_t kNaActive = kNaConst + 2048;                     // one active flag
constexpr size_t kNaOut = kNaActive + 256;                        // kAccMax reduced totals
constexpr size_t kNaHead = kNaOut + 512;
constexpr size_t kNaTiles = kNaHead;                              // TileRef x max tiles
constexpr size_t kNaPartials = kNaTiles + (size_t)kNoAllocMaxTiles * sizeof(TileRef);
constexpr size_t kNoAllocBytes = kNaPartials + (size_t)kNoAllocMaxTiles * kAccMax * sizeof(double);  // ~6.9 MB
static_assert(sizeof(SegInfo) <= kNaConst - kNaSeg, "segment record");
static_assert(sizeof(MassConst) <= 2048 && sizeof(MassTimeConst) <= 2048 && sizeof(AngTimeConst) <= 2048,
              "constant block");
static_assert(kAccMax * sizeof(double) <= kNaHead - kNaOut, "totals");
static_assert(kNaTiles % 256 == 0 && kNaPartials % 256 == 0, "aligned regions");

static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];

constexpr int kMaxDevices = 64;
static std::mutex g_noalloc_mu[kMaxDevices];              // one call at a time per device
static std::atomic<unsigned char*> g_noalloc_ptr[kMaxDevices];

// Called with `device` current (ipx_create).
static ipx_status noalloc_setup(int device) {
  if (device >= kMaxDevices) return fail(IPX_EINVAL, "ipx_create: device %d beyond the %d supported", device, kMaxDevices);
  std::lock_guard<std::mutex> lk(g_noalloc_mu[device]);
  if (g_noalloc_ptr[device].load()) return IPX_OK;
  void* p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !p)
    return fail(IPX_EDEVICE, "ipx_create: hipGetSymbolAddress(scratch) failed: %s", hipGetErrorString(e));
  g_noalloc_ptr[device].store((unsigned char*)p);
  return IPX_OK;
}

__global__ void k_fill_tiles(TileRef* __restrict__ t, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) t[i] = TileRef{0, i};
}

// ---------------------------------------------------------------------------
// Bad events: the per-event contributions w_i ln P_i that are not finite (the
// NLL kernels only see their sum).  A diagnostic pass, not part of an
// evaluation: one count per workgroup, summed on the host.
// ---------------------------------------------------------------------------
template <int MODEL>
__global__ __launch_bounds__(kThreads) void k_count_bad(EventCols cols,
                                                        const typename ModelTraits<MODEL>::Const* __restrict__ k,
                                                        long long* __restrict__ counts) {
  __shared__ int wcount[kThreads / 64];
  int bad = 0;
  const int64_t stride = (int64_t)gridDim.x * kThreads;
  for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < cols.n; i += stride) {
    double acc[1] = {0.0};
    event<MODEL, false>(*k, cols, i, 0u, acc);
    bad += !isfinite(acc[0]);
  }
  for (int off = 32; off >= 1; off >>= 1) bad += __shfl_xor(bad, off, 64);
  if ((threadIdx.x & 63) == 0) wcount[threadIdx.x >> 6] = bad;
  __syncthreads();
  if (threadIdx.x == 0) counts[blockIdx.x] = (long long)wcount[0] + wcount[1] + wcount[2] + wcount[3];
}

template <bool TAG>
__global__ __launch_bounds__(kThreads) void k_count_bad_angtime(EventCols cols, const AngTimeConst* __restrict__ k,
                                                                long long* __restrict__ counts) {
  __shared__ int wcount[kThreads / 64];
  int bad = 0;
  const int64_t stride = (int64_t)gridDim.x * kThreads;
  for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < cols.n; i += stride) {
    double acc[1] = {0.0};
    const double w = cols.w ? cols.w[i] : 1.0;
    event_angtime<false, false, TAG>(*k, &k->C[0][0], cols.c[0][i], cols.c[1][i], cols.c[2][i], cols.c[3][i],
                                     cols.c[4][i], cols.c[5][i], w, acc, nullptr, TAG ? cols.c[6][i] : 1.0);
    bad += !isfinite(acc[0]);
  }
  for (int off = 32; off >= 1; off >>= 1) bad += __shfl_xor(bad, off, 64);
  if ((threadIdx.x & 63) == 0) wcount[threadIdx.x >> 6] = bad;
  __syncthreads();
  if (threadIdx.x == 0) counts[blockIdx.x] = (long long)wcount[0] + wcount[1] + wcount[2] + wcount[3];
}

// ---------------------------------------------------------------------------
// Per-event terms w_i ln P_i (the quantities the evaluation kernels sum), for
// inspection: one lane per event in storage order.  A wave's lanes hold 64
// consecutive events starting at a multiple of 64, as in the tile kernels, so
// the wave-uniform choices (which resolution corrections are evaluated, at
// what continued-fraction depth) are the tile kernels' own.
// ---------------------------------------------------------------------------
template <int MODEL>
__global__ __launch_bounds__(kThreads) void k_event_logp(EventCols cols, typename ModelTraits<MODEL>::Const k,
                                                         double* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (i >= cols.n) return;
  double acc[1] = {0.0};
  event<MODEL, false>(k, cols, i, 0u, acc);
  out[i] = acc[0];
}

template <bool TAG>
__global__ __launch_bounds__(kThreads) void k_event_logp_angtime(EventCols cols, AngTimeConst k,
                                                                 double* __restrict__ out) {
  __shared__ double sC[40];
  if (threadIdx.x < 40) sC[threadIdx.x] = (&k.C[0][0])[threadIdx.x];
  __syncthreads();
  const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (i >= cols.n) return;
  double acc[1] = {0.0};
  const double w = cols.w ? ldg(cols.w + i, 0u) : 1.0;
  event_angtime<false, false, TAG>(k, sC, ldg(cols.c[0] + i, 0u), ldg(cols.c[1] + i, 0u), ldg(cols.c[2] + i, 0u),
                                   ldg(cols.c[3] + i, 0u), ldg(cols.c[4] + i, 0u), ldg(cols.c[5] + i, 0u), w, acc,
                                   nullptr, TAG ? ldg(cols.c[6] + i, 0u) : 1.0);
  out[i] = acc[0];
}

extern "C" {

ipx_status ipx_count_bad_events(ipx_ctx* ctx, const ipx_dataset* d, const double* theta, int np, int64_t* count) {
  if (!ctx || !d || !theta || !count) return fail(IPX_EINVAL, "ipx_count_bad_events: NULL argument");
  const int model = d->model;
  if (np != kNParams[model])
    return fail(IPX_EINVAL, "ipx_count_bad_events: model %d takes %d parameters, got %d", model, kNParams[model], np);
  if (model == kModelIpatia)
    return fail(IPX_EINVAL, "ipx_count_bad_events: use ipx_event_logp for the Ipatia model");
  if (!theta_valid(model, theta)) return fail(IPX_EDOMAIN, "ipx_count_bad_events: parameters outside the domain");
  *count = 0;
  if (d->n == 0) return IPX_OK;
  HIP_TRY(hipSetDevice(ctx->device));
  const unsigned grid = (unsigned)std::min<int64_t>((d->n + kThreads - 1) / kThreads, 4096);
  const size_t kb = 256 * 8;  // room for the largest constant block
  static_assert(sizeof(AngTimeConst) <= 256 * 8 && sizeof(MassTimeConst) <= 256 * 8, "constant block size");
  char* buf = nullptr;
  HIP_TRY(hipMalloc(&buf, kb + grid * sizeof(long long)));
  long long* counts = (long long*)(buf + kb);
  hipError_t e = hipSuccess;
  const EventCols cols = cols_of(d);
  if (model == 1) {
    const MassHoist h = hoist_mass(theta);
    e = hipMemcpyAsync(buf, &h.k, sizeof h.k, hipMemcpyHostToDevice, ctx->stream);
    if (e == hipSuccess) hipLaunchKernelGGL(k_count_bad<1>, dim3(grid), dim3(kThreads), 0, ctx->stream, cols, (const MassConst*)buf, counts);
  } else if (model == 2) {
    const MassTimeHoist h = hoist_masstime(theta);
    e = hipMemcpyAsync(buf, &h.k, sizeof h.k, hipMemcpyHostToDevice, ctx->stream);
    if (e == hipSuccess) hipLaunchKernelGGL(k_count_bad<2>, dim3(grid), dim3(kThreads), 0, ctx->stream, cols, (const MassTimeConst*)buf, counts);
  } else {
    AngTimeHoist h;
    hoist_angtime(theta, d->ang, h);
    e = hipMemcpyAsync(buf, &h.k, sizeof h.k, hipMemcpyHostToDevice, ctx->stream);
    if (e == hipSuccess) {
      if (model == 3) hipLaunchKernelGGL(k_count_bad_angtime<false>, dim3(grid), dim3(kThreads), 0, ctx->stream, cols, (const AngTimeConst*)buf, counts);
      else hipLaunchKernelGGL(k_count_bad_angtime<true>, dim3(grid), dim3(kThreads), 0, ctx->stream, cols, (const AngTimeConst*)buf, counts);
    }
  }
  if (e == hipSuccess) e = hipGetLastError();
  std::vector<long long> hc(grid);
  if (e == hipSuccess) e = hipMemcpyAsync(hc.data(), counts, grid * sizeof(long long), hipMemcpyDeviceToHost, ctx->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
  const hipError_t ef = hipFree(buf);
  if (e != hipSuccess) return fail(IPX_EDEVICE, "ipx_count_bad_events: %s", hipGetErrorString(e));
  if (ef != hipSuccess) return fail(IPX_EDEVICE, "ipx_count_bad_events: hipFree: %s", hipGetErrorString(ef));
  int64_t total = 0;
  for (long long c : hc) total += c;
  *count = total;
  return IPX_OK;
}

ipx_status ipx_event_logp(ipx_ctx* ctx, const ipx_dataset* d, const double* theta, int np, double* out,
                          void* stream) {
  if (!ctx || !d || !theta) return fail(IPX_EINVAL, "ipx_event_logp: NULL argument");
  const int model = d->model;
  if (np != kNParams[model])
    return fail(IPX_EINVAL, "ipx_event_logp: model %d takes %d parameters, got %d", model, kNParams[model], np);
  if (d->n > 0 && !out) return fail(IPX_EINVAL, "ipx_event_logp: out is NULL");
  if (model == kModelIpatia) {
    if (d->n == 0) return IPX_OK;
    HIP_TRY(hipSetDevice(ctx->device));
    hipStream_t s = stream ? (hipStream_t)stream : ctx->stream;
    ipx_dataset* dd = const_cast<ipx_dataset*>(d);
    ipx_status st = ipatia_prepare(ctx, dd, theta, s);
    if (st != IPX_OK) return st;
    hipLaunchKernelGGL(k_event_logp_ipatia, dim3((unsigned)((d->n + kThreads - 1) / kThreads)), dim3(kThreads), 0, s,
                       cols_of(d), (const IpatiaConst*)dd->aux, out);
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipStreamSynchronize(s));
    return IPX_OK;
  }
  if (!theta_valid(model, theta)) return fail(IPX_EDOMAIN, "ipx_event_logp: parameters outside the domain");
  if (d->n == 0) return IPX_OK;
  HIP_TRY(hipSetDevice(ctx->device));
  hipStream_t s = stream ? (hipStream_t)stream : ctx->stream;
  const unsigned grid = (unsigned)((d->n + kThreads - 1) / kThreads);
  const EventCols cols = cols_of(d);
  if (model == 1) {
    const MassHoist h = hoist_mass(theta);
    hipLaunchKernelGGL(k_event_logp<1>, dim3(grid), dim3(kThreads), 0, s, cols, h.k, out);
  } else if (model == 2) {
    const MassTimeHoist h = hoist_masstime(theta);
    hipLaunchKernelGGL(k_event_logp<2>, dim3(grid), dim3(kThreads), 0, s, cols, h.k, out);
  } else {
    AngTimeHoist h;
    hoist_angtime(theta, d->ang, h);
    if (model == 3) hipLaunchKernelGGL(k_event_logp_angtime<false>, dim3(grid), dim3(kThreads), 0, s, cols, h.k, out);
    else hipLaunchKernelGGL(k_event_logp_angtime<true>, dim3(grid), dim3(kThreads), 0, s, cols, h.k, out);
  }
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipStreamSynchronize(s));
  return IPX_OK;
}

ipx_status nll_eval(ipx_ctx* ctx, const ipx_dataset* ds, const double* theta, int np, double* nll, void* stream) {
  return run(ctx, ds, theta, np, nll, nullptr, stream);
}

ipx_status nll_grad(ipx_ctx* ctx, const ipx_dataset* ds, const double* theta, int np, double* nll, double* grad,
                    void* stream) {
  if (!grad) return fail(IPX_EINVAL, "nll_grad: grad is NULL");
  return run(ctx, ds, theta, np, nll, grad, stream);
}

ipx_status nll_eval_noalloc(ipx_ctx* ctx, int model, int64_t n, const double* const* cols, int ncols,
                            const double* w, const double* theta, int np, double* nll, double* grad, void* stream) {
  if (!ctx || !theta || !nll) return fail(IPX_EINVAL, "nll_eval_noalloc: NULL argument");
  if (model < 1 || model > 4) return fail(IPX_EINVAL, "nll_eval_noalloc: unknown model %d (1 .. 4)", model);
  if (ncols != kNCols[model])
    return fail(IPX_EINVAL, "nll_eval_noalloc: model %d takes %d columns, got %d", model, kNCols[model], ncols);
  if (np != kNParams[model])
    return fail(IPX_EINVAL, "nll_eval_noalloc: model %d takes %d parameters, got %d", model, kNParams[model], np);
  if (n < 0) return fail(IPX_EINVAL, "nll_eval_noalloc: negative size");
  if (n > kNoAllocMaxEvents)
    return fail(IPX_EINVAL, "nll_eval_noalloc: %lld events exceed the maximum of %lld (fixed scratch of %zu bytes)",
                (long long)n, (long long)kNoAllocMaxEvents, kNoAllocBytes);
  if (n > 0 && !cols) return fail(IPX_EINVAL, "nll_eval_noalloc: NULL cols");
  for (int c = 0; c < ncols && n > 0; ++c)
    if (!cols[c]) return fail(IPX_EINVAL, "nll_eval_noalloc: column %d is NULL", c);
  {
    ipx_status st = check_theta(model, theta, np, nll, grad);
    if (st != IPX_OK) return st;
  }
  if (ctx->device >= kMaxDevices) return fail(IPX_EINVAL, "nll_eval_noalloc: device %d", ctx->device);
  unsigned char* base = g_noalloc_ptr[ctx->device].load();
  if (!base) return fail(IPX_EDEVICE, "nll_eval_noalloc: scratch address of device %d not set up", ctx->device);
  HIP_TRY(hipSetDevice(ctx->device));
  hipStream_t s = stream ? (hipStream_t)stream : ctx->stream;
  std::lock_guard<std::mutex> lk(g_noalloc_mu[ctx->device]);

  const int64_t n_tiles = (n + kTile - 1) / kTile;
  SegInfo* segs = (SegInfo*)(base + kNaSeg);
  const unsigned char* active = base + kNaActive;
  double* out = (double*)(base + kNaOut);
  TileRef* tiles = (TileRef*)(base + kNaTiles);
  double* partials = (double*)(base + kNaPartials);

  // head of the scratch (segment record, constants, active flag), staged on
  // the host stack and copied in one transfer
  alignas(16) unsigned char head[kNaOut];
  std::memset(head, 0, sizeof head);
  SegInfo seg{};
  for (int c = 0; c < ncols; ++c) seg.cols.c[c] = cols ? cols[c] : nullptr;
  seg.cols.w = w;
  seg.cols.n = n;
  seg.partials = partials;
  seg.n_tiles = n_tiles;
  std::memcpy(head + kNaSeg, &seg, sizeof seg);
  EvalHoist h;
  hoist_eval(model, theta, ang_settings_default(), h);
  std::memcpy(head + kNaConst, h.consts, h.bytes);
  head[kNaActive] = 1;
  HIP_TRY(hipMemcpyAsync(base, head, sizeof head, hipMemcpyHostToDevice, s));
  if (n_tiles > 0) {
    hipLaunchKernelGGL(k_fill_tiles, dim3((unsigned)((n_tiles + 255) / 256)), dim3(256), 0, s, tiles, (int)n_tiles);
    HIP_TRY(hipGetLastError());
  }
  const bool g = grad != nullptr;
  const int nacc = nacc_of(model, g);
  {
    ipx_status st = launch_eval(model, g, (unsigned)std::max<int64_t>(1, n_tiles), segs, tiles, n_tiles,
                                base + kNaConst, active, 1, out, s, nullptr);
    if (st != IPX_OK) return st;
  }
  double a[kAccMax];
  HIP_TRY(hipMemcpyAsync(a, out, nacc * sizeof(double), hipMemcpyDeviceToHost, s));
  if (angular_model(model) && g) angtime_derivatives(theta, h.h3);  // while the kernels run
  HIP_TRY(hipStreamSynchronize(s));
  return finish_eval(model, h, theta, np, a, nll, grad);
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Binned path: histograms, smearing, binned likelihood, toys and CL_s
// ---------------------------------------------------------------------------
struct ipx_hist {
  int n = 0;
  double lo = 0.0, hi = 0.0, dx = 0.0;
  double sig_sum = 0.0;            // sum of the normalised signal template
  double sig_max = 0.0;            // its largest entry
  double* sig = nullptr;           // device [n]: the signal template
  double* cnt = nullptr;           // device [n]: observed counts
  double* work = nullptr;          // device: partials, tables, q_obs, counters
  double* q = nullptr;             // device [2][q_cap]: toy statistics
  int q_cap = 0;
  double* host = nullptr;          // pinned: results read back
  int nwg = 0;
};

static constexpr int kHistMaxBins = 1 << 24;

// partials (kBinnedAcc x nwg) | totals (8) | tables: nu, em, kmax (2n each), L (n) | q_obs (1) |
// counters (2) | (pad to 16 bytes) | CDF heads (2n x kCdfStride)
static size_t hist_cdf_offset(int n, int nwg) {
  const size_t o = (size_t)kBinnedAcc * nwg + 8 + 7 * (size_t)n + 1 + 2;
  return (o + 1) & ~(size_t)1;
}
static size_t hist_work_doubles(int n, int nwg) { return hist_cdf_offset(n, nwg) + 2 * (size_t)n * kCdfStride; }

static ToyTables hist_tables(const ipx_hist* H) {
  double* t = H->work + (size_t)kBinnedAcc * H->nwg + 8;
  return ToyTables{t, t + 2 * (size_t)H->n, t + 4 * (size_t)H->n, t + 6 * (size_t)H->n,
                   H->work + hist_cdf_offset(H->n, H->nwg)};
}
static double* hist_qobs(const ipx_hist* H) { return H->work + (size_t)kBinnedAcc * H->nwg + 8 + 7 * (size_t)H->n; }
static unsigned long long* hist_counters(const ipx_hist* H) { return (unsigned long long*)(hist_qobs(H) + 1); }

static void free_hist(ipx_hist* H) {
  if (H->sig) (void)hipFree(H->sig);
  if (H->cnt) (void)hipFree(H->cnt);
  if (H->work) (void)hipFree(H->work);
  if (H->q) (void)hipFree(H->q);
  if (H->host) (void)hipHostFree(H->host);
  delete H;
}

// sum_{b < n} exp(-k b dx), a geometric sum.
static double geometric_norm(double k, double dx, int n) {
  if (k == 0.0) return (double)n;
  return std::expm1(-k * dx * n) / std::expm1(-k * dx);
}


// Binned-model constants at theta = (ns, nb, k); false outside the domain.
static bool binned_const(const ipx_hist* H, const double* th, BinnedConst* c) {
  const double ns = th[0], nb = th[1], k = th[2];
  if (!std::isfinite(ns) || !std::isfinite(nb) || !std::isfinite(k) || ns < 0.0 || nb < 0.0) return false;
  const double Z = geometric_norm(k, H->dx, H->n);
  if (!(Z > 0.0) || !std::isfinite(Z)) return false;
  *c = BinnedConst{ns, nb, k, 1.0 / Z, H->lo, H->dx, H->n};
  return true;
}

extern "C" {

ipx_status ipx_smear(ipx_ctx* ctx, int n, double dx, double sigma, const double* h, double* out, void* stream) {
  if (!ctx || (n > 0 && (!h || !out))) return fail(IPX_EINVAL, "ipx_smear: NULL argument");
  if (n < 0 || n > kHistMaxBins) return fail(IPX_EINVAL, "ipx_smear: %d bins", n);
  if (!(dx > 0.0) || !(sigma > 0.0) || !std::isfinite(dx) || !std::isfinite(sigma))
    return fail(IPX_EINVAL, "ipx_smear: bin width and sigma must be positive");
  if (n == 0) return IPX_OK;
  HIP_TRY(hipSetDevice(ctx->device));
  hipStream_t s = stream ? (hipStream_t)stream : ctx->stream;
  int chunks = 1, steps = 1;
  smear_grid(n, &chunks, &steps);
  // the kernel table (2n - 1), then the chunk partials (chunks x n), in the
  // context's workspace (allocated on first need, grown, kept until
  // ipx_destroy); calls on one context take turns
  std::lock_guard<std::mutex> lk(ctx->ws_mu);
  const size_t need = (size_t)(2 * n - 1) + (size_t)chunks * n;
  if (need > ctx->smear_ws_doubles) {
    if (ctx->smear_ws) HIP_TRY(hipFree(ctx->smear_ws));
    ctx->smear_ws = nullptr;
    ctx->smear_ws_doubles = 0;
    HIP_TRY(hipMalloc(&ctx->smear_ws, need * sizeof(double)));
    ctx->smear_ws_doubles = need;
  }
  double* kern = ctx->smear_ws;
  double* part = kern + (2 * n - 1);
  hipLaunchKernelGGL(k_smear_kernel, dim3((2 * n - 1 + kThreads - 1) / kThreads), dim3(kThreads), 0, s, kern, n, dx, sigma);
  hipError_t e = hipGetLastError();
  if (e == hipSuccess) {
    hipLaunchKernelGGL(k_smear_part, dim3((n + kSmearOut - 1) / kSmearOut, chunks), dim3(kThreads), 0, s, h, kern, part,
                       n, steps);
    hipLaunchKernelGGL(k_smear_sum, dim3((n + kThreads - 1) / kThreads), dim3(kThreads), 0, s, part, out, n, chunks);
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return fail(IPX_EDEVICE, "ipx_smear: %s", hipGetErrorString(e));
  return IPX_OK;
}

ipx_status ipx_hist_create(ipx_ctx* ctx, int nbins, double lo, double hi, double mu, double sigma_core,
                           double sigma_smear, const double* counts, ipx_hist** out) {
  if (!ctx || !out) return fail(IPX_EINVAL, "ipx_hist_create: NULL argument");
  *out = nullptr;
  if (nbins < 1 || nbins > kHistMaxBins) return fail(IPX_EINVAL, "ipx_hist_create: %d bins", nbins);
  if (!std::isfinite(lo) || !std::isfinite(hi) || !(hi > lo) || !std::isfinite(mu) || !(sigma_core > 0.0) ||
      !(sigma_smear > 0.0) || !std::isfinite(sigma_core) || !std::isfinite(sigma_smear))
    return fail(IPX_EINVAL, "ipx_hist_create: bad range or shape parameters");
  if (counts)
    for (int b = 0; b < nbins; ++b)
      if (!(counts[b] >= 0.0) || !std::isfinite(counts[b]) || counts[b] != std::floor(counts[b]))
        return fail(IPX_EINVAL, "ipx_hist_create: count %d is not a non-negative integer", b);
  HIP_TRY(hipSetDevice(ctx->device));
  ipx_hist* H = new (std::nothrow) ipx_hist();
  if (!H) return fail(IPX_ENOMEM, "ipx_hist_create: host allocation failed");
  H->n = nbins;
  H->lo = lo;
  H->hi = hi;
  H->dx = (hi - lo) / nbins;
  H->nwg = (nbins + kThreads - 1) / kThreads;
  const int n = nbins;
  int chunks = 1, steps = 1;
  smear_grid(n, &chunks, &steps);
  // the smearing's kernel, core and chunk partials first
  const size_t wd = std::max(hist_work_doubles(n, H->nwg), (size_t)(3 * n) + (size_t)chunks * n);
  hipError_t e = hipMalloc(&H->sig, n * sizeof(double));
  if (e == hipSuccess) e = hipMalloc(&H->cnt, n * sizeof(double));
  if (e == hipSuccess) e = hipMalloc(&H->work, wd * sizeof(double));
  if (e == hipSuccess) e = hipHostMalloc((void**)&H->host, 16 * sizeof(double), hipHostMallocDefault);
  if (e != hipSuccess) {
    free_hist(H);
    return fail(IPX_ENOMEM, "ipx_hist_create: allocation failed: %s", hipGetErrorString(e));
  }
  hipStream_t s = ctx->stream;
  double* kern = H->work;              // 2n - 1
  double* core = H->work + 2 * n;      // n (overlaps nothing of kern: 2n - 1 < 2n)
  double* part = H->work + 3 * n;      // chunks x n
  const unsigned g1 = (unsigned)((n + kThreads - 1) / kThreads), g2 = (unsigned)((2 * n - 1 + kThreads - 1) / kThreads);
  hipLaunchKernelGGL(k_gauss_core, dim3(g1), dim3(kThreads), 0, s, core, n, lo, H->dx, mu, sigma_core);
  hipLaunchKernelGGL(k_smear_kernel, dim3(g2), dim3(kThreads), 0, s, kern, n, H->dx, sigma_smear);
  hipLaunchKernelGGL(k_smear_part, dim3((n + kSmearOut - 1) / kSmearOut, chunks), dim3(kThreads), 0, s, core, kern, part,
                     n, steps);
  hipLaunchKernelGGL(k_smear_sum, dim3(g1), dim3(kThreads), 0, s, part, H->sig, n, chunks);
  hipLaunchKernelGGL(k_sum, dim3(1), dim3(kThreads), 0, s, H->sig, n, H->host);
  e = hipGetLastError();
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  const double total = H->host[0];
  if (e == hipSuccess && !(total > 0.0 && std::isfinite(total))) {
    free_hist(H);
    return fail(IPX_EDOMAIN, "ipx_hist_create: the signal shape has no weight in the range");
  }
  if (e == hipSuccess) {
    hipLaunchKernelGGL(k_scale, dim3(g1), dim3(kThreads), 0, s, H->sig, n, 1.0 / total);
    hipLaunchKernelGGL(k_sum, dim3(1), dim3(kThreads), 0, s, H->sig, n, H->host);
    e = hipGetLastError();
  }
  if (e == hipSuccess) {
    if (counts) e = hipMemcpyAsync(H->cnt, counts, n * sizeof(double), hipMemcpyHostToDevice, s);
    else e = hipMemsetAsync(H->cnt, 0, n * sizeof(double), s);
  }
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) {
    free_hist(H);
    return fail(IPX_EDEVICE, "ipx_hist_create: %s", hipGetErrorString(e));
  }
  H->sig_sum = H->host[0];
  {
    std::vector<double> t(n);
    e = hipMemcpy(t.data(), H->sig, n * sizeof(double), hipMemcpyDeviceToHost);
    if (e != hipSuccess) {
      free_hist(H);
      return fail(IPX_EDEVICE, "ipx_hist_create: %s", hipGetErrorString(e));
    }
    for (double v : t) H->sig_max = std::fmax(H->sig_max, v);
  }
  *out = H;
  return IPX_OK;
}

ipx_status ipx_hist_destroy(ipx_ctx* ctx, ipx_hist* H) {
  if (!ctx || !H) return fail(IPX_EINVAL, "ipx_hist_destroy: NULL argument");
  HIP_TRY(hipSetDevice(ctx->device));
  HIP_TRY(hipStreamSynchronize(ctx->stream));
  free_hist(H);
  return IPX_OK;
}

int ipx_hist_nbins(const ipx_hist* H) { return H ? H->n : -1; }

ipx_status ipx_hist_read(ipx_ctx* ctx, const ipx_hist* H, int which, double* host) {
  if (!ctx || !H || !host) return fail(IPX_EINVAL, "ipx_hist_read: NULL argument");
  if (which != 0 && which != 1) return fail(IPX_EINVAL, "ipx_hist_read: which = %d", which);
  HIP_TRY(hipSetDevice(ctx->device));
  HIP_TRY(hipMemcpyAsync(host, which == 0 ? H->sig : H->cnt, H->n * sizeof(double), hipMemcpyDeviceToHost,
                         ctx->stream));
  HIP_TRY(hipStreamSynchronize(ctx->stream));
  return IPX_OK;
}

ipx_status ipx_hist_set_counts(ipx_ctx* ctx, ipx_hist* H, const double* counts) {
  if (!ctx || !H || !counts) return fail(IPX_EINVAL, "ipx_hist_set_counts: NULL argument");
  for (int b = 0; b < H->n; ++b)
    if (!(counts[b] >= 0.0) || !std::isfinite(counts[b]) || counts[b] != std::floor(counts[b]))
      return fail(IPX_EINVAL, "ipx_hist_set_counts: count %d is not a non-negative integer", b);
  HIP_TRY(hipSetDevice(ctx->device));
  HIP_TRY(hipMemcpyAsync(H->cnt, counts, H->n * sizeof(double), hipMemcpyHostToDevice, ctx->stream));
  HIP_TRY(hipStreamSynchronize(ctx->stream));
  return IPX_OK;
}

ipx_status nll_binned(ipx_ctx* ctx, const ipx_hist* H, const double* theta, int np, double* nll, double* grad,
                      void* stream) {
  if (!ctx || !H || !theta || !nll) return fail(IPX_EINVAL, "nll_binned: NULL argument");
  if (np != 3) return fail(IPX_EINVAL, "nll_binned: 3 parameters (ns, nb, k), got %d", np);
  BinnedConst c;
  if (!binned_const(H, theta, &c)) {
    *nll = std::numeric_limits<double>::infinity();
    if (grad)
      for (int i = 0; i < 3; ++i) grad[i] = std::numeric_limits<double>::quiet_NaN();
    return fail(IPX_EDOMAIN, "nll_binned: parameters outside the domain");
  }
  HIP_TRY(hipSetDevice(ctx->device));
  hipStream_t s = stream ? (hipStream_t)stream : ctx->stream;
  double* part = H->work;
  double* tot = H->work + (size_t)kBinnedAcc * H->nwg;
  hipLaunchKernelGGL(k_binned_nll, dim3(H->nwg), dim3(kThreads), 0, s, c, H->sig, H->cnt, part);
  hipLaunchKernelGGL(k_reduce_parts, dim3(kBinnedAcc), dim3(kThreads), 0, s, part, H->nwg, tot);
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipMemcpyAsync(H->host, tot, kBinnedAcc * sizeof(double), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  const double* a = H->host;
  if (!std::isfinite(a[0])) {
    *nll = std::numeric_limits<double>::infinity();
    if (grad)
      for (int i = 0; i < 3; ++i) grad[i] = std::numeric_limits<double>::quiet_NaN();
    return fail(IPX_EDOMAIN, "nll_binned: non-finite likelihood (an expected count is not positive where "
                             "events were seen)");
  }
  *nll = a[0];
  if (grad) {
    const double ybar = a[4] * c.invZ;
    grad[0] = a[1];
    grad[1] = a[2] * c.invZ;
    grad[2] = c.nb * c.invZ * (ybar * a[2] - a[3]);
  }
  return IPX_OK;
}

static ipx_status toy_tables(ipx_ctx* ctx, const ipx_hist* H, const double* theta, BinnedConst* c, hipStream_t s,
                             const char* who) {
  if (!binned_const(H, theta, c) || !(c->nb > 0.0))
    return fail(IPX_EDOMAIN, "%s: parameters outside the domain (ns >= 0, nb > 0, finite k)", who);
  // the inversion starts from p_0 = e^{-nu}: it must not underflow (the
  // background template is monotonic, largest at one end)
  const double emax = std::fmax(1.0, std::exp(-c->k * H->dx * (H->n - 1)));
  const double nu_max = c->ns * H->sig_max + c->nb * emax * c->invZ;
  if (!(nu_max < 700.0))
    return fail(IPX_EDOMAIN, "%s: an expected count reaches %g (the Poisson inversion needs < 700)", who, nu_max);
  hipLaunchKernelGGL(k_toy_tables, dim3(H->nwg), dim3(kThreads), 0, s, *c, H->sig, hist_tables(H));
  HIP_TRY(hipGetLastError());
  return IPX_OK;
}

ipx_status ipx_binned_toy(ipx_ctx* ctx, const ipx_hist* H, const double* theta, uint64_t seed, int hyp,
                          uint64_t toy, double* counts) {
  if (!ctx || !H || !theta || !counts) return fail(IPX_EINVAL, "ipx_binned_toy: NULL argument");
  if (hyp != 0 && hyp != 1) return fail(IPX_EINVAL, "ipx_binned_toy: hypothesis %d", hyp);
  HIP_TRY(hipSetDevice(ctx->device));
  hipStream_t s = ctx->stream;
  BinnedConst c;
  ipx_status st = toy_tables(ctx, H, theta, &c, s, "ipx_binned_toy");
  if (st != IPX_OK) return st;
  double* dev = nullptr;
  HIP_TRY(hipMalloc(&dev, H->n * sizeof(double)));
  const int nblk = (H->n + 3) / 4;
  hipLaunchKernelGGL(k_toy_counts, dim3((nblk + kThreads - 1) / kThreads), dim3(kThreads), 0, s, hist_tables(H), H->n,
                     hyp, seed, toy, dev);
  hipError_t e = hipGetLastError();
  if (e == hipSuccess) e = hipMemcpyAsync(counts, dev, H->n * sizeof(double), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  (void)hipFree(dev);
  if (e != hipSuccess) return fail(IPX_EDEVICE, "ipx_binned_toy: %s", hipGetErrorString(e));
  return IPX_OK;
}

ipx_status cls_toys(ipx_ctx* ctx, ipx_hist* H, const double* theta, uint64_t seed, int ntoys, ipx_cls_result* res,
                    double* q_toys) {
  if (!ctx || !H || !theta || !res) return fail(IPX_EINVAL, "cls_toys: NULL argument");
  if (ntoys < 1 || ntoys > (1 << 24)) return fail(IPX_EINVAL, "cls_toys: %d toys", ntoys);
  HIP_TRY(hipSetDevice(ctx->device));
  hipStream_t s = ctx->stream;
  // q (2 x ntoys) | block partials of the toys (2 x nblk x ntoys) | of the observed counts (nblk)
  const int nblk = ((H->n + 3) / 4 + kClsQuads - 1) / kClsQuads;
  if (H->q_cap < ntoys) {
    if (H->q) (void)hipFree(H->q);
    H->q = nullptr;
    H->q_cap = 0;
    HIP_TRY(hipMalloc(&H->q, (2 * (size_t)ntoys * (1 + (size_t)nblk) + nblk) * sizeof(double)));
    H->q_cap = ntoys;
  }
  double* part = H->q + 2 * (size_t)ntoys;
  double* part_obs = part + 2 * (size_t)nblk * ntoys;
  BinnedConst c;
  ipx_status st = toy_tables(ctx, H, theta, &c, s, "cls_toys");
  if (st != IPX_OK) return st;
  const double S = c.ns * H->sig_sum;
  const ToyTables tb = hist_tables(H);
  hipLaunchKernelGGL(k_cls_block, dim3((unsigned)nblk, 1, 1), dim3(kThreads), 0, s, tb, H->n, seed, 1,
                     (const double*)H->cnt, part_obs);
  hipLaunchKernelGGL(k_cls_q, dim3(1, 1), dim3(kThreads), 0, s, part_obs, nblk, 1, S, hist_qobs(H));
  HIP_TRY(hipGetLastError());
  st = timing_begin(ctx, s);
  if (st != IPX_OK) return st;
  hipLaunchKernelGGL(k_cls_block, dim3((unsigned)nblk, (unsigned)((ntoys + kClsToys - 1) / kClsToys), 2),
                     dim3(kThreads), 0, s, tb, H->n, seed, ntoys, (const double*)nullptr, part);
  HIP_TRY(hipGetLastError());
  st = timing_end(ctx, s);
  if (st != IPX_OK) return st;
  hipLaunchKernelGGL(k_cls_q, dim3((unsigned)((ntoys + kThreads - 1) / kThreads), 2), dim3(kThreads), 0, s, part,
                     nblk, ntoys, S, H->q);
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipMemsetAsync(hist_counters(H), 0, 2 * sizeof(unsigned long long), s));
  hipLaunchKernelGGL(k_count_ge, dim3((unsigned)((ntoys + kThreads - 1) / kThreads), 2), dim3(kThreads), 0, s, H->q,
                     ntoys, hist_qobs(H), hist_counters(H));
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipMemcpyAsync(H->host, hist_qobs(H), 3 * sizeof(double), hipMemcpyDeviceToHost, s));
  if (q_toys) HIP_TRY(hipMemcpyAsync(q_toys, H->q, 2 * (size_t)ntoys * sizeof(double), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  unsigned long long ge[2];
  std::memcpy(ge, H->host + 1, sizeof ge);
  res->q_obs = H->host[0];
  res->n_b = (int64_t)ge[0];
  res->n_sb = (int64_t)ge[1];
  res->cl_b = (double)ge[0] / ntoys;
  res->cl_sb = (double)ge[1] / ntoys;
  res->cl_s = ge[0] > 0 ? res->cl_sb / res->cl_b : std::numeric_limits<double>::quiet_NaN();
  return IPX_OK;
}

}  // extern "C"
