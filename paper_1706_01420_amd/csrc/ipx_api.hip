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
#include <hipcub/hipcub.hpp>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <limits>
#include <string>
#include <algorithm>
#include <vector>

#include "../../include/ipx.h"
#include "ipx_hoist.h"
#include "ipx_kernels.h"
#include "ipx_toys.h"
#include "ipx_batch.h"

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
};

struct ipx_dataset {
  int model = 0;
  int64_t n = 0;
  int64_t n_pad = 0;
  int ncols = 0;
  double* base = nullptr;          // owned column storage (nullptr when borrowed)
  const double* cols[6] = {};
  const double* w = nullptr;
  int64_t n_tiles = 0;
  int64_t n_tiles_outer = 0;       // tiles of the angular coefficient-adjoint kernel
  bool sorted = false;             // events stored in increasing decay time
  double* tau = nullptr;           // 4 x n_pad per-event adjoint factors (angular gradient)
  double* partials = nullptr;      // n_tiles x kAccMax
  double* out_dev = nullptr;       // kAccMax
  double* out_host = nullptr;      // kAccMax, pinned
  size_t bytes = 0;
};

static const int kNParams[4] = {-1, 4, 7, 12};
static const int kNCols[4] = {-1, 1, 3, 6};

// ---------------------------------------------------------------------------
// Event-store ordering: the models with a decay time store their events in
// increasing t, so that the waves whose events need the large-t/sigma
// correction at t are few and contiguous (the NLL is a sum over events; the
// order only changes the rounding of the sum).
// ---------------------------------------------------------------------------
__global__ void k_iota(int* __restrict__ v, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) v[i] = i;
}
__global__ void k_gather(double* __restrict__ dst, const double* __restrict__ src, const int* __restrict__ perm,
                         int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = src[perm[i]];
}

static ipx_status sort_by_time(ipx_dataset* d, hipStream_t s) {
  const int n = (int)d->n;
  const int tcol = d->model == 2 ? 1 : 3;
  double* keys_out = nullptr;
  double* tmp = nullptr;
  int* perm_in = nullptr;
  int* perm = nullptr;
  void* scratch = nullptr;
  size_t scratch_bytes = 0;
  hipError_t e = hipMalloc(&keys_out, (size_t)n * sizeof(double));
  if (e == hipSuccess) e = hipMalloc(&tmp, (size_t)n * sizeof(double));
  if (e == hipSuccess) e = hipMalloc(&perm_in, (size_t)n * sizeof(int));
  if (e == hipSuccess) e = hipMalloc(&perm, (size_t)n * sizeof(int));
  if (e == hipSuccess)
    e = hipcub::DeviceRadixSort::SortPairs(nullptr, scratch_bytes, d->cols[tcol], keys_out, perm_in, perm, n, 0,
                                           64, s);
  if (e == hipSuccess) e = hipMalloc(&scratch, scratch_bytes);
  if (e == hipSuccess) {
    const unsigned blocks = (unsigned)((n + 255) / 256);
    hipLaunchKernelGGL(k_iota, dim3(blocks), dim3(256), 0, s, perm_in, n);
    e = hipGetLastError();
    if (e == hipSuccess)
      e = hipcub::DeviceRadixSort::SortPairs(scratch, scratch_bytes, d->cols[tcol], keys_out, perm_in, perm, n,
                                             0, 64, s);
    const int nstore = d->ncols + (d->w ? 1 : 0);
    for (int c = 0; c < nstore && e == hipSuccess; ++c) {
      double* col = const_cast<double*>(c < d->ncols ? d->cols[c] : d->w);
      hipLaunchKernelGGL(k_gather, dim3(blocks), dim3(256), 0, s, tmp, col, perm, n);
      e = hipGetLastError();
      if (e == hipSuccess) e = hipMemcpyAsync(col, tmp, (size_t)n * sizeof(double), hipMemcpyDeviceToDevice, s);
    }
    if (e == hipSuccess) e = hipStreamSynchronize(s);
  }
  (void)hipFree(keys_out);
  (void)hipFree(tmp);
  (void)hipFree(perm_in);
  (void)hipFree(perm);
  (void)hipFree(scratch);
  if (e != hipSuccess) return fail(IPX_EDEVICE, "ipx_dataset_create: sorting by decay time failed: %s", hipGetErrorString(e));
  d->sorted = true;
  return IPX_OK;
}

extern "C" {

const char* ipx_last_error(void) { return g_last_error.c_str(); }

int ipx_model_nparams(int model) { return (model >= 1 && model <= 3) ? kNParams[model] : -1; }
int ipx_model_ncols(int model) { return (model >= 1 && model <= 3) ? kNCols[model] : -1; }

ipx_status ipx_create(int device, ipx_ctx** out) {
  if (!out) return fail(IPX_EINVAL, "ipx_create: out is NULL");
  *out = nullptr;
  int count = 0;
  HIP_TRY(hipGetDeviceCount(&count));
  if (device < 0 || device >= count) return fail(IPX_EINVAL, "ipx_create: device %d of %d", device, count);
  HIP_TRY(hipSetDevice(device));
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
  delete c;
}

static void free_dataset(ipx_dataset* d) {
  if (d->base) (void)hipFree(d->base);
  if (d->tau) (void)hipFree(d->tau);
  if (d->partials) (void)hipFree(d->partials);
  if (d->out_dev) (void)hipFree(d->out_dev);
  if (d->out_host) (void)hipHostFree(d->out_host);
  delete d;
}

ipx_status ipx_dataset_create(ipx_ctx* ctx, int model, int64_t n, const double* const* cols, int ncols,
                              const double* w, unsigned flags, ipx_dataset** out) {
  if (!ctx || !out) return fail(IPX_EINVAL, "ipx_dataset_create: NULL ctx/out");
  *out = nullptr;
  if (model < 1 || model > 3) return fail(IPX_EINVAL, "ipx_dataset_create: unknown model %d", model);
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
  d->n_tiles_outer = (n + kOuterTile - 1) / kOuterTile;
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
    if (model >= 2 && !(flags & IPX_KEEP_ORDER) && n >= 2 && n <= 0x7fffffff) {
      ipx_status st = sort_by_time(d, ctx->stream);
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
  HIP_TRY(hipSetDevice(ctx->device));
  HIP_TRY(hipStreamSynchronize(ctx->stream));
  free_dataset(d);
  return IPX_OK;
}

size_t ipx_dataset_bytes(const ipx_dataset* d) { return d ? d->bytes : 0; }
int64_t ipx_dataset_size(const ipx_dataset* d) { return d ? d->n : -1; }
int ipx_dataset_model(const ipx_dataset* d) { return d ? d->model : -1; }

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
// Launch helpers
// ---------------------------------------------------------------------------
static EventCols cols_of(const ipx_dataset* d) {
  EventCols c;
  for (int i = 0; i < 6; ++i) c.c[i] = d->cols[i];
  c.w = d->w;
  c.n = d->n;
  return c;
}

template <int MODEL, bool GRAD>
static ipx_status launch_model(ipx_ctx* ctx, const ipx_dataset* d, const typename ModelTraits<MODEL>::Const& k,
                               hipStream_t s) {
  constexpr int nacc = GRAD ? ModelTraits<MODEL>::kAcc : 1;
  if (d->n_tiles == 0) {
    // empty dataset: the reduction of zero tiles writes zeros (no memset, so
    // the call stays capturable in a graph)
    hipLaunchKernelGGL(k_reduce_tiles, dim3(nacc), dim3(kThreads), 0, s, d->partials, (int64_t)0, (int64_t)0, nacc,
                       (int64_t)0, d->out_dev);
    HIP_TRY(hipGetLastError());
    return IPX_OK;
  }
  const int64_t grid = d->n_tiles;  // one workgroup per canonical tile
  const bool timed = ctx->timing;
  if (timed) {
    if (ctx->ev_used == 64) {
      ipx_status st = timing_drain(ctx);
      if (st != IPX_OK) return st;
    }
    HIP_TRY(hipEventRecord(ctx->ev_pool[0][ctx->ev_used], s));
  }
  hipLaunchKernelGGL((k_nll_tiles<MODEL, GRAD>), dim3((unsigned)grid), dim3(kThreads), 0, s, cols_of(d), k,
                     d->partials, d->n_tiles);
  HIP_TRY(hipGetLastError());
  if (timed) {
    HIP_TRY(hipEventRecord(ctx->ev_pool[1][ctx->ev_used], s));
    ctx->ev_used++;
  }
  hipLaunchKernelGGL(k_reduce_tiles, dim3(nacc), dim3(kThreads), 0, s, d->partials, d->n_tiles, d->n_tiles, nacc,
                     (int64_t)0, d->out_dev);
  HIP_TRY(hipGetLastError());
  return IPX_OK;
}

template <bool GRAD>
static ipx_status launch_angtime(ipx_ctx* ctx, ipx_dataset* d, const AngTimeConst& k, hipStream_t s) {
  constexpr int nacc = GRAD ? kAccAngTime : 1;
  if (d->n_tiles == 0) {
    hipLaunchKernelGGL(k_reduce_tiles, dim3(nacc), dim3(kThreads), 0, s, d->partials, (int64_t)0, (int64_t)0, nacc,
                       (int64_t)0, d->out_dev);
    HIP_TRY(hipGetLastError());
    return IPX_OK;
  }
  if (GRAD && !d->tau) {
    hipError_t e = hipMalloc(&d->tau, 4 * (size_t)d->n_pad * sizeof(double));
    if (e != hipSuccess) {
      d->tau = nullptr;
      return fail(IPX_ENOMEM, "nll_grad: per-event scratch allocation failed: %s", hipGetErrorString(e));
    }
    d->bytes += 4 * (size_t)d->n_pad * sizeof(double);
  }
  const bool timed = ctx->timing;
  if (timed) {
    if (ctx->ev_used == 64) {
      ipx_status st = timing_drain(ctx);
      if (st != IPX_OK) return st;
    }
    HIP_TRY(hipEventRecord(ctx->ev_pool[0][ctx->ev_used], s));
  }
  hipLaunchKernelGGL((k_angtime<GRAD>), dim3((unsigned)d->n_tiles), dim3(kThreads), 0, s, cols_of(d), k,
                     d->partials, d->n_tiles, d->tau, d->n_pad);
  HIP_TRY(hipGetLastError());
  if (timed) {
    HIP_TRY(hipEventRecord(ctx->ev_pool[1][ctx->ev_used], s));
    ctx->ev_used++;
  }
  if (GRAD) {
    hipLaunchKernelGGL(k_angtime_outer, dim3((unsigned)d->n_tiles_outer), dim3(kThreads), 0, s, cols_of(d),
                       (const double*)d->tau, d->n_pad, d->partials, d->n_tiles_outer, d->n_tiles);
    HIP_TRY(hipGetLastError());
  }
  hipLaunchKernelGGL(k_reduce_tiles, dim3(nacc), dim3(kThreads), 0, s, d->partials, d->n_tiles, d->n_tiles,
                     kAngInner, d->n_tiles_outer, d->out_dev);
  HIP_TRY(hipGetLastError());
  return IPX_OK;
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
    const AngTimeHoist a = hoist_angtime(th);
    double M = 0.0;
    for (int k = 0; k < 10; ++k) {
      double s = 0.0;
      for (int j = 0; j < 4; ++j) {
        h.C[4 * k + j] = a.k.C[k][j];
        s += std::fabs(a.k.C[k][j]);
      }
      M += kAngMax[k] * s;
    }
    g.M = M;
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

static const double kGenEfficiency[4] = {0.0, 0.25, 0.5, 0.05};  // first-batch guesses
static const int64_t kGenMaxBatch = 1 << 24;

template <int MODEL>
static ipx_status gen_batch(const GenConst& g, GenScratch& sc, uint64_t c0, int64_t count, int64_t got, int64_t need,
                            double* wout, hipStream_t s, int64_t* accepted) {
  const unsigned blocks = (unsigned)((count + 255) / 256);
  hipLaunchKernelGGL((k_gen_flags<MODEL>), dim3(blocks), dim3(256), 0, s, g, (const double*)sc.C, c0, count,
                     sc.flags, sc.counters);
  HIP_TRY(hipGetLastError());
  size_t bytes = sc.scan_bytes;
  HIP_TRY(hipcub::DeviceScan::ExclusiveSum(sc.scan, bytes, sc.flags, sc.rank, (int)count, s));
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

extern "C" ipx_status toy_generate(ipx_ctx* ctx, int model, const double* theta, int np, uint64_t seed,
                                   uint64_t toy_id, int64_t n, unsigned flags, ipx_dataset** out,
                                   ipx_toy_stats* stats) {
  if (!ctx || !theta || !out) return fail(IPX_EINVAL, "toy_generate: NULL argument");
  *out = nullptr;
  if (model < 1 || model > 3) return fail(IPX_EINVAL, "toy_generate: unknown model %d", model);
  if (np != kNParams[model]) return fail(IPX_EINVAL, "toy_generate: model %d takes %d parameters", model, kNParams[model]);
  if (n < 0 || n > 0x7fffffff) return fail(IPX_EINVAL, "toy_generate: n = %lld out of range", (long long)n);
  if (flags & ~IPX_KEEP_ORDER) return fail(IPX_EINVAL, "toy_generate: bad flags %u", flags);
  if (!theta_valid(model, theta)) return fail(IPX_EDOMAIN, "toy_generate: parameters outside the domain");
  HIP_TRY(hipSetDevice(ctx->device));
  hipStream_t s = ctx->stream;
  GenSetup h;
  gen_setup(model, theta, seed, toy_id, h);
  if (!(h.g.M > 0.0) || !std::isfinite(h.g.M)) return fail(IPX_EDOMAIN, "toy_generate: no finite acceptance bound");

  // output dataset, columns written in candidate order
  const int ncols = kNCols[model];
  ipx_dataset* d = new (std::nothrow) ipx_dataset();
  if (!d) return fail(IPX_ENOMEM, "toy_generate: host allocation failed");
  d->model = model;
  d->n = n;
  d->ncols = ncols;
  d->n_pad = (n + 31) / 32 * 32;
  d->n_tiles = (n + kTile - 1) / kTile;
  d->n_tiles_outer = (n + kOuterTile - 1) / kOuterTile;
  const int nstore = ncols + (model == 3 ? 1 : 0);
  const size_t bytes = (size_t)nstore * (size_t)(d->n_pad > 0 ? d->n_pad : 32) * sizeof(double);
  hipError_t e = hipMalloc(&d->base, bytes);
  const int64_t tiles_alloc = d->n_tiles > 0 ? d->n_tiles : 1;
  if (e == hipSuccess) e = hipMalloc(&d->partials, (size_t)tiles_alloc * kAccMax * sizeof(double));
  if (e == hipSuccess) e = hipMalloc(&d->out_dev, kAccMax * sizeof(double));
  if (e == hipSuccess) e = hipHostMalloc(&d->out_host, kAccMax * sizeof(double), hipHostMallocDefault);
  if (e != hipSuccess) {
    free_dataset(d);
    return fail(IPX_ENOMEM, "toy_generate: allocation failed: %s", hipGetErrorString(e));
  }
  d->bytes = bytes + (size_t)tiles_alloc * kAccMax * sizeof(double) + kAccMax * sizeof(double);
  double* colp_host[6] = {};
  for (int c = 0; c < ncols; ++c) {
    colp_host[c] = d->base + (size_t)c * d->n_pad;
    d->cols[c] = colp_host[c];
  }
  double* wout = nullptr;
  if (model == 3) {
    wout = d->base + (size_t)ncols * d->n_pad;
    d->w = wout;
  }

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
    if (e == hipSuccess) e = hipcub::DeviceScan::ExclusiveSum(nullptr, sc.scan_bytes, sc.flags, sc.rank, (int)cap, s);
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
    ipx_status st = sort_by_time(d, s);
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
  TileRef* d_tiles_outer = nullptr;
  int64_t n_tiles = 0, n_tiles_outer = 0;
  void* d_consts = nullptr;
  unsigned char* d_active = nullptr;
  double* d_out = nullptr;
  void* h_consts = nullptr;        // pinned staging, copied by the graph
  unsigned char* h_active = nullptr;
  double* h_out = nullptr;
  hipGraphExec_t exec[2] = {nullptr, nullptr};  // [eval, grad]
  hipStream_t exec_stream[2] = {nullptr, nullptr};
};

static void free_plan(ipx_plan* p) {
  for (int i = 0; i < 2; ++i)
    if (p->exec[i]) (void)hipGraphExecDestroy(p->exec[i]);
  (void)hipFree(p->d_segs); (void)hipFree(p->d_tiles); (void)hipFree(p->d_tiles_outer);
  (void)hipFree(p->d_consts); (void)hipFree(p->d_active); (void)hipFree(p->d_out);
  if (p->h_consts) (void)hipHostFree(p->h_consts);
  if (p->h_active) (void)hipHostFree(p->h_active);
  if (p->h_out) (void)hipHostFree(p->h_out);
  delete p;
}

static size_t const_size_of(int model) {
  return model == 1 ? sizeof(MassConst) : model == 2 ? sizeof(MassTimeConst) : sizeof(AngTimeConst);
}

extern "C" ipx_status ipx_plan_create(ipx_ctx* ctx, int nb, ipx_dataset* const* ds, ipx_plan** out) {
  if (!ctx || !out || (nb > 0 && !ds)) return fail(IPX_EINVAL, "ipx_plan_create: NULL argument");
  *out = nullptr;
  if (nb <= 0) return fail(IPX_EINVAL, "ipx_plan_create: empty batch");
  const int model = ds[0] ? ds[0]->model : 0;
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
  std::vector<TileRef> tiles, outer;
  hipError_t e = hipSuccess;
  for (int j = 0; j < nb && e == hipSuccess; ++j) {
    ipx_dataset* d = ds[j];
    if (model == 3 && !d->tau && d->n > 0) {
      e = hipMalloc(&d->tau, 4 * (size_t)d->n_pad * sizeof(double));
      if (e != hipSuccess) d->tau = nullptr;
      else d->bytes += 4 * (size_t)d->n_pad * sizeof(double);
    }
    SegInfo& S = segs[j];
    S.cols = cols_of(d);
    S.partials = d->partials;
    S.tau = d->tau;
    S.tau_stride = d->n_pad;
    S.n_tiles = d->n_tiles;
    S.n_tiles_outer = d->n_tiles_outer;
    for (int64_t t = 0; t < d->n_tiles; ++t) tiles.push_back(TileRef{j, (int)t});
    for (int64_t t = 0; t < d->n_tiles_outer; ++t) outer.push_back(TileRef{j, (int)t});
  }
  p->n_tiles = (int64_t)tiles.size();
  p->n_tiles_outer = (int64_t)outer.size();
  if (e == hipSuccess) e = hipMalloc(&p->d_segs, nb * sizeof(SegInfo));
  if (e == hipSuccess) e = hipMalloc(&p->d_tiles, std::max<size_t>(1, tiles.size()) * sizeof(TileRef));
  if (e == hipSuccess) e = hipMalloc(&p->d_tiles_outer, std::max<size_t>(1, outer.size()) * sizeof(TileRef));
  if (e == hipSuccess) e = hipMalloc(&p->d_consts, nb * p->const_size);
  if (e == hipSuccess) e = hipMalloc(&p->d_active, nb);
  if (e == hipSuccess) e = hipMalloc(&p->d_out, (size_t)nb * kAccMax * sizeof(double));
  if (e == hipSuccess) e = hipHostMalloc(&p->h_consts, nb * p->const_size, hipHostMallocDefault);
  if (e == hipSuccess) e = hipHostMalloc((void**)&p->h_active, nb, hipHostMallocDefault);
  if (e == hipSuccess) e = hipHostMalloc((void**)&p->h_out, (size_t)nb * kAccMax * sizeof(double), hipHostMallocDefault);
  if (e == hipSuccess) e = hipMemcpy(p->d_segs, segs.data(), nb * sizeof(SegInfo), hipMemcpyHostToDevice);
  if (e == hipSuccess && !tiles.empty())
    e = hipMemcpy(p->d_tiles, tiles.data(), tiles.size() * sizeof(TileRef), hipMemcpyHostToDevice);
  if (e == hipSuccess && !outer.empty())
    e = hipMemcpy(p->d_tiles_outer, outer.data(), outer.size() * sizeof(TileRef), hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    free_plan(p);
    return fail(IPX_ENOMEM, "ipx_plan_create: allocation failed: %s", hipGetErrorString(e));
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

// The body of one batched evaluation, as stream operations (captured once
// into a graph per plan and mode).
static ipx_status enqueue_batch(ipx_plan* p, bool grad, hipStream_t s) {
  const int nb = p->nb;
  HIP_TRY(hipMemcpyAsync(p->d_consts, p->h_consts, nb * p->const_size, hipMemcpyHostToDevice, s));
  HIP_TRY(hipMemcpyAsync(p->d_active, p->h_active, nb, hipMemcpyHostToDevice, s));
  const unsigned grid = (unsigned)std::max<int64_t>(1, p->n_tiles);
  int nacc = 1, split = 1;
  if (p->model == 1) {
    nacc = grad ? kAccMass : 1;
    split = nacc;
    if (grad) hipLaunchKernelGGL((k_nll_batch<1, true>), dim3(grid), dim3(kThreads), 0, s, p->d_segs, p->d_tiles, p->n_tiles, (const MassConst*)p->d_consts, p->d_active);
    else hipLaunchKernelGGL((k_nll_batch<1, false>), dim3(grid), dim3(kThreads), 0, s, p->d_segs, p->d_tiles, p->n_tiles, (const MassConst*)p->d_consts, p->d_active);
  } else if (p->model == 2) {
    nacc = grad ? kAccMassTime : 1;
    split = nacc;
    if (grad) hipLaunchKernelGGL((k_nll_batch<2, true>), dim3(grid), dim3(kThreads), 0, s, p->d_segs, p->d_tiles, p->n_tiles, (const MassTimeConst*)p->d_consts, p->d_active);
    else hipLaunchKernelGGL((k_nll_batch<2, false>), dim3(grid), dim3(kThreads), 0, s, p->d_segs, p->d_tiles, p->n_tiles, (const MassTimeConst*)p->d_consts, p->d_active);
  } else {
    nacc = grad ? kAccAngTime : 1;
    split = grad ? kAngInner : 1;
    if (grad) hipLaunchKernelGGL((k_angtime_batch<true>), dim3(grid), dim3(kThreads), 0, s, p->d_segs, p->d_tiles, p->n_tiles, (const AngTimeConst*)p->d_consts, p->d_active);
    else hipLaunchKernelGGL((k_angtime_batch<false>), dim3(grid), dim3(kThreads), 0, s, p->d_segs, p->d_tiles, p->n_tiles, (const AngTimeConst*)p->d_consts, p->d_active);
    HIP_TRY(hipGetLastError());
    if (grad) {
      const unsigned go = (unsigned)std::max<int64_t>(1, p->n_tiles_outer);
      hipLaunchKernelGGL(k_angtime_outer_batch, dim3(go), dim3(kThreads), 0, s, p->d_segs, p->d_tiles_outer,
                         p->n_tiles_outer, p->d_active);
    }
  }
  HIP_TRY(hipGetLastError());
  hipLaunchKernelGGL(k_reduce_batch, dim3(nacc, nb), dim3(kThreads), 0, s, p->d_segs, p->d_active, split, p->d_out);
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipMemcpyAsync(p->h_out, p->d_out, (size_t)nb * kAccMax * sizeof(double), hipMemcpyDeviceToHost, s));
  return IPX_OK;
}

extern "C" ipx_status nll_eval_batch(ipx_ctx* ctx, ipx_plan* p, const double* theta, const unsigned char* active,
                                     double* nll, double* grad, void* stream) {
  if (!ctx || !p || !theta || !nll) return fail(IPX_EINVAL, "nll_eval_batch: NULL argument");
  if (p->ctx != ctx) return fail(IPX_EINVAL, "nll_eval_batch: plan belongs to another context");
  HIP_TRY(hipSetDevice(ctx->device));
  const int model = p->model, nb = p->nb, np = kNParams[model];
  std::vector<MassHoist> h1;
  std::vector<MassTimeHoist> h2;
  std::vector<AngTimeHoist> h3;
  if (model == 1) h1.resize(nb);
  else if (model == 2) h2.resize(nb);
  else h3.resize(nb);
  int n_active = 0;
  for (int j = 0; j < nb; ++j) {
    const double* th = theta + (size_t)j * np;
    bool on = active ? active[j] != 0 : true;
    if (on && !theta_valid(model, th)) {
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
    else { h3[j] = hoist_angtime(th); std::memcpy(dst, &h3[j].k, sizeof(AngTimeConst)); }
  }
  if (n_active > 0) {
    hipStream_t s = stream ? (hipStream_t)stream : ctx->stream;
    const int mode = grad ? 1 : 0;
    if (!p->exec[mode]) {
      hipGraph_t g = nullptr;
      HIP_TRY(hipStreamBeginCapture(ctx->stream, hipStreamCaptureModeThreadLocal));
      ipx_status st = enqueue_batch(p, grad != nullptr, ctx->stream);
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
    HIP_TRY(hipGraphLaunch(p->exec[mode], s));
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

static ipx_status run(ipx_ctx* ctx, const ipx_dataset* dc, const double* theta, int np, double* nll,
                      double* grad, void* stream) {
  if (!ctx || !dc || !theta || !nll) return fail(IPX_EINVAL, "NULL argument");
  ipx_dataset* d = const_cast<ipx_dataset*>(dc);  // lazily allocated scratch only
  const int model = d->model;
  if (np != kNParams[model]) return fail(IPX_EINVAL, "model %d takes %d parameters, got %d", model, kNParams[model], np);
  if (!theta_valid(model, theta)) {
    *nll = std::numeric_limits<double>::infinity();
    if (grad)
      for (int i = 0; i < np; ++i) grad[i] = std::numeric_limits<double>::quiet_NaN();
    return fail(IPX_EDOMAIN, "parameters outside the domain of model %d", model);
  }
  HIP_TRY(hipSetDevice(ctx->device));
  hipStream_t s = stream ? (hipStream_t)stream : ctx->stream;
  ipx_status st = IPX_OK;
  MassHoist h1;
  MassTimeHoist h2;
  AngTimeHoist h3;
  const bool g = grad != nullptr;
  if (model == 1) {
    h1 = hoist_mass(theta);
    st = g ? launch_model<1, true>(ctx, d, h1.k, s) : launch_model<1, false>(ctx, d, h1.k, s);
  } else if (model == 2) {
    h2 = hoist_masstime(theta);
    st = g ? launch_model<2, true>(ctx, d, h2.k, s) : launch_model<2, false>(ctx, d, h2.k, s);
  } else {
    h3 = hoist_angtime(theta);
    st = g ? launch_angtime<true>(ctx, d, h3.k, s) : launch_angtime<false>(ctx, d, h3.k, s);
  }
  if (st != IPX_OK) return st;
  const int nacc = g ? (model == 1 ? kAccMass : model == 2 ? kAccMassTime : kAccAngTime) : 1;
  HIP_TRY(hipMemcpyAsync(d->out_host, d->out_dev, nacc * sizeof(double), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  const double* a = d->out_host;
  if (!std::isfinite(a[0])) {
    *nll = std::numeric_limits<double>::infinity();
    if (grad)
      for (int i = 0; i < np; ++i) grad[i] = std::numeric_limits<double>::quiet_NaN();
    return fail(IPX_EDOMAIN, "non-finite likelihood (an event has P <= 0 or a non-finite term)");
  }
  *nll = -a[0];
  if (g) {
    if (model == 1) grad_mass(h1, theta, a, grad);
    else if (model == 2) grad_masstime(h2, theta, a, grad);
    else grad_angtime(h3, theta, a, grad);
  }
  return IPX_OK;
}

extern "C" {

ipx_status nll_eval(ipx_ctx* ctx, const ipx_dataset* ds, const double* theta, int np, double* nll, void* stream) {
  return run(ctx, ds, theta, np, nll, nullptr, stream);
}

ipx_status nll_grad(ipx_ctx* ctx, const ipx_dataset* ds, const double* theta, int np, double* nll, double* grad,
                    void* stream) {
  if (!grad) return fail(IPX_EINVAL, "nll_grad: grad is NULL");
  return run(ctx, ds, theta, np, nll, grad, stream);
}

}  // extern "C"
