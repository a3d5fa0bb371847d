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

#include "../../include/ipx.h"
#include "ipx_hoist.h"
#include "ipx_kernels.h"

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
  double* partials = nullptr;      // n_tiles x kAccMax
  double* out_dev = nullptr;       // kAccMax
  double* out_host = nullptr;      // kAccMax, pinned
  size_t bytes = 0;
};

static const int kNParams[4] = {-1, 4, 7, 12};
static const int kNCols[4] = {-1, 1, 3, 6};

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
  if (flags > IPX_BORROW_DEVICE) return fail(IPX_EINVAL, "ipx_dataset_create: bad flags %u", flags);
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
  if (flags == IPX_BORROW_DEVICE) {
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
    const hipMemcpyKind kind = flags == IPX_COPY_HOST ? hipMemcpyHostToDevice : hipMemcpyDeviceToDevice;
    for (int c = 0; c < nstore; ++c) {
      double* dst = d->base + (size_t)c * d->n_pad;
      const double* src = c < ncols ? cols[c] : w;
      if (n > 0) e = hipMemcpyAsync(dst, src, (size_t)n * sizeof(double), kind, ctx->stream);
      if (e != hipSuccess) break;
      if (c < ncols) d->cols[c] = dst; else d->w = dst;
    }
    if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
    if (e != hipSuccess) {
      free_dataset(d);
      return fail(IPX_EDEVICE, "ipx_dataset_create: copy failed: %s", hipGetErrorString(e));
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
    hipLaunchKernelGGL(k_reduce_tiles, dim3(nacc), dim3(kThreads), 0, s, d->partials, (int64_t)0, d->out_dev);
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
  hipLaunchKernelGGL(k_reduce_tiles, dim3(nacc), dim3(kThreads), 0, s, d->partials, d->n_tiles, d->out_dev);
  HIP_TRY(hipGetLastError());
  return IPX_OK;
}

static ipx_status run(ipx_ctx* ctx, const ipx_dataset* d, const double* theta, int np, double* nll,
                      double* grad, void* stream) {
  if (!ctx || !d || !theta || !nll) return fail(IPX_EINVAL, "NULL argument");
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
    st = g ? launch_model<3, true>(ctx, d, h3.k, s) : launch_model<3, false>(ctx, d, h3.k, s);
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
