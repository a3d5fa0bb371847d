"""Thin ctypes binding of libipx (include/ipx.h): argument marshalling only.

Every function keeps the C name.  Device work happens in the library's HIP
kernels; nothing here computes a likelihood.  Importing this module imports
torch first, so that libipx binds to the HIP runtime torch has already mapped
(one runtime per process; torch tensors and streams can then be passed in).
If libipx.so is missing the import fails: there is no fallback path.
"""
import ctypes
import os
import threading

import numpy as np
import torch  # noqa: F401  (maps torch's HIP runtime before libipx is loaded)

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libipx.so")

IPX_OK = 0
IPX_EINVAL = -1
IPX_ENOMEM = -2
IPX_EDEVICE = -3
IPX_EBUSY = -4
IPX_ENOTFOUND = -5
IPX_ETIMEOUT = -6
IPX_EDOMAIN = -7
IPX_ECANCELED = -8
STATUS_NAMES = {0: "IPX_OK", -1: "IPX_EINVAL", -2: "IPX_ENOMEM", -3: "IPX_EDEVICE", -4: "IPX_EBUSY",
                -5: "IPX_ENOTFOUND", -6: "IPX_ETIMEOUT", -7: "IPX_EDOMAIN", -8: "IPX_ECANCELED"}

IPX_MODEL_MASS = 1
IPX_MODEL_MASSTIME = 2
IPX_MODEL_ANGTIME = 3
IPX_MODEL_ANGTIME_TAGGED = 4
IPX_MODEL_IPATIA = 5

IPX_COPY_HOST = 0
IPX_COPY_DEVICE = 1
IPX_BORROW_DEVICE = 2
IPX_KEEP_ORDER = 4
IPX_NO_WEIGHTS = 8
IPX_FN_EXP, IPX_FN_LOG, IPX_FN_SINCOS, IPX_FN_ERFCX, IPX_FN_FADDEEVA = 0, 1, 2, 3, 4

_c_double_p = ctypes.POINTER(ctypes.c_double)
_c_void_pp = ctypes.POINTER(ctypes.c_void_p)

# (name, restype, argtypes) of every exported function
_SIGNATURES = [
    ("ipx_create", ctypes.c_int, [ctypes.c_int, _c_void_pp]),
    ("ipx_destroy", None, [ctypes.c_void_p]),
    ("ipx_last_error", ctypes.c_char_p, []),
    ("ipx_model_nparams", ctypes.c_int, [ctypes.c_int]),
    ("ipx_model_ncols", ctypes.c_int, [ctypes.c_int]),
    ("ipx_dataset_create", ctypes.c_int,
     [ctypes.c_void_p, ctypes.c_int, ctypes.c_int64, ctypes.POINTER(ctypes.c_void_p), ctypes.c_int,
      ctypes.c_void_p, ctypes.c_uint, _c_void_pp]),
    ("ipx_dataset_destroy", ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p]),
    ("ipx_dataset_bytes", ctypes.c_size_t, [ctypes.c_void_p]),
    ("ipx_dataset_size", ctypes.c_int64, [ctypes.c_void_p]),
    ("ipx_dataset_model", ctypes.c_int, [ctypes.c_void_p]),
    ("ipx_dataset_column", ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, _c_void_pp]),
    ("ipx_dataset_set_angular", ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_double]),
    ("ipx_dataset_read", ctypes.c_int,
     [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int, ctypes.c_int64, ctypes.c_int64, _c_double_p]),
    # pointer arguments as plain addresses (the per-call marshalling below)
    ("nll_eval", ctypes.c_int,
     [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p]),
    ("nll_grad", ctypes.c_int,
     [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p,
      ctypes.c_void_p]),
    ("nll_eval_noalloc", ctypes.c_int,
     [ctypes.c_void_p, ctypes.c_int, ctypes.c_int64, ctypes.POINTER(ctypes.c_void_p), ctypes.c_int,
      ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    ("ipx_sim_create", ctypes.c_int,
     [ctypes.c_void_p, ctypes.c_int, ctypes.POINTER(ctypes.c_void_p), ctypes.POINTER(ctypes.c_int), ctypes.c_int,
      _c_void_pp]),
    ("ipx_sim_destroy", None, [ctypes.c_void_p]),
    ("ipx_sim_nparams", ctypes.c_int, [ctypes.c_void_p]),
    ("nll_sim", ctypes.c_int,
     [ctypes.c_void_p, ctypes.c_void_p, _c_double_p, ctypes.c_int, _c_double_p, ctypes.c_void_p, ctypes.c_void_p]),
    ("ipx_plan_create", ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.POINTER(ctypes.c_void_p), _c_void_pp]),
    ("ipx_plan_destroy", None, [ctypes.c_void_p]),
    ("nll_eval_batch", ctypes.c_int,
     [ctypes.c_void_p, ctypes.c_void_p, _c_double_p, ctypes.c_void_p, _c_double_p, ctypes.c_void_p,
      ctypes.c_void_p]),
    ("ipx_server_start", ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, _c_void_pp]),
    ("ipx_submit", ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.POINTER(ctypes.c_uint64)]),
    ("ipx_poll", ctypes.c_int, [ctypes.c_void_p, ctypes.c_uint64, ctypes.c_void_p]),
    ("ipx_wait", ctypes.c_int, [ctypes.c_void_p, ctypes.c_uint64, ctypes.c_int64, ctypes.c_void_p]),
    ("ipx_server_drain", ctypes.c_int, [ctypes.c_void_p]),
    ("ipx_cancel", ctypes.c_int, [ctypes.c_void_p, ctypes.c_uint64]),
    ("ipx_server_stop", ctypes.c_int, [ctypes.c_void_p]),
    ("ipx_server_stats_read", ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p]),
    ("toy_generate", ctypes.c_int,
     [ctypes.c_void_p, ctypes.c_int, _c_double_p, ctypes.c_int, ctypes.c_uint64, ctypes.c_uint64, ctypes.c_int64,
      ctypes.c_uint, _c_void_pp, ctypes.c_void_p]),
    ("toy_generate_batch", ctypes.c_int,
     [ctypes.c_void_p, ctypes.c_int, _c_double_p, ctypes.c_int, ctypes.c_uint64, ctypes.c_int, ctypes.c_void_p,
      ctypes.c_void_p, ctypes.c_uint, ctypes.c_void_p, ctypes.c_void_p]),
    ("ipx_smear", ctypes.c_int,
     [ctypes.c_void_p, ctypes.c_int, ctypes.c_double, ctypes.c_double, ctypes.c_void_p, ctypes.c_void_p,
      ctypes.c_void_p]),
    ("ipx_hist_create", ctypes.c_int,
     [ctypes.c_void_p, ctypes.c_int, ctypes.c_double, ctypes.c_double, ctypes.c_double, ctypes.c_double,
      ctypes.c_double, ctypes.c_void_p, _c_void_pp]),
    ("ipx_hist_destroy", ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p]),
    ("ipx_hist_nbins", ctypes.c_int, [ctypes.c_void_p]),
    ("ipx_hist_read", ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int, _c_double_p]),
    ("ipx_hist_set_counts", ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, _c_double_p]),
    ("nll_binned", ctypes.c_int,
     [ctypes.c_void_p, ctypes.c_void_p, _c_double_p, ctypes.c_int, _c_double_p, ctypes.c_void_p, ctypes.c_void_p]),
    ("ipx_binned_toy", ctypes.c_int,
     [ctypes.c_void_p, ctypes.c_void_p, _c_double_p, ctypes.c_uint64, ctypes.c_int, ctypes.c_uint64, _c_double_p]),
    ("cls_toys", ctypes.c_int,
     [ctypes.c_void_p, ctypes.c_void_p, _c_double_p, ctypes.c_uint64, ctypes.c_int, ctypes.c_void_p,
      ctypes.c_void_p]),
    ("ipx_timing_enable", ctypes.c_int, [ctypes.c_void_p, ctypes.c_int]),
    ("ipx_timing_read", ctypes.c_int,
     [ctypes.c_void_p, _c_double_p, ctypes.POINTER(ctypes.c_int64), ctypes.c_int]),
    ("ipx_plan_set_schedule", ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p]),
    ("ipx_plan_get_schedule", ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p]),
    ("ipx_plan_autotune", ctypes.c_int,
     [ctypes.c_void_p, ctypes.c_void_p, _c_double_p, ctypes.c_int, ctypes.c_int, ctypes.c_void_p, _c_double_p,
      ctypes.c_void_p, ctypes.POINTER(ctypes.c_int)]),
    ("ipx_count_bad_events", ctypes.c_int,
     [ctypes.c_void_p, ctypes.c_void_p, _c_double_p, ctypes.c_int, ctypes.POINTER(ctypes.c_int64)]),
    ("ipx_event_logp", ctypes.c_int,
     [ctypes.c_void_p, ctypes.c_void_p, _c_double_p, ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p]),
    ("ipx_fp64_peak_probe", ctypes.c_int, [ctypes.c_void_p, _c_double_p, _c_double_p]),
    ("ipx_math_eval", ctypes.c_int,
     [ctypes.c_void_p, ctypes.c_int, ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
      ctypes.c_void_p]),
]
EXPORTED = [s[0] for s in _SIGNATURES]


class IpxError(RuntimeError):
    def __init__(self, status, message):
        super().__init__("%s: %s" % (STATUS_NAMES.get(status, status), message))
        self.status = status


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError("libipx.so is not built (python -m paper_1706_01420_amd.build)")
    lib = ctypes.CDLL(LIB_PATH)
    for name, res, args in _SIGNATURES:
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib


_lib = _load()


def _check(status):
    if status != IPX_OK:
        raise IpxError(status, _lib.ipx_last_error().decode())
    return status


def _stream_ptr(stream):
    if stream is None:
        return None
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream  # torch.cuda.Stream


def _dbl(a):
    return a.ctypes.data_as(_c_double_p)


# ---------------------------------------------------------------------------
# C functions (same names)
# ---------------------------------------------------------------------------
def ipx_create(device=0):
    h = ctypes.c_void_p()
    _check(_lib.ipx_create(int(device), ctypes.byref(h)))
    return h


def ipx_destroy(ctx):
    _lib.ipx_destroy(ctx)


def ipx_last_error():
    return _lib.ipx_last_error().decode()


def ipx_model_nparams(model):
    return _lib.ipx_model_nparams(int(model))


def ipx_model_ncols(model):
    return _lib.ipx_model_ncols(int(model))


def ipx_dataset_create(ctx, model, cols, w=None, flags=IPX_COPY_HOST):
    """cols: list of 1-D float64 arrays (host numpy arrays for IPX_COPY_HOST,
    CUDA torch tensors for the device flags)."""
    ncols = len(cols)
    keep = []
    ptrs = (ctypes.c_void_p * max(ncols, 1))()
    n = None
    kind = flags & 3
    for i, c in enumerate(cols):
        if kind == IPX_COPY_HOST:
            c = np.ascontiguousarray(c, dtype=np.float64)
            keep.append(c)
            ptrs[i] = c.ctypes.data
            length = c.shape[0]
        else:
            if not (isinstance(c, torch.Tensor) and c.is_cuda and c.dtype == torch.float64 and c.is_contiguous()):
                raise TypeError("device columns must be contiguous float64 CUDA tensors")
            ptrs[i] = c.data_ptr()
            length = c.shape[0]
        if n is None:
            n = length
        elif n != length:
            raise ValueError("columns differ in length")
    wp = None
    if w is not None:
        if kind == IPX_COPY_HOST:
            w = np.ascontiguousarray(w, dtype=np.float64)
            keep.append(w)
            wp = w.ctypes.data
        else:
            wp = w.data_ptr()
        if w.shape[0] != n:
            raise ValueError("weights differ in length")
    h = ctypes.c_void_p()
    _check(_lib.ipx_dataset_create(ctx, int(model), int(n or 0), ptrs, ncols, wp, int(flags), ctypes.byref(h)))
    return h


def ipx_dataset_destroy(ctx, ds):
    _check(_lib.ipx_dataset_destroy(ctx, ds))


def ipx_dataset_bytes(ds):
    return _lib.ipx_dataset_bytes(ds)


def ipx_dataset_size(ds):
    return _lib.ipx_dataset_size(ds)


def ipx_dataset_model(ds):
    return _lib.ipx_dataset_model(ds)


def ipx_dataset_column(ds, col):
    p = ctypes.c_void_p()
    _check(_lib.ipx_dataset_column(ds, int(col), ctypes.byref(p)))
    return p.value


def ipx_dataset_set_angular(ctx, ds, xi=None, c_sp=1.0):
    """Normalisation weights xi (10 values, None: flat efficiency) and S-P
    factor c_sp of an angular dataset."""
    xp = None
    if xi is not None:
        xi = np.ascontiguousarray(xi, dtype=np.float64)
        if xi.shape != (10,):
            raise ValueError("xi takes 10 values")
        xp = xi.ctypes.data
    _check(_lib.ipx_dataset_set_angular(ctx, ds, xp, float(c_sp)))


def ipx_dataset_read(ctx, ds, col, offset=0, count=None):
    """Host copy (numpy) of column `col` of a dataset, in storage order."""
    n = ipx_dataset_size(ds)
    count = n - offset if count is None else count
    out = np.empty(count)
    _check(_lib.ipx_dataset_read(ctx, ds, int(col), int(offset), int(count), _dbl(out)))
    return out


class _CallBuffers:
    """Per-thread argument buffers of the single-dataset calls: theta is copied
    into a fixed array whose address is taken once, so a call costs one small
    copy instead of building ctypes pointer objects."""
    CAP = 64

    def __init__(self):
        self.th = np.empty(self.CAP)
        self.g = np.empty(self.CAP)
        self.out = np.empty(1)
        self.th_p, self.g_p, self.out_p = self.th.ctypes.data, self.g.ctypes.data, self.out.ctypes.data


_tls = threading.local()


def _buffers(theta):
    b = getattr(_tls, "b", None)
    if b is None:
        b = _tls.b = _CallBuffers()
    n = len(theta)
    if n > b.CAP:
        raise ValueError("theta has %d entries" % n)
    b.th[:n] = theta
    return b, n


def nll_eval(ctx, ds, theta, stream=None):
    """-sum w ln P at theta; +inf for IPX_EDOMAIN (parameters outside the domain
    or a non-finite likelihood), an exception for any other error."""
    b, n = _buffers(theta)
    st = _lib.nll_eval(ctx, ds, b.th_p, n, b.out_p, None if stream is None else _stream_ptr(stream))
    if st == IPX_EDOMAIN:
        return float("inf")
    _check(st)
    return float(b.out[0])


def nll_grad(ctx, ds, theta, stream=None):
    """(NLL, dNLL/dtheta); (+inf, NaN) for IPX_EDOMAIN."""
    b, n = _buffers(theta)
    st = _lib.nll_grad(ctx, ds, b.th_p, n, b.out_p, b.g_p, None if stream is None else _stream_ptr(stream))
    if st == IPX_EDOMAIN:
        return float("inf"), np.full(n, np.nan)
    _check(st)
    return float(b.out[0]), b.g[:n].copy()


def nll_eval_noalloc(ctx, model, cols, w, theta, grad=False, stream=None):
    """nll_eval (grad=False: returns NLL) or nll_grad (grad=True: returns
    (NLL, gradient)) over contiguous float64 CUDA tensors used in place, with
    the library's fixed scratch (no allocation); +inf (and NaN gradients) for
    IPX_EDOMAIN."""
    ncols = len(cols)
    ptrs = (ctypes.c_void_p * max(ncols, 1))()
    n = None
    for i, c in enumerate(cols):
        if not (isinstance(c, torch.Tensor) and c.is_cuda and c.dtype == torch.float64 and c.is_contiguous()):
            raise TypeError("columns must be contiguous float64 CUDA tensors")
        ptrs[i] = c.data_ptr()
        if n is None:
            n = c.shape[0]
        elif n != c.shape[0]:
            raise ValueError("columns differ in length")
    wp = None
    if w is not None:
        if not (isinstance(w, torch.Tensor) and w.is_cuda and w.dtype == torch.float64 and w.is_contiguous()):
            raise TypeError("weights must be a contiguous float64 CUDA tensor")
        if w.shape[0] != n:
            raise ValueError("weights differ in length")
        wp = w.data_ptr()
    b, npar = _buffers(theta)
    st = _lib.nll_eval_noalloc(ctx, int(model), int(n or 0), ptrs, ncols, wp, b.th_p, npar, b.out_p,
                               b.g_p if grad else None, None if stream is None else _stream_ptr(stream))
    if st == IPX_EDOMAIN:
        return (float("inf"), np.full(npar, np.nan)) if grad else float("inf")
    _check(st)
    return (float(b.out[0]), b.g[:npar].copy()) if grad else float(b.out[0])


class _NLL(torch.autograd.Function):
    """-ln L as a differentiable torch scalar: the forward runs nll_grad and
    keeps the gradient, the backward scales it by the incoming gradient."""

    @staticmethod
    def forward(fctx, theta, ctx, ds):
        f, g = nll_grad(ctx, ds, theta.detach().to("cpu", torch.float64).numpy())
        fctx.save_for_backward(torch.from_numpy(g))
        return torch.tensor(f, dtype=theta.dtype, device=theta.device)

    @staticmethod
    def backward(fctx, grad_out):
        (g,) = fctx.saved_tensors
        return grad_out * g.to(device=grad_out.device, dtype=grad_out.dtype), None, None


def nll(ctx, ds, theta):
    """NLL of dataset ds at theta (a 1-D float64 torch tensor); differentiable
    with respect to theta through the analytic gradient."""
    return _NLL.apply(theta, ctx, ds)


def ipx_sim_create(ctx, datasets, bins, nbins):
    """Simultaneous set of angular categories (dataset c in KK-mass bin bins[c])."""
    arr = (ctypes.c_void_p * len(datasets))(*[d.value for d in datasets])
    b = (ctypes.c_int * len(datasets))(*[int(x) for x in bins])
    h = ctypes.c_void_p()
    _check(_lib.ipx_sim_create(ctx, len(datasets), arr, b, int(nbins), ctypes.byref(h)))
    return h


def ipx_sim_destroy(sim):
    _lib.ipx_sim_destroy(sim)


def ipx_sim_nparams(sim):
    return _lib.ipx_sim_nparams(sim)


def nll_sim(ctx, sim, theta, grad=False, stream=None):
    """Joint NLL of the set's categories (and its gradient); +inf (NaN
    gradient) for IPX_EDOMAIN."""
    th = np.ascontiguousarray(theta, dtype=np.float64)
    out = np.empty(1)
    g = np.empty(th.shape[0]) if grad else None
    st = _lib.nll_sim(ctx, sim, _dbl(th), th.shape[0], _dbl(out), None if g is None else g.ctypes.data,
                      None if stream is None else _stream_ptr(stream))
    if st == IPX_EDOMAIN:
        return (float("inf"), np.full(th.shape[0], np.nan)) if grad else float("inf")
    _check(st)
    return (float(out[0]), g) if grad else float(out[0])


def ipx_plan_create(ctx, datasets):
    arr = (ctypes.c_void_p * len(datasets))(*[d.value for d in datasets])
    h = ctypes.c_void_p()
    _check(_lib.ipx_plan_create(ctx, len(datasets), arr, ctypes.byref(h)))
    return h


def ipx_plan_destroy(plan):
    _lib.ipx_plan_destroy(plan)


class _Schedule(ctypes.Structure):
    _fields_ = [("workgroups", ctypes.c_int), ("order", ctypes.c_int), ("graph", ctypes.c_int),
                ("variant", ctypes.c_int)]


class _TuneEntry(ctypes.Structure):
    _fields_ = [("schedule", _Schedule), ("us", ctypes.c_double)]


def _sched_dict(sc):
    return {"workgroups": sc.workgroups, "order": sc.order, "graph": sc.graph, "variant": sc.variant}


def ipx_plan_set_schedule(plan, workgroups=0, order=0, graph=1, variant=0):
    """Launch schedule of the plan's per-event kernel (results do not depend on it)."""
    sc = _Schedule(int(workgroups), int(order), int(graph), int(variant))
    _check(_lib.ipx_plan_set_schedule(plan, ctypes.byref(sc)))


def ipx_plan_get_schedule(plan):
    sc = _Schedule()
    _check(_lib.ipx_plan_get_schedule(plan, ctypes.byref(sc)))
    return _sched_dict(sc)


def ipx_plan_autotune(ctx, plan, theta, grad=True, reps=5):
    """Time the candidate schedules at theta (nb, np), keep the fastest on the
    plan; returns (best schedule dict, its median us, [(schedule dict, us), ...])."""
    th = np.ascontiguousarray(theta, dtype=np.float64)
    best = _Schedule()
    best_us = ctypes.c_double()
    table = (_TuneEntry * 64)()
    n = ctypes.c_int(64)
    _check(_lib.ipx_plan_autotune(ctx, plan, _dbl(th), 1 if grad else 0, int(reps), ctypes.byref(best),
                                  ctypes.byref(best_us), table, ctypes.byref(n)))
    rows = [(_sched_dict(table[i].schedule), table[i].us) for i in range(n.value)]
    return _sched_dict(best), best_us.value, rows


def nll_eval_batch(ctx, plan, theta, active=None, grad=False, stream=None):
    """theta: (nb, np).  Returns nll (nb,) and, with grad=True, (nll, grad (nb, np)).
    Entries outside the domain / non-finite come back as +inf (NaN gradient)."""
    th = np.ascontiguousarray(theta, dtype=np.float64)
    nb, np_ = th.shape
    nll = np.full(nb, np.nan)
    g = np.full((nb, np_), np.nan) if grad else None
    act = None
    if active is not None:
        act = np.ascontiguousarray(active, dtype=np.uint8)
    st = _lib.nll_eval_batch(ctx, plan, _dbl(th), None if act is None else act.ctypes.data, _dbl(nll),
                             None if g is None else g.ctypes.data, _stream_ptr(stream))
    if st not in (IPX_OK, IPX_EDOMAIN):
        _check(st)
    return (nll, g) if grad else nll


class ServerCfg(ctypes.Structure):
    _fields_ = [("slots", ctypes.c_int), ("scratch_bytes", ctypes.c_size_t), ("workgroups", ctypes.c_int),
                ("idle_iterations", ctypes.c_int), ("max_pending", ctypes.c_int), ("policy", ctypes.c_int)]


class _Request(ctypes.Structure):
    _fields_ = [("ds", ctypes.c_void_p), ("theta", _c_double_p), ("np", ctypes.c_int), ("want_grad", ctypes.c_int)]


class _Result(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int), ("np", ctypes.c_int), ("nll", ctypes.c_double),
                ("grad", ctypes.c_double * 12), ("latency_us", ctypes.c_double)]


def _result_dict(r):
    return {"status": r.status, "nll": r.nll, "grad": np.array(r.grad[:r.np]), "latency_us": r.latency_us}


SERVE_SPREAD = 0
SERVE_OLDEST_FIRST = 1
SERVE_FEWEST_FIRST = 2


def ipx_server_start(ctx, slots=0, scratch_bytes=0, workgroups=0, idle_iterations=0, max_pending=0,
                     policy=SERVE_SPREAD):
    cfg = ServerCfg(slots, scratch_bytes, workgroups, idle_iterations, max_pending, policy)
    h = ctypes.c_void_p()
    _check(_lib.ipx_server_start(ctx, ctypes.byref(cfg), ctypes.byref(h)))
    return h


def ipx_submit(srv, ds, theta, want_grad=False):
    th = np.ascontiguousarray(theta, dtype=np.float64)
    req = _Request(ds.value if isinstance(ds, ctypes.c_void_p) else ds, _dbl(th), th.shape[0], 1 if want_grad else 0)
    t = ctypes.c_uint64()
    _check(_lib.ipx_submit(srv, ctypes.byref(req), ctypes.byref(t)))
    return t.value


def ipx_poll(srv, ticket):
    """Result dict when done (taken once), None while running."""
    r = _Result()
    st = _lib.ipx_poll(srv, ctypes.c_uint64(ticket), ctypes.byref(r))
    if st == IPX_EBUSY:
        return None
    if st not in (IPX_OK, IPX_EDOMAIN, IPX_ETIMEOUT, IPX_ECANCELED):
        _check(st)
    return _result_dict(r)


def ipx_wait(srv, ticket, timeout_s=-1.0):
    r = _Result()
    st = _lib.ipx_wait(srv, ctypes.c_uint64(ticket), int(timeout_s * 1e9) if timeout_s >= 0 else -1, ctypes.byref(r))
    if st not in (IPX_OK, IPX_EDOMAIN, IPX_ECANCELED):
        _check(st)
    return _result_dict(r)


def ipx_cancel(srv, ticket):
    """Withdraw a request still waiting for a slot (its result, status
    IPX_ECANCELED, is then taken as usual); IpxError with IPX_EBUSY if it is
    on the device or finished."""
    _check(_lib.ipx_cancel(srv, ctypes.c_uint64(ticket)))


def ipx_server_drain(srv):
    """Block until every request submitted so far has finished (results stay
    available to ipx_poll / ipx_wait)."""
    _check(_lib.ipx_server_drain(srv))


def ipx_server_stop(srv):
    _check(_lib.ipx_server_stop(srv))


class _ServerStats(ctypes.Structure):
    _fields_ = [("published", ctypes.c_uint64), ("completed", ctypes.c_uint64), ("launches", ctypes.c_uint64),
                ("pending", ctypes.c_uint64), ("in_flight", ctypes.c_uint64), ("cancelled", ctypes.c_uint64)]


def ipx_server_stats_read(srv):
    r = _ServerStats()
    _check(_lib.ipx_server_stats_read(srv, ctypes.byref(r)))
    return {k: int(getattr(r, k)) for k, _ in _ServerStats._fields_}


class _ToyStats(ctypes.Structure):
    _fields_ = [("n_candidates", ctypes.c_uint64), ("n_violations", ctypes.c_uint64)]


def toy_generate(ctx, model, theta_gen, seed, toy_id, n, flags=0):
    """Generate n events; returns (dataset handle, {"n_candidates", "n_violations"})."""
    th = np.ascontiguousarray(theta_gen, dtype=np.float64)
    h = ctypes.c_void_p()
    st = _ToyStats()
    _check(_lib.toy_generate(ctx, int(model), _dbl(th), th.shape[0], ctypes.c_uint64(seed), ctypes.c_uint64(toy_id),
                             int(n), int(flags), ctypes.byref(h), ctypes.byref(st)))
    return h, {"n_candidates": st.n_candidates, "n_violations": st.n_violations}


def toy_generate_batch(ctx, model, theta_gen, seed, toy_ids, sizes, flags=0):
    """Generate many toys at once; returns (list of dataset handles, list of
    stats dicts), toy j equal to toy_generate(..., toy_ids[j], sizes[j], flags)."""
    th = np.ascontiguousarray(theta_gen, dtype=np.float64)
    ids = np.ascontiguousarray(toy_ids, dtype=np.uint64)
    ns = np.ascontiguousarray(sizes, dtype=np.int64)
    k = ids.shape[0]
    if ns.shape[0] != k:
        raise ValueError("toy_ids and sizes differ in length")
    outs = (ctypes.c_void_p * max(k, 1))()
    st = (_ToyStats * max(k, 1))()
    _check(_lib.toy_generate_batch(ctx, int(model), _dbl(th), th.shape[0], ctypes.c_uint64(seed), k,
                                   ids.ctypes.data, ns.ctypes.data, int(flags), outs, st))
    return ([ctypes.c_void_p(outs[j]) for j in range(k)],
            [{"n_candidates": st[j].n_candidates, "n_violations": st[j].n_violations} for j in range(k)])


def ipx_timing_enable(ctx, enable=True):
    _check(_lib.ipx_timing_enable(ctx, 1 if enable else 0))


def ipx_timing_read(ctx, reset=False):
    ms = ctypes.c_double()
    n = ctypes.c_int64()
    _check(_lib.ipx_timing_read(ctx, ctypes.byref(ms), ctypes.byref(n), 1 if reset else 0))
    return ms.value, n.value


def ipx_math_eval(ctx, fn, x, x2=None):
    """Device elementary function fn (IPX_FN_*) on the array x (and x2 for the
    Faddeeva function); returns y, or (y, y2) for IPX_FN_SINCOS and
    IPX_FN_FADDEEVA."""
    x = np.ascontiguousarray(x, np.float64).ravel()
    n = x.size
    two_out = fn in (IPX_FN_SINCOS, IPX_FN_FADDEEVA)
    if fn == IPX_FN_FADDEEVA:
        x2 = np.ascontiguousarray(x2, np.float64).ravel()
        if x2.size != n:
            raise ValueError("x2 must have the size of x")
    y = np.empty(n)
    y2 = np.empty(n) if two_out else None
    _check(_lib.ipx_math_eval(ctx, int(fn), n, x.ctypes.data, x2.ctypes.data if x2 is not None else None,
                              y.ctypes.data, y2.ctypes.data if two_out else None))
    return (y, y2) if two_out else y


def ipx_count_bad_events(ctx, ds, theta):
    """Number of events of ds whose contribution w ln P at theta is not finite."""
    th = np.ascontiguousarray(theta, np.float64)
    n = ctypes.c_int64()
    _check(_lib.ipx_count_bad_events(ctx, ds, _dbl(th), th.size, ctypes.byref(n)))
    return n.value


def ipx_event_logp(ctx, ds, theta, out=None, stream=None):
    """Per-event terms w_i ln P_i at theta in storage order, written by the
    library into a float64 CUDA tensor (out, or a new one); returns it."""
    th = np.ascontiguousarray(theta, np.float64)
    n = _lib.ipx_dataset_size(ds)
    if out is None:
        out = torch.empty(max(n, 0), dtype=torch.float64, device="cuda")
    elif not (isinstance(out, torch.Tensor) and out.is_cuda and out.dtype == torch.float64
              and out.is_contiguous() and out.numel() >= n):
        raise TypeError("out must be a contiguous float64 CUDA tensor of at least %d elements" % n)
    _check(_lib.ipx_event_logp(ctx, ds, _dbl(th), th.size, out.data_ptr() if n > 0 else None,
                               _stream_ptr(stream)))
    return out


def ipx_fp64_peak_probe(ctx):
    """Attainable FP64 rate of the device: (TFLOP/s of an FMA loop, its median shader clock in GHz)."""
    tf = ctypes.c_double()
    ghz = ctypes.c_double()
    _check(_lib.ipx_fp64_peak_probe(ctx, ctypes.byref(tf), ctypes.byref(ghz)))
    return tf.value, ghz.value


# ---------------------------------------------------------------------------
# Binned path
# ---------------------------------------------------------------------------
class _ClsResult(ctypes.Structure):
    _fields_ = [("cl_sb", ctypes.c_double), ("cl_b", ctypes.c_double), ("cl_s", ctypes.c_double),
                ("q_obs", ctypes.c_double), ("n_sb", ctypes.c_int64), ("n_b", ctypes.c_int64)]


def ipx_smear(ctx, h, dx, sigma, out=None, stream=None):
    """Gaussian smearing of the binned shape h (a float64 CUDA tensor); returns out."""
    if not (isinstance(h, torch.Tensor) and h.is_cuda and h.dtype == torch.float64 and h.is_contiguous()):
        raise TypeError("h must be a contiguous float64 CUDA tensor")
    if out is None:
        out = torch.empty_like(h)
    _check(_lib.ipx_smear(ctx, int(h.shape[0]), float(dx), float(sigma), h.data_ptr(), out.data_ptr(),
                          None if stream is None else _stream_ptr(stream)))
    return out


def ipx_hist_create(ctx, nbins, lo, hi, mu, sigma_core, sigma_smear, counts=None):
    cp = None
    if counts is not None:
        counts = np.ascontiguousarray(counts, dtype=np.float64)
        if counts.shape != (nbins,):
            raise ValueError("counts must have nbins entries")
        cp = counts.ctypes.data
    h = ctypes.c_void_p()
    _check(_lib.ipx_hist_create(ctx, int(nbins), float(lo), float(hi), float(mu), float(sigma_core),
                                float(sigma_smear), cp, ctypes.byref(h)))
    return h


def ipx_hist_destroy(ctx, hist):
    _check(_lib.ipx_hist_destroy(ctx, hist))


def ipx_hist_read(ctx, hist, which=0):
    out = np.empty(_lib.ipx_hist_nbins(hist))
    _check(_lib.ipx_hist_read(ctx, hist, int(which), _dbl(out)))
    return out


def ipx_hist_set_counts(ctx, hist, counts):
    c = np.ascontiguousarray(counts, dtype=np.float64)
    _check(_lib.ipx_hist_set_counts(ctx, hist, _dbl(c)))


def nll_binned(ctx, hist, theta, grad=False, stream=None):
    th = np.ascontiguousarray(theta, dtype=np.float64)
    out = np.empty(1)
    g = np.empty(3) if grad else None
    st = _lib.nll_binned(ctx, hist, _dbl(th), th.shape[0], _dbl(out), None if g is None else g.ctypes.data,
                         None if stream is None else _stream_ptr(stream))
    if st == IPX_EDOMAIN:
        return (float("inf"), np.full(3, np.nan)) if grad else float("inf")
    _check(st)
    return (float(out[0]), g) if grad else float(out[0])


def ipx_binned_toy(ctx, hist, theta, seed, hyp, toy):
    th = np.ascontiguousarray(theta, dtype=np.float64)
    out = np.empty(_lib.ipx_hist_nbins(hist))
    _check(_lib.ipx_binned_toy(ctx, hist, _dbl(th), ctypes.c_uint64(seed), int(hyp), ctypes.c_uint64(toy), _dbl(out)))
    return out


def cls_toys(ctx, hist, theta, seed, ntoys, want_q=False):
    """dict(cl_sb, cl_b, cl_s, q_obs, n_sb, n_b[, q_b, q_sb])."""
    th = np.ascontiguousarray(theta, dtype=np.float64)
    r = _ClsResult()
    q = np.empty(2 * ntoys) if want_q else None
    _check(_lib.cls_toys(ctx, hist, _dbl(th), ctypes.c_uint64(seed), int(ntoys), ctypes.byref(r),
                         None if q is None else q.ctypes.data))
    out = {k: getattr(r, k) for k, _ in _ClsResult._fields_}
    if q is not None:
        out["q_b"], out["q_sb"] = q[:ntoys], q[ntoys:]
    return out
