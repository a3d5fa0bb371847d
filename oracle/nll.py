"""Negative log-likelihood and its gradient (oracle test infrastructure).

NLL(theta) = - sum_i w_i ln P(x_i | theta), the FCN that the paper's examples
hand to the minimizer (Example 1 and Example 2: "-2 log L, or just -log L";
this code returns -ln L).  The sum is taken with ``math.fsum`` (exactly
rounded), so the only rounding left is in the per-event terms.

The gradient comes from forward-mode dual numbers pushed through the same PDF
definitions (``oracle.dual``), not from hand-derived formulas.
"""
import math

import numpy as np

from . import dual as D
from . import models

CHUNK = 1 << 16


def _as_cols(model, cols):
    cols = [np.ascontiguousarray(c, dtype=np.float64) for c in cols]
    if len(cols) != models.NCOLS[model]:
        raise ValueError("model %d takes %d columns" % (model, models.NCOLS[model]))
    n = cols[0].shape[0]
    if any(c.shape != (n,) for c in cols):
        raise ValueError("columns differ in length")
    return cols, n


def log_pdf(model, cols, theta, settings=None):
    """Per-event ln P as an array (value only); settings as models.pdf."""
    cols, n = _as_cols(model, cols)
    out = np.empty(n)
    th = [float(x) for x in theta]
    for lo in range(0, n, CHUNK):
        hi = min(n, lo + CHUNK)
        out[lo:hi] = np.log(models.pdf(model, [c[lo:hi] for c in cols], th, settings))
    return out


def nll(model, cols, theta, w=None, settings=None):
    """-sum_i w_i ln P_i, exactly summed; +inf outside the parameter domain or
    when any event has P <= 0 or a non-finite P."""
    if not models.theta_valid(model, theta):
        return math.inf
    lp = log_pdf(model, cols, theta, settings)
    if w is not None:
        lp = lp * np.asarray(w, dtype=np.float64)
    if not np.all(np.isfinite(lp)):
        return math.inf
    return -math.fsum(lp.tolist())


def nll_grad(model, cols, theta, w=None, settings=None):
    """(NLL, dNLL/dtheta) with the gradient from forward-mode dual numbers."""
    if not models.theta_valid(model, theta):
        return math.inf, np.full(len(theta), np.nan)
    cols, n = _as_cols(model, cols)
    K = len(theta)
    wv = None if w is None else np.asarray(w, dtype=np.float64)
    vals = np.empty(n)
    ders = np.empty((K, n))
    for lo in range(0, n, CHUNK):
        hi = min(n, lo + CHUNK)
        th = D.seed(theta)
        lp = D.log(models.pdf(model, [c[lo:hi] for c in cols], th, settings))
        v, d = lp.v, np.broadcast_to(lp.d, (K, hi - lo))
        if wv is not None:
            v = v * wv[lo:hi]
            d = d * wv[lo:hi]
        vals[lo:hi] = v
        ders[:, lo:hi] = d
    if not np.all(np.isfinite(vals)):
        return math.inf, np.full(K, np.nan)
    f = -math.fsum(vals.tolist())
    g = np.array([-math.fsum(ders[j].tolist()) for j in range(K)])
    return f, g


def nll_grad_scale(model, cols, theta, w=None, settings=None):
    """(NLL, gradient, scale): nll_grad's values plus, per parameter, the sum
    of the absolute per-event terms sum_i |w_i d ln P_i / d theta_j| (the size
    of the sum the gradient cancels down from, which bounds its rounding)."""
    if not models.theta_valid(model, theta):
        return math.inf, np.full(len(theta), np.nan), np.full(len(theta), np.nan)
    cols, n = _as_cols(model, cols)
    K = len(theta)
    wv = None if w is None else np.asarray(w, dtype=np.float64)
    vals = np.empty(n)
    ders = np.empty((K, n))
    for lo in range(0, n, CHUNK):
        hi = min(n, lo + CHUNK)
        lp = D.log(models.pdf(model, [c[lo:hi] for c in cols], D.seed(theta), settings))
        v, d = lp.v, np.broadcast_to(lp.d, (K, hi - lo))
        if wv is not None:
            v = v * wv[lo:hi]
            d = d * wv[lo:hi]
        vals[lo:hi] = v
        ders[:, lo:hi] = d
    if not np.all(np.isfinite(vals)):
        return math.inf, np.full(K, np.nan), np.full(K, np.nan)
    f = -math.fsum(vals.tolist())
    g = np.array([-math.fsum(ders[j].tolist()) for j in range(K)])
    return f, g, np.abs(ders).sum(axis=1)


def event_grad(model, cols, theta, settings=None):
    """Per-event d ln P_i / d theta, shape (K, n) (used by tolerance budgets)."""
    cols, n = _as_cols(model, cols)
    K = len(theta)
    out = np.empty((K, n))
    for lo in range(0, n, CHUNK):
        hi = min(n, lo + CHUNK)
        lp = D.log(models.pdf(model, [c[lo:hi] for c in cols], D.seed(theta), settings))
        out[:, lo:hi] = np.broadcast_to(lp.d, (K, hi - lo))
    return out
