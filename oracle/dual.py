"""Forward-mode dual numbers over numpy arrays (oracle test infrastructure).

A ``Dual`` carries a value ``v`` (scalar or array, real or complex) and its
derivatives ``d`` with respect to K free parameters, shaped ``(K,) + v.shape``.
Every operation applies the chain rule of elementary calculus; nothing here is
specific to the likelihood.  The oracle evaluates its PDFs with these objects
to get the exact analytic gradient that the GPU adjoint kernels are compared
with, without any hand-derived derivative formula.

Functions accept either ``Dual`` or plain numpy values, so one definition of a
PDF serves both the value-only and the gradient evaluation.
"""
import numpy as np
from scipy import special as sp

_SQRT_PI = np.sqrt(np.pi)


class Dual:
    __slots__ = ("v", "d")
    __array_priority__ = 1000

    def __init__(self, v, d):
        self.v = np.asarray(v)
        self.d = np.asarray(d)

    @property
    def K(self):
        return self.d.shape[0]

    # -- helpers -----------------------------------------------------------
    def _dexp(self, ndim):
        """Derivative array broadcastable against a result of ``ndim`` dims."""
        extra = ndim - self.v.ndim
        if extra <= 0:
            return self.d
        return self.d.reshape((self.d.shape[0],) + (1,) * extra + self.v.shape)

    # -- arithmetic --------------------------------------------------------
    def __add__(self, o):
        if isinstance(o, Dual):
            v = self.v + o.v
            return Dual(v, self._dexp(v.ndim) + o._dexp(v.ndim))
        v = self.v + o
        return Dual(v, self._dexp(v.ndim) + np.zeros_like(v))

    __radd__ = __add__

    def __neg__(self):
        return Dual(-self.v, -self.d)

    def __sub__(self, o):
        return self + (-o)

    def __rsub__(self, o):
        return (-self) + o

    def __mul__(self, o):
        if isinstance(o, Dual):
            v = self.v * o.v
            return Dual(v, self._dexp(v.ndim) * o.v + o._dexp(v.ndim) * self.v)
        v = self.v * o
        return Dual(v, self._dexp(v.ndim) * o)

    __rmul__ = __mul__

    def __truediv__(self, o):
        if isinstance(o, Dual):
            v = self.v / o.v
            return Dual(v, (self._dexp(v.ndim) - o._dexp(v.ndim) * v) / o.v)
        v = self.v / o
        return Dual(v, self._dexp(v.ndim) / o)

    def __rtruediv__(self, o):
        # o / self
        v = o / self.v
        return Dual(v, -self._dexp(v.ndim) * v / self.v)

    def __pow__(self, n):
        if isinstance(n, Dual):
            raise TypeError("Dual exponent not supported")
        v = self.v ** n
        return Dual(v, self._dexp(v.ndim) * (n * self.v ** (n - 1)))

    def __getitem__(self, idx):
        return Dual(self.v[idx], self.d[(slice(None),) + (idx if isinstance(idx, tuple) else (idx,))])


def value(x):
    return x.v if isinstance(x, Dual) else np.asarray(x)


def _chain(x, fv, dfdx):
    """Result of applying f to x, given f(x.v) and a callable for f'(x.v)."""
    if isinstance(x, Dual):
        return Dual(fv, x._dexp(np.ndim(fv)) * dfdx())
    return fv


def exp(x):
    v = np.exp(value(x))
    return _chain(x, v, lambda: v)


def expm1(x):
    xv = value(x)
    return _chain(x, np.expm1(xv), lambda: np.exp(xv))


def log(x):
    xv = value(x)
    return _chain(x, np.log(xv), lambda: 1.0 / xv)


def sqrt(x):
    """Square root.  Its slope is infinite at 0; a direction along which the
    argument does not change leaves the root unchanged there as well (zero
    derivative, not 0 x inf), so only the directions that move a vanishing
    argument get a non-finite derivative."""
    v = np.sqrt(value(x))
    if not isinstance(x, Dual):
        return v
    d = x._dexp(np.ndim(v))
    with np.errstate(divide="ignore", invalid="ignore"):
        dv = np.where(d == 0.0, 0.0, d * (0.5 / v))
    return Dual(v, dv)


def sin(x):
    xv = value(x)
    return _chain(x, np.sin(xv), lambda: np.cos(xv))


def cos(x):
    xv = value(x)
    return _chain(x, np.cos(xv), lambda: -np.sin(xv))


def erfc(x):
    """Complementary error function of a real argument; d/dx = -2/sqrt(pi) e^{-x^2}."""
    xv = value(x)
    return _chain(x, sp.erfc(xv), lambda: -2.0 / _SQRT_PI * np.exp(-xv * xv))


def wofz(x):
    """Faddeeva function w(z) = e^{-z^2} erfc(-iz); w'(z) = -2 z w(z) + 2i/sqrt(pi)."""
    xv = value(x)
    w = sp.wofz(xv)
    return _chain(x, w, lambda: -2.0 * xv * w + 2j / _SQRT_PI)


def real(x):
    if isinstance(x, Dual):
        return Dual(np.real(x.v), np.real(x.d))
    return np.real(x)


def imag(x):
    if isinstance(x, Dual):
        return Dual(np.imag(x.v), np.imag(x.d))
    return np.imag(x)


def where(mask, a, b):
    """Elementwise select; mask is a plain boolean array."""
    if not isinstance(a, Dual) and not isinstance(b, Dual):
        return np.where(mask, a, b)
    av, bv = value(a), value(b)
    v = np.where(mask, av, bv)
    K = a.K if isinstance(a, Dual) else b.K
    ad = a._dexp(v.ndim) if isinstance(a, Dual) else np.zeros((K,) + (1,) * v.ndim)
    bd = b._dexp(v.ndim) if isinstance(b, Dual) else np.zeros((K,) + (1,) * v.ndim)
    return Dual(v, np.where(mask, ad, bd))


def seed(theta):
    """Independent variables: theta[j] gets unit derivative along direction j."""
    theta = np.asarray(theta, dtype=np.float64)
    K = theta.shape[0]
    eye = np.eye(K)
    return [Dual(theta[j], eye[:, j].copy()) for j in range(K)]
