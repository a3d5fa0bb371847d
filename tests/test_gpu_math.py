"""Device elementary functions (the inline exp, ln, sin/cos, erfcx and Faddeeva
w that the event kernels use), element by element through ipx_math_eval,
against independent references: numpy in 80-bit extended precision for exp,
ln, sin and cos (errors in ulp of the double result), scipy.special.erfcx and
scipy.special.wofz for the resolution functions (relative error of |w|; the
device routines are the Jacobi continued fraction and Weideman's rational
series, the references a separate algorithm, so agreement pins both)."""
import sys

import numpy as np
import pytest
from scipy import special

pytestmark = pytest.mark.gpu


def say(*a):
    print("[gpu]", *a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def lib():
    from paper_1706_01420_amd import ipx
    return ipx


@pytest.fixture(scope="module")
def ctx(lib):
    c = lib.ipx_create(0)
    yield c
    lib.ipx_destroy(c)


def ulp_err(y, ref, floor=0.0):
    """|y - ref| in units of the last place of max(|ref|, floor) (as double)."""
    r = ref.astype(np.float64)
    scale = np.maximum(np.abs(r), floor)
    return np.abs(y.astype(np.longdouble) - ref) / np.spacing(scale).astype(np.longdouble)


def test_exp(lib, ctx):
    rng = np.random.default_rng(11)
    x = np.concatenate([rng.uniform(-745.0, 709.7, 200000), rng.uniform(-2.0, 2.0, 100000),
                        np.array([0.0, -0.0, 1.0, -1.0, 0.5 * np.log(2.0), 1e-300, -1e-300])])
    say("exp", x.size)
    y = lib.ipx_math_eval(ctx, lib.IPX_FN_EXP, x)
    ref = np.exp(x.astype(np.longdouble))
    normal = ref.astype(np.float64) >= np.finfo(np.float64).tiny
    e = ulp_err(y[normal], ref[normal])
    say("exp max ulp", float(e.max()))
    assert e.max() <= 2.0
    # subnormal results: absolute error within one subnormal step
    sub = ~normal
    assert np.all(np.abs(y[sub] - ref[sub].astype(np.float64)) <= 2 * 4.95e-324)
    sp = lib.ipx_math_eval(ctx, lib.IPX_FN_EXP, np.array([-800.0, -1e300, -np.inf, 710.0, 1e300, np.inf, np.nan]))
    assert np.all(sp[:3] == 0.0)
    assert np.all(np.isposinf(sp[3:6]))
    assert np.isnan(sp[6])


def test_log(lib, ctx):
    rng = np.random.default_rng(12)
    x = np.concatenate([np.exp(rng.uniform(-700.0, 700.0, 200000)), rng.uniform(0.5, 2.0, 100000),
                        1.0 + rng.uniform(-1e-8, 1e-8, 1000), np.array([1.0, 2.0, 0.5, np.sqrt(0.5), 4.9e-324,
                                                                            2.2250738585072014e-308,
                                                                            1.7976931348623157e308])])
    say("log", x.size)
    y = lib.ipx_math_eval(ctx, lib.IPX_FN_LOG, x)
    ref = np.log(x.astype(np.longdouble))
    e = ulp_err(y, ref)
    e = e[np.abs(ref.astype(np.float64)) > 0]
    say("log max ulp", float(e.max()))
    assert e.max() <= 3.0
    assert lib.ipx_math_eval(ctx, lib.IPX_FN_LOG, np.array([1.0]))[0] == 0.0
    sp = lib.ipx_math_eval(ctx, lib.IPX_FN_LOG, np.array([0.0, -0.0, -1.0, np.inf, np.nan]))
    assert np.isneginf(sp[0]) and np.isneginf(sp[1])
    assert np.isnan(sp[2]) and np.isposinf(sp[3]) and np.isnan(sp[4])


def test_sincos(lib, ctx):
    rng = np.random.default_rng(13)
    x = np.concatenate([rng.uniform(-np.pi, np.pi, 100000), rng.uniform(-400.0, 400.0, 200000),
                        np.arange(-200, 201) * (np.pi / 2), rng.uniform(-1e6, 1e6, 1000),
                        np.array([0.0, 1e-300, -1e-20, 2.0 ** 19, -(2.0 ** 19) - 1.0, 1e9])])
    say("sincos", x.size)
    s, c = lib.ipx_math_eval(ctx, lib.IPX_FN_SINCOS, x)
    xl = x.astype(np.longdouble)
    # near the zeros of sin/cos the reduced argument carries an absolute
    # error below 2e-27 (|x| <= 2^19): errors in ulp of max(|ref|, 1e-9)
    es = ulp_err(s, np.sin(xl), 1e-9)
    ec = ulp_err(c, np.cos(xl), 1e-9)
    say("sin max ulp", float(es.max()), "cos max ulp", float(ec.max()))
    assert es.max() <= 2.0 and ec.max() <= 2.0
    assert s[-6] == 0.0 and c[-6] == 1.0 and s[-5] == 1e-300


def test_erfcx(lib, ctx):
    x = np.concatenate([np.linspace(0.0, 8.0, 20001), np.geomspace(1e-6, 1e7, 20000)])
    say("erfcx", x.size)
    y = lib.ipx_math_eval(ctx, lib.IPX_FN_ERFCX, x)
    ref = special.erfcx(x)
    rel = np.abs(y - ref) / ref
    say("erfcx max rel", float(rel.max()))
    assert rel.max() < 1e-13


def test_faddeeva(lib, ctx):
    rng = np.random.default_rng(14)
    # the convolution's arguments: |Re| up to a few, Im from 0 to large, both
    # branches (series |z| < 6 with Im z < 3.4, fraction elsewhere) and the
    # branch boundaries
    re = np.concatenate([rng.uniform(-8.0, 8.0, 100000), rng.uniform(-0.5, 0.5, 20000),
                         np.full(2000, 6.0), np.linspace(-5.9, 5.9, 2000), rng.uniform(-1e4, 1e4, 2000)])
    im = np.concatenate([rng.uniform(0.0, 12.0, 100000), np.geomspace(1e-3, 1e5, 20000),
                         rng.uniform(0.0, 6.0, 2000), np.full(2000, 3.4), rng.uniform(0.0, 1e4, 2000)])
    say("faddeeva", re.size)
    wr, wi = lib.ipx_math_eval(ctx, lib.IPX_FN_FADDEEVA, re, im)
    ref = special.wofz(re + 1j * im)
    rel = np.abs((wr + 1j * wi) - ref) / np.abs(ref)
    say("faddeeva max rel", float(rel.max()))
    assert rel.max() < 1e-13


def test_math_eval_errors(lib, ctx):
    with pytest.raises(lib.IpxError):
        lib.ipx_math_eval(ctx, 99, np.zeros(3))
    assert lib.ipx_math_eval(ctx, lib.IPX_FN_EXP, np.zeros(0)).size == 0
