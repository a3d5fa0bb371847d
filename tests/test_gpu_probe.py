"""The FP64 ceiling probe returns a plausible rate and clock (an FMA loop on
all compute units: between 10 % and 105 % of the nominal 78.6 TFLOP/s, clock
between 0.5 and 3 GHz)."""
import pytest

pytestmark = pytest.mark.gpu


def test_fp64_peak_probe():
    from paper_1706_01420_amd import ipx
    ctx = ipx.ipx_create(0)
    try:
        tf, ghz = ipx.ipx_fp64_peak_probe(ctx)
        assert 7.86 < tf < 82.5, tf
        assert 0.5 < ghz < 3.0, ghz
    finally:
        ipx.ipx_destroy(ctx)
