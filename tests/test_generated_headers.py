"""The generated headers of the device code (Weideman series coefficients,
continued-fraction depth thresholds, near-minimax polynomial coefficients)
are what their generator scripts write today: each script is re-run and its
output compared with the committed header byte for byte."""
import os
import subprocess
import sys

import pytest

CSRC = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_1706_01420_amd", "csrc")


@pytest.mark.parametrize("script,header", [("gen_weideman.py", "weideman_coeffs.h"),
                                           ("gen_cfdepth.py", "cf_depth.h"),
                                           ("gen_minimax.py", "minimax_coeffs.h"),
                                           ("gen_rgamma.py", "rgamma_coeffs.h")])
def test_header_matches_generator(script, header):
    out = subprocess.run([sys.executable, os.path.join(CSRC, script)], cwd=CSRC, check=True,
                         capture_output=True, text=True, timeout=600).stdout
    with open(os.path.join(CSRC, header)) as f:
        assert out == f.read()
