"""Device-code hygiene (CPU only): the gfx950 assembly of libipx contains no
writes through the scalar data cache (scalar stores, scalar atomics, scalar
cache write-back or invalidate-with-write-back), and no packed-FP32 math."""
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
FORBIDDEN = [r"\bs_store", r"\bs_buffer_store", r"\bs_scratch_store", r"\bs_atomic", r"\bs_buffer_atomic",
             r"\bs_dcache_wb", r"\bs_dcache_discard", r"\bv_pk_add_f32", r"\bv_pk_mul_f32", r"\bv_pk_fma_f32"]


@pytest.fixture(scope="module")
def asm(tmp_path_factory):
    from paper_1706_01420_amd import build
    out = str(tmp_path_factory.mktemp("isa") / "ipx.s")
    cmd = build.command(out, extra=("--offload-device-only", "-S"))
    cmd = [c for c in cmd if c != "-shared"]
    subprocess.run(cmd, check=True, capture_output=True)
    return open(out).read()


def test_no_scalar_cache_writes_or_packed_fp32(asm):
    body = [l for l in asm.splitlines() if l.startswith("\t") and not l.strip().startswith((";", "."))]
    for pat in FORBIDDEN:
        hits = [l for l in body if re.search(pat, l)]
        assert not hits, (pat, hits[:3])
