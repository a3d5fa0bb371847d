"""The C ABI library loads on a host without a GPU, exports every function the
public header declares, binds to the single HIP runtime torch maps, and fails
cleanly (an error status, no crash) when no device is present."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADERS = [os.path.join(ROOT, "include", f) for f in sorted(os.listdir(os.path.join(ROOT, "include")))
           if f.endswith(".h")]


def declared_functions():
    names = []
    for h in HEADERS:
        text = open(h).read()
        names += re.findall(r"^IPX_API\s+[^(;]*?\b([A-Za-z_][A-Za-z0-9_]*)\s*\(", text, re.M)
    return names


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("nll_eval", "nll_grad", "ipx_create", "ipx_dataset_create"):
        assert required in names


def test_library_exports_every_declared_symbol():
    from paper_1706_01420_amd import ipx
    lib = ctypes.CDLL(ipx.LIB_PATH)
    for name in declared_functions():
        assert hasattr(lib, name), name
    assert sorted(ipx.EXPORTED) == sorted(declared_functions())


def test_one_hip_runtime_in_process():
    from paper_1706_01420_amd import ipx  # noqa: F401
    maps = open("/proc/self/maps").read()
    hip = {l.split()[-1] for l in maps.splitlines() if "libamdhip64" in l}
    assert len(hip) == 1, hip


def test_host_only_queries():
    from paper_1706_01420_amd import ipx
    assert [ipx.ipx_model_nparams(m) for m in (1, 2, 3, 4, 5)] == [4, 7, 12, 12, 11]
    assert [ipx.ipx_model_ncols(m) for m in (1, 2, 3, 4, 5)] == [1, 3, 6, 7, 1]
    assert ipx.ipx_model_nparams(0) == -1 and ipx.ipx_model_ncols(6) == -1


def test_create_without_device_is_an_error_not_a_crash():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    from paper_1706_01420_amd import ipx
    with pytest.raises(ipx.IpxError) as e:
        ipx.ipx_create(0)
    assert e.value.status == ipx.IPX_EDEVICE
    assert ipx.ipx_last_error() != ""
