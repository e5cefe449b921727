"""The C-ABI library loads and exports every function include/nphc.h declares
(no compute calls: these run without a GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "nphc.h")
LIB = os.path.join(ROOT, "paper_1104_5497_amd", "libnphc.so")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"\b(nphc_[a-z_0-9]+)\s*\(", src)
    return sorted(set(names))


def test_header_declares_the_entry_points():
    names = declared_functions()
    for n in ("nphc_track_paths", "nphc_refine_certify", "nphc_classify", "nphc_adjoint",
              "nphc_mark_duplicates", "nphc_select"):
        assert n in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="libnphc.so not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    for n in declared_functions():
        assert hasattr(lib, n), f"{n} declared in nphc.h but not exported"


@pytest.mark.skipif(not os.path.exists(LIB), reason="libnphc.so not built")
def test_host_only_calls():
    from paper_1104_5497_amd import _lib as L
    assert L.lib().nphc_version().startswith(b"nphc")
    assert L.lib().nphc_strerror(L.NPHC_EINVAL) == b"invalid argument"
    o = L.default_track_opts(L.NPHC_FP64)
    assert o.max_corr == 3 and o.hmax == 0.05
    assert L.default_track_opts(L.NPHC_FP32).max_corr == 2
    c = L.default_cert_opts()
    assert c.real_tol == 1e-7
