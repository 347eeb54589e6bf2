"""The C ABI on the CPU: the library loads and exports every function include/rgf.h declares.

No compute call is made (there is no GPU here); argument checks that fail
before any device work are exercised too.
"""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2609_37058_amd", "librgf.so")
HEADER = os.path.join(ROOT, "include", "rgf.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\*?\s*([a-z_][a-z0-9_]*)\s*\(", text, flags=re.M)
    return sorted(set(n for n in names if n not in ("if", "return")))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        pytest.skip("librgf.so not built")
    return C.CDLL(LIB)


def test_header_declares_the_boundary():
    names = declared_functions()
    for n in ("rgf_transmission", "lead_self_energy", "transport_open", "transport_submit",
              "transport_poll", "transport_close"):
        assert n in names


def test_every_declared_symbol_is_exported(lib):
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_signatures_cover_the_header():
    from paper_2609_37058_amd import rgf
    assert set(declared_functions()) <= set(rgf.SIGNATURES)


def test_argument_errors_before_device_work(lib):
    from paper_2609_37058_amd import rgf
    rgf.load()
    L = rgf._lib
    assert L.rgf_transmission(None, None, 0, 1e-6, 0, None, None, None) == rgf.RGF_EINVAL
    d = rgf.rgf_device(0, 4, None, None, None, None, rgf.rgf_lead(), rgf.rgf_lead())
    assert L.rgf_transmission(C.byref(d), None, 1, 1e-6, 0, None, None, None) == rgf.RGF_EINVAL
    assert b"N < 1" in L.rgf_last_error()
    assert L.rgf_set_tile(0, 96) == rgf.RGF_EINVAL
    assert L.rgf_set_mixed_parts(8) == rgf.RGF_EINVAL
    assert L.rgf_version().startswith(b"librgf")
