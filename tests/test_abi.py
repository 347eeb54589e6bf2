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
    assert L.rgf_ldos(C.byref(d), None, 1, 1e-6, None, None, None, None, None) == rgf.RGF_EINVAL
    assert L.rgf_kpm_moments(None, -1.0, 1.0, 10, None, 4, None, None) == rgf.RGF_EINVAL
    assert L.rgf_kpm_fermi(None, 10, 1.0, -1.0, 3.0, None, None) == rgf.RGF_EINVAL
    assert L.rgf_kpm_dos(None, 0, -1.0, 1.0, None, 5, None, None) == rgf.RGF_EINVAL
    assert L.rgf_profile(-1) == rgf.RGF_EINVAL
    assert L.rgf_check_device(None, 1e-10, None, None) == rgf.RGF_EINVAL
    assert L.rgf_check_device(C.byref(d), 1e-10, None, None) == rgf.RGF_EINVAL  # null blocks, no device work
    assert L.rgf_set_checks(1) == rgf.RGF_OK and L.rgf_get_checks() == 1
    assert L.rgf_set_checks(0) == rgf.RGF_OK and L.rgf_get_checks() == 0
    assert L.rgf_profile(16) == rgf.RGF_OK and L.rgf_profile(0) == rgf.RGF_OK
    assert L.rgf_profile_classes(1, 1 << 8) == rgf.RGF_EINVAL  # no class 8
    assert L.rgf_profile_classes(-1, 1) == rgf.RGF_EINVAL
    assert L.rgf_profile_classes(3, (1 << 8) - 1) == rgf.RGF_OK and L.rgf_profile_classes(0, 0) == rgf.RGF_OK
    n = C.c_int64()
    assert L.rgf_profile_read_class(8, C.byref(n), None, None, None, None) == rgf.RGF_EINVAL


def test_decimation_cap_setting(lib):
    """rgf_set_sr_maxit: [1, 100] sets the cap, 0 restores 100, anything else is rejected."""
    from paper_2609_37058_amd import rgf
    rgf.load()
    L = rgf._lib
    assert L.rgf_get_sr_maxit() == 100
    assert L.rgf_set_sr_maxit(101) == rgf.RGF_EINVAL and L.rgf_get_sr_maxit() == 100
    assert L.rgf_set_sr_maxit(-1) == rgf.RGF_EINVAL
    rgf.set_sr_maxit(3)
    assert rgf.get_sr_maxit() == 3
    rgf.set_sr_maxit(0)
    assert rgf.get_sr_maxit() == 100


def test_noalloc_rejects_blocks_beyond_its_scratch(lib):
    """A block size whose one-energy workspace exceeds the static scratch array is refused with
    RGF_ETOOBIG before any device work (the pointers below are never dereferenced)."""
    from paper_2609_37058_amd import rgf
    rgf.load()
    L = rgf._lib
    fake = 256  # non-null, never read: the size check comes first
    for M, ok in ((768, False), (2048, False)):
        lead = rgf.rgf_lead(M, fake, fake, fake, fake)
        d = rgf.rgf_device(3, M, fake, fake, fake, fake, lead, lead)
        rc = L.rgf_transmission_noalloc(C.byref(d), fake, 4, 1e-6, 0, fake, None, None)
        assert rc == rgf.RGF_ETOOBIG, (M, rc)
        assert b"scratch" in L.rgf_last_error()
    assert L.rgf_transmission_noalloc(None, None, 0, 1e-6, 0, None, None, None) == rgf.RGF_EINVAL


def test_binding_rejects_wrong_dtypes():
    """The binding checks what the C calls read and write through each pointer (CPU tensors are
    refused before any dtype question, so this runs without a GPU)."""
    import torch
    from paper_2609_37058_amd import rgf
    with pytest.raises(ValueError, match="float64"):
        rgf._energies(torch.zeros(4, dtype=torch.float32))
    with pytest.raises(ValueError, match="device tensors"):
        rgf._ptr(torch.zeros(4, dtype=torch.float64), torch.float64, "E")


def test_tuning_table_on_the_host(tmp_path):
    """Set/get of the tuning table and its JSON round trip (no device work)."""
    from paper_2609_37058_amd import rgf
    rgf.load()
    assert rgf.get_tuning(100, "fp64") == (128, 1)      # defaults: 128 tiles, one lane below Mp = 256
    assert rgf.get_tuning(1024, "mixed") == (128, 2)
    assert rgf.get_tuning(256, "fp64") == (64, 2)       # the measured built-in choice at Mp = 256
    assert rgf.get_tuning(256, "mixed") == (128, 2)
    rgf.set_tuning(100, "fp64", 64, 2)
    assert rgf.get_tuning(128, "fp64") == (64, 2)       # same padded size class
    assert rgf.get_tuning(129, "fp64") == (128, 1)
    path = str(tmp_path / "tune.json")
    rgf.save_tuning(path, [100, 1024])
    rgf.set_tuning(100, "fp64", 0, 0)
    assert rgf.get_tuning(100, "fp64") == (128, 1)
    assert rgf.load_tuning(path) == 4
    assert rgf.get_tuning(100, "fp64") == (64, 2)
    rgf.set_tuning(100, "fp64", 0, 0)
    L = rgf._lib
    assert L.rgf_set_tuning(0, 0, 64, 1) == rgf.RGF_EINVAL
    assert L.rgf_set_tuning(100, 0, 96, 1) == rgf.RGF_EINVAL
    assert L.rgf_set_tuning(100, 0, 64, 5) == rgf.RGF_EINVAL
    assert L.rgf_autotune(0, 0, 0, None, None, None) == rgf.RGF_EINVAL
