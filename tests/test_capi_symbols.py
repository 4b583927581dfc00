"""The C-ABI library loads (no GPU needed) and exports every entry point that
include/nnp.h declares; the binding declares the same set."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2310_03121_amd", "libnnp.so")


def declared():
    hdr = open(os.path.join(ROOT, "include", "nnp.h")).read()
    hdr = re.sub(r"/\*.*?\*/", "", hdr, flags=re.S)
    return sorted(set(re.findall(r"\b(nnp_[a-z0-9_]+)\s*\(", hdr)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        pytest.fail("libnnp.so is not built: run python -m paper_2310_03121_amd.build")
    return ctypes.CDLL(LIB)


def test_every_declared_symbol_is_exported(lib):
    names = declared()
    assert len(names) >= 20
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_covers_the_header():
    from paper_2310_03121_amd import capi
    assert sorted(capi.SYMBOLS) == declared()


def test_status_strings_without_gpu(lib):
    f = lib.nnp_status_string
    f.restype = ctypes.c_char_p
    assert f(0) == b"ok"
    assert b"cutoff" in f(3)
    assert lib.nnp_profile_stage_count() > 5


def test_host_argument_errors_without_gpu(lib):
    # null handle and null parameter structs are rejected before any device work
    lib.nnp_create.restype = ctypes.c_int
    out = ctypes.c_void_p()
    assert lib.nnp_create(None, None, 0, ctypes.byref(out)) == 1
    lib.nnp_workspace_bytes.restype = ctypes.c_size_t
    assert lib.nnp_workspace_bytes(None, 10, 1, None) == 0
