"""The C-ABI library loads and exports every function declared in include/*.h
(no compute call: this runs without a GPU)."""
import ctypes
import glob
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PKG = os.path.join(ROOT, "paper_2605_03561_amd")


def declared(header):
    src = open(header).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(ta_[a-z0-9_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def built():
    lib = os.path.join(PKG, "libta.so")
    if not os.path.exists(lib):
        from paper_2605_03561_amd import build
        build.build_ta()
    return lib


def test_exports_match_header(built):
    lib = ctypes.CDLL(built)
    names = declared(os.path.join(ROOT, "include", "ta.h"))
    assert len(names) >= 14
    for n in names:
        assert hasattr(lib, n), f"{n} declared in ta.h but not exported"


def test_every_header_is_exported(built):
    libs = {"ta.h": built}
    for hdr in glob.glob(os.path.join(ROOT, "include", "*.h")):
        base = os.path.basename(hdr)
        so = libs.get(base) or os.path.join(PKG, "lib" + base[:-2] + ".so")
        if not os.path.exists(so):
            from paper_2605_03561_amd import build
            build.build_all()
        lib = ctypes.CDLL(so)
        for n in declared(hdr):
            assert hasattr(lib, n), f"{n} ({base}) not exported by {os.path.basename(so)}"


def test_status_strings(built):
    lib = ctypes.CDLL(built)
    lib.ta_status_string.restype = ctypes.c_char_p
    assert lib.ta_status_string(0) == b"ok"
    assert lib.ta_status_string(3) == b"context id out of range"
    lib.ta_last_error.restype = ctypes.c_char_p
    lib.ta_last_error.argtypes = [ctypes.c_void_p]
    assert lib.ta_last_error(None) == b"NULL handle"


def test_create_rejects_null_out(built):
    lib = ctypes.CDLL(built)
    assert lib.ta_create(None, 0) == 1
