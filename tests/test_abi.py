"""The C ABI: the header is plain C, and libotm.so exports every function it
declares (no compute call: this runs without a GPU)."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "otm.h")
LIB = os.path.join(ROOT, "paper_1309_0787_amd", "libotm.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"\b(otm_[a-z0-9_]+)\s*\(", text)
    return sorted(set(names))


def test_header_is_plain_c():
    subprocess.check_call(["gcc", "-std=c99", "-Wall", "-Werror", "-fsyntax-only", "-x", "c", HEADER])


def test_library_exports_every_declared_function():
    if not os.path.exists(LIB):
        pytest.skip("libotm.so not built")
    lib = ctypes.CDLL(LIB)
    names = declared_functions()
    assert len(names) >= 20
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing


def test_python_binding_covers_the_header():
    from paper_1309_0787_amd import otm
    assert set(declared_functions()) == set(otm._SIGS)


def test_status_strings_without_gpu():
    if not os.path.exists(LIB):
        pytest.skip("libotm.so not built")
    lib = ctypes.CDLL(LIB)
    lib.otm_status_string.restype = ctypes.c_char_p
    assert lib.otm_status_string(-4) == b"second moment not positive definite on the projection"
    assert lib.otm_max_k() == 128 and lib.otm_max_batch() == 128
