"""The C-ABI library loads on a CPU-only host and exports every function that
include/mlcc3.h declares (no compute calls)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SO = os.path.join(ROOT, "paper_2202_08612_amd", "libmlcc3.so")


def declared():
    src = open(os.path.join(ROOT, "include", "mlcc3.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(mlcc3_[a-z0-9_]+)\s*\(", src)))


@pytest.mark.skipif(not os.path.exists(SO), reason="libmlcc3.so not built")
def test_exports_every_declared_symbol():
    lib = ctypes.CDLL(SO)
    names = declared()
    assert len(names) >= 10
    for n in names:
        assert hasattr(lib, n), n


@pytest.mark.skipif(not os.path.exists(SO), reason="libmlcc3.so not built")
def test_host_only_helpers():
    lib = ctypes.CDLL(SO)
    lib.mlcc3_num_triples.restype = ctypes.c_int64
    for n in range(0, 20):
        assert lib.mlcc3_num_triples(n) == n * (n + 1) * (n + 2) // 6 - n
    lib.mlcc3_status_string.restype = ctypes.c_char_p
    assert lib.mlcc3_status_string(-2).decode().startswith("omega")
