"""The C-ABI library loads and exports every symbol include/mctrg.h declares
(CPU only: no compute calls)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_1710_03757_amd", "libmctrg.so")
HDR = os.path.join(ROOT, "include", "mctrg.h")


def declared():
    txt = open(HDR).read()
    return sorted(set(re.findall(r"^\s*(?:int|void|const char\*|int32_t)\s+(mctrg_\w+)\s*\(", txt, re.M)))


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_every_declared_symbol_is_exported():
    lib = ctypes.CDLL(LIB)
    names = declared()
    assert len(names) >= 11
    for n in names:
        assert hasattr(lib, n), n


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_host_only_calls():
    lib = ctypes.CDLL(LIB)
    lib.mctrg_capacity_dim.restype = ctypes.c_int32
    assert lib.mctrg_capacity_dim(2, 32, 0) == 2
    assert lib.mctrg_capacity_dim(2, 32, 1) == 4
    assert lib.mctrg_capacity_dim(2, 32, 2) == 16
    assert lib.mctrg_capacity_dim(2, 32, 3) == 32
    assert lib.mctrg_capacity_dim(2, 8, 10) == 8
    lib.mctrg_status_string.restype = ctypes.c_char_p
    assert lib.mctrg_status_string(-1) == b"invalid argument"
    # argument errors are caught before any device work
    out = ctypes.c_void_p()
    assert lib.mctrg_init_tensor(7, 1, None, None, 0, None, ctypes.byref(out)) == -1
    assert lib.mctrg_run_samples(None, None, 1, None, None, None, None, None, None) == -1


def test_python_binding_names_match_header():
    import importlib.util
    if not os.path.exists(LIB):
        pytest.skip("library not built")
    import paper_1710_03757_amd as m
    assert sorted(m.EXPORTED) == declared()
