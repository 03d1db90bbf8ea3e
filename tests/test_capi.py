"""The C-ABI library loads and exports every symbol its header declares (CPU only:
no call here touches a GPU; only host-side argument checks are exercised)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "lob.h")
LIB = os.path.join(ROOT, "paper_2511_02136_amd", "liblob.so")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_ \*]*?\b(lob_[a-z_0-9]+)\s*\(", src, flags=re.M)
    return sorted(set(names))


def test_header_declares_the_entry_points():
    names = declared_functions()
    for n in ("lob_init", "lob_reset", "lob_step", "lob_rollout", "lob_observe", "lob_export_books",
              "lob_export_state", "lob_destroy", "lob_strerror"):
        assert n in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="liblob.so not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    for n in declared_functions():
        assert hasattr(lib, n), n


@pytest.mark.skipif(not os.path.exists(LIB), reason="liblob.so not built")
def test_host_side_argument_checks():
    lib = ctypes.CDLL(LIB)
    lib.lob_strerror.restype = ctypes.c_char_p
    assert lib.lob_strerror(0) == b"ok"
    assert lib.lob_strerror(-1) == b"invalid argument"
    assert lib.lob_strerror(-4).startswith(b"call out of order")
    # NULL arguments are rejected before any device call
    lib.lob_init.argtypes = [ctypes.c_void_p, ctypes.c_void_p]
    assert lib.lob_init(None, None) == -1
    lib.lob_step.argtypes = [ctypes.c_void_p] * 5
    assert lib.lob_step(None, None, None, None, None) == -1
    lib.lob_rollout.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p,
                                ctypes.c_void_p, ctypes.c_void_p]
    assert lib.lob_rollout(None, None, 1, None, None, None) == -1
    lib.lob_destroy.argtypes = [ctypes.c_void_p]
    assert lib.lob_destroy(None) == 0
