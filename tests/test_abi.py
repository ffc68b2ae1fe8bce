"""CPU checks of the C ABI: the library loads, exports every entry point that
include/*.h declares, and rejects bad arguments before touching a device."""
import ctypes
import glob
import os
import re

import numpy as np
import pytest

import paper_1706_00773_amd as eu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_functions():
    names = set()
    for h in glob.glob(os.path.join(ROOT, "include", "*.h")):
        src = open(h).read()
        src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
        for m in re.finditer(r"^\s*(?:const\s+)?[A-Za-z_][\w\s\*]*?\b(eig_\w+)\s*\(", src, re.M):
            names.add(m.group(1))
    return names


def test_header_declares_entry_points():
    names = _declared_functions()
    assert {"eig_state_create", "eig_state_upload", "eig_update_rankk", "eig_query",
            "eig_state_destroy", "eig_status_str", "eig_debug_fetch"} <= names


def test_library_exports_every_declared_symbol():
    lib = eu.load_library()
    for name in _declared_functions():
        assert hasattr(lib, name), name
    assert set(eu.EXPORTED) == _declared_functions()


def test_status_strings():
    for code in range(0, -10, -1):
        s = eu.eig_status_str(code)
        assert isinstance(s, str) and s and s != "unknown status"
    assert eu.eig_status_str(123) == "unknown status"


def test_info_struct_layout():
    # int64 x7, int32 x2, double x3, int64, double[8]
    assert ctypes.sizeof(eu.eig_info) == 7 * 8 + 2 * 4 + 3 * 8 + 8 + 8 * 8


def test_create_rejects_bad_size_without_device():
    lib = eu.load_library()
    h = ctypes.c_void_p()
    assert lib.eig_state_create(ctypes.byref(h), 0, 0) == eu.EIG_EINVAL
    assert lib.eig_state_create(ctypes.byref(h), -5, 0) == eu.EIG_EINVAL
    assert lib.eig_state_create(None, 10, 0) == eu.EIG_EINVAL


def test_null_state_is_rejected():
    lib = eu.load_library()
    K = np.zeros((4, 2), order="F")
    sig = (ctypes.c_int8 * 2)(1, -1)
    assert lib.eig_update_rankk(None, 2, K.ctypes.data, 4, sig, 0, None) == eu.EIG_EINVAL
    assert lib.eig_query(None, None, None, 1, 0, None, None) == eu.EIG_EINVAL
    assert lib.eig_state_destroy(None) == eu.EIG_EINVAL
    assert lib.eig_state_upload(None, None, None, 1, 0, None) == eu.EIG_EINVAL
    assert lib.eig_debug_fetch(None, 1, None, 0, None) == eu.EIG_EINVAL


def test_no_device_reports_edevice():
    import torch

    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    lib = eu.load_library()
    h = ctypes.c_void_p()
    assert lib.eig_state_create(ctypes.byref(h), 16, 0) == eu.EIG_EDEVICE
