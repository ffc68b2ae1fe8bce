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
    for code in range(0, -11, -1):
        s = eu.eig_status_str(code)
        assert isinstance(s, str) and s and s != "unknown status"
    assert eu.eig_status_str(123) == "unknown status"


def _c_layout(struct, fields):
    """sizeof and offsetof as the C compiler lays out `struct` from include/eigupd.h."""
    import subprocess
    import tempfile

    inc = os.path.join(ROOT, "include")
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "eigupd.h"', "int main(void) {",
             f'  printf("%zu\\n", sizeof({struct}));']
    lines += [f'  printf("%zu\\n", offsetof({struct}, {f}));' for f in fields]
    lines += ["  return 0;", "}"]
    with tempfile.TemporaryDirectory() as d:
        src, exe = os.path.join(d, "l.c"), os.path.join(d, "l")
        with open(src, "w") as fh:
            fh.write("\n".join(lines) + "\n")
        subprocess.run(["gcc", "-I", inc, src, "-o", exe], check=True)
        out = subprocess.run([exe], check=True, capture_output=True, text=True).stdout.split()
    return [int(v) for v in out]


@pytest.mark.parametrize("cls", ["eig_info", "eig_batch_item", "eig_completion",
                                 "eig_server_info", "eig_chain_info"])
def test_struct_layouts_match_the_header(cls):
    st = getattr(eu, cls)
    names = [f for f, _ in st._fields_]
    c = _c_layout(cls, names)
    assert ctypes.sizeof(st) == c[0]
    assert [getattr(st, f).offset for f in names] == c[1:]


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
    info = eu.eig_chain_info()
    assert lib.eig_sturm_chain(None, 2, K.ctypes.data, 4, sig, None, 0, None, 0, None, None, 0,
                               ctypes.byref(info), None) == eu.EIG_EINVAL


def test_no_device_reports_edevice():
    import torch

    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    lib = eu.load_library()
    h = ctypes.c_void_p()
    assert lib.eig_state_create(ctypes.byref(h), 16, 0) == eu.EIG_EDEVICE


def test_noalloc_checks_arguments_before_the_device():
    """The no-allocation entry point rejects bad sizes, ranks and modes before it
    looks for a device (the pointers are never read on these paths)."""
    import torch

    lib = eu.load_library()
    f = lib.eig_eigvals_rankk_noalloc
    x = np.zeros(4)
    p = x.ctypes.data
    sig = (ctypes.c_int8 * 2)(1, -1)
    nmax = eu.EIG_NOALLOC_NMAX
    assert f(nmax + 1, 2, p, p, nmax + 1, p, nmax + 1, sig, 0, p, p, 0, None) == \
        eu.EIG_EUNSUPPORTED
    assert f(16, 9, p, p, 16, p, 16, sig, 0, p, p, 0, None) == eu.EIG_EUNSUPPORTED
    assert f(16, 2, p, p, 16, p, 16, sig, eu.EIG_VALUES_ONLY, p, p, 0, None) == \
        eu.EIG_EUNSUPPORTED
    assert f(16, 2, p, p, 15, p, 16, sig, 0, p, p, 0, None) == eu.EIG_EINVAL
    assert f(16, 2, p, p, 16, p, 16, sig, 0, p, None, 0, None) == eu.EIG_EINVAL
    assert f(0, 2, p, p, 16, p, 16, sig, 0, p, p, 0, None) == eu.EIG_EINVAL
    if not torch.cuda.is_available():
        assert f(16, 2, p, p, 16, p, 16, sig, 0, p, p, 0, None) == eu.EIG_EDEVICE


def test_c_client_compiles(tmp_path):
    """The plain C client (tests/c_client/eigupd_client.c) builds against the header
    and the library with gcc alone, no Python or torch types involved."""
    import importlib.util

    spec = importlib.util.spec_from_file_location(
        "c_client_build", os.path.join(ROOT, "tests", "c_client", "build.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    out = mod.build(str(tmp_path / "client"))
    assert os.path.exists(out)
