"""Host-side checks of the C ABI that need no GPU: the library loads, exports
every symbol include/phia.h declares, and rejects invalid instances with the
documented status codes before touching the device."""
import os
import re
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "phia.h")


@pytest.fixture(scope="module")
def phia():
    from paper_2407_10205_amd import phia as P
    if not os.path.exists(P.LIB_PATH):
        pytest.skip("libphia.so not built")
    P.lib()
    return P


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(phia_[a-z0-9_]+)\s*\(", src)))


def test_header_and_binding_agree(phia):
    assert declared_functions() == sorted(phia.EXPORTS)


def test_library_exports_every_declared_symbol(phia):
    out = subprocess.run(["nm", "-D", "--defined-only", phia.LIB_PATH], capture_output=True, text=True,
                         check=True).stdout
    exported = set(re.findall(r"\bT (phia_[a-z0-9_]+)", out))
    missing = [f for f in declared_functions() if f not in exported]
    assert not missing, missing


def test_version_and_empty_error(phia):
    assert b"gfx950" in phia.lib().phia_version()
    assert phia.lib().phia_last_error() is not None


def _code(phia, J, h=None, **kw):
    try:
        phia.Problem(J, h, **kw)
    except phia.PhiaError as e:
        return e.code
    return 0


def test_validation_codes(phia):
    asym = np.array([[0, 1.0], [2.0, 0]])
    assert _code(phia, asym) == -2                       # PHIA_ENOTSYM
    assert _code(phia, np.array([[1.0, 0], [0, 0]])) == -3  # PHIA_EDIAG
    off = np.array([[0, 0.3], [0.3, 0]])
    assert _code(phia, off, frac_bits=2) == -4           # off the 2^-2 grid
    assert _code(phia, off) == -4                        # no grid f <= 15 holds 0.3
    big = np.array([[0, 200.0], [200.0, 0]])
    assert _code(phia, big, path="i8") == -4             # outside int8
    wide = np.array([[0, 40000.0], [40000.0, 0]])
    assert _code(phia, wide, path="ell") == -4           # outside the 16 bits of an ELL slot
    assert _code(phia, big, path=5) == -1                # unknown path
    assert _code(phia, np.array([[0, np.nan], [np.nan, 0]])) == -1
    assert _code(phia, np.zeros((2, 2)), frac_bits=16) == -1


def test_null_and_size_arguments(phia):
    import ctypes as C
    L = phia.lib()
    p = C.c_void_p()
    assert L.phia_create(None, None, 4, None, C.byref(p)) == -1
    J = np.zeros((2, 2))
    assert L.phia_create(J.ctypes.data_as(C.c_void_p), None, 0, None, C.byref(p)) == -1
    assert L.phia_create(J.ctypes.data_as(C.c_void_p), None, 20000, None, C.byref(p)) == -1
    assert L.phia_create(J.ctypes.data_as(C.c_void_p), None, 2, None, None) == -1
    assert L.phia_sync(None) == -1
    assert L.phia_set_incremental(None, 1) == -1
    out = (C.c_int64 * 3)()
    assert L.phia_incremental_stats(None, out) == -1
    L.phia_destroy(None)


@pytest.mark.parametrize("path,N", [("i8", 5056), ("bf16hilo", 2496), ("fp32", 4096), ("ell", 4096)])
def test_size_limits_per_path(phia, path, N):
    """Each path's largest instance passes the size check (on a machine
    without a GPU it then fails for want of a device); one spin more is
    PHIA_ERANGE before any device call."""
    J = np.zeros((N + 1, N + 1))
    J[0, 1] = J[1, 0] = 1.0
    assert _code(phia, J, path=path) == -4
    code = _code(phia, J[:N, :N].copy(), path=path)
    assert code != -4


def test_product_and_oracle_share_no_code():
    """The HIP path and the CPU oracle are independent: no source of the
    package (kernels, runtime, binding) refers to the oracle, and the oracle
    includes no header of the package nor imports its binding."""
    pkg = os.path.join(ROOT, "paper_2407_10205_amd")
    for d, _, files in os.walk(pkg):
        if "_build" in d or "__pycache__" in d:
            continue
        for f in files:
            if f.endswith((".py", ".hip", ".cpp", ".h")):
                assert "oracle" not in open(os.path.join(d, f)).read().lower(), os.path.join(d, f)
    assert "oracle" not in open(HEADER).read().lower()
    odir = os.path.join(ROOT, "oracle")
    for f in os.listdir(odir):
        if f.endswith((".c", ".h")):
            incs = re.findall(r'#include\s+[<"]([^>"]+)[>"]', open(os.path.join(odir, f)).read())
            assert all(i in ("phia_oracle.h", "math.h", "stdlib.h", "string.h", "stdint.h", "omp.h") for i in incs), (f, incs)
        if f.endswith(".py"):
            src = open(os.path.join(odir, f)).read()
            assert "paper_2407_10205_amd" not in src and "libphia" not in src, f
