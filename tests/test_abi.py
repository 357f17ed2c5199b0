"""C ABI: the library loads, exports every function include/pdfmi.h declares,
and its host-only validation rejects malformed input (no GPU calls)."""
import ctypes
import os
import subprocess
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "pdfmi.h")
LIB = os.path.join(ROOT, "paper_2009_06635_amd", "libpdfmi.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:int|const char\*)\s+(pdf_\w+)\s*\(", text, flags=re.M)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        pytest.fail("libpdfmi.so not built")
    import torch  # noqa: F401  -- same HIP runtime as torch
    return ctypes.CDLL(LIB)


def test_exports_every_declared_symbol(lib):
    names = declared_functions()
    assert {"pdf_load_grid", "pdf_xfxq2", "pdf_alphas_q2"} <= set(names)
    for n in names:
        assert hasattr(lib, n), n


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def _validate(lib, shape, pids, knots, values):
    shape = np.ascontiguousarray(shape, np.int32)
    pids = np.ascontiguousarray(pids, np.int32)
    knots = np.ascontiguousarray(knots, np.float64)
    values = np.ascontiguousarray(values, np.float64)
    f = lib.pdf_validate_grid
    f.argtypes = [ctypes.c_int32, ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
    return f(len(shape), _p(shape), len(pids), _p(pids), _p(knots), _p(values))


def _good():
    xk = [1e-3, 1e-2, 0.1, 1.0]
    q1 = [2.0, 4.0, 8.0]
    q2 = [8.0, 16.0, 32.0]
    shape = [[4, 3], [4, 3]]
    knots = xk + q1 + xk + q2
    values = np.ones(2 * 4 * 3 * 2)
    return shape, [21, 1], knots, values


def test_validation_accepts_good_grid(lib):
    assert _validate(lib, *_good()) == 0


@pytest.mark.parametrize("case", ["nx1", "nonmono_x", "x_gt_1", "x_le_0", "q_nonmono", "threshold_gap",
                                  "nan_value", "xrange_differs"])
def test_validation_rejects_malformed_grid(lib, case):
    shape, pids, knots, values = _good()
    knots = list(knots)
    values = values.copy()
    if case == "nx1":
        shape = [[1, 3], [4, 3]]
    elif case == "nonmono_x":
        knots[1], knots[2] = knots[2], knots[1]
    elif case == "x_gt_1":
        knots[3] = 1.5
    elif case == "x_le_0":
        knots[0] = 0.0
    elif case == "q_nonmono":
        knots[5] = 1.0
    elif case == "threshold_gap":
        knots[7] = 9.0
    elif case == "nan_value":
        values[5] = np.nan
    elif case == "xrange_differs":
        knots[10] = 0.5
    if case == "nx1":
        knots = knots[:1] + knots[4:]
        values = np.ones(1 * 3 * 2 + 4 * 3 * 2)
    assert _validate(lib, shape, pids, knots, values) == -2


@pytest.mark.parametrize("pids", [[21, 7], [21, 21], [0, 21], [-7, 1]])
def test_validation_rejects_bad_pids(lib, pids):
    shape, _, knots, values = _good()
    assert _validate(lib, shape, pids, knots, values) == -4


def test_validate_alphas(lib):
    f = lib.pdf_validate_alphas
    f.argtypes = [ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p]

    def v(q, a):
        q = np.ascontiguousarray(q, np.float64)
        a = np.ascontiguousarray(a, np.float64)
        return f(len(q), _p(q), _p(a))

    assert v([1, 2, 3, 3, 4], [0.1] * 5) == 0
    assert v([1], [0.1]) == -2
    assert v([1, 2, 2, 2, 3], [0.1] * 5) == -2     # a one-knot segment
    assert v([1, 3, 2], [0.1] * 3) == -2
    assert v([1, 2, 3], [0.1, np.nan, 0.1]) == -2
    assert v([0, 2, 3], [0.1] * 3) == -2


def test_capi_demo_is_built_against_the_library():
    """tests/capi_demo (a plain C consumer of include/pdfmi.h) is built with the library."""
    exe = os.path.join(os.path.dirname(os.path.abspath(__file__)), "capi_demo")
    if not os.path.exists(exe):
        pytest.skip("library not built")
    assert os.access(exe, os.X_OK)
    out = subprocess.run(["ldd", exe], capture_output=True, text=True).stdout
    assert "libpdfmi.so" in out


def test_tune_cache_file_handling(lib, tmp_path):
    """pdf_batch_tune_cache is host-only: a missing file holds no entries, lines
    that do not parse or hold an invalid choice are skipped, NULL stops it."""
    f = lib.pdf_batch_tune_cache
    f.argtypes = [ctypes.c_char_p]
    assert f(os.fsencode(str(tmp_path / "none.txt"))) == 0
    p = tmp_path / "tune.txt"
    p.write_text("not a line\nkey-a 4096 1\nkey-b 100 0\nkey-c 8192 7\n\n")
    assert f(os.fsencode(str(p))) == 0
    assert f(None) == 0
    assert f(b"") == 0
