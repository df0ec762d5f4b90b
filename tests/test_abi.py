"""C ABI: the library loads, exports what include/h2mv.h declares, and rejects
bad arguments before touching the device (CPU only)."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_1902_01829_amd import h2mv

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_exports_every_declared_symbol():
    with open(os.path.join(ROOT, "include", "h2mv.h")) as f:
        text = f.read()
    declared = set(re.findall(r"\b(h2_[a-z_]+)\s*\(", text))
    assert declared == set(h2mv.EXPORTS)
    lib = ctypes.CDLL(h2mv.LIB_PATH)
    for name in declared:
        assert hasattr(lib, name), name


def test_free_null_is_noop():
    h2mv.h2_free(0)


def _pts(n=100, d=2):
    return np.random.Generator(np.random.PCG64(3)).random((n, d))


@pytest.mark.parametrize("kw,code", [
    (dict(n=0), h2mv.H2_ERR_INVALID_ARG),
    (dict(dim=4), h2mv.H2_ERR_INVALID_ARG),
    (dict(leaf=1), h2mv.H2_ERR_INVALID_ARG),
    (dict(p=0), h2mv.H2_ERR_INVALID_ARG),
    (dict(eta=0.0), h2mv.H2_ERR_INVALID_ARG),
    (dict(eta=float("nan")), h2mv.H2_ERR_INVALID_ARG),
    (dict(ell=-0.1), h2mv.H2_ERR_INVALID_ARG),
    (dict(storage=7), h2mv.H2_ERR_INVALID_ARG),
    (dict(nan_point=True), h2mv.H2_ERR_INVALID_ARG),
    (dict(p=9), h2mv.H2_ERR_UNSUPPORTED),
    (dict(dim=3, p=5), h2mv.H2_ERR_UNSUPPORTED),
    (dict(leaf=65), h2mv.H2_ERR_UNSUPPORTED),
])
def test_invalid_arguments(kw, code):
    d = kw.get("dim", 2)
    P = _pts(max(kw.get("n", 100), 1), 3 if d == 4 else d)[:kw.get("n", 100)]
    if kw.get("nan_point"):
        P = P.copy()
        P[5, 0] = np.nan
    with pytest.raises(h2mv.H2Error) as e:
        h2mv.h2_build_from_points(P, d, kw.get("leaf", 16), kw.get("p", 2), kw.get("eta", 0.9),
                                  kw.get("ell", 0.1), storage=kw.get("storage", 0),
                                  flags=h2mv.H2_FLAG_STRUCTURE_ONLY)
    assert e.value.code == code
    assert h2mv.h2_last_error()


def test_structure_only_handle_rejects_products():
    h = h2mv.h2_build_from_points(_pts(), 2, 16, 2, 0.9, 0.1, flags=h2mv.H2_FLAG_STRUCTURE_ONLY)
    try:
        with pytest.raises(h2mv.H2Error) as e:
            h2mv.h2_matvec(h, 8, 16)
        assert e.value.code == h2mv.H2_ERR_INVALID_ARG
        with pytest.raises(h2mv.H2Error):
            h2mv.h2_matmat(h, 8, 100, 16, 100, 2)
    finally:
        h2mv.h2_free(h)


def test_null_arguments():
    with pytest.raises(h2mv.H2Error):
        h2mv.h2_matvec(0, 8, 16)
    with pytest.raises(h2mv.H2Error):
        h2mv.h2_get_info(0)


def _valid_arrays():
    """A small, consistent H^2 given by arrays: 8 rows, q = 1, ranks (2, 3),
    one coupling block per leaf pair, dense diagonal blocks."""
    n = 8
    b = np.array([0, 0, 4], dtype=np.int64)
    e = np.array([8, 4, 8], dtype=np.int64)
    return {"n": n, "q": 1, "level_rank": np.array([2, 3], dtype=np.int32), "begin": b, "end": e,
            "U": np.ones(8 * 3), "V": np.ones(8 * 3), "E": np.ones(2 * 3 * 2), "F": np.ones(2 * 3 * 2),
            "S_rowptr": [np.array([0, 0], dtype=np.int32), np.array([0, 1, 2], dtype=np.int32)],
            "S_colidx": [np.zeros(0, dtype=np.int32), np.array([1, 0], dtype=np.int32)],
            "S": [np.zeros(0), np.ones(2 * 9)],
            "D_rowptr": np.array([0, 1, 2], dtype=np.int32), "D_colidx": np.array([0, 1], dtype=np.int32),
            "D": np.ones(2 * 16)}


def _bad(field, value):
    a = _valid_arrays()
    a[field] = value
    return a


@pytest.mark.parametrize("arr,storage,code", [
    (_bad("n", 0), 0, h2mv.H2_ERR_INVALID_ARG),
    (_bad("q", 30), 0, h2mv.H2_ERR_UNSUPPORTED),
    (_bad("q", -1), 0, h2mv.H2_ERR_INVALID_ARG),
    (_bad("level_rank", np.array([2, 0], dtype=np.int32)), 0, h2mv.H2_ERR_INVALID_ARG),
    (_bad("level_rank", np.array([2, 65], dtype=np.int32)), 0, h2mv.H2_ERR_UNSUPPORTED),
    (_bad("end", np.array([7, 4, 8], dtype=np.int64)), 0, h2mv.H2_ERR_INVALID_ARG),      # root not [0, n)
    (_bad("begin", np.array([0, 0, 5], dtype=np.int64)), 0, h2mv.H2_ERR_INVALID_ARG),    # gap between children
    (_bad("D_rowptr", np.array([0, 2, 1], dtype=np.int32)), 0, h2mv.H2_ERR_INVALID_ARG),  # decreasing
    (_bad("D_colidx", np.array([0, 2], dtype=np.int32)), 0, h2mv.H2_ERR_INVALID_ARG),     # column out of range
    (_bad("U", None), 0, h2mv.H2_ERR_INVALID_ARG),                                         # coupling without U
    (_valid_arrays(), 5, h2mv.H2_ERR_INVALID_ARG),
])
def test_build_from_arrays_rejects(arr, storage, code):
    with pytest.raises(h2mv.H2Error) as e:
        h2mv.h2_build_from_arrays(arr, storage)
    assert e.value.code == code
    assert h2mv.h2_last_error()


def test_build_from_arrays_rejects_wide_leaf():
    a = _valid_arrays()
    n = 130
    a.update(n=n, begin=np.array([0, 0, 65], dtype=np.int64), end=np.array([n, 65, n], dtype=np.int64))
    with pytest.raises(h2mv.H2Error) as e:
        h2mv.h2_build_from_arrays(a, 0)
    assert e.value.code == h2mv.H2_ERR_UNSUPPORTED


def test_read_probe_rejects_bad_arguments():
    for args in ((0, 16, 1, 8), (8, 16, 1, 0), (8, 8, 1, 8), (8, 24, 1, 8), (8, 16, 0, 8), (8, 16, 70000, 8)):
        with pytest.raises(h2mv.H2Error) as e:
            h2mv.h2_read_probe(*args)
        assert e.value.code == h2mv.H2_ERR_INVALID_ARG


def test_set_schedule_rejects_without_a_product_handle():
    with pytest.raises(h2mv.H2Error) as e:
        h2mv.h2_set_schedule(0, h2mv.H2_SCHEDULE_STREAMED)
    assert e.value.code == h2mv.H2_ERR_INVALID_ARG
    h = h2mv.h2_build_from_points(_pts(), 2, 16, 2, 0.9, 0.1, flags=h2mv.H2_FLAG_STRUCTURE_ONLY)
    try:
        with pytest.raises(h2mv.H2Error) as e:
            h2mv.h2_set_schedule(h, h2mv.H2_SCHEDULE_STREAMED)
        assert e.value.code == h2mv.H2_ERR_INVALID_ARG
    finally:
        h2mv.h2_free(h)
