"""The C ABI library loads on a host without a GPU and exports every function
include/knnd.h declares; argument errors are reported before any device work."""
import ctypes
import os
import re

import numpy as np
import pytest

import paper_2202_00517_amd as knnd

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    text = open(os.path.join(ROOT, "include", "knnd.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(knnd_\w+)\s*\(", text)))


def test_header_declares_the_bound_functions():
    assert _declared() == sorted(knnd.EXPORTED)


def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(knnd.LIB_PATH)
    for name in _declared():
        assert hasattr(lib, name), name


def test_abi_version_and_status_strings():
    text = open(os.path.join(ROOT, "include", "knnd.h")).read()
    ver = int(re.search(r"#define KNND_ABI_VERSION (\d+)", text).group(1))
    assert knnd.lib().knnd_abi_version() == ver
    for code, name in [(0, "KNND_OK"), (1, "KNND_WARN_MAX_ROUNDS"), (-1, "KNND_ERR_ARG"),
                       (-2, "KNND_ERR_DOMAIN"), (-3, "KNND_ERR_NOMEM"), (-4, "KNND_ERR_DEVICE"),
                       (-5, "KNND_ERR_UNSUPPORTED")]:
        assert knnd.status_string(code) == name


def test_params_struct_layout_matches_header():
    assert ctypes.sizeof(knnd.knnd_params) == 40
    assert knnd.knnd_params.delta.offset == 32
    assert ctypes.sizeof(knnd.knnd_round_stats) == 88
    p = knnd.default_params()
    assert (p.precision, p.dtype, p.fcr_samples, p.max_rounds, p.flags) == (0, 0, 0, 100, 0)
    assert (p.stop_rule, p.comparator, p.delta) == (knnd.KNND_STOP_FCR, knnd.KNND_CMP_KL, 0.0)


@pytest.mark.parametrize("kw", [dict(stop_rule=3), dict(stop_rule=-1), dict(comparator=4), dict(comparator=-1),
                                dict(stop_rule=2, delta=-0.5), dict(stop_rule=2, delta=float("nan")),
                                dict(stop_rule=2, delta=float("inf")), dict(precision=4)])
def test_bad_params_are_argument_errors_before_device_work(kw):
    P = np.full((10, 4), 0.25, dtype=np.float32)
    idx = np.empty((10, 3), dtype=np.int32)
    r = ctypes.c_int32()
    p = knnd.default_params(**kw)
    st = knnd.lib().knnd_build_ex(P.ctypes.data, 10, 3, 3, 1, ctypes.byref(p), 0, None,
                                  idx.ctypes.data, None, None, ctypes.byref(r))
    assert st == knnd.KNND_ERR_ARG
    arr = (knnd.knnd_instance * 1)()
    arr[0].points, arr[0].n, arr[0].d, arr[0].K, arr[0].seed = P.ctypes.data, 10, 3, 3, 1
    arr[0].out_idx = idx.ctypes.data
    arr[0].out_rounds = ctypes.pointer(r)
    assert knnd.lib().knnd_build_batched(arr, 1, ctypes.byref(p), 0, None) == knnd.KNND_ERR_ARG


@pytest.mark.parametrize("n,d,K", [(1, 3, 2), (10, 0, 2), (10, 3, 1), (10, 3, 10), (200, 3, 65)])
def test_shape_errors_return_before_device_work(n, d, K):
    P = np.full((max(n, 1), d + 1), 1.0 / (d + 1), dtype=np.float32)
    idx = np.empty((max(n, 1), max(K, 1)), dtype=np.int32)
    upd = np.empty(4, dtype=np.int64)
    r = ctypes.c_int32()
    st = knnd.lib().knnd_build(P.ctypes.data, n, d, K, 1, idx.ctypes.data, upd.ctypes.data, 4,
                               ctypes.byref(r))
    assert st == knnd.KNND_ERR_ARG


def test_null_pointers_are_argument_errors():
    lib = knnd.lib()
    r = ctypes.c_int32()
    assert lib.knnd_build(None, 10, 3, 2, 1, None, None, 4, ctypes.byref(r)) == knnd.KNND_ERR_ARG
    assert lib.knnd_ctx_round(None, None) == knnd.KNND_ERR_ARG
    assert lib.knnd_ctx_round_share(None, 0, 1, None) == knnd.KNND_ERR_ARG
    assert lib.knnd_ctx_destroy(None) == knnd.KNND_ERR_ARG
    assert lib.knnd_ctx_rounds(None) == -1


def test_batched_struct_layout_and_argument_errors():
    assert ctypes.sizeof(knnd.knnd_instance) == 72
    lib = knnd.lib()
    assert lib.knnd_build_batched(None, 1, None, 0, None) == knnd.KNND_ERR_ARG
    arr = (knnd.knnd_instance * 2)()
    P = np.full((10, 4), 0.25, dtype=np.float32)
    idx = np.empty((10, 3), dtype=np.int32)
    r = ctypes.c_int32()
    for b in range(2):
        arr[b].points, arr[b].n, arr[b].d, arr[b].K, arr[b].seed = P.ctypes.data, 10, 3, 3, b
        arr[b].out_idx = idx.ctypes.data
        arr[b].out_rounds = ctypes.pointer(r)
    assert lib.knnd_build_batched(arr, 0, None, 0, None) == knnd.KNND_ERR_ARG
    arr[1].K = 10  # K > n - 1 in the second instance
    assert lib.knnd_build_batched(arr, 2, None, 0, None) == knnd.KNND_ERR_ARG
