"""The C ABI on the host: every declared symbol is exported, and invalid
inputs are rejected with the documented status before any device work."""

import ctypes

import numpy as np
import pytest

from paper_1204_6255_amd import di

pytestmark = pytest.mark.filterwarnings("ignore")


def _has_gpu():
    try:
        import torch
        return torch.cuda.is_available()
    except Exception:
        return False


def test_every_declared_symbol_is_exported():
    names = di.declared_functions()
    assert {"di_graph_create", "di_solve", "di_solve_dev", "di_last_error"} <= set(names)
    L = di.lib()
    for name in names:
        assert hasattr(L, name), name


def test_version_and_defaults():
    assert di.di_version() >> 16 == 1
    o = di.di_opts_default()
    assert o.method == di.DI_SOP and o.precision == di.DI_FP64 and o.stop == di.DI_STOP_RESID
    assert o.max_cycles > 0 and o.inner_tol > 0


def test_struct_layouts_match_header():
    # sizes follow from the field lists in include/di.h
    assert ctypes.sizeof(di.di_opts) == 40
    assert ctypes.sizeof(di.di_stats) == 4 * 4 + 8 + 13 * 8


@pytest.mark.parametrize("n,src,dst,expect", [
    (3, [0, 1, 1], [1, 0, 0], di.DI_E_DUP),
    (3, [0, 1, 0], [1, 0, 2], di.DI_E_UNSORTED),
    (3, [0, 0], [2, 1], di.DI_E_UNSORTED),
    (3, [0, 1], [1, 3], di.DI_E_RANGE),
    (3, [-1, 1], [1, 2], di.DI_E_RANGE),
    (0, [], [], di.DI_E_INVAL),
    (-5, [], [], di.DI_E_INVAL),
])
def test_graph_create_rejects_bad_link_lists(n, src, dst, expect):
    st, h = di.di_graph_create(n, np.array(src, np.int32), np.array(dst, np.int32))
    assert st == expect, (di.STATUS_NAMES.get(st), di.di_last_error())
    assert not h
    assert di.di_last_error()


def test_graph_create_rejects_flags():
    st, h = di.di_graph_create(3, np.array([0], np.int32), np.array([1], np.int32), flags=4)
    assert st == di.DI_E_INVAL


def test_graph_create_null_arrays():
    h = ctypes.c_void_p()
    assert di.lib().di_graph_create(4, 2, None, None, 0, ctypes.byref(h)) == di.DI_E_INVAL
    assert di.lib().di_graph_create(4, 0, None, None, 0, None) == di.DI_E_INVAL


def test_solve_rejects_null_graph():
    X = np.zeros(4)
    st, _ = di.di_solve(None, None, 0.85, 1e-9, None, X)
    assert st == di.DI_E_INVAL


@pytest.mark.skipif(_has_gpu(), reason="checks the no-GPU path")
def test_valid_graph_without_gpu_reports_device_error():
    st, h = di.di_graph_create(3, np.array([0, 1], np.int32), np.array([1, 2], np.int32))
    assert st == di.DI_E_DEVICE
    assert "no CPU fallback" in di.di_last_error()


def test_serving_struct_layout():
    assert ctypes.sizeof(di.di_serve_stats) == 6 * 8 + 8 + 8


@pytest.mark.skipif(_has_gpu(), reason="checks the no-GPU path")
def test_serving_without_gpu_reports_device_error():
    st, h = di.di_serve_create(1 << 30, 8)
    assert st == di.DI_E_DEVICE and not h.value
    st, _ = di.di_serve_create(1 << 30, 0)
    assert st == di.DI_E_INVAL


def test_batch_rejects_bad_arguments_before_device_work():
    st, _, _ = di.di_solve_batch(None, 2, None, 0.85, [1e-9, 1e-9])
    assert st == di.DI_E_INVAL


def test_cycle_record_layout():
    # double r, int64 links, int32 selected, int32 senders
    assert ctypes.sizeof(di.di_cycle_rec) == 24


def test_trace_rejects_bad_arguments_before_device_work():
    L = di.lib()
    recs = (di.di_cycle_rec * 4)()
    count = ctypes.c_int32(-1)
    st = di.di_stats()
    o = di.di_opts_default()
    # no graph
    assert L.di_solve_trace_dev(None, None, 0.85, 1e-9, ctypes.byref(o), None, ctypes.byref(st),
                                recs, 4, ctypes.byref(count)) == di.DI_E_INVAL
    assert count.value == 0
    # negative capacity, records missing for a positive capacity, no count
    assert L.di_solve_trace_dev(None, None, 0.85, 1e-9, ctypes.byref(o), None, ctypes.byref(st),
                                recs, -1, ctypes.byref(count)) == di.DI_E_INVAL
    assert L.di_solve_trace_dev(None, None, 0.85, 1e-9, ctypes.byref(o), None, ctypes.byref(st),
                                None, 4, ctypes.byref(count)) == di.DI_E_INVAL
    assert L.di_solve_trace_dev(None, None, 0.85, 1e-9, ctypes.byref(o), None, ctypes.byref(st),
                                recs, 4, None) == di.DI_E_INVAL
    # the asynchronous Gauss-Seidel baseline has no cycles to trace
    o.method = di.DI_GS_ASYNC
    assert L.di_solve_trace_dev(None, None, 0.85, 1e-9, ctypes.byref(o), None, ctypes.byref(st),
                                recs, 4, ctypes.byref(count)) == di.DI_E_INVAL
    assert "Gauss" in di.di_last_error() or "DI_GS_ASYNC" in di.di_last_error()
