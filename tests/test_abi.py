"""C ABI contract checks that need no GPU: the library loads, exports every entry
point the header declares, and rejects bad arguments before touching the device."""
import ctypes
import os
import re

import pytest

import paper_2403_01596_amd as p2p

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    text = open(os.path.join(ROOT, "include", "p2p.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(p2p_[a-z_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for n in ("p2p_plan_create", "p2p_apply", "p2p_apply_backward", "p2p_plan_destroy", "p2p_box_ids",
              "p2p_plan_info", "p2p_plan_export", "p2p_status_str", "p2p_last_error"):
        assert n in names


def test_library_exports_every_declared_symbol():
    L = p2p.lib()
    for n in declared_functions():
        assert hasattr(L, n), n


def test_status_strings():
    L = p2p.lib()
    for s in range(7):
        assert len(L.p2p_status_str(s)) > 0
    assert L.p2p_status_str(99) == b"unknown status"


def test_argument_errors_before_device_work():
    L = p2p.lib()
    out = ctypes.c_void_p()
    assert L.p2p_plan_create(None, None, 0, 1.0, None, None, None) == 1
    assert b"out" in L.p2p_last_error()
    assert L.p2p_plan_create(None, None, -1, 1.0, None, None, ctypes.byref(out)) == 1
    assert L.p2p_plan_create(None, None, 5, 1.0, None, None, ctypes.byref(out)) == 1  # NULL arrays
    dummy = ctypes.c_void_p(16)
    assert L.p2p_plan_create(dummy, dummy, 5, -1.0, None, None, ctypes.byref(out)) == 2
    assert L.p2p_plan_create(dummy, dummy, 5, float("nan"), None, None, ctypes.byref(out)) == 2
    assert L.p2p_plan_create(dummy, dummy, 10 ** 9, 1.0, None, None, ctypes.byref(out)) == 2
    bad = p2p._Opts(7, 0, 1, 0, None)
    assert L.p2p_plan_create(dummy, dummy, 5, 1.0, ctypes.byref(bad), None, ctypes.byref(out)) == 1
    bad = p2p._Opts(1, 0, 0, 0, None)
    assert L.p2p_plan_create(dummy, dummy, 5, 1.0, ctypes.byref(bad), None, ctypes.byref(out)) == 1
    bad = p2p._Opts(1, 0, 1, 4, None)
    assert L.p2p_plan_create(dummy, dummy, 5, 1.0, ctypes.byref(bad), None, ctypes.byref(out)) == 1
    assert out.value is None
    # invalid handles
    assert L.p2p_apply(None, None, None, 1, 1, None) == 6
    assert L.p2p_apply_backward(None, None, None, None, None, 1, 1, None) == 6
    assert L.p2p_plan_info(None, None) == 6
    assert L.p2p_plan_destroy(None) == 0
    assert L.p2p_batch_destroy(None) == 0

    origin = (ctypes.c_double * 3)(0, 0, 0)
    assert L.p2p_box_ids(None, -1, origin, 1.0, None, None) == 1
    assert L.p2p_box_ids(dummy, 5, origin, 0.0, dummy, None) == 2
    assert L.p2p_box_ids(dummy, 5, None, 1.0, dummy, None) == 1
    # the plan from a leaf grid
    assert L.p2p_plan_create_grid(dummy, 5, None, 1.0, 1.0, None, None, ctypes.byref(out)) == 1
    assert L.p2p_plan_create_grid(dummy, 5, origin, 0.0, 1.0, None, None, ctypes.byref(out)) == 2
    assert L.p2p_plan_create_grid(dummy, 5, origin, float("nan"), 1.0, None, None, ctypes.byref(out)) == 2
    assert L.p2p_plan_create_grid(dummy, 5, (ctypes.c_double * 3)(0, float("inf"), 0), 1.0, 1.0, None, None,
                                  ctypes.byref(out)) == 2
    assert L.p2p_plan_create_grid(dummy, -1, origin, 1.0, 1.0, None, None, ctypes.byref(out)) == 1
    assert L.p2p_plan_create_grid(None, 5, origin, 1.0, 1.0, None, None, ctypes.byref(out)) == 1
    assert L.p2p_plan_create_grid(dummy, 5, origin, 1.0, -2.0, None, None, ctypes.byref(out)) == 2
    assert L.p2p_plan_create_grid(dummy, 5, origin, 1.0, 1.0, None, None, None) == 1
    assert out.value is None


def test_foreign_handles_are_not_read():
    # pointers that were never handed out by the library (as a destroyed handle
    # would be): looked up among the live handles, so nothing is dereferenced
    L = p2p.lib()
    for h in (ctypes.c_void_p(16), ctypes.c_void_p(0xdead0000), ctypes.c_void_p(ctypes.addressof(ctypes.c_int64(7)))):
        assert L.p2p_plan_destroy(h) == 6
        assert L.p2p_apply(h, None, None, 1, 1, None) == 6
        assert L.p2p_apply_backward(h, None, None, None, None, 1, 1, None) == 6
        assert L.p2p_plan_info(h, None) == 6
        assert L.p2p_plan_export(h, None, None, None, None, None) == 6
        assert L.p2p_plan_timing(h, 1) == 6
        assert L.p2p_batch_destroy(h) == 6
        assert L.p2p_batch_apply(h, None, None, None) == 6
        assert b"invalid" in L.p2p_last_error()

def test_missing_library_fails_loudly(monkeypatch, tmp_path):
    monkeypatch.setattr(p2p, "_lib", None)
    monkeypatch.setattr(p2p, "LIB_PATH", str(tmp_path / "absent.so"))
    with pytest.raises(ImportError):
        p2p.lib()
