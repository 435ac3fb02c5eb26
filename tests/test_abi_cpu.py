"""C-ABI checks that need no GPU: the library loads, exports every function include/stp.h declares,
and rejects invalid arguments on the host before any device work."""
import ctypes as C
import os
import re

import pytest

from paper_2003_12787_amd import stp

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    text = open(os.path.join(ROOT, "include", "stp.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^\s*[A-Za-z_][\w \*]*?\b(stp_\w+)\s*\(", text, flags=re.M)))


@pytest.fixture(scope="module")
def L():
    if not os.path.exists(stp.LIB_PATH):
        import paper_2003_12787_amd.build as b
        b.build()
    return stp.lib()


def test_header_declares_the_abi():
    assert declared_functions() == sorted(stp.SYMBOLS)


def test_library_exports_every_declared_symbol(L):
    for name in declared_functions():
        assert hasattr(L, name), name


def _desc(classes, prec=stp.FP32, device=0, variant=0):
    arr = (stp.Class * len(classes))(*[stp.Class(*c) for c in classes])
    d = stp.PlanDesc(len(classes), arr, prec, 0, device, variant, 0)
    d._arr = arr
    return d


@pytest.mark.parametrize("classes,prec,expect", [
    ([(0, 9, stp.ELASTIC, 0)], stp.FP32, stp.E_UNSUPPORTED),     # order below 1
    ([(10, 9, stp.ELASTIC, 0)], stp.FP32, stp.E_UNSUPPORTED),    # order above 9
    ([(3, 4, stp.ELASTIC, 0)], stp.FP32, stp.E_UNSUPPORTED),     # elastic needs m = 9
    ([(3, 9, stp.ACOUSTIC, 0)], stp.FP32, stp.E_UNSUPPORTED),    # acoustic needs m = 4
    ([(3, 17, stp.GENERIC, 0)], stp.FP32, stp.E_UNSUPPORTED),    # generic m <= 16
    ([(3, 0, stp.GENERIC, 0)], stp.FP32, stp.E_UNSUPPORTED),
    ([(3, 9, 7, 0)], stp.FP32, stp.E_INVAL),                     # unknown physics
    ([(3, 9, stp.ELASTIC, 1 << 9)], stp.FP32, stp.E_INVAL),      # unknown flag
    ([(3, 9, stp.ELASTIC, stp.A_PRESENT)], stp.FP32, stp.E_INVAL),  # A only for generic
    ([(3, 4, stp.GENERIC, stp.PARAM_PER_ELEMENT)], stp.FP32, stp.E_INVAL),
    ([(3, 9, stp.ELASTIC, 0)], 7, stp.E_INVAL),                  # unknown precision
    ([(3, 4, stp.ELASTIC_CURV, 0)], stp.FP32, stp.E_UNSUPPORTED),  # curvilinear elastic needs m = 9
    ([(3, 9, stp.ELASTIC_CURV, stp.COEF_PER_ELEMENT)], stp.FP32, stp.E_INVAL),  # params, not A/B
])
def test_plan_rejects_invalid_classes_on_host(L, classes, prec, expect):
    d = _desc(classes, prec)
    h = C.c_void_p()
    assert L.stp_plan(C.byref(d), C.byref(h)) == expect


def test_plan_rejects_unknown_node_family(L):
    d = _desc([(3, 9, stp.ELASTIC, 0)])
    d.nodes = 2
    h = C.c_void_p()
    assert L.stp_plan(C.byref(d), C.byref(h)) == stp.E_INVAL
    assert "nodes" in stp.last_error()


@pytest.mark.parametrize("mode", [-1, 3])
def test_plan_rejects_unknown_autotune_mode(L, mode):
    d = _desc([(3, 9, stp.ELASTIC, 0)])
    d.autotune = mode
    h = C.c_void_p()
    assert L.stp_plan(C.byref(d), C.byref(h)) == stp.E_INVAL
    assert "autotune" in stp.last_error()
    assert h.value is None
    assert stp.last_error() != ""


def test_plan_rejects_null_and_bad_counts(L):
    h = C.c_void_p()
    assert L.stp_plan(None, C.byref(h)) == stp.E_INVAL
    d = _desc([(3, 9, stp.ELASTIC, 0)])
    assert L.stp_plan(C.byref(d), None) == stp.E_INVAL
    d.nclass = 0
    assert L.stp_plan(C.byref(d), C.byref(h)) == stp.E_INVAL
    d = _desc([(3, 9, stp.ELASTIC, 0)], device=-1)
    assert L.stp_plan(C.byref(d), C.byref(h)) == stp.E_INVAL
    d = _desc([(3, 9, stp.ELASTIC, 0)], variant=99)
    assert L.stp_plan(C.byref(d), C.byref(h)) == stp.E_INVAL


def test_null_plan_entry_points(L):
    b = stp.Batch()
    assert L.stp_run(None, C.byref(b), None) == stp.E_INVAL
    t = C.c_uint64()
    assert L.stp_submit(None, C.byref(b), C.byref(t)) == stp.E_INVAL
    assert L.stp_poll(None, 1, None) == stp.E_INVAL
    assert L.stp_drain(None) == stp.E_INVAL
    assert L.stp_reserve(None, 10) == stp.E_INVAL
    assert L.stp_plan_describe(None, None, 0) == stp.E_INVAL
    assert L.stp_correct(None, None, None) == stp.E_INVAL
    assert L.stp_face_params(None, 1, 16, 1 << 20, None) == stp.E_INVAL
    assert L.stp_class_cost(None, 0, None, None) == stp.E_INVAL
    L.stp_plan_free(None)  # no-op
    assert "NULL" in stp.last_error()
