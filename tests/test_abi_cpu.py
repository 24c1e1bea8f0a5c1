"""Host-side checks of the C ABI library: it loads, exports every symbol the
header declares, and its pure host logic (defaults, parameter validation,
null handles, status strings) behaves as documented.  No GPU needed."""
import ctypes
import os
import re

import pytest

from paper_1203_0889_amd import fmm

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_symbols():
    txt = open(os.path.join(ROOT, "include", "fmm.h")).read()
    return sorted(set(re.findall(r"^\s*(?:const char \*|fmm_status )(fmm_\w+)\(", txt, re.M)))


def test_library_exports_every_declared_symbol():
    lib = fmm.load_library()
    syms = header_symbols()
    assert len(syms) >= 16
    for s in syms:
        assert hasattr(lib, s), s
    assert set(syms) == set(fmm.EXPORTS)


def test_default_params_and_status_strings():
    lib = fmm.load_library()
    prm = fmm.fmm_params()
    assert lib.fmm_default_params(ctypes.byref(prm)) == 0
    assert (prm.p, prm.ncrit, prm.theta_num, prm.theta_den, prm.max_level, prm.precision) == (8, 64, 1, 2, 21, 1)
    assert lib.fmm_default_params(None) == -1
    for code, name in fmm.STATUS.items():
        assert lib.fmm_status_string(code).decode()
    assert lib.fmm_status_string(0).decode() == "ok"


@pytest.mark.parametrize("field,value", [("p", -1), ("p", 17), ("ncrit", 0), ("theta_num", 0), ("theta_den", 0),
                                         ("theta_num", 3), ("max_level", 0), ("max_level", 22), ("precision", 7),
                                         ("flags", 8)])
def test_create_rejects_bad_params_before_touching_a_device(field, value):
    lib = fmm.load_library()
    prm = fmm.fmm_params()
    lib.fmm_default_params(ctypes.byref(prm))
    if field == "theta_num" and value == 3:
        prm.theta_den = 2   # theta >= 1
    setattr(prm, field, value)
    h = ctypes.c_void_p()
    assert lib.fmm_create(ctypes.byref(prm), 0, None, ctypes.byref(h)) == -1
    assert not h.value


def test_create_rejects_bad_user_box():
    lib = fmm.load_library()
    prm = fmm.fmm_params()
    lib.fmm_default_params(ctypes.byref(prm))
    prm.flags = fmm.FLAG_USER_BOX
    prm.box_side = 0.0
    h = ctypes.c_void_p()
    assert lib.fmm_create(ctypes.byref(prm), 0, None, ctypes.byref(h)) == -1


def test_null_plan_is_rejected_everywhere():
    lib = fmm.load_library()
    off = (ctypes.c_int64 * 2)(0, 0)
    assert lib.fmm_build_tree(None, 1, off, None, None) == -1
    assert lib.fmm_upward(None) == -1
    assert lib.fmm_evaluate(None, None, None, None, None) == -1
    assert lib.fmm_backward(None, None, None, None) == -1
    assert lib.fmm_sync(None) == -1
    assert lib.fmm_get_counts(None, None, None, None, None) == -1
    assert lib.fmm_copy_tree(None, None, None, None) == -1
    assert lib.fmm_copy_lists(None, None, None, None, None) == -1
    assert lib.fmm_get_tuning(None, None) == -1
    assert lib.fmm_set_tuning(None, None) == -1
    assert lib.fmm_destroy(None) == 0
    assert lib.fmm_last_error(None).decode() == "null plan"


def test_python_binding_validates_tensors():
    import torch
    with pytest.raises((TypeError, ValueError)):
        fmm._check_dev(torch.zeros(4, 3, dtype=torch.float64), "pos", shape_tail=(3,))   # host tensor


def test_autotune_rejects_null_plan():
    lib = fmm.load_library()
    assert lib.fmm_autotune(None, 1, None, None) == -1
