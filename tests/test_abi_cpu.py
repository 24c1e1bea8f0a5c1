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


def _create_status(**fields):
    lib = fmm.load_library()
    prm = fmm.fmm_params()
    lib.fmm_default_params(ctypes.byref(prm))
    for k, v in fields.items():
        setattr(prm, k, v)
    h = ctypes.c_void_p()
    st = lib.fmm_create(ctypes.byref(prm), 0, None, ctypes.byref(h))
    if st == 0:
        lib.fmm_destroy(h)
    else:
        assert not h.value
    return st


@pytest.mark.parametrize("fields", [dict(p=-1), dict(p=17), dict(ncrit=0), dict(theta_num=0), dict(theta_den=0),
                                    dict(theta_num=3, theta_den=2), dict(theta_num=1, theta_den=1),
                                    dict(max_level=0), dict(max_level=22), dict(precision=7),
                                    dict(flags=1 << 8),
                                    dict(flags=fmm.FLAG_INCREMENTAL, theta_num=4, theta_den=5),
                                    dict(flags=fmm.FLAG_MUTUAL),   # mixed precision
                                    dict(flags=fmm.FLAG_MUTUAL_M2L), dict(flags=fmm.FLAG_MUTUAL_P2P),
                                    dict(precision=0, flags=fmm.FLAG_MUTUAL_P2P | fmm.FLAG_DETERMINISTIC)])
def test_create_rejects_bad_params_before_touching_a_device(fields):
    assert _create_status(**fields) == -1


@pytest.mark.parametrize("fields", [dict(), dict(flags=fmm.FLAG_DETERMINISTIC), dict(precision=0),
                                    dict(precision=0, flags=fmm.FLAG_MUTUAL),
                                    dict(precision=0, flags=fmm.FLAG_MUTUAL_M2L),
                                    dict(flags=fmm.FLAG_INCREMENTAL | fmm.FLAG_COST_REUSE, theta_num=2, theta_den=5)])
def test_create_accepts_good_params(fields):
    # past the parameter checks: a plan where a GPU is present, otherwise
    # the device error, never FMM_ERR_INVALID_ARG
    assert _create_status(**fields) in (0, -4)


def test_create_rejects_bad_user_box():
    lib = fmm.load_library()
    prm = fmm.fmm_params()
    lib.fmm_default_params(ctypes.byref(prm))
    prm.flags = fmm.FLAG_USER_BOX
    prm.box_side = 0.0
    h = ctypes.c_void_p()
    assert lib.fmm_create(ctypes.byref(prm), 0, None, ctypes.byref(h)) == -1


def test_python_binding_rejects_unknown_mutual_value():
    with pytest.raises(ValueError):
        fmm.Plan(p=4, precision="fp64", device=0, mutual="l2l")


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


def test_trace_rejects_null_plan_and_bad_capacity():
    lib = fmm.load_library()
    n = ctypes.c_int64(7)
    assert lib.fmm_get_trace(None, None, 0, ctypes.byref(n)) == -1


def test_trace_record_layout_matches_header():
    # fmm_task_record: two uint64 then six 32-bit fields, 40 bytes
    assert ctypes.sizeof(fmm.fmm_task_record) == 40
    assert fmm.TASK_DTYPE.itemsize == 40
    assert [f for f, _ in fmm.fmm_task_record._fields_] == list(fmm.TASK_DTYPE.names)


def test_trace_summary_on_synthetic_records():
    """Host logic of the trace summary: two compute units, one M2L task
    (4 waves) on the first and two P2P tasks on the second."""
    import numpy as np
    from paper_1203_0889_amd import trace
    rec = np.zeros(3, dtype=fmm.TASK_DTYPE)
    rec["start"] = [1000, 1000, 1500]
    rec["end"] = [2000, 1400, 2500]          # ticks: 10, 4 and 10 us
    rec["kind"] = [0, 1, 1]
    rec["kernel"] = [0, 1, 1]
    rec["hw_id"] = [3 << 8, 5 << 8, 5 << 8]   # CU 3 and CU 5
    rec["xcc"] = [0, 0, 0]
    s = trace.summarize(rec)
    assert s["tasks"] == 3 and s["compute_units"] == 2
    assert abs(s["span_us"] - 15.0) < 1e-9
    assert s["m2l"]["tasks"] == 1 and abs(s["m2l"]["mean_us"] - 10.0) < 1e-9
    assert s["p2p"]["tasks"] == 2 and s["p2p"]["by_side_kernel"] == 2
    # busy wave-time: CU 3 = 4 x 10 us, CU 5 = 4 + 10 us
    assert abs(s["cu_busy_wave_us"]["max"] - 40.0) < 1e-9 and abs(s["cu_busy_wave_us"]["min"] - 14.0) < 1e-9
    assert abs(s["cu_busy_imbalance"] - 40.0 / 27.0) < 1e-12
    assert trace.summarize(rec[:0]) == {"tasks": 0}


C_CONSUMER = r"""
#include <stdio.h>
#include "fmm.h"
int main(void) {
    fmm_params prm;
    fmm_plan *plan = NULL;
    if (fmm_default_params(&prm) != FMM_OK) return 1;
    prm.flags = FMM_FLAG_MUTUAL;   /* needs FP64: refused before any device call */
    if (fmm_create(&prm, 0, NULL, &plan) != FMM_ERR_INVALID_ARG || plan) return 2;
    printf("%d %d %s\n", prm.p, prm.ncrit, fmm_status_string(FMM_ERR_CAPACITY));
    return 0;
}
"""


def test_c_consumer_compiles_links_and_runs(tmp_path):
    # the header is plain C99 and the library links into a C program
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    pkg = os.path.join(root, "paper_1203_0889_amd")
    src, exe = tmp_path / "consumer.c", tmp_path / "consumer"
    src.write_text(C_CONSUMER)
    cmd = ["gcc", "-std=c99", "-pedantic", "-Wall", "-Wextra", "-Werror", "-I", os.path.join(root, "include"),
           str(src), "-o", str(exe), "-L", pkg, "-lfmm_mi355x", "-Wl,-rpath," + pkg]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, (r.returncode, r.stderr)
    p, ncrit, msg = r.stdout.split(" ", 2)
    assert (int(p), int(ncrit)) == (8, 64) and msg.strip()

