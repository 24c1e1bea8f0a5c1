"""Device task trace (FMM_FLAG_TRACE, fmm_get_trace) on the GPU: every task
of the work queue is recorded exactly once, with sane times and units, and
tracing does not change the results.  The uniform input (2e5 particles,
seed 71) is one whose M2L target count the group build used to overcount
(see the target-count test of the mixed path)."""
import numpy as np
import pytest
import torch

from paper_1203_0889_amd import fmm, trace, workloads as W

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def run(dist, traced, n=200000, prec="mixed"):
    pos, q = W.uniform_cube(n, 71) if dist == "uniform" else W.plummer(n, 72)
    plan = fmm.Plan(p=8, ncrit=64, theta=(1, 2), precision=prec, device=0, trace=traced)
    plan.build_tree(torch.from_numpy(pos).cuda(), torch.from_numpy(q).cuda())
    plan.upward()
    out = {k: v.cpu().numpy() for k, v in plan.evaluate().items() if v is not None}
    torch.cuda.synchronize()
    return plan, out


@pytest.mark.parametrize("dist", ["uniform", "plummer"])
def test_trace_records_every_task_once(dist):
    plan, out = run(dist, True)
    rec = plan.trace()
    _, _, cells = plan.copy_tree()
    leaves = np.nonzero((cells[:, 6] < 0) & (cells[:, 5] > 0))[0]
    m2l = rec[rec["kind"] == 0]
    p2p = rec[rec["kind"] == 1]
    say(dist, "records", len(rec), "m2l", len(m2l), "p2p", len(p2p), "leaves", len(leaves))
    assert len(m2l) + len(p2p) == len(rec)
    # M2L task indices are a permutation of the task table; P2P tasks are the leaves
    assert np.array_equal(np.sort(m2l["task"]), np.arange(len(m2l)))
    assert np.array_equal(np.sort(p2p["task"]), leaves)
    assert np.all(rec["end"] >= rec["start"])
    assert set(np.unique(rec["kernel"])) <= {0, 1}
    assert np.all(m2l["kernel"] == 0)
    assert np.all(rec["xcc"] < 8)
    s = trace.summarize(rec)
    say(dist, s)
    assert s["compute_units"] > 1 and s["span_us"] > 0 and s["cu_busy_imbalance"] >= 1.0
    # tracing changes no result (other builds of the same input differ only
    # by the FP32 summation order of the per-target source lists)
    _, ref = run(dist, False)
    assert rel(out["phi"], ref["phi"]) < 1e-6 and rel(out["field"], ref["field"]) < 1e-6


def test_trace_off_and_fp64_record_nothing():
    plan, _ = run("uniform", False, n=20000)
    assert len(plan.trace()) == 0
    plan, _ = run("uniform", True, n=20000, prec="fp64")
    assert len(plan.trace()) == 0


def test_trace_capacity_argument():
    plan, _ = run("uniform", True, n=20000)
    full = plan.trace()
    lib = fmm.load_library()
    import ctypes
    part = np.zeros(5, dtype=fmm.TASK_DTYPE)
    n = ctypes.c_int64()
    assert lib.fmm_get_trace(plan._h, ctypes.c_void_p(part.ctypes.data), 5, ctypes.byref(n)) == 0
    assert n.value == len(full) and len(full) > 5
    assert np.array_equal(part, full[:5])
