"""The work-queue autotuner (fmm_autotune): it picks a setting from its
candidate set, reports a positive kernel time, leaves the plan ready for
fmm_evaluate, and the tuned results agree with the default setting's up to
the FP32 rounding of the regrouped task sums."""
import numpy as np
import pytest
import torch

import oracle
from paper_1203_0889_amd import fmm, workloads as W
from parity import check_mixed, leaf_ids

pytestmark = pytest.mark.gpu


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def test_autotune_mixed():
    pos, q = W.uniform_cube(200000, 51)
    plan = fmm.Plan(p=8, ncrit=64, theta=(1, 2), precision="mixed", device=0)
    plan.build_tree(torch.from_numpy(pos).cuda(), torch.from_numpy(q).cuda())
    plan.upward()
    ref = {k: v.cpu().numpy() for k, v in plan.evaluate().items() if v is not None}
    tuning, ms = plan.autotune(repeats=2)
    print("autotune:", tuning, ms, flush=True)
    assert tuning["m2l_task_entries"] in (32, 64, 96, 128)
    assert (tuning["grid_per_cu"], tuning["p2p_per_cu"]) in ((1, 1), (1, 2), (1, 3), (2, 0), (3, 0), (2, 1), (2, 2))
    assert tuning["early_p2p_per_cu"] == 0
    assert ms > 0
    assert plan.get_tuning() == tuning
    out = {k: v.cpu().numpy() for k, v in plan.evaluate().items() if v is not None}
    torch.cuda.synchronize()
    assert rel(out["phi"], ref["phi"]) < 1e-6 and rel(out["field"], ref["field"]) < 1e-6
    # a later build keeps the tuned setting
    plan.build_tree(torch.from_numpy(pos).cuda(), torch.from_numpy(q).cuda())
    plan.upward()
    out2 = {k: v.cpu().numpy() for k, v in plan.evaluate().items() if v is not None}
    assert plan.get_tuning() == tuning
    assert rel(out2["phi"], ref["phi"]) < 1e-6


def test_autotune_fp64_task_size():
    # the FP64 path tunes the task size of its matrix-core M2L (the launch
    # shape untouched); results stay the FP64 path's to rounding
    pos, q = W.uniform_cube(20000, 52)
    dpos, dq = torch.from_numpy(pos).cuda(), torch.from_numpy(q).cuda()
    plan = fmm.Plan(p=6, ncrit=32, theta=(1, 2), precision="fp64", device=0)
    plan.build_tree(dpos, dq)
    plan.upward()
    ref = {k: v.cpu().numpy() for k, v in plan.evaluate().items()}
    shape = {k: v for k, v in plan.get_tuning().items() if k != "m2l_task_entries"}
    tuning, ms = plan.autotune(repeats=1)
    assert ms > 0 and tuning["m2l_task_entries"] in (16, 32, 64, 128)
    assert {k: v for k, v in tuning.items() if k != "m2l_task_entries"} == shape
    assert plan.get_tuning() == tuning
    out = {k: v.cpu().numpy() for k, v in plan.evaluate().items()}
    assert rel(out["phi"], ref["phi"]) < 1e-13 and rel(out["field"], ref["field"]) < 1e-13
    # deterministic mode: another plan with the chosen task size gives the
    # same bits
    plans = []
    for _ in range(2):
        pl = fmm.Plan(p=6, ncrit=32, theta=(1, 2), precision="fp64", device=0, deterministic=True)
        pl.set_tuning(**tuning)
        pl.build_tree(dpos, dq)
        pl.upward()
        plans.append({k: v.cpu().numpy() for k, v in pl.evaluate().items()})
    assert all(np.array_equal(plans[0][k], plans[1][k]) for k in ("phi", "field", "energy"))
    # nothing to tune where M2L runs per pair
    for kw in (dict(p=13), dict(p=6, mutual="m2l")):
        plan = fmm.Plan(ncrit=32, theta=(1, 2), precision="fp64", device=0, **kw)
        plan.build_tree(dpos, dq)
        plan.upward()
        assert plan.autotune()[1] == -1.0


def test_default_task_size_by_precision():
    # the FP64 path's matrix-core M2L runs its tasks as one plain launch and
    # takes smaller tasks by default than the mixed path's work queue
    assert fmm.Plan(p=4, precision="fp64", device=0).get_tuning()["m2l_task_entries"] == 32
    assert fmm.Plan(p=4, precision="mixed", device=0).get_tuning()["m2l_task_entries"] == 128


def test_tuning_validation():
    plan = fmm.Plan(p=4, precision="mixed", device=0)
    with pytest.raises(fmm.FMMError):
        plan.set_tuning(m2l_task_entries=0)
    with pytest.raises(fmm.FMMError):
        plan.set_tuning(grid_per_cu=9)
    with pytest.raises(fmm.FMMError):
        plan.set_tuning(p2p_per_cu=9)
    with pytest.raises(fmm.FMMError):
        plan.set_tuning(p2p_per_cu=-1)
    with pytest.raises(fmm.FMMError):
        plan.set_tuning(p2p_per_cu=1, early_p2p_per_cu=2)   # more early workgroups than side ones
    with pytest.raises(fmm.FMMError):
        plan.set_tuning(early_p2p_per_cu=-1)
    with pytest.raises(fmm.FMMError) as ei:
        plan.autotune()
    assert ei.value.status == -2


def test_autotune_right_after_upward():
    """Regression: the autotuner must size the evaluate workspaces itself
    (here no fmm_evaluate has run on the plan yet)."""
    pos, q = W.uniform_cube(60000, 53)
    plan = fmm.Plan(p=8, ncrit=64, theta=(1, 2), precision="mixed", device=0)
    plan.build_tree(torch.from_numpy(pos).cuda(), torch.from_numpy(q).cuda())
    plan.upward()
    tuning, ms = plan.autotune(repeats=1)
    assert ms > 0
    out = plan.evaluate()
    ref = fmm.Plan(p=8, ncrit=64, theta=(1, 2), precision="mixed", device=0)
    ref.build_tree(torch.from_numpy(pos).cuda(), torch.from_numpy(q).cuda())
    ref.upward()
    r = ref.evaluate()
    torch.cuda.synchronize()
    assert rel(out["phi"].cpu().numpy(), r["phi"].cpu().numpy()) < 1e-6


@pytest.mark.parametrize("dist", ["uniform", "plummer"])
def test_launch_shapes_agree(dist):
    """The queue with and without the P2P side kernel, and with several
    workgroup counts, on one tree: the near field is summed per leaf in a
    fixed order, and the locals differ only by the order of FP64 atomic
    additions of FP32 task sums.  (The launch shape is read at evaluate
    time; the task tables depend only on m2l_task_entries.)"""
    n = 150000
    pos, q = W.uniform_cube(n, 61) if dist == "uniform" else W.plummer(n, 62)
    plan = fmm.Plan(p=8, ncrit=64, theta=(1, 2), precision="mixed", device=0)
    plan.build_tree(torch.from_numpy(pos).cuda(), torch.from_numpy(q).cuda())
    ref = None
    for shape in ((1, 2), (2, 0), (1, 1), (3, 0), (1, 3), (4, 4)):
        plan.set_tuning(grid_per_cu=shape[0], p2p_per_cu=shape[1])
        plan.upward()
        out = {k: v.cpu().numpy() for k, v in plan.evaluate().items() if v is not None}
        torch.cuda.synchronize()
        if ref is None:
            ref = out
            continue
        e = (rel(out["phi"], ref["phi"]), rel(out["field"], ref["field"]))
        print(dist, "shape", shape, e, flush=True)
        assert max(e) < 1e-12


@pytest.mark.parametrize("entries", [1, 16, 96])
def test_task_sizes_match_oracle(entries):
    """The task-size knob (M2L class entries per task, the analogue of the
    paper's granularity Q) away from its default: the results still match
    the FP64 oracle FMM to the mixed path's bound, with a non-default launch
    shape too."""
    pos, q = W.plummer(25000, 64)
    ref_phi, ref_fld, _ = oracle.fmm(pos, q, 6, 32, 1, 2)
    plan = fmm.Plan(p=6, ncrit=32, theta=(1, 2), precision="mixed", device=0)
    plan.set_tuning(m2l_task_entries=entries, grid_per_cu=2, p2p_per_cu=1)
    plan.build_tree(torch.from_numpy(pos).cuda(), torch.from_numpy(q).cuda())
    plan.upward()
    out = {k: v.cpu().numpy() for k, v in plan.evaluate().items() if v is not None}
    torch.cuda.synchronize()
    e = (rel(out["phi"], ref_phi), rel(out["field"], ref_fld))
    print("entries", entries, "vs oracle", e, flush=True)
    assert max(e) < 1e-5
    _, perm, cells = plan.copy_tree()
    check_mixed(out, ref_phi, ref_fld, leaf_ids(perm, cells), label="entries %d" % entries)


def test_early_near_field_changes_no_result():
    """The near field started by the build (early_p2p_per_cu > 0, beside the
    upward pass and the far-field build) gives bitwise the results of the
    near field started with the queue, in deterministic mode: after a full
    build, after a kept-topology rebuild, from a step graph, through the
    evaluation that cannot allocate (other claim counters: the early kernel
    is waited for and the near field recomputed), and for a second
    evaluation of the same build (the queue's own near field)."""
    pos, q = W.uniform_cube(100000, 54)
    v = W.velocities(100000, 55, 1e-4)
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    res = {}
    for early in (0, 1):
        plan = fmm.Plan(p=8, ncrit=64, theta=(1, 2), precision="mixed", device=0, incremental=True,
                        deterministic=True)
        plan.set_tuning(grid_per_cu=1, p2p_per_cu=2, early_p2p_per_cu=early)
        got = []
        plan.build_tree(dev(pos), dev(q))
        plan.upward()
        got.append(plan.evaluate())
        got.append(plan.evaluate())                      # no new particles: the queue's near field
        plan.build_tree(dev(pos + v), dev(q))            # kept topology
        assert plan.build_info()["kept"] == 1
        plan.upward()
        got.append(plan.evaluate())
        plan.build_tree(dev(pos + 2 * v), dev(q))
        plan.upward()
        outs = {"phi": torch.empty(100000, dtype=torch.float64, device="cuda"),
                "field": torch.empty((100000, 3), dtype=torch.float64, device="cuda")}
        plan.evaluate_noalloc_into(**outs)
        got.append(dict(outs))
        gpos = dev(pos + 3 * v)
        g = {"phi": torch.empty(100000, dtype=torch.float64, device="cuda"),
             "field": torch.empty((100000, 3), dtype=torch.float64, device="cuda")}
        plan.graph_capture_step(gpos, dev(q), **g)
        gpos.copy_(dev(pos + 4 * v))
        plan.graph_launch()
        plan.sync()
        got.append(dict(g))
        res[early] = [{k: t.cpu().numpy() for k, t in o.items() if t is not None and k in ("phi", "field")}
                      for o in got]
        plan.close()
    for i, (a, b) in enumerate(zip(res[0], res[1])):
        for k in ("phi", "field"):
            assert np.array_equal(a[k], b[k]), (i, k)
