"""Time stepping on a kept topology (FMM_FLAG_INCREMENTAL, FMM_FLAG_COST_REUSE,
fmm_graph_capture_step).

Particles move along straight lines; every step is checked against the
oracle evaluated with the tree and lists of the first build and the moved
particles (the frozen-tree evaluation of the oracle, itself pinned against
the direct sum on the CPU).  A kept step must match it to the parity bounds
of a fresh build; a move beyond the widened leaves must trigger a full
rebuild, checked against a fresh oracle build.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_1203_0889_amd import fmm, workloads as W
from parity import check_fp64, check_mixed, leaf_ids, rel

pytestmark = pytest.mark.gpu

N = 20000
P = 8
NCRIT = 64


def say(*a):
    print(*a, flush=True)


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def host(out):
    return {k: v.cpu().numpy() for k, v in out.items() if v is not None}


def leaf_sides(T):
    """Side of the leaf cell holding every particle (input order)."""
    lv, cf = T.cell("level"), T.cell("child_first")
    first, cnt = T.cell("first"), T.cell("count")
    side = np.zeros(T.n)
    for c in np.nonzero(cf < 0)[0]:
        side[T.perm[first[c]:first[c] + cnt[c]]] = T.box[3] / 2.0 ** lv[c]
    return side


def setup(seed=81):
    pos0, q = W.uniform_cube(N, seed)
    T = oracle.Tree(pos0, NCRIT)
    T.lists(1, 2)
    side = leaf_sides(T)
    v = W.velocities(N, seed + 1, side)     # one leaf side per unit of time
    return pos0, q, T, v, side


def check(prec, out, ref, ids, label):
    if prec == "fp64":
        e = (rel(out["phi"], ref[0]), rel(out["field"], ref[1]))
        say(label, "rel L2 vs the oracle", e)
        assert max(e) < 1e-11
        check_fp64(out, ref[0], ref[1], ids, say, label)
    else:
        e = (rel(out["phi"], ref[0]), rel(out["field"], ref[1]))
        say(label, "rel L2 vs the oracle", e)
        assert max(e) < 1e-5
        check_mixed(out, ref[0], ref[1], ids, say, label)


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_incremental_steps_match_frozen_oracle(prec):
    say("incremental", prec, "N", N)
    pos0, q, T, v, side = setup()
    plan = fmm.Plan(p=P, ncrit=NCRIT, theta=(1, 2), precision=prec, device=0, incremental=True)
    plan.build_tree(dev(pos0), dev(q))
    _, perm, cells = plan.copy_tree()
    ids = leaf_ids(perm, cells)
    assert plan.build_info() == {"full": 1, "kept": 0}
    for k in (1, 2, 3):
        # at most 0.09 of a leaf side per axis: inside the widened leaves
        pos = pos0 + 0.03 * k * v
        qk = q * (1.0 + 0.1 * k)
        plan.build_tree(dev(pos), dev(qk))
        assert plan.build_info() == {"full": 1, "kept": k}
        plan.upward()
        out = host(plan.evaluate())
        check(prec, out, T.fmm(qk, P, pos=pos), ids, "step %d" % k)
        assert out["energy"][0] == pytest.approx(0.5 * np.dot(qk, out["phi"]), rel=1e-12)
    # a third of a leaf side: particles leave their widened leaves, so the
    # tree is built again from these positions
    pos = pos0 + 0.3 * v
    plan.build_tree(dev(pos), dev(q))
    assert plan.build_info() == {"full": 2, "kept": 3}
    plan.upward()
    out = host(plan.evaluate())
    T2 = oracle.Tree(pos, NCRIT)
    T2.lists(1, 2)
    _, perm, cells = plan.copy_tree()
    check(prec, out, T2.fmm(q, P), leaf_ids(perm, cells), "rebuilt")


def test_keep_topology_never_rebuilds():
    pos0, q, T, v, side = setup(83)
    plan = fmm.Plan(p=P, ncrit=NCRIT, theta=(1, 2), precision="fp64", device=0, keep_topology=True)
    plan.build_tree(dev(pos0), dev(q))
    pos = pos0 + 0.3 * v                      # beyond the widened leaves: kept all the same
    plan.build_tree(dev(pos), dev(q))
    assert plan.build_info() == {"full": 1, "kept": 1}
    plan.upward()
    out = host(plan.evaluate())
    _, perm, cells = plan.copy_tree()
    check("fp64", out, T.fmm(q, P, pos=pos), leaf_ids(perm, cells), "kept beyond the leaves")


def test_incremental_needs_theta_below_four_fifths():
    with pytest.raises(fmm.FMMError) as ei:
        fmm.Plan(p=4, ncrit=64, theta=(4, 5), precision="mixed", device=0, incremental=True)
    assert ei.value.status == -1
    fmm.Plan(p=4, ncrit=64, theta=(3, 4), precision="mixed", device=0, incremental=True).close()


def other_work():
    pos, q = W.uniform_cube(2000, 99)
    plan = fmm.Plan(p=4, ncrit=32, theta=(1, 2), precision="mixed", device=0)
    plan.build_tree(dev(pos), dev(q))
    plan.upward()
    plan.evaluate()
    x = torch.randn(1 << 20, device="cuda")
    (x * 2.0).sum().item()


@pytest.mark.parametrize("prec", ["mixed", "fp64"])
def test_step_graph_replays(prec):
    """One captured graph per time step (rebuild on the kept topology,
    upward, evaluate): each replay reads the positions written into the
    captured input tensor and matches, bit for bit, an eager step of a
    second plan (deterministic mode) and the frozen-tree oracle."""
    say("step graph", prec)
    pos0, q, T, v, side = setup(85)
    kw = dict(p=P, ncrit=NCRIT, theta=(1, 2), precision=prec, device=0, incremental=True, deterministic=True)
    plan, ref_plan = fmm.Plan(**kw), fmm.Plan(**kw)
    plan.build_tree(dev(pos0), dev(q))
    ref_plan.build_tree(dev(pos0), dev(q))
    _, perm, cells = plan.copy_tree()
    ids = leaf_ids(perm, cells)
    pos_t, q_t = dev(pos0 + 0.02 * v), dev(q)
    out = {"phi": torch.empty(N, dtype=torch.float64, device="cuda"),
           "field": torch.empty((N, 3), dtype=torch.float64, device="cuda"),
           "force": torch.empty((N, 3), dtype=torch.float64, device="cuda"),
           "energy": torch.empty(1, dtype=torch.float64, device="cuda")}
    plan.graph_capture_step(pos_t, q_t, **out)
    for k in (2, 3, 4):
        pos = pos0 + 0.02 * k * v
        pos_t.copy_(dev(pos))
        for t in out.values():
            t.zero_()
        torch.cuda.synchronize()
        plan.graph_launch()
        plan.sync()
        got = host(out)
        ref_plan.build_tree(dev(pos), dev(q))
        ref_plan.upward()
        ref = host(ref_plan.evaluate())
        for name in ("phi", "field", "force", "energy"):
            assert np.array_equal(got[name], ref[name]), (k, name)
        check(prec, got, T.fmm(q, P, pos=pos), ids, "replay %d" % k)
        other_work()
    assert plan.build_info() == {"full": 1, "kept": 1}   # the capture's own eager step
    # a particle beyond its widened leaf: the replay reports it
    bad = pos0.copy()
    bad[7, np.argmax(np.abs(v[7]))] += 0.5 * side[7] * np.sign(v[7, np.argmax(np.abs(v[7]))])   # half a leaf side
    pos_t.copy_(dev(bad))
    torch.cuda.synchronize()
    plan.graph_launch()
    with pytest.raises(fmm.FMMError) as ei:
        plan.sync()
    assert ei.value.status == -2
    # an eager build from those positions rebuilds and drops the graph
    plan.build_tree(dev(bad), dev(q))
    assert plan.build_info()["full"] == 2
    with pytest.raises(fmm.FMMError):
        plan.graph_launch()


@pytest.mark.parametrize("prec", ["mixed", "fp64"])
def test_step_graph_batch(prec):
    """A batch of instances in one step graph (kept topology): every replay
    with new positions and charges equals, bit for bit, an eager step of a
    second plan (deterministic mode), per-instance energies included."""
    pos0, q0, offsets = W.batch(6, 17)
    offs = [int(o) for o in offsets]
    n = len(q0)
    say("step graph batch", prec, "N", n)
    kw = dict(p=6, ncrit=64, theta=(1, 2), precision=prec, device=0, keep_topology=True, deterministic=True)
    plan, ref_plan = fmm.Plan(**kw), fmm.Plan(**kw)
    plan.build_tree(dev(pos0), dev(q0), offs)
    ref_plan.build_tree(dev(pos0), dev(q0), offs)
    pos_t, q_t = dev(pos0), dev(q0)
    out = {"phi": torch.empty(n, dtype=torch.float64, device="cuda"),
           "field": torch.empty((n, 3), dtype=torch.float64, device="cuda"),
           "energy": torch.empty(6, dtype=torch.float64, device="cuda")}
    plan.graph_capture_step(pos_t, q_t, **out)
    rng = np.random.default_rng(3)
    for k in range(3):
        pos = pos0 + 1e-4 * rng.standard_normal(pos0.shape)
        q = q0 * (1.0 + 0.1 * k)
        pos_t.copy_(dev(pos))
        q_t.copy_(dev(q))
        for t in out.values():
            t.zero_()
        torch.cuda.synchronize()
        plan.graph_launch()
        plan.sync()
        got = host(out)
        ref_plan.build_tree(dev(pos), dev(q), offs)
        ref_plan.upward()
        ref = host(ref_plan.evaluate())
        for name in ("phi", "field", "energy"):
            assert np.array_equal(got[name], ref[name]), (k, name)
        other_work()


def test_step_graph_needs_a_kept_topology():
    pos, q = W.uniform_cube(2000, 86)
    plan = fmm.Plan(p=4, ncrit=32, theta=(1, 2), precision="mixed", device=0)
    plan.build_tree(dev(pos), dev(q))
    phi = torch.empty(2000, dtype=torch.float64, device="cuda")
    with pytest.raises(fmm.FMMError) as ei:
        plan.graph_capture_step(dev(pos), dev(q), phi=phi)
    assert ei.value.status == -2


def test_cost_reuse_orders_by_measured_costs():
    """The P2P tasks of a step on a kept topology are ordered by the
    durations the previous evaluation measured: every task still runs once
    (task trace) and the results are bitwise those of a plan without it."""
    n = 200000
    pos, q = W.uniform_cube(n, 87)
    kw = dict(p=P, ncrit=NCRIT, theta=(1, 2), precision="mixed", device=0, incremental=True, deterministic=True)
    plans = (fmm.Plan(cost_reuse=True, **kw), fmm.Plan(cost_reuse=True, trace=True, **kw), fmm.Plan(**kw))
    res = []
    for pl in plans:
        pl.build_tree(dev(pos), dev(q))
        pl.upward()
        host(pl.evaluate())
        for _ in range(2):
            pl.build_tree(dev(pos), dev(q))       # kept: with cost reuse, reordered by the measured costs
            pl.upward()
            res.append(host(pl.evaluate()))
        assert pl.build_info() == {"full": 1, "kept": 2}
    for r in res[1:]:
        for name in ("phi", "field", "force", "energy"):
            assert np.array_equal(r[name], res[0][name]), name
    rec = plans[1].trace()
    _, _, cells = plans[1].copy_tree()
    leaves = np.nonzero((cells[:, 6] < 0) & (cells[:, 5] > 0))[0]
    p2p = rec[rec["kind"] == 1]
    assert np.array_equal(np.sort(p2p["task"]), leaves)
    assert np.array_equal(np.sort(rec[rec["kind"] == 0]["task"]), np.arange(len(rec) - len(p2p)))


def test_step_graph_with_cost_reuse():
    """The captured step reorders the P2P tasks at every replay by the
    durations the previous replay measured; results stay bitwise those of
    an eager step without cost reuse."""
    pos0, q, T, v, side = setup(89)
    kw = dict(p=P, ncrit=NCRIT, theta=(1, 2), precision="mixed", device=0, incremental=True, deterministic=True)
    plan, ref_plan = fmm.Plan(cost_reuse=True, **kw), fmm.Plan(**kw)
    plan.build_tree(dev(pos0), dev(q))
    ref_plan.build_tree(dev(pos0), dev(q))
    plan.upward()
    plan.evaluate()                               # first measurement
    pos_t, q_t = dev(pos0 + 0.02 * v), dev(q)
    phi = torch.empty(N, dtype=torch.float64, device="cuda")
    field = torch.empty((N, 3), dtype=torch.float64, device="cuda")
    plan.graph_capture_step(pos_t, q_t, phi=phi, field=field)
    for k in (2, 3, 4):
        pos = pos0 + 0.02 * k * v
        pos_t.copy_(dev(pos))
        torch.cuda.synchronize()
        plan.graph_launch()
        plan.sync()
        got = (phi.cpu().numpy(), field.cpu().numpy())
        ref_plan.build_tree(dev(pos), dev(q))
        ref_plan.upward()
        ref = host(ref_plan.evaluate())
        assert np.array_equal(got[0], ref["phi"]) and np.array_equal(got[1], ref["field"]), k
        other_work()
