"""HIP graph of the numeric part of a solve (fmm_graph_capture / launch).

Each graph is replayed several times with unrelated eager GPU work and
synchronisations between the replays, and every replay is checked against
the eager result of the same plan.  FP64 atomics make the mixed path's
summation order vary from run to run, so values are compared to 1e-12
relative, not bitwise.
"""
import numpy as np
import pytest
import torch

from paper_1203_0889_amd import fmm, workloads as W

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)


def rel(a, b):
    a, b = np.asarray(a), np.asarray(b)
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def eager(plan):
    plan.upward()
    out = plan.evaluate()
    torch.cuda.synchronize()
    return {k: v.cpu().numpy() for k, v in out.items()}


def other_work():
    """Unrelated eager GPU work between replays."""
    pos, q = W.uniform_cube(2000, 99)
    plan = fmm.Plan(p=4, ncrit=32, theta=(1, 2), precision="mixed", device=0)
    plan.build_tree(dev(pos), dev(q))
    eager(plan)
    x = torch.randn(1 << 20, device="cuda")
    (x * 2.0).sum().item()


@pytest.mark.parametrize("prec", ["mixed", "fp64"])
def test_graph_replays_match_eager_batched(prec):
    sizes = [4000, 0, 9000, 2500]
    parts = [W.uniform_cube(4000, 1), W.uniform_cube(0, 2), W.plummer(9000, 3), W.uniform_cube(2500, 4)]
    pos = np.concatenate([a for a, _ in parts])
    q = np.concatenate([b for _, b in parts])
    offs = np.concatenate([[0], np.cumsum(sizes)]).tolist()
    n = len(q)
    plan = fmm.Plan(p=6, ncrit=48, theta=(1, 2), precision=prec, device=0)
    plan.build_tree(dev(pos), dev(q), offs)
    ref = eager(plan)
    phi = torch.empty(n, dtype=torch.float64, device="cuda")
    field = torch.empty((n, 3), dtype=torch.float64, device="cuda")
    energy = torch.empty(len(sizes), dtype=torch.float64, device="cuda")
    plan.graph_capture(phi=phi, field=field, energy=energy)
    for r in range(3):
        phi.zero_()
        field.zero_()
        energy.zero_()
        torch.cuda.synchronize()
        plan.graph_launch()
        torch.cuda.synchronize()
        e = (rel(phi.cpu().numpy(), ref["phi"]), rel(field.cpu().numpy(), ref["field"]),
             rel(energy.cpu().numpy(), ref["energy"]))
        say(prec, "replay", r, e)
        assert max(e) < 1e-12
        other_work()


def test_graph_follows_frozen_topology_refresh():
    n = 20000
    pos, q = W.plummer(n, 7)
    q2 = np.random.default_rng(8).uniform(-1.0, 1.0, n)
    plan = fmm.Plan(p=8, ncrit=64, theta=(1, 2), precision="mixed", device=0, keep_topology=True)
    plan.build_tree(dev(pos), dev(q))
    eager(plan)
    phi = torch.empty(n, dtype=torch.float64, device="cuda")
    field = torch.empty((n, 3), dtype=torch.float64, device="cuda")
    plan.graph_capture(phi=phi, field=field)
    for r, charges in enumerate((q2, q, q2)):
        plan.build_tree(dev(pos), dev(charges))       # refresh: same tree, new charges
        plan.graph_launch()
        torch.cuda.synchronize()
        got = (phi.cpu().numpy(), field.cpu().numpy())
        ref = eager(plan)                             # same plan, eager
        e = (rel(got[0], ref["phi"]), rel(got[1], ref["field"]))
        say("refresh replay", r, e)
        assert max(e) < 1e-12
        other_work()


def test_graph_with_backward_fp64():
    n = 8000
    pos, q = W.uniform_cube(n, 12)
    plan = fmm.Plan(p=6, ncrit=48, theta=(1, 2), precision="fp64", device=0)
    plan.build_tree(dev(pos), dev(q))
    eager(plan)
    g = dev(np.array([1.5]))
    rp, rq = plan.backward(g)
    torch.cuda.synchronize()
    rp, rq = rp.cpu().numpy(), rq.cpu().numpy()
    energy = torch.empty(1, dtype=torch.float64, device="cuda")
    gp = torch.empty((n, 3), dtype=torch.float64, device="cuda")
    gq = torch.empty(n, dtype=torch.float64, device="cuda")
    plan.graph_capture(energy=energy, grad_energy=g, grad_pos=gp, grad_q=gq)
    for r in range(3):
        gp.zero_()
        gq.zero_()
        torch.cuda.synchronize()
        plan.graph_launch()
        torch.cuda.synchronize()
        e = (rel(gp.cpu().numpy(), rp), rel(gq.cpu().numpy(), rq))
        say("backward replay", r, e)
        assert max(e) < 1e-12
        other_work()


def test_graph_errors():
    plan = fmm.Plan(p=4, ncrit=64, theta=(1, 2), precision="mixed", device=0)
    with pytest.raises(fmm.FMMError) as ei:
        plan.graph_launch()
    assert ei.value.status == -2
    with pytest.raises(fmm.FMMError) as ei:
        plan.graph_capture()
    assert ei.value.status == -2
