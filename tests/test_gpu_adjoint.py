"""GPU checks of the adjoint (fmm_backward) through the C ABI.

The FMM applies a fixed (for a given tree and lists) non-symmetric matrix A:
E = 1/2 q^T A q per instance.  Pins that do not rely on the adjoint code:
  * dot-product identity <w, A q> = <A^T w, q>, with A q from fmm_evaluate
    and A^T w = 2 grad_q(w) - phi(w) from fmm_backward (g = 1);
  * charge finite differences, exact because E is quadratic in q;
  * position finite differences with the topology frozen
    (FMM_FLAG_KEEP_TOPOLOGY), plain central and Richardson-extrapolated;
  * the direct-sum gradient: dE/dq = phi_direct, dE/dx = -F_direct up to the
    FMM's truncation error;
  * batched instances = single solves scaled by their upstream weights.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_1203_0889_amd import fmm, workloads as W
from paper_1203_0889_amd.autograd import FMMEnergy

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b)))


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def forward(plan, pos, q, offsets=None):
    plan.build_tree(dev(pos), dev(q), offsets)
    plan.upward()
    out = plan.evaluate()
    torch.cuda.synchronize()
    return {k: v.cpu().numpy() for k, v in out.items()}


def backward(plan, g):
    gp, gq = plan.backward(dev(np.atleast_1d(g)))
    torch.cuda.synchronize()
    return gp.cpu().numpy(), gq.cpu().numpy()


DOT_CASES = [
    ("uniform4k_p4_fp64", "uniform", 4096, 1, 4, 64, (1, 2), "fp64", 1e-12),
    ("plummer12k_p6_fp64", "plummer", 12000, 4, 6, 32, (1, 2), "fp64", 1e-12),
    ("uniform20k_p8_mixed", "uniform", 20000, 2, 8, 64, (1, 2), "mixed", 2e-5),
    ("plummer15k_p8_mixed", "plummer", 15000, 4, 8, 64, (1, 2), "mixed", 2e-5),
]


@pytest.mark.parametrize("case", DOT_CASES, ids=[c[0] for c in DOT_CASES])
def test_dot_product_identity(case):
    name, dist, n, seed, p, ncrit, theta, prec, tol = case
    say("case", name)
    pos, q = W.uniform_cube(n, seed) if dist == "uniform" else W.plummer(n, seed)
    w = np.random.default_rng(seed + 7).uniform(-1.0, 1.0, n)
    pa = fmm.Plan(p=p, ncrit=ncrit, theta=theta, precision=prec, device=0)
    phi_q = forward(pa, pos, q)["phi"]
    pb = fmm.Plan(p=p, ncrit=ncrit, theta=theta, precision=prec, device=0)
    phi_w = forward(pb, pos, w)["phi"]
    _, gq_w = backward(pb, 1.0)
    at_w = 2.0 * gq_w - phi_w
    lhs, rhs = float(np.dot(w, phi_q)), float(np.dot(at_w, q))
    scale = float(np.linalg.norm(w) * np.linalg.norm(phi_q))
    say(name, "<w,Aq>", lhs, "<A^T w,q>", rhs, "rel", abs(lhs - rhs) / scale)
    assert abs(lhs - rhs) <= tol * scale
    # A is not symmetric (non-mutual M2L), but close to it: A^T w ~ A w
    say(name, "|A^T w - A w| / |A w|", rel(at_w, phi_w))
    assert rel(at_w, phi_w) < 1e-2


# exact for FP64 (E is quadratic in q); the mixed path's rounding is not
# smooth in q, so its differences carry that noise
@pytest.mark.parametrize("prec,tol", [("fp64", 1e-9), ("mixed", 1e-3)])
def test_charge_finite_differences(prec, tol):
    n, p = 4096, 6
    pos, q = W.uniform_cube(n, 11)
    plan = fmm.Plan(p=p, ncrit=40, theta=(1, 2), precision=prec, device=0)
    forward(plan, pos, q)
    _, gq = backward(plan, 1.0)
    idx = np.random.default_rng(3).choice(n, 8, replace=False)
    h = 1.0
    fd = []
    for i in idx:
        e = []
        for sgn in (1.0, -1.0):
            qq = q.copy()
            qq[i] += sgn * h
            e.append(forward(fmm.Plan(p=p, ncrit=40, theta=(1, 2), precision=prec, device=0), pos, qq)["energy"][0])
        fd.append((e[0] - e[1]) / (2 * h))
    fd = np.array(fd)
    say(prec, "charge FD rel", rel(gq[idx], fd))
    assert rel(gq[idx], fd) < tol


def isolated(pos, count, min_dist, seed):
    """Indices of particles whose nearest neighbour is farther than min_dist."""
    from scipy.spatial import cKDTree
    d, _ = cKDTree(pos).query(pos, k=2)
    good = np.nonzero(d[:, 1] > min_dist)[0]
    return np.random.default_rng(seed).choice(good, count, replace=False)


def test_position_finite_differences_fp64():
    n, p = 3000, 6
    pos, q = W.uniform_cube(n, 21)
    plan = fmm.Plan(p=p, ncrit=32, theta=(1, 2), precision="fp64", device=0, keep_topology=True)
    forward(plan, pos, q)
    gp, _ = backward(plan, 1.0)
    h = 1e-5
    idx = isolated(pos, 12, 100 * h, 5)

    def energy(x):
        return forward(plan, x, q)["energy"][0]

    def central(i, d, hh):
        xp, xm = pos.copy(), pos.copy()
        xp[i, d] += hh
        xm[i, d] -= hh
        return (energy(xp) - energy(xm)) / (2 * hh)

    plain, rich, ana = [], [], []
    for i in idx:
        for d in range(3):
            d1, d2 = central(i, d, h), central(i, d, h / 2)
            plain.append(d1)
            rich.append((4 * d2 - d1) / 3)
            ana.append(gp[i, d])
    plain, rich, ana = map(np.array, (plain, rich, ana))
    say("position FD: plain", rel(ana, plain), "Richardson", rel(ana, rich))
    assert rel(ana, plain) < 1e-4
    assert rel(ana, rich) < 1e-6


def test_gradient_matches_direct_mixed():
    n = 30000
    pos, q = W.plummer(n, 4)
    plan = fmm.Plan(p=8, ncrit=64, theta=(1, 2), precision="mixed", device=0)
    out = forward(plan, pos, q)
    gp, gq = backward(plan, 1.0)
    tg = W.error_sample(n, 17, 2048)
    phi_d, fld_d = oracle.direct(pos, q, tg)
    f_d = q[tg, None] * fld_d
    e_q, e_x = rel(gq[tg], phi_d), rel(gp[tg], -f_d)
    say("gradient vs direct: dE/dq", e_q, "dE/dx", e_x)
    assert e_q < 1e-4 and e_x < 1e-4
    # and against the forward's own outputs (A nearly symmetric)
    assert rel(gq, out["phi"]) < 1e-4
    assert rel(gp, -out["force"]) < 1e-4


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-12), ("mixed", 1e-5)])
def test_batched_backward_equals_single(prec, tol):
    sizes = [3000, 0, 5000, 1200]
    parts = [W.uniform_cube(sizes[0], 31), W.uniform_cube(0, 32), W.plummer(sizes[2], 33), W.uniform_cube(sizes[3], 34)]
    pos = np.concatenate([a for a, _ in parts])
    q = np.concatenate([b for _, b in parts])
    offs = np.concatenate([[0], np.cumsum(sizes)]).tolist()
    g = np.array([1.0, 3.0, 0.5, -2.0])
    plan = fmm.Plan(p=6, ncrit=48, theta=(1, 2), precision=prec, device=0)
    forward(plan, pos, q, offs)
    gp, gq = backward(plan, g)
    for k in range(len(sizes)):
        a, b = offs[k], offs[k + 1]
        if a == b:
            continue
        single = fmm.Plan(p=6, ncrit=48, theta=(1, 2), precision=prec, device=0)
        forward(single, pos[a:b], q[a:b])
        sp, sq = backward(single, g[k])
        say(prec, "instance", k, rel(gq[a:b], sq), rel(gp[a:b], sp))
        assert rel(gq[a:b], sq) < tol and rel(gp[a:b], sp) < tol


def test_autograd_function():
    n = 6000
    pos, q = W.uniform_cube(n, 41)
    plan = fmm.Plan(p=6, ncrit=64, theta=(1, 2), precision="fp64", device=0)
    x = dev(pos).requires_grad_(True)
    c = dev(q).requires_grad_(True)
    E = FMMEnergy.apply(x, c, plan)
    (3.0 * E.sum()).backward()
    torch.cuda.synchronize()
    ref = fmm.Plan(p=6, ncrit=64, theta=(1, 2), precision="fp64", device=0)
    out = forward(ref, pos, q)
    assert abs(E.item() - out["energy"][0]) <= 1e-12 * abs(out["energy"][0])
    rp, rq = backward(ref, 3.0)
    assert rel(x.grad.cpu().numpy(), rp) < 1e-12
    assert rel(c.grad.cpu().numpy(), rq) < 1e-12


def test_backward_state_errors():
    plan = fmm.Plan(p=4, ncrit=64, theta=(1, 2), precision="fp64", device=0)
    pos, q = W.uniform_cube(500, 1)
    plan.build_tree(dev(pos), dev(q))
    plan.upward()
    with pytest.raises(fmm.FMMError) as ei:
        plan.backward(dev(np.ones(1)))
    assert ei.value.status == -2  # FMM_ERR_STATE before fmm_evaluate
