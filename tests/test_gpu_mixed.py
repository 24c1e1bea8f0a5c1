"""GPU parity of the mixed-precision path (FP32 P2P on the vector units, M2L
on the bf16 matrix cores with split operands and FP32 accumulation, FP64
elsewhere and in the final per-particle / per-cell accumulation) against the
FP64 CPU oracle, and of batched instances against single solves."""
import numpy as np
import pytest
import torch

import oracle
from paper_1203_0889_amd import fmm, workloads as W
from parity import check_fp64, check_mixed, leaf_ids

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b)))


def gpu_run(pos, q, p, ncrit, theta, precision, offsets=None):
    plan = fmm.Plan(p=p, ncrit=ncrit, theta=theta, precision=precision, device=0)
    plan.build_tree(torch.from_numpy(np.ascontiguousarray(pos)).cuda(),
                    torch.from_numpy(np.ascontiguousarray(q)).cuda(), offsets)
    plan.upward()
    out = plan.evaluate()
    torch.cuda.synchronize()
    return plan, {k: v.cpu().numpy() for k, v in out.items()}


# FP32 rounding of the near field and of M2L bounds the agreement with the
# FP64 oracle FMM (same tree, lists and truncation): 1e-5 relative L2, and
# no single particle off by more than MAX_MIXED of the rms.  The last case
# has the shape of the Plummer-sphere configuration at p = 10 (equal
# charges 1/N, 32 particles per leaf, theta = 2/5) at a size the oracle
# finishes in seconds.
MIXED_CASES = [
    ("uniform4k_p4", "uniform", 4096, 1, 4, 64, (1, 2)),
    ("uniform70k_p8", "uniform", 70000, 2, 8, 64, (1, 2)),
    ("uniform33k_p6_ragged", "uniform", 33333, 8, 6, 50, (1, 2)),
    ("plummer30k_p8", "plummer", 30000, 4, 8, 64, (1, 2)),
    ("plummer20k_p10_theta04", "plummer", 20000, 3, 10, 32, (2, 5)),
    ("plummer12k_p10_theta04_equal_q", "plummer_equal", 12000, 3, 10, 32, (2, 5)),
]


def make_case(dist, n, seed):
    if dist == "uniform":
        return W.uniform_cube(n, seed)
    return W.plummer(n, seed, equal_charges=dist == "plummer_equal")


@pytest.mark.parametrize("case", MIXED_CASES, ids=[c[0] for c in MIXED_CASES])
def test_mixed_matches_oracle_fmm(case):
    name, dist, n, seed, p, ncrit, theta = case
    say("case", name)
    pos, q = make_case(dist, n, seed)
    plan, out = gpu_run(pos, q, p, ncrit, theta, "mixed")
    phi_ref, fld_ref, T = oracle.fmm(pos, q, p, ncrit, *theta)
    e_phi, e_fld = rel(out["phi"], phi_ref), rel(out["field"], fld_ref)
    say(name, "mixed vs oracle fmm", e_phi, e_fld)
    assert e_phi < 1e-5 and e_fld < 1e-5
    # tree and lists are those of the FP64 path: bit-exact vs the oracle
    keys, perm, cells = plan.copy_tree()
    assert np.array_equal(cells[:, :9], T.cells)
    check_mixed(out, phi_ref, fld_ref, leaf_ids(perm, cells), say, name)
    tg = W.error_sample(n, 13, 2048)
    pd, fd = oracle.direct(pos, q, tg)
    e_phi_d, e_fld_d = rel(out["phi"][tg], pd), rel(out["field"][tg], fd)
    say(name, "mixed vs direct", e_phi_d, e_fld_d)
    tol = {4: (1e-3, 1e-2), 6: (1e-4, 1e-3), 8: (1e-4, 1e-4), 10: (1e-4, 1e-4)}[p]
    assert e_phi_d < tol[0] and e_fld_d < tol[1]
    assert out["energy"][0] == pytest.approx(0.5 * np.dot(q, out["phi"]), rel=1e-12)


def test_mixed_root_leaf_and_single_particle():
    pos, q = W.uniform_cube(40, 5)
    plan, out = gpu_run(pos, q, 8, 64, (1, 2), "mixed")
    pd, fd = oracle.direct(pos, q)
    assert rel(out["phi"], pd) < 1e-5 and rel(out["field"], fd) < 1e-5
    plan, out = gpu_run(np.array([[0.5, 0.5, 0.5]]), np.array([1.0]), 8, 64, (1, 2), "mixed")
    assert out["phi"][0] == 0.0 and np.all(out["field"] == 0.0)


# The orders at both ends of the mixed path: p = 0..2 use one 32-row MFMA
# tile of the class operator, p = 11 and 12 five and six (the largest queue
# kernel); same FP32 bound against the FP64 oracle FMM as above.
@pytest.mark.parametrize("p", [0, 1, 2, 11, 12])
def test_mixed_orders_at_the_ends(p):
    say("mixed order", p)
    pos, q = W.uniform_cube(5000, 30 + p)
    plan, out = gpu_run(pos, q, p, 48, (1, 2), "mixed")
    phi_ref, fld_ref, _ = oracle.fmm(pos, q, p, 48, 1, 2)
    e_phi, e_fld = rel(out["phi"], phi_ref), rel(out["field"], fld_ref)
    say("p", p, "vs oracle FMM: phi", e_phi, "field", e_fld)
    assert e_phi < 1e-5 and e_fld < 1e-5
    _, perm, cells = plan.copy_tree()
    check_mixed(out, phi_ref, fld_ref, leaf_ids(perm, cells), say, "p=%d" % p)
    # the FP64 path's class-table M2L at the same orders
    _, out = gpu_run(pos, q, p, 48, (1, 2), "fp64")
    e = (rel(out["phi"], phi_ref), rel(out["field"], fld_ref))
    say("p", p, "fp64 vs oracle FMM", e)
    assert max(e) < 1e-11
    check_fp64(out, phi_ref, fld_ref, leaf_ids(perm, cells), say, "p=%d fp64" % p)


# The odd orders the other cases skip, on an adaptive tree (pairs outside
# the class table go through the per-pair FP64 kernel): every order-templated
# kernel of both paths (the work queue, the FP64 class-table M2L, the
# per-pair M2L) at p = 3, 5, 7, 9 against the oracle FMM.
@pytest.mark.parametrize("p", [3, 5, 7, 9])
def test_odd_orders_both_paths(p):
    say("odd order", p)
    pos, q = W.plummer(4000, 71)
    phi_ref, fld_ref, _ = oracle.fmm(pos, q, p, 16, 1, 2)
    for precision, tol in (("fp64", 1e-11), ("mixed", 1e-5)):
        plan, out = gpu_run(pos, q, p, 16, (1, 2), precision)
        e = (rel(out["phi"], phi_ref), rel(out["field"], fld_ref))
        say("p", p, precision, "vs oracle FMM", e, "pairs outside the class table", plan.queue_info()["nextra"])
        assert max(e) < tol
        _, perm, cells = plan.copy_tree()
        check = check_fp64 if precision == "fp64" else check_mixed
        check(out, phi_ref, fld_ref, leaf_ids(perm, cells), say, "p=%d %s" % (p, precision))
    assert plan.queue_info()["nextra"] > 0


def test_mixed_coincident_cluster_reaches_max_level():
    # 24 coincident particles (no leaf can split them below ncrit = 8, so the
    # tree goes down to level 21) inside a uniform background: the coincident
    # pairs contribute nothing, and the deep levels give the M2L classes of
    # large level differences
    bg, qb = W.uniform_cube(3000, 41)
    pos = np.concatenate([bg, np.tile(np.array([[0.3, 0.6, 0.45]]), (24, 1))])
    q = np.concatenate([qb, np.linspace(-1.0, 1.0, 24)])
    plan, out = gpu_run(pos, q, 6, 8, (1, 2), "mixed")
    T = oracle.Tree(pos, 8)
    assert int(T.cells[:, 0].max()) == 21
    phi_ref, fld_ref, _ = oracle.fmm(pos, q, 6, 8, 1, 2)
    assert np.all(np.isfinite(out["phi"])) and np.all(np.isfinite(out["field"]))
    e_phi, e_fld = rel(out["phi"], phi_ref), rel(out["field"], fld_ref)
    say("coincident cluster vs oracle FMM: phi", e_phi, "field", e_fld)
    assert e_phi < 1e-5 and e_fld < 1e-5
    _, perm, cells = plan.copy_tree()
    check_mixed(out, phi_ref, fld_ref, leaf_ids(perm, cells), say, "coincident cluster")


def test_mixed_repeated_builds_reuse_operator_cache():
    plan = fmm.Plan(p=6, ncrit=32, precision="mixed", device=0)
    for n, seed, dist in ((8000, 1, "uniform"), (12000, 2, "plummer"), (5000, 3, "uniform")):
        say("rebuild", n, dist)
        pos, q = W.uniform_cube(n, seed) if dist == "uniform" else W.plummer(n, seed)
        plan.build_tree(torch.from_numpy(pos).cuda(), torch.from_numpy(q).cuda())
        plan.upward()
        out = plan.evaluate()
        phi_ref, fld_ref, _ = oracle.fmm(pos, q, 6, 32, 1, 2)
        o = {k: v.cpu().numpy() for k, v in out.items()}
        assert rel(o["phi"], phi_ref) < 1e-5
        assert rel(o["field"], fld_ref) < 1e-5
        _, perm, cells = plan.copy_tree()
        check_mixed(o, phi_ref, fld_ref, leaf_ids(perm, cells), say, "rebuild %d" % n)


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-12), ("mixed", 1e-5)])
def test_batched_instances_equal_single_solves(precision, tol):
    # uneven sizes, an empty instance, uniform and Plummer mixed
    parts = [W.uniform_cube(3000, 1), W.plummer(5000, 2), (np.zeros((0, 3)), np.zeros(0)),
             W.uniform_cube(1500, 3), W.plummer(800, 4)]
    pos = np.concatenate([p for p, _ in parts])
    q = np.concatenate([c for _, c in parts])
    offsets = np.cumsum([0] + [len(c) for _, c in parts])
    plan, out = gpu_run(pos, q, 6, 32, (1, 2), precision, list(offsets))
    _, _, cells = plan.copy_tree()
    for k, (pk, qk) in enumerate(parts):
        a, b = offsets[k], offsets[k + 1]
        if b == a:
            assert out["energy"][k] == 0.0
            continue
        say("instance", k, b - a)
        _, single = gpu_run(pk, qk, 6, 32, (1, 2), precision)
        assert rel(out["phi"][a:b], single["phi"]) < tol and rel(out["field"][a:b], single["field"]) < tol
        phi_ref, fld_ref, T = oracle.fmm(pk, qk, 6, 32, 1, 2)
        assert rel(out["phi"][a:b], phi_ref) < max(tol, 1e-11)
        ids = leaf_ids(T.perm, T.cells)
        mine = {"phi": out["phi"][a:b], "field": out["field"][a:b]}
        (check_fp64 if precision == "fp64" else check_mixed)(mine, phi_ref, fld_ref, ids, say, "instance %d" % k)
        mine = cells[cells[:, 9] == k]
        assert np.array_equal(mine[:, :4], T.cells[:, :4])   # same cells (level, coords) per instance
        assert out["energy"][k] == pytest.approx(0.5 * np.dot(qk, out["phi"][a:b]), rel=1e-12)


@pytest.mark.parametrize("shape", [(1, 2), (2, 0)], ids=["side_kernel_deferred_join", "queue_only"])
def test_output_subsets_agree(shape):
    """The outputs do not depend on which of them are asked for: the
    evaluation writes them from L2P (queue without a P2P side kernel), from
    the energy pass or from a separate pass after the join (with one).
    Same plan and tree, so every result must be bit-identical; the force is
    q E and the energy half the sum of q phi."""
    say("output subsets", shape)
    pos, q = W.uniform_cube(20000, 5)
    plan = fmm.Plan(p=6, ncrit=32, theta=(1, 2), precision="mixed", device=0)
    plan.build_tree(torch.from_numpy(pos).cuda(), torch.from_numpy(q).cuda())
    plan.upward()
    plan.set_tuning(grid_per_cu=shape[0], p2p_per_cu=shape[1])
    full = {k: v.cpu().numpy() for k, v in plan.evaluate().items()}
    no_energy = {k: v.cpu().numpy() for k, v in plan.evaluate(energy=False).items() if v is not None}
    only_energy = plan.evaluate(phi=False, field=False, force=False)["energy"].cpu().numpy()
    only_phi = plan.evaluate(field=False, force=False, energy=False)["phi"].cpu().numpy()
    torch.cuda.synchronize()
    for k in ("phi", "field", "force"):
        assert np.array_equal(full[k], no_energy[k]), k
    assert np.array_equal(full["phi"], only_phi)
    assert np.array_equal(full["energy"], only_energy)
    qn = q.astype(np.float64)
    assert np.allclose(full["force"], qn[:, None] * full["field"], rtol=1e-15, atol=0)
    assert abs(full["energy"][0] - 0.5 * np.dot(qn, full["phi"])) <= 1e-10 * abs(full["energy"][0])


def table_targets(T):
    """Cells owning at least one M2L pair of the class table (level
    difference at most 2, integer centre offset in units of the smaller cell
    at most 24 per axis), from the oracle's lists: the targets of the
    batched M2L; and the number of pairs outside the table."""
    c, m = T.cells, T.m2l
    A, B = m[:, 0], m[:, 1]
    la, lb = c[A, 0], c[B, 0]
    SA, SB = np.left_shift(1, 21 - la), np.left_shift(1, 21 - lb)
    sh = 21 - np.maximum(la, lb)
    ok = np.abs(la - lb) <= 2
    for d in range(3):
        rho = np.right_shift((2 * c[A, 1 + d] + 1) * SA - (2 * c[B, 1 + d] + 1) * SB, sh)
        ok &= np.abs(rho) <= 24
    has = np.zeros(T.ncell, dtype=bool)
    has[A[ok]] = True
    return int(has.sum()), int((~ok).sum())


# Regression: the count of batched M2L targets came from a sampled search
# of the sorted target keys that missed the first cell without table pairs
# when it lay after the last sampled key (an overcount of up to ncell / 256,
# whose extra "targets" had cell index -1 and made the group kernels read
# outside the lists; a GPU memory fault when the bytes before the list held
# a negative value).  These inputs were all overcounted.
COUNT_CASES = [("uniform200k_s71", "uniform", 200000, 71), ("plummer150k_s62", "plummer", 150000, 62),
               ("uniform200k_s51", "uniform", 200000, 51)]


@pytest.mark.parametrize("case", COUNT_CASES, ids=[c[0] for c in COUNT_CASES])
def test_m2l_target_count(case):
    name, dist, n, seed = case
    pos, q = make_case(dist, n, seed)
    T = oracle.Tree(pos, 64)
    T.lists(1, 2)
    plan = fmm.Plan(p=8, ncrit=64, theta=(1, 2), precision="mixed", device=0)
    plan.build_tree(torch.from_numpy(pos).cuda(), torch.from_numpy(q).cuda())
    info = plan.queue_info()
    say(name, "ncell", T.ncell, info)
    ntarget, nextra = table_targets(T)
    assert info["ntarget"] == ntarget and info["nextra"] == nextra
    assert info["ngroup"] == (info["ntarget"] + 255) // 256
