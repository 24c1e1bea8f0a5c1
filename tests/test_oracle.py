"""Pins of the FP64 CPU oracle against what mathematics fixes independently of
it: closed forms, invariants, exact identities, bounds, brute force on tiny
inputs and hand-derived interaction lists.  CPU only."""
import math

import numpy as np
import pytest

import oracle
from paper_1203_0889_amd import workloads as W

LEVELS = 21


def rel(a, b):
    return np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b))


# --------------------------------------------------------------------------
# Direct sum: the plain definition (problem of Sec. 2.1)
# --------------------------------------------------------------------------

def test_direct_two_charges_closed_form():
    pos = np.array([[0.1, -0.2, 0.3], [0.1 + 3.0, -0.2 + 4.0, 0.3]])  # r = 5
    q = np.array([2.0, -0.5])
    phi, E = oracle.direct(pos, q)
    assert phi[0] == pytest.approx(-0.5 / 5.0, rel=1e-15)
    assert phi[1] == pytest.approx(2.0 / 5.0, rel=1e-15)
    # E_0 = q_1 (x_0 - x_1) / r^3
    assert np.allclose(E[0], -0.5 * np.array([-3.0, -4.0, 0.0]) / 125.0, rtol=1e-15, atol=0)
    assert np.allclose(E[1], 2.0 * np.array([3.0, 4.0, 0.0]) / 125.0, rtol=1e-15, atol=0)


def test_direct_cube_corners_closed_form():
    # 8 equal charges on the corners of a cube of side a, probe of zero charge at the centre
    a, q0 = 0.7, 1.3
    corners = np.array([[i, j, k] for i in (0, 1) for j in (0, 1) for k in (0, 1)], float) * a
    pos = np.vstack([corners, [[a / 2, a / 2, a / 2]]])
    q = np.r_[np.full(8, q0), 0.0]
    phi, E = oracle.direct(pos, q)
    assert phi[8] == pytest.approx(8 * q0 / (math.sqrt(3) * a / 2), rel=1e-14)
    assert np.abs(E[8]).max() < 1e-13
    # a corner sees 3 edges (a), 3 face diagonals (a sqrt2), 1 body diagonal (a sqrt3)
    assert phi[0] == pytest.approx(q0 * (3 / a + 3 / (a * math.sqrt(2)) + 1 / (a * math.sqrt(3))), rel=1e-14)
    # field at corner 0 points away from the cube along (-1,-1,-1) by symmetry
    Ecomp = q0 * (1 / a ** 2 + 2 * (1 / math.sqrt(2)) / (2 * a * a) + (1 / math.sqrt(3)) / (3 * a * a))
    assert np.allclose(E[0], -Ecomp * np.ones(3), rtol=1e-13)


def test_direct_invariants():
    pos, q = W.uniform_cube(300, 11)
    phi, E = oracle.direct(pos, q)
    # Newton's third law: total force vanishes
    F = q[:, None] * E
    assert np.abs(F.sum(0)).max() < 1e-12 * np.abs(F).sum()
    # translation invariance
    phi2, E2 = oracle.direct(pos + np.array([10.0, -3.0, 7.5]), q)
    assert rel(phi2, phi) < 1e-12 and rel(E2, E) < 1e-10
    # scaling phi(l x) = phi / l, E(l x) = E / l^2
    phi3, E3 = oracle.direct(2.5 * pos, q)
    assert rel(phi3, phi / 2.5) < 1e-14 and rel(E3, E / 6.25) < 1e-14
    # linearity in q
    q2 = W.uniform_cube(300, 12)[1]
    pa, Ea = oracle.direct(pos, q2)
    pb, Eb = oracle.direct(pos, 2 * q - 3 * q2)
    assert rel(pb, 2 * phi - 3 * pa) < 1e-13 and rel(Eb, 2 * E - 3 * Ea) < 1e-13
    # permutation equivariance
    perm = np.random.default_rng(0).permutation(300)
    pp, Ep = oracle.direct(pos[perm], q[perm])
    assert rel(pp, phi[perm]) < 1e-13 and rel(Ep, E[perm]) < 1e-12
    # target subset = same rows
    tg = np.array([5, 17, 299, 0])
    pt, Et = oracle.direct(pos, q, tg)
    assert np.array_equal(pt, phi[tg]) and np.array_equal(Et, E[tg])


def test_direct_skips_coincident_pairs():
    pos = np.array([[0.0, 0, 0], [0.0, 0, 0], [1.0, 0, 0]])
    q = np.array([1.0, 2.0, 4.0])
    phi, E = oracle.direct(pos, q)
    assert phi[0] == 4.0 and phi[1] == 4.0 and phi[2] == 3.0
    assert np.all(np.isfinite(E))


# --------------------------------------------------------------------------
# Keys, sort, tree (Sec. 2.1, 2.2)
# --------------------------------------------------------------------------

def _grid_point(ix, iy, iz):
    # point inside grid cell (ix, iy, iz) of the unit box (side 1, scale 2^21)
    return np.array([(ix + 0.5), (iy + 0.5), (iz + 0.5)]) / 2.0 ** LEVELS


def test_keys_worked_examples():
    box = np.array([0.0, 0.0, 0.0, 1.0])
    scale = 2.0 ** LEVELS
    pts = np.array([_grid_point(0, 0, 0), _grid_point(1, 0, 0), _grid_point(0, 1, 0), _grid_point(0, 0, 1),
                    _grid_point(5, 3, 6), _grid_point(2 ** 21 - 1, 2 ** 21 - 1, 2 ** 21 - 1),
                    [1.0, 1.0, 1.0]])
    keys = oracle.morton_keys(pts, box, scale)
    # ix=5=101b, iy=3=011b, iz=6=110b -> digits (z y x) per bit: 011, 110, 101 -> 3 + 6*8 + 5*64
    assert list(keys[:5]) == [0, 1, 2, 4, 371]
    assert keys[5] == 2 ** 63 - 1
    assert keys[6] == 2 ** 63 - 1   # the max corner clamps to the last cell


def test_keys_golden_file():
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", "morton_keys.txt")
    rows = [list(map(int, l.split())) for l in open(path) if l.strip() and not l.startswith("#")]
    pts = np.array([_grid_point(ix, iy, iz) for ix, iy, iz, _ in rows])
    keys = oracle.morton_keys(pts, np.array([0.0, 0.0, 0.0, 1.0]), 2.0 ** LEVELS)
    assert [int(k) for k in keys] == [r[3] for r in rows]


def test_bounding_cube():
    pos = np.array([[0.5, 2.0, -1.0], [1.5, 2.25, 3.0], [1.0, 2.1, 0.0]])
    box = oracle.bounding_cube(pos)
    assert list(box) == [0.5, 2.0, -1.0, 4.0]
    assert list(oracle.bounding_cube(np.array([[3.0, 3.0, 3.0]]))) == [3.0, 3.0, 3.0, 1.0]


def test_sort_is_stable_permutation():
    rng = np.random.default_rng(3)
    keys = rng.integers(0, 20, 500).astype(np.uint64)
    perm = oracle.sort_keys(keys)
    assert np.array_equal(np.sort(perm), np.arange(500))
    sk = keys[perm]
    assert np.all(sk[1:] >= sk[:-1])
    ties = sk[1:] == sk[:-1]
    assert np.all(perm[1:][ties] > perm[:-1][ties])


def _naive_tree(icoord, ncrit, max_level=LEVELS):
    """Brute-force recursive octree from integer grid coordinates: a cell is
    a set of particles; split while count > ncrit. Returns {(level, ix, iy, iz): count}."""
    out = {}

    def rec(level, c, idx):
        out[(level,) + c] = len(idx)
        if len(idx) <= ncrit or level == max_level:
            return
        sh = LEVELS - level - 1
        sub = icoord[idx] >> sh
        for o in range(8):
            want = (2 * c[0] + (o & 1), 2 * c[1] + ((o >> 1) & 1), 2 * c[2] + ((o >> 2) & 1))
            m = np.all(sub == np.array(want), axis=1)
            if m.any():
                rec(level + 1, want, idx[m])

    rec(0, (0, 0, 0), np.arange(icoord.shape[0]))
    return out


@pytest.mark.parametrize("dist,n,ncrit", [("uniform", 1500, 16), ("plummer", 1500, 8), ("uniform", 40, 64)])
def test_tree_matches_brute_force(dist, n, ncrit):
    pos, q = W.uniform_cube(n, 7) if dist == "uniform" else W.plummer(n, 7)
    T = oracle.Tree(pos, ncrit)
    box, scale = T.box, T.scale
    ic = np.minimum(np.floor((pos - box[:3]) * scale), 2 ** LEVELS - 1).astype(np.int64)
    naive = _naive_tree(ic, ncrit)
    got = {(int(c[0]), int(c[1]), int(c[2]), int(c[3])): int(c[5]) for c in T.cells}
    assert got == naive
    # level-major, Morton order within a level
    lv = T.cell("level")
    assert np.all(np.diff(lv) >= 0)
    # leaves partition [0, N); sizes within ncrit; children sum to parent
    leaf = T.cell("child_first") < 0
    first, count = T.cell("first"), T.cell("count")
    cov = np.zeros(n, int)
    for f, c in zip(first[leaf], count[leaf]):
        cov[f:f + c] += 1
    assert np.all(cov == 1)
    assert np.all(count[leaf] <= ncrit)
    for c in np.nonzero(~leaf)[0]:
        cf, nch = T.cells[c, 6], T.cells[c, 7]
        assert count[cf:cf + nch].sum() == count[c]
    # keys of particles carry the prefix of their leaf
    sk = T.keys[T.perm]
    for c in np.nonzero(leaf)[0][:200]:
        l = lv[c]
        pre = sk[first[c]:first[c] + count[c]] >> np.uint64(3 * (LEVELS - l))
        assert np.all(pre == pre[0])


# --------------------------------------------------------------------------
# Dual tree traversal lists (Sec. 4)
# --------------------------------------------------------------------------

def _cover_matrix(T, m2l, p2p):
    n = T.n
    first, count = T.cell("first"), T.cell("count")
    perm = T.perm
    C = np.zeros((n, n), np.int32)
    for A, B in np.vstack([m2l, p2p]):
        ia = perm[first[A]:first[A] + count[A]]
        ib = perm[first[B]:first[B] + count[B]]
        C[np.ix_(ia, ib)] += 1
    return C


def _mac_int(T, A, B, a, b):
    lv = T.cell("level")
    SA, SB = 1 << (LEVELS - int(lv[A])), 1 << (LEVELS - int(lv[B]))
    d2 = 0
    for name in ("ix", "iy", "iz"):
        ca, cb = int(T.cell(name)[A]), int(T.cell(name)[B])
        d2 += ((2 * ca + 1) * SA - (2 * cb + 1) * SB) ** 2
    return 3 * b * b * (SA + SB) ** 2 < a * a * d2


@pytest.mark.parametrize("dist,n,ncrit,theta", [("uniform", 1200, 8, (1, 2)), ("plummer", 1500, 4, (2, 5)),
                                                ("uniform", 700, 1, (1, 2))])
def test_lists_cover_every_pair_once(dist, n, ncrit, theta):
    pos, q = W.uniform_cube(n, 5) if dist == "uniform" else W.plummer(n, 5)
    T = oracle.Tree(pos, ncrit)
    m2l, p2p = T.lists(*theta)
    C = _cover_matrix(T, m2l, p2p)
    assert np.all(C == 1)
    leaf = T.cell("child_first") < 0
    assert np.all(leaf[p2p[:, 0]]) and np.all(leaf[p2p[:, 1]])
    a, b = theta
    assert all(_mac_int(T, A, B, a, b) for A, B in m2l[:500])
    assert not any(_mac_int(T, A, B, a, b) for A, B in p2p[:500])
    # MAC, float form with half diagonal radii (R_A + R_B < theta d), away from the boundary
    ctr = T.centres()
    side = T.box[3] / 2.0 ** T.cell("level")
    R = math.sqrt(3) / 2 * side
    for arr, want in ((m2l, True), (p2p, False)):
        d = np.linalg.norm(ctr[arr[:, 0]] - ctr[arr[:, 1]], axis=1)
        lhs = R[arr[:, 0]] + R[arr[:, 1]]
        margin = np.abs(lhs - (a / b) * d) > 1e-9 * lhs
        assert np.all(((lhs < (a / b) * d) == want)[margin])
    # sorted by (target, source), no duplicates
    for arr in (m2l, p2p):
        key = arr[:, 0].astype(np.int64) * (1 << 32) + arr[:, 1]
        assert np.all(np.diff(key) > 0)


@pytest.mark.parametrize("dist,n,ncrit,theta", [("uniform", 3000, 16, (1, 2)), ("plummer", 4000, 8, (2, 5)),
                                                ("plummer", 2500, 4, (99, 100))])
def test_p2p_lists_are_symmetric(dist, n, ncrit, theta):
    # For theta < 1 a failed MAC stays failed when a cell is replaced by its
    # parent (the radius doubles while the centre moves by at most the old
    # radius), so every ancestor pair of a P2P leaf pair is split and the
    # traversal reaches the pair in both orders: the P2P list equals its
    # transpose (the mutual P2P evaluates each such pair once).  An M2L
    # pair need not come in both orders: (A_i <- B_j) may be reached through
    # (A_i <- B) while the reverse stops one level up at (B_j <- A), so the
    # M2L list is only partly symmetric.
    pos, q = W.uniform_cube(n, 8) if dist == "uniform" else W.plummer(n, 8)
    T = oracle.Tree(pos, ncrit)
    m2l, p2p = T.lists(*theta)
    key = lambda a, b: a.astype(np.int64) * (1 << 32) + b
    assert np.array_equal(np.sort(key(p2p[:, 0], p2p[:, 1])), np.sort(key(p2p[:, 1], p2p[:, 0])))
    both = np.isin(key(m2l[:, 1], m2l[:, 0]), key(m2l[:, 0], m2l[:, 1]))
    assert 0.5 < both.mean() < 1.0


def _grid_particles(level):
    k = 2 ** level
    g = np.array([[i, j, l] for l in range(k) for j in range(k) for i in range(k)], float)
    return (g + 0.5) / k


def test_lists_uniform_level2_grid_hand_derived():
    # One particle at the centre of each of the 64 level-2 cells, ncrit = 1:
    # level 1 pairs never pass the MAC (|di|^2 <= 3), nor do (level-2, level-1)
    # pairs (|dC|^2 <= 75 S^2 < 108 S^2), so every level-2 pair is visited and
    # (A <- B) is M2L iff 3*4*(2S)^2 < |2S di|^2, i.e. |di|^2 > 12 (strict).
    pos = _grid_particles(2)
    T = oracle.Tree(pos, 1)
    m2l, p2p = T.lists(1, 2)
    lv = T.cell("level")
    assert np.all(lv[m2l] == 2) and np.all(lv[p2p] == 2)
    icoord = np.stack([T.cell("ix"), T.cell("iy"), T.cell("iz")], 1)
    l2 = np.nonzero(lv == 2)[0]
    want_m2l, want_p2p = set(), set()
    for A in l2:
        for B in l2:
            d2 = int(((icoord[A] - icoord[B]) ** 2).sum())
            (want_m2l if d2 > 12 else want_p2p).add((int(A), int(B)))
    assert set(map(tuple, m2l.tolist())) == want_m2l
    assert set(map(tuple, p2p.tolist())) == want_p2p
    # the boundary case |di|^2 == 12 is P2P (strict MAC)
    assert any(int(((icoord[A] - icoord[B]) ** 2).sum()) == 12 for A, B in p2p)


def test_lists_uniform_level3_grid_hand_derived():
    # One particle per level-3 cell (512), ncrit = 1, theta = 1/2.  With ties
    # splitting the target, a pair of level-3 leaves (a, b) with parents
    # (A, B) is covered by exactly one of, in this order:
    #   M2L(A <- B)  if MAC(A, B)              (same level 2)
    #   M2L(a <- B)  if MAC(a, B)              (target one level finer)
    #   M2L(a <- b)  if MAC(a, b)
    #   P2P(a <- b)  otherwise.
    # (No level-1 or (2,1) pair passes the MAC on this grid.)
    pos = _grid_particles(3)
    T = oracle.Tree(pos, 1)
    m2l, p2p = T.lists(1, 2)
    lv = T.cell("level")
    par = T.cell("parent")
    l3 = np.nonzero(lv == 3)[0]
    want_m2l, want_p2p = set(), set()
    for a_ in l3:
        for b_ in l3:
            A, B = int(par[a_]), int(par[b_])
            if A != B and _mac_int(T, A, B, 1, 2):
                want_m2l.add((A, B))
            elif _mac_int(T, a_, B, 1, 2):
                want_m2l.add((int(a_), B))
            elif a_ != b_ and _mac_int(T, a_, b_, 1, 2):
                want_m2l.add((int(a_), int(b_)))
            else:
                want_p2p.add((int(a_), int(b_)))
    assert set(map(tuple, m2l.tolist())) == want_m2l
    assert set(map(tuple, p2p.tolist())) == want_p2p
    assert np.any(lv[m2l[:, 0]] == lv[m2l[:, 1]] + 1)   # mixed-level pairs exist


def test_single_leaf_root_is_direct():
    pos, q = W.uniform_cube(50, 9)
    T = oracle.Tree(pos, 64)
    m2l, p2p = T.lists(1, 2)
    assert T.ncell == 1 and len(m2l) == 0 and p2p.tolist() == [[0, 0]]
    phi, E = T.fmm(q, 4)
    pd, Ed = oracle.direct(pos, q)
    assert rel(phi, pd) < 1e-15 and rel(E, Ed) < 1e-15


# --------------------------------------------------------------------------
# Expansion operators (Cartesian Taylor form)
# --------------------------------------------------------------------------

def test_taylor_coefficients_closed_forms():
    r = np.array([0.3, -0.7, 1.1])
    x, y, z = r
    rr = np.linalg.norm(r)
    b = oracle.taylor(4, r)
    mi = oracle.multi_indices(4)
    idx = {m: i for i, m in enumerate(mi)}
    assert b[idx[(0, 0, 0)]] == pytest.approx(1 / rr, rel=1e-15)
    assert b[idx[(1, 0, 0)]] == pytest.approx(-x / rr ** 3, rel=1e-14)
    assert b[idx[(0, 0, 1)]] == pytest.approx(-z / rr ** 3, rel=1e-14)
    assert b[idx[(2, 0, 0)]] == pytest.approx((3 * x * x - rr * rr) / (2 * rr ** 5), rel=1e-13)
    assert b[idx[(1, 1, 0)]] == pytest.approx(3 * x * y / rr ** 5, rel=1e-13)
    assert b[idx[(1, 1, 1)]] == pytest.approx(-15 * x * y * z / rr ** 7, rel=1e-13)
    # 1/|r| is harmonic: sum_k d^(g+2e_k) G = 0 for every g, i.e.
    # sum_k (g+2e_k)! b_(g+2e_k) = 0
    f = math.factorial
    for g in oracle.multi_indices(2):
        s = 0.0
        scale = 0.0
        for k in range(3):
            h = list(g)
            h[k] += 2
            h = tuple(h)
            t = f(h[0]) * f(h[1]) * f(h[2]) * b[idx[h]]
            s += t
            scale += abs(t)
        assert abs(s) <= 1e-13 * scale


def test_taylor_coefficients_vs_finite_differences():
    r = np.array([0.9, 0.4, -0.6])
    mi = oracle.multi_indices(3)
    b = oracle.taylor(3, r)
    h = 1e-3
    for i, m in enumerate(mi):
        if sum(m) != 3:
            continue
        # third derivatives from second-order-accurate nested central differences
        def G(p):
            return 1 / np.linalg.norm(p)

        def D(fn, k):
            e = np.zeros(3)
            e[k] = h
            return lambda p: (fn(p + e) - fn(p - e)) / (2 * h)
        fn = G
        for k in range(3):
            for _ in range(m[k]):
                fn = D(fn, k)
        fd = fn(r) / (math.factorial(m[0]) * math.factorial(m[1]) * math.factorial(m[2]))
        assert fd == pytest.approx(b[i], rel=1e-3)


def test_p2m_moments_exact():
    src = np.array([[0.1, 0.2, -0.05], [-0.12, 0.03, 0.07], [0.0, -0.1, 0.1]])
    q = np.array([0.5, -1.25, 2.0])
    c = np.zeros(3)
    M = oracle.p2m(4, src, q, c)
    mi = oracle.multi_indices(4)
    assert M[0] == pytest.approx(q.sum(), rel=1e-15)
    # dipole +-q at +-delta/2: zero monopole, dipole moment q*delta
    d = np.array([0.02, -0.01, 0.03])
    Md = oracle.p2m(4, np.array([d / 2, -d / 2]), np.array([3.0, -3.0]), c)
    assert Md[0] == 0.0
    for k, e in enumerate([(1, 0, 0), (0, 1, 0), (0, 0, 1)]):
        assert Md[mi.index(e)] == pytest.approx(3.0 * d[k], rel=1e-14)


@pytest.mark.parametrize("p", [2, 4, 6, 8, 10])
def test_p2m_m2p_greengard_rokhlin_bound(p):
    # unit charge at offset a, targets on a sphere of radius rho > |a|
    rng = np.random.default_rng(p)
    a = np.array([0.2, -0.1, 0.15])
    na = np.linalg.norm(a)
    M = oracle.p2m(p, a[None], np.array([1.0]), np.zeros(3))
    for rho in (2 * na, 4 * na):
        v = rng.normal(size=(50, 3))
        x = rho * v / np.linalg.norm(v, axis=1)[:, None]
        phi, _ = oracle.m2p(p, M, np.zeros(3), x)
        exact = 1 / np.linalg.norm(x - a, axis=1)
        bound = (na / rho) ** (p + 1) / (rho - na)
        assert np.all(np.abs(phi - exact) <= bound * (1 + 1e-9) + 1e-15)


def test_m2p_field_matches_direct_far():
    rng = np.random.default_rng(1)
    src = rng.uniform(-0.1, 0.1, (20, 3))
    q = rng.uniform(-1, 1, 20)
    tgt = rng.normal(size=(10, 3))
    tgt = 3 * tgt / np.linalg.norm(tgt, axis=1)[:, None]
    M = oracle.p2m(10, src, q, np.zeros(3))
    phi, E = oracle.m2p(10, M, np.zeros(3), tgt)
    allpos = np.vstack([tgt, src])
    pd, Ed = oracle.direct(allpos, np.r_[np.zeros(10), q], np.arange(10))
    assert rel(phi, pd) < 1e-12 and rel(E, Ed) < 1e-11


@pytest.mark.parametrize("p", [3, 8])
def test_m2m_is_exact(p):
    rng = np.random.default_rng(2)
    src = rng.uniform(-0.25, 0.25, (30, 3)) + np.array([0.25, -0.25, 0.25])
    q = rng.uniform(-1, 1, 30)
    c_child = np.array([0.25, -0.25, 0.25])
    c_par = np.zeros(3)
    M1 = oracle.m2m(p, oracle.p2m(p, src, q, c_child), c_child, c_par)
    M2 = oracle.p2m(p, src, q, c_par)
    assert np.abs(M1 - M2).max() <= 1e-14 * np.abs(M2).max()


@pytest.mark.parametrize("p", [3, 8])
def test_l2l_is_exact(p):
    rng = np.random.default_rng(4)
    L = rng.normal(size=oracle.nk_cart(p))
    c = np.zeros(3)
    c2 = np.array([-0.25, 0.25, 0.25])
    L2 = oracle.l2l(p, L, c, c2)
    x = c2 + rng.uniform(-0.25, 0.25, (40, 3))
    p1, E1 = oracle.l2p(p, L, c, x)
    p2, E2 = oracle.l2p(p, L2, c2, x)
    assert rel(p2, p1) < 1e-13 and rel(E2, E1) < 1e-13


def test_l2p_field_is_minus_gradient():
    rng = np.random.default_rng(6)
    L = rng.normal(size=oracle.nk_cart(5))
    x = rng.uniform(-0.3, 0.3, (5, 3))
    phi, E = oracle.l2p(5, L, np.zeros(3), x)
    h = 1e-6
    for k in range(3):
        e = np.zeros(3)
        e[k] = h
        fp, _ = oracle.l2p(5, L, np.zeros(3), x + e)
        fm, _ = oracle.l2p(5, L, np.zeros(3), x - e)
        assert np.allclose(-(fp - fm) / (2 * h), E[:, k], rtol=1e-6, atol=1e-7)


def test_m2l_single_pair_converges_in_p():
    # equal cells of side 1 just inside the MAC (theta = 1/2: d > 2 sqrt3 = 3.46)
    rng = np.random.default_rng(8)
    cB = np.zeros(3)
    cA = np.array([3.6, 0.0, 0.0])
    src = cB + rng.uniform(-0.5, 0.5, (64, 3))
    tgt = cA + rng.uniform(-0.5, 0.5, (64, 3))
    q = rng.uniform(-1, 1, 64)
    allpos = np.vstack([tgt, src])
    pd, Ed = oracle.direct(allpos, np.r_[np.zeros(64), q], np.arange(64))
    errs = []
    for p in (2, 4, 6, 8, 10):
        L = oracle.m2l(p, oracle.p2m(p, src, q, cB), cB, cA)
        phi, E = oracle.l2p(p, L, cA, tgt)
        errs.append((rel(phi, pd), rel(E, Ed)))
    for (a1, b1), (a2, b2) in zip(errs, errs[1:]):
        assert a2 < a1 and b2 < b1
    assert errs[3][0] < 1e-5 and errs[3][1] < 1e-4   # p = 8


# --------------------------------------------------------------------------
# Whole FMM
# --------------------------------------------------------------------------

def test_fmm_error_decreases_with_p():
    pos, q = W.uniform_cube(3000, 21)
    pd, Ed = oracle.direct(pos, q)
    T = oracle.Tree(pos, 32)
    T.lists(1, 2)
    prev = (1.0, 1.0)
    for p in (2, 4, 6, 8):
        phi, E = T.fmm(q, p)
        e = (rel(phi, pd), rel(E, Ed))
        assert e[0] < prev[0] and e[1] < prev[1]
        prev = e
    assert prev[0] < 1e-6 and prev[1] < 1e-6


def test_fmm_uniform4k_p4_tolerance():
    pos, q, w = W.make("uniform4k_p4")
    pd, Ed = oracle.direct(pos, q)
    phi, E, T = oracle.fmm(pos, q, w["p"], w["ncrit"], *w["theta"])
    assert rel(phi, pd) < 1e-3 and rel(E, Ed) < 1e-2


def test_fmm_plummer_adaptive():
    pos, q = W.plummer(4000, 31)
    pd, Ed = oracle.direct(pos, q)
    phi, E, T = oracle.fmm(pos, q, 8, 16, 1, 2)
    lv = T.cell("level")
    assert lv.max() - lv[T.cell("child_first") < 0].min() >= 3   # really adaptive
    assert rel(phi, pd) < 1e-5 and rel(E, Ed) < 1e-4


def test_fmm_translation_and_linearity():
    pos, q = W.uniform_cube(2000, 41)
    T = oracle.Tree(pos, 16)
    T.lists(1, 2)
    phi, E = T.fmm(q, 6)
    q2 = W.uniform_cube(2000, 42)[1]
    p2, E2 = T.fmm(q2, 6)
    p3, E3 = T.fmm(2 * q - q2, 6)
    assert rel(p3, 2 * phi - p2) < 1e-13 and rel(E3, 2 * E - E2) < 1e-13
    # a shifted copy builds the same tree; result is the same to rounding
    phis, Es, _ = oracle.fmm(pos + 5.0, q, 6, 16, 1, 2)
    assert rel(phis, phi) < 1e-10 and rel(Es, E) < 1e-9


def test_workload_generators():
    p1, q1 = W.uniform_cube(1000, 3)
    p2, q2 = W.uniform_cube(1000, 3)
    assert np.array_equal(p1, p2) and np.array_equal(q1, q2)
    assert p1.min() >= 0 and p1.max() < 1 and q1.min() >= -1 and q1.max() <= 1
    pp, qp = W.plummer(200000, 3)
    r = np.linalg.norm(pp, axis=1)
    assert r.max() <= 20.0
    # half of the (truncated) mass lies inside the Plummer half-mass radius
    mt = 20.0 ** 3 / (1 + 20.0 ** 2) ** 1.5
    rh = 1.0 / math.sqrt((0.5 * mt) ** (-2.0 / 3.0) - 1)
    assert abs(np.mean(r < rh) - 0.5) < 0.005
    sizes = W.batch_sizes()
    assert sizes.min() >= 1024 and sizes.max() <= 65536 and len(sizes) == 256
    s = W.error_sample(1 << 20, 2)
    assert len(np.unique(s)) == 4096


def leaf_sides(T):
    """Side of the leaf cell holding every particle (input order)."""
    lv, cf = T.cell("level"), T.cell("child_first")
    first, cnt = T.cell("first"), T.cell("count")
    side = np.zeros(T.n)
    for c in np.nonzero(cf < 0)[0]:
        side[T.perm[first[c]:first[c] + cnt[c]]] = T.box[3] / 2.0 ** lv[c]
    return side


def test_fmm_frozen_tree_moved_particles():
    """Evaluation on a kept tree with moved particles (time stepping without
    a rebuild): each particle moves by up to 1/10 of its leaf side per axis,
    so it stays inside its leaf widened by 1/8; the result is still the
    potential of the moved particles to the FMM's accuracy at p = 8, and far
    from that of the old positions (the new ones are really read)."""
    pos0, q = W.uniform_cube(3000, 51)
    T = oracle.Tree(pos0, 32)
    T.lists(1, 2)
    side = leaf_sides(T)
    assert np.all(side > 0)
    phi0, E0 = T.fmm(q, 8)
    phis, Es = T.fmm(q, 8, pos=pos0)
    assert np.array_equal(phi0, phis) and np.array_equal(E0, Es)
    pos1 = pos0 + W.velocities(3000, 52, 0.1 * side)
    phi1, E1 = T.fmm(q, 8, pos=pos1)
    pd, Ed = oracle.direct(pos1, q)
    assert rel(phi1, pd) < 1e-6 and rel(E1, Ed) < 1e-6
    pd0, Ed0 = oracle.direct(pos0, q)
    assert rel(phi1, pd0) > 1e-2 and rel(E1, Ed0) > 1e-1
