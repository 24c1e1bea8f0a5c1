"""ctypes binding of the FP64 CPU oracle (oracle.c).

TEST INFRASTRUCTURE ONLY.  The product path never imports this module.

Everything here is FP64 and follows the readings R1-R8 stated at the top of
oracle.c:
  * direct(pos, q, targets=None)      -- the exact sums of Sec. 2.1's problem
  * Tree(pos, ncrit, max_level, box)  -- Morton keys / sort / adaptive octree
                                         (Sec. 2.1, 2.2)
  * Tree.lists(theta_num, theta_den)  -- dual tree traversal (Sec. 4)
  * Tree.fmm(pos, q, p)               -- the six FMM stages (Sec. 2.1)
  * p2m / m2p / m2m / m2l / l2l / l2p -- single operators, Cartesian Taylor
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

_d = ctypes.POINTER(ctypes.c_double)
_i64 = ctypes.POINTER(ctypes.c_int64)
_u64 = ctypes.POINTER(ctypes.c_uint64)
_i32 = ctypes.POINTER(ctypes.c_int32)
_vp = ctypes.c_void_p


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        from . import build as _b
        _b.build()
    lib = ctypes.CDLL(_LIB_PATH)
    I64, I32 = ctypes.c_int64, ctypes.c_int
    lib.orc_direct.argtypes = [I64, _d, _d, I64, _i64, _d, _d]
    lib.orc_bounding_cube.argtypes = [I64, _d, _d]
    lib.orc_morton_keys.argtypes = [I64, _d, _d, ctypes.c_double, _u64]
    lib.orc_sort_keys.argtypes = [I64, _u64, _i64]
    lib.orc_tree_build.argtypes = [I64, _d, _d, I32, I32]
    lib.orc_tree_build.restype = _vp
    lib.orc_tree_free.argtypes = [_vp]
    lib.orc_tree_ncell.argtypes = [_vp]
    lib.orc_tree_ncell.restype = I64
    lib.orc_tree_box.argtypes = [_vp, _d, _d]
    lib.orc_tree_copy.argtypes = [_vp, _u64, _i64, _i64]
    lib.orc_tree_lists.argtypes = [_vp, I32, I32, _i64, _i64]
    lib.orc_tree_copy_lists.argtypes = [_vp, _i32, _i32, _i32, _i32]
    lib.orc_fmm_eval.argtypes = [_vp, _d, _d, I32, _d, _d, _d, _d]
    lib.orc_fmm_eval.restype = I32
    lib.orc_nk.argtypes = [I32]
    lib.orc_nk.restype = I32
    lib.orc_p2m.argtypes = [I32, I64, _d, _d, _d, _d]
    lib.orc_m2p.argtypes = [I32, _d, _d, I64, _d, _d, _d]
    lib.orc_m2m.argtypes = [I32, _d, _d, _d, _d]
    lib.orc_m2l.argtypes = [I32, _d, _d, _d, _d]
    lib.orc_l2l.argtypes = [I32, _d, _d, _d, _d]
    lib.orc_l2p.argtypes = [I32, _d, _d, I64, _d, _d, _d]
    lib.orc_taylor.argtypes = [I32, _d, _d]
    lib.orc_num_threads.restype = I32
    lib.orc_set_num_threads.argtypes = [I32]
    _lib = lib
    return lib


def _f64(a, shape=None):
    a = np.ascontiguousarray(a, dtype=np.float64)
    if shape is not None:
        a = a.reshape(shape)
    return a


def _p(a, t):
    return a.ctypes.data_as(t) if a is not None else None


def num_threads() -> int:
    """OpenMP threads the oracle uses."""
    return int(_load().orc_num_threads())


def set_num_threads(n: int) -> None:
    """OpenMP threads of the oracle's later calls."""
    _load().orc_set_num_threads(int(n))


def direct(pos, q, targets=None):
    """Exact potential and field (phi, E) at the targets, FP64, O(N * targets).

    phi_i = sum_{j: r_ij > 0} q_j / r_ij ;  E_i = sum_{j: r_ij > 0} q_j (x_i - x_j) / r_ij^3
    """
    lib = _load()
    pos = _f64(pos, (-1, 3))
    q = _f64(q)
    n = pos.shape[0]
    if targets is None:
        nt, tidx = n, None
    else:
        tidx = np.ascontiguousarray(targets, dtype=np.int64)
        nt = tidx.shape[0]
    phi = np.zeros(nt)
    field = np.zeros((nt, 3))
    lib.orc_direct(n, _p(pos, _d), _p(q, _d), nt, _p(tidx, _i64), _p(phi, _d), _p(field, _d))
    return phi, field


def bounding_cube(pos):
    """(min_x, min_y, min_z, side) per reading R2."""
    pos = _f64(pos, (-1, 3))
    box = np.zeros(4)
    _load().orc_bounding_cube(pos.shape[0], _p(pos, _d), _p(box, _d))
    return box


def morton_keys(pos, box, scale):
    pos = _f64(pos, (-1, 3))
    box = _f64(box)
    keys = np.zeros(pos.shape[0], dtype=np.uint64)
    _load().orc_morton_keys(pos.shape[0], _p(pos, _d), _p(box, _d), float(scale), _p(keys, _u64))
    return keys


def sort_keys(keys):
    keys = np.ascontiguousarray(keys, dtype=np.uint64)
    perm = np.zeros(keys.shape[0], dtype=np.int64)
    _load().orc_sort_keys(keys.shape[0], _p(keys, _u64), _p(perm, _i64))
    return perm


CELL_FIELDS = ("level", "ix", "iy", "iz", "first", "count", "child_first", "nchild", "parent")


class Tree:
    """Keys, sort and adaptive octree of one particle set (FP64 oracle)."""

    def __init__(self, pos, ncrit, max_level=21, box=None):
        lib = _load()
        self._lib = lib
        self.pos = _f64(pos, (-1, 3))
        self.n = self.pos.shape[0]
        b = None if box is None else _f64(box)
        self._h = lib.orc_tree_build(self.n, _p(self.pos, _d), _p(b, _d), int(ncrit), int(max_level))
        self.ncell = int(lib.orc_tree_ncell(self._h))
        box4 = np.zeros(4)
        sc = ctypes.c_double()
        lib.orc_tree_box(self._h, _p(box4, _d), ctypes.byref(sc))
        self.box = box4
        self.scale = sc.value
        self.keys = np.zeros(self.n, dtype=np.uint64)
        self.perm = np.zeros(self.n, dtype=np.int64)
        self.cells = np.zeros((self.ncell, 9), dtype=np.int64)
        lib.orc_tree_copy(self._h, _p(self.keys, _u64), _p(self.perm, _i64), _p(self.cells, _i64))
        self.m2l = None
        self.p2p = None

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            self._lib.orc_tree_free(h)
            self._h = None

    def cell(self, name):
        return self.cells[:, CELL_FIELDS.index(name)]

    def lists(self, theta_num, theta_den):
        """Dual tree traversal; returns (m2l, p2p) as (k, 2) int32 arrays of
        (target, source), each sorted by (target, source)."""
        nm, npp = ctypes.c_int64(), ctypes.c_int64()
        self._lib.orc_tree_lists(self._h, int(theta_num), int(theta_den), ctypes.byref(nm), ctypes.byref(npp))
        m2l = np.zeros((nm.value, 2), dtype=np.int32)
        p2p = np.zeros((npp.value, 2), dtype=np.int32)
        mt = np.zeros(nm.value, dtype=np.int32)
        ms = np.zeros(nm.value, dtype=np.int32)
        pt = np.zeros(npp.value, dtype=np.int32)
        ps = np.zeros(npp.value, dtype=np.int32)
        self._lib.orc_tree_copy_lists(self._h, _p(mt, _i32), _p(ms, _i32), _p(pt, _i32), _p(ps, _i32))
        m2l[:, 0], m2l[:, 1] = mt, ms
        p2p[:, 0], p2p[:, 1] = pt, ps
        self.m2l, self.p2p = m2l, p2p
        return m2l, p2p

    def fmm(self, q, p, pos=None, want_expansions=False):
        """FMM potential and field in input order (lists() must have run).

        pos defaults to the positions the tree was built from (a different
        array of the same shape evaluates with the frozen tree and lists)."""
        if self.m2l is None:
            raise RuntimeError("call lists() first")
        q = _f64(q)
        pos = self.pos if pos is None else _f64(pos, (-1, 3))
        phi = np.zeros(self.n)
        field = np.zeros((self.n, 3))
        nk = nk_cart(p)
        M = L = None
        if want_expansions:
            M = np.zeros((self.ncell, nk))
            L = np.zeros((self.ncell, nk))
        rc = self._lib.orc_fmm_eval(self._h, _p(pos, _d), _p(q, _d), int(p), _p(phi, _d), _p(field, _d),
                                    _p(M, _d), _p(L, _d))
        if rc != 0:
            raise RuntimeError("oracle fmm failed")
        if want_expansions:
            return phi, field, M, L
        return phi, field

    def centres(self):
        """Geometric cell centres per reading R8 (FP64)."""
        lv = self.cell("level")
        out = np.zeros((self.ncell, 3))
        for d, name in enumerate(("ix", "iy", "iz")):
            out[:, d] = self.box[d] + ((2 * self.cell(name) + 1).astype(np.float64) * self.box[3]) / np.ldexp(1.0, lv + 1)
        return out


def nk_cart(p):
    """|K_p| = number of Cartesian multi-indices with |alpha| <= p."""
    return (p + 1) * (p + 2) * (p + 3) // 6


def multi_indices(order):
    """Multi-indices with |alpha| <= order in the oracle's order (degree,
    then a0 descending, then a1 descending)."""
    out = []
    for n in range(order + 1):
        for a0 in range(n, -1, -1):
            for a1 in range(n - a0, -1, -1):
                out.append((a0, a1, n - a0 - a1))
    return out


def p2m(p, src, q, c):
    src = _f64(src, (-1, 3))
    q = _f64(q)
    c = _f64(c)
    M = np.zeros(nk_cart(p))
    _load().orc_p2m(p, src.shape[0], _p(src, _d), _p(q, _d), _p(c, _d), _p(M, _d))
    return M


def m2p(p, M, c, tgt):
    tgt = _f64(tgt, (-1, 3))
    M = _f64(M)
    c = _f64(c)
    phi = np.zeros(tgt.shape[0])
    field = np.zeros((tgt.shape[0], 3))
    _load().orc_m2p(p, _p(M, _d), _p(c, _d), tgt.shape[0], _p(tgt, _d), _p(phi, _d), _p(field, _d))
    return phi, field


def m2m(p, M, c, c2):
    M, c, c2 = _f64(M), _f64(c), _f64(c2)
    out = np.zeros(nk_cart(p))
    _load().orc_m2m(p, _p(M, _d), _p(c, _d), _p(c2, _d), _p(out, _d))
    return out


def m2l(p, M, cB, cA):
    M, cB, cA = _f64(M), _f64(cB), _f64(cA)
    out = np.zeros(nk_cart(p))
    _load().orc_m2l(p, _p(M, _d), _p(cB, _d), _p(cA, _d), _p(out, _d))
    return out


def l2l(p, L, c, c2):
    L, c, c2 = _f64(L), _f64(c), _f64(c2)
    out = np.zeros(nk_cart(p))
    _load().orc_l2l(p, _p(L, _d), _p(c, _d), _p(c2, _d), _p(out, _d))
    return out


def l2p(p, L, c, tgt):
    tgt = _f64(tgt, (-1, 3))
    L, c = _f64(L), _f64(c)
    phi = np.zeros(tgt.shape[0])
    field = np.zeros((tgt.shape[0], 3))
    _load().orc_l2p(p, _p(L, _d), _p(c, _d), tgt.shape[0], _p(tgt, _d), _p(phi, _d), _p(field, _d))
    return phi, field


def taylor(order, r):
    """b_gamma(r) = d^gamma (1/|r|) / gamma! for |gamma| <= order."""
    r = _f64(r)
    out = np.zeros(nk_cart(order))
    _load().orc_taylor(order, _p(r, _d), _p(out, _d))
    return out


def fmm(pos, q, p, ncrit, theta_num, theta_den, max_level=21, box=None):
    """Convenience: build tree, lists and evaluate.  Returns (phi, field, tree)."""
    t = Tree(pos, ncrit, max_level, box)
    t.lists(theta_num, theta_den)
    phi, field = t.fmm(q, p)
    return phi, field, t
