"""The level-by-level M2M and L2L on adaptive trees, where most cells of
the deep levels are leaves: the kernels take a level's cells with children
from a list the build makes, so each case first checks (on the host, from
the oracle's tree) that its tree has what the kernels must handle:

  * levels with more than 256 cells but few enough parents that the
    per-(parent, octant) kernel runs, where launches over every cell used
    the register-tiled one;
  * levels in the tiled kernel whose parents fill some tiles only
    partly, the grid covering a bound (the smaller of the level's and the
    next level's cell counts) with the blocks beyond the parents idle;
  * parents without a child in some octants.

FP64 path against the oracle FMM (Cartesian Taylor, the same tree and
lists): 1e-11 relative L2 and the per-particle bounds of the FP64 tests;
the mixed path, whose M2M and L2L are the same FP64 kernels, at its 1e-5.
Expansions and lists are the paper's (Sec. 2.1, 2.2, 4)."""
import numpy as np
import pytest
import torch

import oracle
from paper_1203_0889_amd import fmm, workloads as W
from parity import check_fp64, check_mixed, leaf_ids, rel

pytestmark = pytest.mark.gpu

SMALL_LEVEL = 256   # parents per level up to which one block per (parent, octant) runs


def say(*a):
    print(*a, flush=True)


def level_shape(T):
    """Per level with a level below it: cells, parents, bound on parents."""
    c = T.cells
    lev, nch = c[:, 0], c[:, 7]
    L = int(lev.max()) + 1
    cells = [int(np.sum(lev == l)) for l in range(L)]
    return [(cells[l], int(np.sum(nch[lev == l] > 0)), min(cells[l], cells[l + 1])) for l in range(L - 1)]


# (name, n, seed, ncrit, p, precision, a level of more than 256 cells in the small kernel)
CASES = [
    ("plummer12k_ncrit4_p6", 12000, 7, 4, 6, "fp64", True),
    ("plummer30k_ncrit8_p5", 30000, 5, 8, 5, "fp64", False),
    ("plummer20k_ncrit16_p7", 20000, 3, 16, 7, "fp64", True),
    ("plummer20k_ncrit16_p7_mixed", 20000, 3, 16, 7, "mixed", True),
]


@pytest.mark.parametrize("name,n,seed,ncrit,p,precision,small_wide", CASES, ids=[c[0] for c in CASES])
def test_level_kernels_on_adaptive_trees(name, n, seed, ncrit, p, precision, small_wide):
    pos, q = W.plummer(n, seed)
    T = oracle.Tree(pos, ncrit)
    T.lists(1, 2)
    shape = level_shape(T)
    say(name, "levels (cells, parents, bound):", shape)
    if small_wide:
        assert any(c > SMALL_LEVEL and b <= SMALL_LEVEL for c, _, b in shape)
    assert any(b > SMALL_LEVEL and par < b for c, par, b in shape)   # tiled, with idle blocks
    assert any(b > SMALL_LEVEL and par % 32 for c, par, b in shape)  # a partly filled tile
    nch = T.cells[:, 7]
    assert np.any((nch > 0) & (nch < 8))                               # octants without a child
    phi_ref, fld_ref = T.fmm(q, p)
    plan = fmm.Plan(p=p, ncrit=ncrit, theta=(1, 2), precision=precision, device=0)
    plan.build_tree(torch.from_numpy(pos).cuda(), torch.from_numpy(q).cuda())
    plan.upward()
    out = {k: v.cpu().numpy() for k, v in plan.evaluate().items()}
    torch.cuda.synchronize()
    e = (rel(out["phi"], phi_ref), rel(out["field"], fld_ref))
    say(name, precision, "vs oracle fmm", e)
    ids = leaf_ids(T.perm, T.cells)
    if precision == "fp64":
        assert max(e) < 1e-11
        check_fp64(out, phi_ref, fld_ref, ids, say, name)
    else:
        assert max(e) < 1e-5
        check_mixed(out, phi_ref, fld_ref, ids, say, name)
