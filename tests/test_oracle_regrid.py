"""Pins of the oracle's regrid (explosion / coalescence operators applied to
whole blocks, eq. ctof and eq. ftoc).

* splitting a block and merging its 8 children again is the identity
  (the 1/8 mean of 8 copies is the copy);
* volume-weighted mass and momentum are unchanged by any regrid;
* a uniform flow stays uniform;
* the new forest is 2:1 balanced and all-zero flags change nothing.
"""

import numpy as np
import pytest

from oracle import Forest, RefinedOracle
from oracle.regrid import regrid_forest


def three_level(n=4):
    def refine(L, x, y, z):
        return (L == 0 and (x, y, z) == (1, 1, 1)) or (L == 1 and (x, y, z) == (3, 3, 2))
    return Forest.build((3, 3, 3), n, 2, refine)


def _state(o, seed):
    rng = np.random.default_rng(seed)
    N = o.total_cells()
    o.init_pdfs(1.0 + 0.01 * rng.uniform(-1, 1, N), 0.04 * rng.uniform(-1, 1, (N, 3)))
    o.step(2)


def test_zero_flags_identity():
    o = RefinedOracle(three_level(), 1.3)
    _state(o, 1)
    o2 = o.regrid(np.zeros(len(o.forest.leaves), dtype=np.int8), 3)
    assert o2.forest.canonical_leaves() == o.forest.canonical_leaves()
    for L in range(o.num_levels):
        assert np.array_equal(o2.interior_pdfs(L), o.interior_pdfs(L))


def test_split_then_merge_is_identity():
    o = RefinedOracle(three_level(), 1.3)
    _state(o, 2)
    leaves = o.forest.canonical_leaves()
    flags = np.array([1 if (L == 1 and x % 2 == 0 and y % 2 == 0) else 0 for (L, x, y, z) in leaves], dtype=np.int8)
    o2 = o.regrid(flags, 3)
    # merge every group that the split created (children of the split blocks)
    split = {leaf for leaf, f in zip(leaves, flags) if f > 0}
    back = np.array([-1 if (L >= 1 and (L - 1, x >> 1, y >> 1, z >> 1) in split) else 0
                     for (L, x, y, z) in o2.forest.canonical_leaves()], dtype=np.int8)
    o3 = o2.regrid(back, 3)
    # blocks the balance also split stay split; compare the blocks that came back
    old = {l: i for i, l in enumerate(leaves)}
    n3 = o.n ** 3
    got = {l: i for i, l in enumerate(o3.forest.canonical_leaves())}
    for leaf in split:
        if leaf in got:
            a = o.interior_pdfs(leaf[0])[o.forest.level_blocks(leaf[0]).tolist().index(list(leaf[1:])) * n3:][:n3]
            b = o3.interior_pdfs(leaf[0])[o3.forest.level_blocks(leaf[0]).tolist().index(list(leaf[1:])) * n3:][:n3]
            assert np.max(np.abs(a - b)) < 1e-16
    assert any(leaf in got for leaf in split)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_regrid_conserves_and_balances(seed):
    o = RefinedOracle(three_level(), 1.3)
    _state(o, seed)
    rng = np.random.default_rng(seed)
    flags = rng.choice([-1, 0, 1], size=len(o.forest.leaves), p=[0.5, 0.3, 0.2]).astype(np.int8)
    M0, J0 = o.mass()
    o2 = o.regrid(flags, 3)
    assert o2.forest.is_balanced()
    o2.forest.check_cover()
    M1, J1 = o2.mass()
    assert abs(M1 - M0) / M0 < 1e-14
    assert np.max(np.abs(J1 - J0)) / M0 < 1e-14
    o2.step(2)
    M2, J2 = o2.mass()
    assert abs(M2 - M0) / M0 < 1e-13


def test_uniform_flow_survives_regrid():
    o = RefinedOracle(three_level(), 1.6)
    N = o.total_cells()
    U = np.array([0.02, 0.01, -0.03])
    o.init_pdfs(np.ones(N), np.tile(U, (N, 1)))
    o.step(2)
    rng = np.random.default_rng(5)
    o2 = o.regrid(rng.choice([-1, 0, 1], size=len(o.forest.leaves)).astype(np.int8), 3)
    o2.step(3)
    rho, u = o2.moments()
    assert np.max(np.abs(u - U)) < 1e-14
    assert np.max(np.abs(rho - 1)) < 1e-14


def test_merge_blocked_by_balance():
    # a level-2 group next to level-3 leaves cannot merge
    def refine(L, x, y, z):
        return (L == 0 and (x, y, z) == (1, 1, 1)) or (L == 1 and (x, y, z) == (3, 3, 3)) or \
               (L == 2 and (x, y, z) == (7, 7, 7))
    f = Forest.build((3, 3, 3), 4, 3, refine)
    flags = [-1 if L == 2 else 0 for (L, x, y, z) in f.canonical_leaves()]
    f2 = regrid_forest(f, flags, 3)
    assert f2.is_balanced()
    # every level-3 leaf still has level-2 neighbours: some level-2 leaves remain
    assert any(l[0] == 2 for l in f2.leaves)
