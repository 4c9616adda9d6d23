"""Host-side checks of the C ABI (no device work).

* the library loads and exports every entry point the header declares;
* the library's own forest builder gives, leaf for leaf, the same balanced
  forest and canonical order as the oracle's independent builder;
* its level tables give the same coalescence set size as the oracle's set
  definition (which is written in terms of children, not neighbour blocks);
* error codes for invalid descriptions.
"""

import os
import re

import numpy as np
import pytest

from oracle import Forest, RefinedOracle
from paper_1508_07982_amd import lbm
from paper_1508_07982_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _lib():
    if not os.path.exists(lbm.LIB_PATH):
        from paper_1508_07982_amd import build
        build.build()
    return lbm.load_library()


def test_exports_every_declared_symbol():
    lib = _lib()
    names = set()
    for hdr in os.listdir(os.path.join(ROOT, "include")):
        if hdr.endswith(".h"):
            text = open(os.path.join(ROOT, "include", hdr)).read()
            names |= set(re.findall(r"^(?:int|const char \*)\s*(lbm_\w+)\s*\(", text, flags=re.M))
    assert len(names) >= 20
    for name in sorted(names):
        assert hasattr(lib, name), name


def test_lattice_convention_matches_oracle():
    from oracle import refined as orc
    _lib()
    e, w = lbm.lattice()
    eo, wo = orc.lattice()
    assert np.array_equal(e, eo)
    assert np.array_equal(w, wo)


PERIODIC = (True, True, True)


def _forests():
    def three(L, x, y, z):
        return (L == 0 and (x, y, z) == (1, 1, 1)) or (L == 1 and (x, y, z) == (3, 3, 2))

    def corner(L, x, y, z):  # refinement in the corner of the root grid, next to the walls
        return (L == 0 and (x, y, z) == (0, 0, 0)) or (L == 1 and (x, y, z) == (0, 0, 1))
    w1 = W.config_two_level()
    w2 = W.config_sphere(32, 4)
    w4 = W.config_slab_sphere()
    return [
        ("two_level", (2, 2, 2), 16, 1, w1.refine, PERIODIC),
        ("three_level", (3, 3, 3), 4, 2, three, PERIODIC),
        ("sphere_shell", w2.R, 32, 3, w2.refine, PERIODIC),
        ("slab_sphere", w4.R, 16, 3, w4.refine, PERIODIC),
        ("uniform", (2, 3, 4), 8, 0, None, PERIODIC),
        ("corner_walls_y", (3, 3, 3), 4, 2, corner, (True, False, True)),
        ("corner_walls_xz", (3, 3, 3), 4, 2, corner, (False, True, False)),
        ("corner_closed_box", (3, 3, 3), 8, 2, corner, (False, False, False)),
    ]


@pytest.mark.parametrize("name, R, n, Lmax, refine, periodic", _forests())
def test_forest_builder_matches_oracle(name, R, n, Lmax, refine, periodic):
    _lib()
    got = lbm.build_leaves(R, n, Lmax, refine=refine, periodic=periodic)
    ref = Forest.build(R, n, Lmax, refine, periodic=periodic)
    assert got.tolist() == [list(t) for t in ref.canonical_leaves()]


def test_walls_change_the_balance():
    """Across a periodic wrap the corner refinement touches the far side of
    the root grid and the 2:1 balance refines it there; with walls it does
    not, so the forest has fewer leaves."""
    _lib()
    name, R, n, Lmax, refine, _ = [f for f in _forests() if f[0] == "corner_closed_box"][0]
    open_box = lbm.build_leaves(R, n, Lmax, refine=refine)
    closed = lbm.build_leaves(R, n, Lmax, refine=refine, periodic=(False, False, False))
    assert len(closed) < len(open_box)


@pytest.mark.parametrize("name, R, n, Lmax, refine, periodic",
                         [f for f in _forests() if f[0] in ("two_level", "three_level") or "corner" in f[0]])
def test_level_tables_match_oracle_sets(name, R, n, Lmax, refine, periodic):
    _lib()
    forest = Forest.build(R, n, Lmax, refine, periodic=periodic)
    o = RefinedOracle(forest, 1.5)
    for L in range(forest.max_level + 1):
        st = lbm.plan_level_stats(R, n, Lmax, L, refine=refine, periodic=periodic)
        c = o.tables[L].cells
        assert st["interior_cells"] == c.n_int
        assert st["coalesced_pairs"] == len(o.tables[L].coal_cell)


def test_sphere_shell_sizes():
    _lib()
    w = W.config_sphere(32, 4)
    leaves = lbm.build_leaves(w.R, w.n, w.max_level, refine=w.refine)
    counts = [int(np.sum(leaves[:, 0] == L)) for L in range(4)]
    assert counts == [0, 352, 984, 2368]


def test_error_codes():
    _lib()
    with pytest.raises(lbm.LBMError) as e:
        lbm.build_leaves((2, 2, 2), 12, 1)
    assert e.value.name == "LBM_E_INVALID"
    with pytest.raises(lbm.LBMError) as e:
        lbm.build_leaves((2, 2, 2), 8, 1, periodic=(True, 2, True))
    assert e.value.name == "LBM_E_INVALID"
    # leaves that leave a hole
    with pytest.raises(lbm.LBMError) as e:
        lbm.build_leaves((2, 1, 1), 8, 0, leaves=[(0, 0, 0, 0)])
    assert e.value.name == "LBM_E_COVER"
    # level-2 blocks next to a level-0 block
    leaves = [(0, 1, 0, 0)] + [(1, x, y, z) for x in (0, 1) for y in (0, 1) for z in (0, 1) if (x, y, z) != (1, 0, 0)]
    leaves += [(2, 2 + x, y, z) for x in (0, 1) for y in (0, 1) for z in (0, 1)]
    with pytest.raises(lbm.LBMError) as e:
        lbm.build_leaves((2, 1, 1), 8, 2, leaves=leaves, balance=False)
    assert e.value.name == "LBM_E_UNBALANCED"
    fixed = lbm.build_leaves((2, 1, 1), 8, 2, leaves=leaves, balance=True)
    ref = Forest((2, 1, 1), 8, leaves)
    ref.balance()
    assert fixed.tolist() == [list(t) for t in ref.canonical_leaves()]
