"""Forest of octrees over a periodic uniform root grid (oracle side).

Section 3.2: the domain is a uniform grid of root blocks; refining a block
splits it into 8 children of half the edge length, and every block, on every
level, holds the same n^3 cells, so level transitions coincide with block
boundaries (section 4).  Section 2.3: neighbouring cells may differ by at
most one level (2:1 balance).  Section 3.3: the forest is built by
repeatedly splitting blocks selected by user callbacks, and additional splits
enforce the 2:1 balance.

Readings:
* Balance is enforced over face, edge and corner neighbours, across the
  periodic wrap.  D3Q19 itself only exchanges across faces and edges
  (section 2), but corner balance guarantees that every halo cell near a fine
  block has a parent exactly one level coarser.
* Build order: for l = 0 .. Lmax-1 the callback is asked once for every leaf
  on level l; afterwards the 2:1 balance is enforced by splitting the
  coarser block of every violating pair until none is left.  That fixed point
  is the unique smallest balanced refinement of the callback's forest.
* Canonical block order: level-major, then the Morton (Z-order) index of the
  block position on its level, x in the lowest bit.

A leaf is the tuple (L, x, y, z): level and integer block position on that
level; level L has R_a * 2^L positions along axis a.

An axis may be non-periodic (section 2.2: domain boundaries get a boundary
treatment instead of the periodic copy): positions beyond its ends lie
outside the domain, are no neighbours for the 2:1 balance and hold no-slip
walls (see tables.py).
"""

from __future__ import annotations

import itertools

import numpy as np

NEIGHBOUR_OFFSETS = [d for d in itertools.product((-1, 0, 1), repeat=3) if d != (0, 0, 0)]


def morton_key(x: int, y: int, z: int) -> int:
    """Interleave the bits of (x, y, z), x lowest."""
    key = 0
    bit = 0
    while (x | y | z) >> bit:
        key |= ((x >> bit) & 1) << (3 * bit)
        key |= ((y >> bit) & 1) << (3 * bit + 1)
        key |= ((z >> bit) & 1) << (3 * bit + 2)
        bit += 1
    return key


class Forest:
    """A 2:1 balanced forest: root grid R, n^3 cells per block, leaf set."""

    def __init__(self, roots, n: int, leaves, periodic=(True, True, True)):
        self.R = tuple(int(r) for r in roots)
        self.n = int(n)
        self.periodic = tuple(bool(p) for p in periodic)
        self.leaves = set(tuple(int(v) for v in leaf) for leaf in leaves)
        if not self.leaves:
            raise ValueError("empty forest")
        self.max_level = max(leaf[0] for leaf in self.leaves)

    # -- construction --------------------------------------------------------
    @classmethod
    def build(cls, roots, n: int, max_level: int, refine=None, periodic=(True, True, True)):
        """Roots, then callback splits level by level, then 2:1 balance."""
        R = tuple(int(r) for r in roots)
        leaves = {(0, x, y, z) for x in range(R[0]) for y in range(R[1]) for z in range(R[2])}
        for level in range(max_level):
            if refine is None:
                break
            for leaf in sorted(leaf for leaf in leaves if leaf[0] == level):
                if refine(leaf[0], leaf[1], leaf[2], leaf[3]):
                    leaves.remove(leaf)
                    leaves.update(cls._children(leaf))
        forest = cls(R, n, leaves, periodic)
        forest.balance()
        forest.check_cover()
        return forest

    @staticmethod
    def _children(leaf):
        L, x, y, z = leaf
        return [(L + 1, 2 * x + ox, 2 * y + oy, 2 * z + oz)
                for oz in (0, 1) for oy in (0, 1) for ox in (0, 1)]

    def covering_leaf(self, level: int, pos):
        """Leaf of level <= `level` that contains block position `pos` of
        `level` (wrapped along periodic axes), or None if that position is
        split into finer leaves or lies beyond a non-periodic end."""
        dims = [r << level for r in self.R]
        if any(not self.periodic[a] and not 0 <= int(pos[a]) < dims[a] for a in range(3)):
            return None
        p = [int(pos[a]) % dims[a] for a in range(3)]
        for lv in range(level, -1, -1):
            s = level - lv
            cand = (lv, p[0] >> s, p[1] >> s, p[2] >> s)
            if cand in self.leaves:
                return cand
        return None

    def balance(self):
        """Split coarse leaves until no two touching leaves differ by > 1 level."""
        changed = True
        while changed:
            changed = False
            for leaf in sorted(self.leaves, key=lambda t: -t[0]):
                if leaf not in self.leaves:
                    continue
                L = leaf[0]
                if L < 2:
                    continue
                for d in NEIGHBOUR_OFFSETS:
                    q = (leaf[1] + d[0], leaf[2] + d[1], leaf[3] + d[2])
                    cov = self.covering_leaf(L, q)
                    if cov is not None and cov[0] < L - 1:
                        self.leaves.remove(cov)
                        self.leaves.update(self._children(cov))
                        changed = True
        self.max_level = max(leaf[0] for leaf in self.leaves)

    def is_balanced(self) -> bool:
        for leaf in self.leaves:
            for d in NEIGHBOUR_OFFSETS:
                q = (leaf[1] + d[0], leaf[2] + d[1], leaf[3] + d[2])
                cov = self.covering_leaf(leaf[0], q)
                if cov is not None and cov[0] < leaf[0] - 1:
                    return False
        return True

    def check_cover(self):
        """Every finest-level position is covered by exactly one leaf."""
        Lm = self.max_level
        dims = [r << Lm for r in self.R]
        count = np.zeros(dims, dtype=np.int32)
        for (L, x, y, z) in self.leaves:
            if any(v < 0 or v >= (r << L) for v, r in zip((x, y, z), self.R)):
                raise ValueError(f"leaf {(L, x, y, z)} outside the root grid")
            s = 1 << (Lm - L)
            count[x * s:(x + 1) * s, y * s:(y + 1) * s, z * s:(z + 1) * s] += 1
        if not np.all(count == 1):
            raise ValueError("leaves do not cover the domain exactly once")

    # -- queries ---------------------------------------------------------------
    def canonical_leaves(self):
        """Leaves sorted level-major, then by Morton index."""
        return sorted(self.leaves, key=lambda t: (t[0], morton_key(t[1], t[2], t[3])))

    def level_blocks(self, level: int) -> np.ndarray:
        """(B, 3) block positions of level `level` in canonical order."""
        pos = [t[1:] for t in self.canonical_leaves() if t[0] == level]
        return np.array(pos, dtype=np.int64).reshape(-1, 3)

    def num_cells(self, level: int) -> int:
        return len(self.level_blocks(level)) * self.n ** 3

    def coverage_grid(self, level: int) -> np.ndarray:
        """Per block position of `level`: the level of the leaf covering it if
        that leaf is on `level` or coarser, else FINER (= level + 1)."""
        dims = [r << level for r in self.R]
        grid = np.full(dims, -1, dtype=np.int16)
        for (L, x, y, z) in self.leaves:
            if L <= level:
                s = 1 << (level - L)
                grid[x * s:(x + 1) * s, y * s:(y + 1) * s, z * s:(z + 1) * s] = L
            else:
                s = L - level
                grid[x >> s, y >> s, z >> s] = level + 1
        assert np.all(grid >= 0)
        return grid
