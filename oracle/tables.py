"""Per-level cell sets and index tables of the refined step (oracle side).

Definitions (section 2.3, section 4, section 4.3, section 4.4):

* Level L has cell index space G_L = Z^3 modulo (R * n * 2^L) (periodic).
  Leaf (L, b) covers cells n*b + [0, n)^3; I_L is the union of the cells of
  level-L leaves, region(L) the volume those leaves cover.
* parent(x) = floor(x / 2) in G_{L-1}; children(X) = {2X + o, o in {0,1}^3}.
* dist_L(x): periodic Chebyshev distance from x to I_L.
* H_L = {x in region(L-1) : dist_L(x) <= 2}: the two innermost ghost layers
  that are streamed but never collided (section 4: both stream and boundary
  handling include them, collision does not).
* E_L = {x in region(L-1) : dist_L(x) <= 4}: the four fine ghost layers
  filled from two coarse layers by the explosion (section 4, section 4.3):
  homogeneously, every cell takes its parent's 19 values (eq. ctof), or, as
  the interpolation of the exploded values that Algorithm 2 adds (section
  4.1), a limited linear reconstruction of each PDF inside the parent (see
  refined_oracle.c).
* Stream (pull form): for x in I_L u H_L and every direction a, the new value
  is the old value at x - e_a.  A source inside region(L+1) has no level-L
  value; such an (x, a) must be in the coalescence set.
* Walls (section 2.2): along a non-periodic axis every cell beyond the
  domain is a no-slip boundary cell.  The boundary treatment stores, after
  the collision, in the boundary cell the value the neighbouring fluid cell
  sent towards it, reversed; the fluid cell then pulls it unchanged.  So a
  pull of (x, a) from a boundary cell x - e_a takes x's own value of the
  opposite direction (halfway bounce-back: the wall lies midway between the
  cells).  Section 4.1 extends the boundary treatment to the two innermost
  ghost layers of fine blocks, so halo cells bounce back their own
  (exploded) values the same way.  Cells outside the domain are never
  interior, ghost or explosion cells and never take part in coalescence.
* Coalescence set P_L.  Section 4.4 sends only the PDFs "streaming into" the
  coarse block from the two innermost fine ghost layers, averaged over the 8
  fine cells of a coarse cell (eq. ftoc).  Reading used by default
  ("virtual"): (X, a) with X in I_L is coalesced if some child c of X has
  c - e_a or c - 2 e_a in I_{L+1}, i.e. if the value arriving in a child
  after the two fine substeps has passed through the fine interior.  The
  alternative ("literal"): X - e_a lies in region(L+1).  They differ only
  for diagonal directions that graze a convex edge of the fine region.

Index layout of the stored cells S_L = I_L u E_L:
  [0, n_int)             I_L, canonical order (blocks canonical, x fastest)
  [n_int, n_int + n_h)   H_L
  [n_int + n_h, n_store) E_L \\ H_L
"""

from __future__ import annotations

import numpy as np

from .forest import NEIGHBOUR_OFFSETS

WALL = -2  # pull-table code: the source lies beyond a non-periodic end (bounce-back)


def d3q19_velocities() -> np.ndarray:
    """Discrete velocities of D3Q19 (section 2, Qian et al.): the rest
    vector, the 6 face neighbours and the 12 edge neighbours.  Index order
    is a data convention: opposite directions are adjacent (a, a+1 for odd a)."""
    return np.array([
        (0, 0, 0),
        (1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1),
        (1, 1, 0), (-1, -1, 0), (1, -1, 0), (-1, 1, 0),
        (1, 0, 1), (-1, 0, -1), (1, 0, -1), (-1, 0, 1),
        (0, 1, 1), (0, -1, -1), (0, 1, -1), (0, -1, 1),
    ], dtype=np.int64)


E = d3q19_velocities()


def _axis_dist(n: int, d: int) -> np.ndarray:
    """Chebyshev distance along one axis from local coordinate i of a block
    to the adjacent block at offset d (-1, 0, +1) on the same level."""
    i = np.arange(n)
    if d == 1:
        return n - i
    if d == -1:
        return i + 1
    return np.zeros(n, dtype=np.int64)


def _pattern_distance(n: int, offsets) -> np.ndarray:
    """Distance of every cell of a block to the union of its neighbour blocks
    at `offsets`; array indexed [z, y, x] (ravel gives x fastest)."""
    dist = np.full((n, n, n), 1 << 30, dtype=np.int64)
    for d in offsets:
        dx, dy, dz = _axis_dist(n, d[0]), _axis_dist(n, d[1]), _axis_dist(n, d[2])
        box = np.maximum(np.maximum(dz[:, None, None], dy[None, :, None]), dx[None, None, :])
        dist = np.minimum(dist, box)
    return dist


def _shift(arr: np.ndarray, d, periodic) -> np.ndarray:
    """arr shifted so that out[p] = arr[p + d]; along a non-periodic axis the
    entries beyond the end are False (no block there)."""
    out = np.roll(arr, shift=(-d[0], -d[1], -d[2]), axis=(0, 1, 2))
    for ax in range(3):
        if not periodic[ax] and d[ax] != 0:
            sl = [slice(None)] * 3
            sl[ax] = slice(-1, None) if d[ax] > 0 else slice(0, 1)
            out[tuple(sl)] = False
    return out


class LevelCells:
    """Cell sets I_L, H_L, E_L of one level and a coordinate -> index map."""

    def __init__(self, forest, L: int):
        n = forest.n
        self.L, self.n = L, n
        self.periodic = tuple(getattr(forest, "periodic", (True, True, True)))
        self.n3 = n ** 3
        self.pdims = np.array([r << L for r in forest.R], dtype=np.int64)
        self.cdims = self.pdims * n
        self.cov = forest.coverage_grid(L)
        self.blocks = forest.level_blocks(L)
        self.finer = L + 1
        nb = len(self.blocks)
        self.real_slot = np.full(self.cov.shape, -1, dtype=np.int64)
        if nb:
            self.real_slot[tuple(self.blocks.T)] = np.arange(nb)
        self.n_int = nb * self.n3

        # ghost positions: in region(L-1) and touching a level-L block
        is_real = self.cov == L
        touch = np.zeros(self.cov.shape, dtype=bool)
        pattern = np.zeros(self.cov.shape, dtype=np.int64)
        for bit, d in enumerate(NEIGHBOUR_OFFSETS):
            # neighbour at offset d of position p is real  <=> shift by -d
            nbr_real = _shift(is_real, d, self.periodic)
            touch |= nbr_real
            pattern |= nbr_real.astype(np.int64) << bit
        cand = touch & ~is_real & (self.cov < L)
        if np.any(cand & (self.cov < L - 1)):
            raise AssertionError("2:1 balance violated: level-%d block touches level <= %d" % (L, L - 2))
        self.ghost_pos = np.argwhere(cand).astype(np.int64)
        # order ghosts by linear position (x fastest) for determinism
        lin = self.ghost_pos[:, 0] + self.pdims[0] * (self.ghost_pos[:, 1] + self.pdims[1] * self.ghost_pos[:, 2])
        self.ghost_pos = self.ghost_pos[np.argsort(lin, kind="stable")]
        ng = len(self.ghost_pos)
        self.ghost_slot = np.full(self.cov.shape, -1, dtype=np.int64)
        if ng:
            self.ghost_slot[tuple(self.ghost_pos.T)] = np.arange(ng)

        # per-ghost cell distance to I_L (only 26-neighbour blocks can be
        # within 4 cells when n >= 4)
        gdist = np.empty((ng, self.n3), dtype=np.int64)
        pats = pattern[tuple(self.ghost_pos.T)] if ng else np.zeros(0, dtype=np.int64)
        for p in np.unique(pats):
            offs = [d for bit, d in enumerate(NEIGHBOUR_OFFSETS) if (p >> bit) & 1]
            gdist[pats == p] = _pattern_distance(n, offs).ravel()
        self.ghost_index = np.full((ng, self.n3), -1, dtype=np.int64)
        h_mask = gdist <= 2
        e_mask = (gdist > 2) & (gdist <= 4)
        self.n_h = int(h_mask.sum())
        self.n_far = int(e_mask.sum())
        self.ghost_index[h_mask] = self.n_int + np.arange(self.n_h)
        self.ghost_index[e_mask] = self.n_int + self.n_h + np.arange(self.n_far)
        self.n_live = self.n_int + self.n_h
        self.n_store = self.n_live + self.n_far

        # coordinates of every stored cell, in index order
        loc = np.stack(np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij"), -1)
        loc = loc.transpose(2, 1, 0, 3).reshape(-1, 3)  # x fastest: (i, j, k) per local index
        self.local_xyz = loc
        coords = np.empty((self.n_store, 3), dtype=np.int64)
        if nb:
            coords[:self.n_int] = (self.blocks[:, None, :] * n + loc[None, :, :]).reshape(-1, 3)
        if ng:
            gall = (self.ghost_pos[:, None, :] * n + loc[None, :, :])
            coords[self.n_int:self.n_live] = gall[h_mask]
            coords[self.n_live:] = gall[e_mask]
        self.coords = coords

    def outside(self, g: np.ndarray) -> np.ndarray:
        """Whether global level-L cells g lie beyond a non-periodic end."""
        out = np.zeros(len(g), dtype=bool)
        for ax in range(3):
            if not self.periodic[ax]:
                out |= (g[:, ax] < 0) | (g[:, ax] >= self.cdims[ax])
        return out

    def lookup(self, g: np.ndarray):
        """Index in S_L of global level-L cells g (M, 3), -1 if not stored,
        WALL beyond a non-periodic end; and whether each cell lies in
        region(L+1)."""
        wall = self.outside(g)
        g = np.mod(g, self.cdims)
        pos = g // self.n
        loc = g % self.n
        lin = loc[:, 0] + self.n * (loc[:, 1] + self.n * loc[:, 2])
        pos_t = (pos[:, 0], pos[:, 1], pos[:, 2])
        rs = self.real_slot[pos_t]
        gs = self.ghost_slot[pos_t]
        idx = np.full(len(g), -1, dtype=np.int64)
        m = rs >= 0
        idx[m] = rs[m] * self.n3 + lin[m]
        m2 = (~m) & (gs >= 0)
        idx[m2] = self.ghost_index[gs[m2], lin[m2]]
        fine = (self.cov[pos_t] == self.finer) & ~wall
        idx[wall] = WALL
        return idx, fine

    def in_interior(self, g: np.ndarray) -> np.ndarray:
        """Whether global level-L cells g lie in I_L."""
        wall = self.outside(g)
        g = np.mod(g, self.cdims)
        pos = g // self.n
        return (self.cov[(pos[:, 0], pos[:, 1], pos[:, 2])] == self.L) & ~wall


class LevelTables:
    """Index tables of one level, ready for the C loops."""

    def __init__(self, cells, coarser, finer, coalescence: str = "virtual"):
        L = cells.L
        self.cells = cells
        # stream: pull source of every live cell and direction
        live = cells.coords[:cells.n_live]
        pull = np.empty((cells.n_live, 19), dtype=np.int64)
        for a in range(19):
            idx, fine = cells.lookup(live - E[a])
            bad = (idx == -1) & ~(fine & (np.arange(cells.n_live) < cells.n_int))
            if np.any(bad):
                raise AssertionError(f"level {L}: stream source missing for direction {a}")
            pull[:, a] = idx
        self.pull = pull.astype(np.int32)

        # explosion: parent (in I_{L-1}) of every E_L cell; for the
        # interpolated explosion also the cell's octant inside its parent and
        # the parent's 6 face neighbours (+x, -x, +y, -y, +z, -z) in I_{L-1},
        # -1 where that neighbour is no level-(L-1) interior cell
        far = cells.coords[cells.n_int:]
        if len(far):
            par = far // 2
            idx, _ = coarser.lookup(par)
            if np.any(idx < 0) or np.any(idx >= coarser.n_int):
                raise AssertionError(f"level {L}: explosion parent not in I_{L-1}")
            self.expl_src = idx.astype(np.int32)
            self.expl_oct = (far - 2 * par).astype(np.int32)
            nbr = np.empty((len(far), 6), dtype=np.int64)
            for d in range(3):
                for side, sgn in ((0, 1), (1, -1)):
                    step = np.zeros(3, dtype=np.int64)
                    step[d] = sgn
                    q, _ = coarser.lookup(par + step)
                    nbr[:, 2 * d + side] = np.where((q >= 0) & (q < coarser.n_int), q, -1)
            self.expl_nbr = nbr.astype(np.int32)
        else:
            self.expl_src = np.zeros(0, dtype=np.int32)
            self.expl_oct = np.zeros((0, 3), dtype=np.int32)
            self.expl_nbr = np.zeros((0, 6), dtype=np.int32)

        # coalescence pairs
        cc, cd, ch = [], [], []
        if finer is not None and cells.n_int:
            n = cells.n
            nbr_fine = np.zeros(len(cells.blocks), dtype=bool)
            for d in NEIGHBOUR_OFFSETS:
                p = np.mod(cells.blocks + np.array(d), cells.pdims)
                nbr_fine |= cells.cov[(p[:, 0], p[:, 1], p[:, 2])] == cells.finer
            cand_blocks = np.nonzero(nbr_fine)[0]
            loc = cells.local_xyz
            shell = np.nonzero(np.any((loc == 0) | (loc == n - 1), axis=1))[0]
            X_idx = (cand_blocks[:, None] * cells.n3 + shell[None, :]).ravel()
            X = cells.coords[X_idx] if len(X_idx) else np.zeros((0, 3), dtype=np.int64)
            offs = np.array([(ox, oy, oz) for oz in (0, 1) for oy in (0, 1) for ox in (0, 1)])
            for a in range(1, 19):
                if coalescence == "virtual":
                    hit = np.zeros(len(X), dtype=bool)
                    for o in offs:
                        c = 2 * X + o
                        hit |= finer.in_interior(c - E[a]) | finer.in_interior(c - 2 * E[a])
                elif coalescence == "literal":
                    _, hit = cells.lookup(X - E[a])
                else:
                    raise ValueError(coalescence)
                sel = np.nonzero(hit)[0]
                if not len(sel):
                    continue
                kids = np.empty((len(sel), 8), dtype=np.int64)
                for j, o in enumerate(offs):
                    idx, _ = finer.lookup(2 * X[sel] + o)
                    if np.any(idx < finer.n_int) or np.any(idx >= finer.n_live):
                        raise AssertionError(f"level {L}: coalescence child outside H_{L+1}")
                    kids[:, j] = idx
                cc.append(X_idx[sel])
                cd.append(np.full(len(sel), a))
                ch.append(kids)
        if cc:
            self.coal_cell = np.concatenate(cc).astype(np.int32)
            self.coal_dir = np.concatenate(cd).astype(np.int32)
            self.coal_child = np.concatenate(ch).astype(np.int32)
        else:
            self.coal_cell = np.zeros(0, dtype=np.int32)
            self.coal_dir = np.zeros(0, dtype=np.int32)
            self.coal_child = np.zeros((0, 8), dtype=np.int32)

        # every interior pull from region(L+1) must be overwritten by coalescence
        missing = np.argwhere(self.pull[:cells.n_int] == -1)
        if len(missing):
            have = set(zip(self.coal_cell.tolist(), self.coal_dir.tolist()))
            for x, a in missing.tolist():
                if (x, a) not in have:
                    raise AssertionError(f"level {L}: cell {x} dir {a} pulls from the fine region but is not coalesced")


def build_tables(forest, coalescence: str = "virtual"):
    cells = [LevelCells(forest, L) for L in range(forest.max_level + 1)]
    tabs = []
    for L, c in enumerate(cells):
        coarser = cells[L - 1] if L > 0 else None
        finer = cells[L + 1] if L < forest.max_level else None
        tabs.append(LevelTables(c, coarser, finer, coalescence))
    return tabs
