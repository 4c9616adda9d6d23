"""Pins of the oracle's interpolated explosion (section 4.1, Algorithm 2's
interpolation of the exploded values; the scheme is a reading, see
refined_oracle.c): a limited linear reconstruction of every PDF inside its
coarse parent.

* A field linear in position is reproduced exactly at the child centres
  (the limited slope of a linear field is its slope), with the slope of an
  axis set to 0 where a face neighbour of the parent is no coarse interior
  cell -- validity decided here from the forest's coverage, not from the
  oracle's tables.
* The 8 children of every parent average to its values (mass and momentum
  of the exploded cells equal the parent's).
* Zero slopes give eq. ctof: a uniform state explodes bitwise into its
  parents' values, and a uniform flow runs as with the homogeneous
  explosion up to rounding.
* Mass and momentum are conserved to roundoff over many steps.
* An independent dense formulation (slopes from np.roll on the coarse copy)
  agrees with the Algorithm 1 oracle.
* Against a uniformly fine run of the same flow, the interpolated
  explosion roughly halves the deviation of the refined run.
"""

import math

import numpy as np
import pytest

from oracle import Forest, RefinedOracle
from oracle import refined as orc


def three_level(n=4):
    def refine(L, x, y, z):
        return (L == 0 and (x, y, z) == (1, 1, 1)) or (L == 1 and (x, y, z) == (3, 3, 2))
    return Forest.build((3, 3, 3), n, 2, refine)


def two_level(n=4):
    return Forest.build((2, 2, 2), n, 1, lambda L, x, y, z: L == 0 and (x, y, z) == (0, 0, 0))


def interior_coords(o, L):
    c = o.tables[L].cells
    return c.coords[:c.n_int]


def coarse_interior(forest, L, cells):
    """Whether level-L cells (M, 3) are level-L interior cells (no wrap:
    callers keep away from the ends)."""
    cov = forest.coverage_grid(L)
    pos = cells // forest.n
    inside = np.all((pos >= 0) & (pos < np.array(cov.shape)), axis=1)
    out = np.zeros(len(cells), dtype=bool)
    out[inside] = cov[tuple(pos[inside].T)] == L
    return out


def test_linear_field_is_reproduced_at_the_child_centres():
    f = three_level(4)
    o = RefinedOracle(f, 1.5, interpolation=True)
    rng = np.random.default_rng(3)
    c0 = rng.uniform(0.01, 0.05, 19)
    grad = rng.uniform(-1e-3, 1e-3, (19, 3))
    xc = interior_coords(o, 0).astype(float) + 0.5  # level-0 cell centres
    o.set_interior_pdfs(0, c0[None, :] + xc @ grad.T)
    o.explode(1)
    cells, vals = o.exploded(1)
    par = cells // 2
    # exact linear value at the child centre, per axis only where both face
    # neighbours of the parent are level-0 interior cells
    want = c0[None, :] + (par + 0.5) @ grad.T
    for d in range(3):
        step = np.zeros(3, dtype=np.int64)
        step[d] = 1
        ok = coarse_interior(f, 0, par + step) & coarse_interior(f, 0, par - step)
        off = (cells[:, d] - 2 * par[:, d] - 0.5) * 0.5
        want += np.where(ok[:, None], off[:, None] * grad[None, :, d], 0.0)
    assert np.max(np.abs(vals - want)) < 1e-15
    full = np.ones(len(par), dtype=bool)
    for d in range(3):
        step = np.zeros(3, dtype=np.int64)
        step[d] = 1
        full &= coarse_interior(f, 0, par + step) & coarse_interior(f, 0, par - step)
    assert full.sum() > 100  # many parents away from the fine region use all three slopes


@pytest.mark.parametrize("make, L", [(two_level, 1), (three_level, 1), (three_level, 2)])
def test_children_average_to_the_parent(make, L):
    o = RefinedOracle(make(4), 1.5, interpolation=True)
    rng = np.random.default_rng(4)
    _, w = orc.lattice()
    for lv in range(o.num_levels):
        o.set_interior_pdfs(lv, w[None, :] * (1.0 + 0.3 * rng.uniform(-1, 1, (o.n_int(lv), 19))))
    o.explode(L)
    cells, vals = o.exploded(L)
    pc = interior_coords(o, L - 1)
    pf = o.interior_pdfs(L - 1)
    index = {tuple(c): i for i, c in enumerate(pc)}
    groups = {}
    for c, v in zip(cells, vals):
        groups.setdefault(tuple(c // 2), []).append(v)
    complete = 0
    for p, vs in groups.items():
        if len(vs) == 8:
            complete += 1
            assert np.max(np.abs(np.mean(vs, axis=0) - pf[index[p]])) < 1e-15
    assert complete > 10


@pytest.mark.parametrize("make", [two_level, three_level])
def test_zero_slopes_give_the_homogeneous_explosion(make):
    """A uniform state has zero slopes: every exploded cell takes its
    parent's values bitwise (eq. ctof).  Over several steps the 8-child sums
    of the coalescence round (3x is not exact in binary), slopes of rounding
    size appear, and the runs with and without interpolation stay within
    rounding of each other."""
    o = RefinedOracle(make(4), 1.7, interpolation=True)
    N = o.total_cells()
    o.init_pdfs(np.full(N, 1.01), np.tile([0.03, -0.02, 0.01], (N, 1)))
    for L in range(1, o.num_levels):
        o.explode(L)
        _, vals = o.exploded(L)
        assert np.array_equal(vals, np.broadcast_to(o.interior_pdfs(L - 1)[0], vals.shape))
    runs = []
    for interp in (False, True):
        o = RefinedOracle(make(4), 1.7, interpolation=interp)
        o.init_pdfs(np.full(N, 1.01), np.tile([0.03, -0.02, 0.01], (N, 1)))
        o.step(5)
        runs.append(np.concatenate([o.interior_pdfs(L) for L in range(o.num_levels)]))
    assert np.max(np.abs(runs[0] - runs[1])) < 1e-15


@pytest.mark.parametrize("make", [two_level, three_level])
def test_interpolation_conserves_mass_and_momentum(make):
    o = RefinedOracle(make(4), 1.6, interpolation=True)
    rng = np.random.default_rng(6)
    _, w = orc.lattice()
    for L in range(o.num_levels):
        o.set_interior_pdfs(L, w[None, :] * (1.0 + 0.2 * rng.uniform(-1, 1, (o.n_int(L), 19))))
    M0, J0 = o.mass()
    o.step(20)
    M1, J1 = o.mass()
    assert abs(M1 - M0) / M0 < 1e-13
    assert np.max(np.abs(J1 - J0)) < 1e-12


class VirtualFineInterp:
    """Dense copies of the whole domain per level (as in the homogeneous
    brute force), with the coarse copy exploded by a limited linear
    reconstruction: slopes from np.roll of the coarse copy, kept only where
    both face neighbours are own coarse cells."""

    def __init__(self, forest, omega0):
        self.n = forest.n
        self.Lmax = forest.max_level
        self.omega = [orc.omega_level(omega0, L) for L in range(self.Lmax + 1)]
        self.e, _ = orc.lattice()
        self.D, self.own, self.coarser = [], [], []
        for L in range(self.Lmax + 1):
            cov = forest.coverage_grid(L)
            cc = np.repeat(np.repeat(np.repeat(cov, self.n, 0), self.n, 1), self.n, 2)
            self.own.append(cc == L)
            self.coarser.append(cc < L)
            self.D.append(np.full(cc.shape + (19,), np.nan))

    def load(self, L, coords, f):
        self.D[L][coords[:, 0], coords[:, 1], coords[:, 2]] = f

    def _stream(self, L):
        for a in range(19):
            self.D[L][..., a] = np.roll(self.D[L][..., a], shift=tuple(int(v) for v in self.e[a]), axis=(0, 1, 2))

    def _collide(self, L):
        m = self.own[L]
        self.D[L][m] = orc.collide(self.D[L][m], self.omega[L])

    def _explode(self, L):
        C = np.nan_to_num(self.D[L - 1])
        own = self.own[L - 1]
        up = np.repeat(np.repeat(np.repeat(C, 2, 0), 2, 1), 2, 2)
        for d in range(3):
            plus = np.roll(C, -1, axis=d) - C
            minus = C - np.roll(C, 1, axis=d)
            ok = np.roll(own, -1, axis=d) & np.roll(own, 1, axis=d)
            g = np.where((plus * minus > 0) & ok[..., None], np.where(np.abs(plus) < np.abs(minus), plus, minus), 0.0)
            g = np.repeat(np.repeat(np.repeat(g, 2, 0), 2, 1), 2, 2)
            odd = (np.arange(g.shape[d]) % 2 - 0.5) * 0.5
            shape = [1, 1, 1, 1]
            shape[d] = -1
            up = up + odd.reshape(shape) * g
        m = self.coarser[L]
        self.D[L][m] = up[m]

    def _coalesce(self, L):
        fine = self.D[L + 1]
        s = fine.shape
        mean = fine.reshape(s[0] // 2, 2, s[1] // 2, 2, s[2] // 2, 2, 19).mean(axis=(1, 3, 5))
        m = self.own[L]
        self.D[L][m] = mean[m]

    def step_level(self, L):
        if L > 0:
            self._explode(L)
        for _ in range(1 if L == 0 else 2):
            self._collide(L)
            if L < self.Lmax:
                self.step_level(L + 1)
            self._stream(L)
            if L < self.Lmax:
                self._coalesce(L)


@pytest.mark.parametrize("make, omega0", [(two_level, 1.3), (three_level, 1.7)])
def test_matches_dense_formulation(make, omega0):
    forest = make(4)
    o = RefinedOracle(forest, omega0, interpolation=True)
    vf = VirtualFineInterp(forest, omega0)
    rng = np.random.default_rng(29)
    _, w = orc.lattice()
    for L in range(o.num_levels):
        f = w[None, :] * (1.0 + 0.3 * rng.uniform(-1, 1, (o.n_int(L), 19)))
        o.set_interior_pdfs(L, f)
        vf.load(L, interior_coords(o, L), f)
    for _ in range(3):
        o.step(1)
        vf.step_level(0)
        for L in range(o.num_levels):
            c = interior_coords(o, L)
            ref = vf.D[L][c[:, 0], c[:, 1], c[:, 2]]
            assert np.all(np.abs(o.interior_pdfs(L) - ref) < 1e-13)


def _shear_run(forest, interp, T=100, n=8, N0=16, U=1e-3, omega0=1.6):
    o = RefinedOracle(forest, omega0, interpolation=interp)
    k = 2 * math.pi / N0
    xy = np.concatenate([(interior_coords(o, L)[:, :2] + 0.5) / 2 ** L for L in range(o.num_levels)])
    u = np.zeros((len(xy), 3))
    u[:, 0] = U * np.sin(k * xy[:, 1])
    u[:, 1] = 0.5 * U * np.sin(k * xy[:, 0])
    o.init_pdfs(np.ones(len(xy)), u)
    o.step(T)
    return o


def test_interpolation_brings_the_refined_run_closer_to_the_fine_one():
    """A shear flow on 2x2x2 roots of 8^3 with one octant refined, against
    the same flow with every root refined (the uniformly fine solution),
    after 100 coarse steps: coarse cells compare with the mean of their
    fine children.  Measured: 3.4e-2 (eq. ctof) and 1.8e-2 (interpolated)."""
    n, N0 = 8, 16
    fine = _shear_run(Forest.build((2, 2, 2), n, 1, lambda L, x, y, z: L == 0), False)
    _, uf = fine.moments()
    cf = interior_coords(fine, 1)
    dense = np.zeros((2 * N0,) * 3 + (3,))
    dense[cf[:, 0], cf[:, 1], cf[:, 2]] = uf
    coarse_mean = dense.reshape(N0, 2, N0, 2, N0, 2, 3).mean(axis=(1, 3, 5))
    errs = {}
    for interp in (False, True):
        o = _shear_run(two_level(n), interp)
        _, u = o.moments()
        c0, c1 = interior_coords(o, 0), interior_coords(o, 1)
        ref = np.concatenate([coarse_mean[c0[:, 0], c0[:, 1], c0[:, 2]], dense[c1[:, 0], c1[:, 1], c1[:, 2]]])
        w = o.level_weights()
        errs[interp] = np.sqrt(np.sum(w[:, None] * (u - ref) ** 2) / np.sum(w[:, None] * ref ** 2))
    assert errs[True] < 0.7 * errs[False]
    assert errs[False] < 0.05
