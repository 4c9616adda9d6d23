"""Pins of the oracle's no-slip walls (section 2.2) on refined grids.

Walls sit on the non-periodic ends of the y axis, halfway between the last
fluid cell and the boundary cell beyond it (entire cells are fluid or
boundary, section 5).  Each pin fixes the result by something other than the
oracle's own tables:

* plane Poiseuille flow driven by a constant acceleration, TRT with
  Lambda_eo = 3/16 (section 2, eq. lambda_eo; section 5.1): the steady state
  is the parabola u_x = a y (H - y) / (2 nu) at the cell centres to rounding,
  on a uniform grid and with refinement at one wall, at both walls and in
  the middle (the paper reports L-infinity close to machine accuracy for
  exactly these layouts);
* bounce-back conserves mass exactly, so the volume-weighted mass of a
  random state stays constant on refined grids whose level interfaces are
  parallel to the walls; where an interface meets a wall, the fine ghost
  layers bounce packets back at the fine resolution (which moves them along
  the wall into the neighbouring coarse cell's children) while the coarse
  level bounces them back in place, so mass is kept only to the size of the
  non-equilibrium part (measured and bounded here);
* a hand-traced packet hitting a wall comes back reversed;
* an independent dense "virtual fine" formulation with walls (np.roll with
  reversal at the ends) agrees with the Algorithm 1 oracle.
"""

import numpy as np
import pytest

from oracle import Forest, RefinedOracle
from oracle import refined as orc

WALLS_Y = (True, False, True)
LAMBDA_EO = 3.0 / 16.0


def interior_coords(o, L):
    c = o.tables[L].cells
    return c.coords[:c.n_int]


def cell_y(o):
    """Cell-centre y of every interior cell in level-0 cell units."""
    return np.concatenate([(interior_coords(o, L)[:, 1] + 0.5) / 2 ** L for L in range(o.num_levels)])


# ----------------------------------------------------------------------------
# plane Poiseuille flow (section 5.1)
# ----------------------------------------------------------------------------

LAYOUTS = {
    "uniform": ((1, 2, 1), 0, None),
    "bottom_wall": ((1, 2, 1), 1, lambda L, x, y, z: L == 0 and y == 0),
    "both_walls": ((1, 3, 1), 1, lambda L, x, y, z: L == 0 and y != 1),
    "middle": ((1, 3, 1), 1, lambda L, x, y, z: L == 0 and y == 1),
    "bottom_two_levels": ((1, 2, 1), 2, lambda L, x, y, z: y == 0),
}


def poiseuille(layout, steps, n=8, lambda_e=1.0, a0=1e-6):
    R, Lmax, refine = LAYOUTS[layout]
    o = RefinedOracle(Forest.build(R, n, Lmax, refine, periodic=WALLS_Y), lambda_e, lambda_eo=LAMBDA_EO,
                      accel0=(a0, 0.0, 0.0))
    H = R[1] * n
    nu = (1.0 / lambda_e - 0.5) / 3.0  # level-0 lattice units (eq. viscosity_trt)
    y = cell_y(o)
    exact = a0 / (2.0 * nu) * y * (H - y)
    u = np.zeros((len(y), 3))
    u[:, 0] = exact
    o.init_pdfs(np.ones(len(y)), u)  # relaxes from the equilibrium of the parabola
    o.step(steps)
    _, got = o.moments()
    return o, got, exact


@pytest.mark.parametrize("layout", sorted(LAYOUTS))
def test_poiseuille_steady_state_to_rounding(layout):
    # the transient decays on the viscous time H^2 / nu (H = 16 or 24 level-0 cells)
    steps = 4000 if LAYOUTS[layout][0][1] == 2 else 7000
    o, u, exact = poiseuille(layout, steps)
    err = np.max(np.abs(u[:, 0] - exact)) / np.max(exact)
    assert err < 1e-9, err
    assert np.max(np.abs(u[:, 1:])) < 1e-14
    # flow rate per unit width: Q = (2/3) u_max H for the parabola (section 5.1);
    # the volume-weighted mean of the discrete profile over the channel
    w = np.concatenate([np.full(o.n_int(L), 8.0 ** -L) for L in range(o.num_levels)])
    R = LAYOUTS[layout][0]
    H = R[1] * o.n
    mean = np.sum(w * u[:, 0]) / np.sum(w)
    # cell-centred midpoint sum of the parabola: exact mean minus u''h^2/24 per level
    assert abs(mean - np.sum(w * exact) / np.sum(w)) < 1e-9 * np.max(exact)
    assert np.max(exact) == pytest.approx(1e-6 * H * H / 8.0 / (1.0 / 6.0), rel=2e-2)


def test_poiseuille_without_magic_parameter_is_not_exact():
    """Control: with SRT-like rates (Lambda_eo = 1/4 at lambda_e = 1) the
    bounce-back wall is not exactly halfway and the profile is off by a
    visible amount; the pin above is not met by any scheme."""
    R, Lmax, refine = LAYOUTS["uniform"]
    n, a0 = 8, 1e-6
    o = RefinedOracle(Forest.build(R, n, Lmax, refine, periodic=WALLS_Y), 1.6, lambda_eo=0.4,
                      accel0=(a0, 0.0, 0.0))
    nu = (1.0 / 1.6 - 0.5) / 3.0
    y = cell_y(o)
    exact = a0 / (2.0 * nu) * y * (R[1] * n - y)
    u = np.zeros((len(y), 3))
    u[:, 0] = exact
    o.init_pdfs(np.ones(len(y)), u)
    o.step(4000)
    _, got = o.moments()
    assert np.max(np.abs(got[:, 0] - exact)) / np.max(exact) > 1e-4


# ----------------------------------------------------------------------------
# conservation and hand traces
# ----------------------------------------------------------------------------

def three_level_walls(n=4):
    def refine(L, x, y, z):
        return (L == 0 and (x, y, z) == (1, 0, 1)) or (L == 1 and (x, y, z) == (3, 0, 2))
    return Forest.build((3, 3, 3), n, 2, refine, periodic=WALLS_Y)


def two_level_walls(n=4):
    return Forest.build((2, 2, 2), n, 1, lambda L, x, y, z: L == 0 and (x, y, z) == (0, 0, 0),
                        periodic=WALLS_Y)


def slab_walls(n=4, levels=1):
    """Roots (2, 3, 2); the bottom layer of roots refined, and for two levels
    the bottom layer of level-1 blocks once more: every level interface is a
    plane parallel to the walls."""
    return Forest.build((2, 3, 2), n, levels, lambda L, x, y, z: y == 0, periodic=WALLS_Y)


def _random_state_drift(f, steps=20, omega0=1.7):
    o = RefinedOracle(f, omega0)
    rng = np.random.default_rng(5)
    _, w = orc.lattice()
    for L in range(o.num_levels):
        o.set_interior_pdfs(L, w[None, :] * (1.0 + 0.2 * rng.uniform(-1, 1, (o.n_int(L), 19))))
    M0, _ = o.mass()
    o.step(steps)
    M1, _ = o.mass()
    return abs(M1 - M0) / M0


@pytest.mark.parametrize("levels", [1, 2])
def test_mass_conserved_with_walls_parallel_to_interfaces(levels):
    f = slab_walls(4, levels)
    assert f.max_level == levels
    assert _random_state_drift(f) < 1e-13


@pytest.mark.parametrize("make", [two_level_walls, three_level_walls])
def test_mass_where_an_interface_meets_a_wall(make):
    """The refined blocks touch the bottom wall, so level interfaces meet it
    at right angles: the drift is no longer roundoff but stays at the size
    of the non-equilibrium part (random PDFs of +-20 % here: about 1e-6 after
    20 steps; 2e-14 per coarse step for the smooth Poiseuille flow)."""
    f = make(4)
    assert any(leaf[2] == 0 for leaf in f.leaves if leaf[0] == f.max_level)
    drift = _random_state_drift(f)
    assert 1e-12 < drift < 1e-5


def test_packet_bounces_back_at_a_wall():
    """omega = 0: a packet in the cell next to the bottom wall moving down
    (direction 4 = (0, -1, 0)) is in the same cell one step later, moving up
    (direction 3); a diagonal one keeps its x motion: (1, -1, 0) -> (1, 1, 0)
    lands in the same cell (halfway bounce-back reverses the whole vector)."""
    f = Forest.build((2, 2, 2), 4, 0, None, periodic=WALLS_Y)
    o = RefinedOracle(f, 0.0)
    c = interior_coords(o, 0)
    X = int(np.nonzero(np.all(c == (3, 0, 2), axis=1))[0][0])
    e, _ = orc.lattice()
    down = int(np.nonzero(np.all(e == (0, -1, 0), axis=1))[0][0])
    up = int(np.nonzero(np.all(e == (0, 1, 0), axis=1))[0][0])
    diag = int(np.nonzero(np.all(e == (1, -1, 0), axis=1))[0][0])
    back = int(np.nonzero(np.all(e == (-1, 1, 0), axis=1))[0][0])
    f0 = np.zeros((o.n_int(0), 19))
    f0[X, down] = 1.0
    f0[X, diag] = 2.0
    o.set_interior_pdfs(0, f0)
    o.step(1)
    got = o.interior_pdfs(0)
    nz = {(int(i), int(a)): got[i, a] for i, a in zip(*np.nonzero(got))}
    assert nz == {(X, up): 1.0, (X, back): 2.0}


# ----------------------------------------------------------------------------
# brute-force virtual-fine formulation with walls
# ----------------------------------------------------------------------------

class VirtualFineWalls:
    """Every level keeps a dense copy of the whole domain at its resolution.
    Streaming is np.roll along every axis, after which the cells whose source
    lies beyond the y ends take their own value of the opposite direction.
    Coarse regions are exploded into the finer copy, only own cells collide,
    and an own coarse (cell, direction) takes the mean of its 8 children after
    the finer level's two substeps where the value arriving in a child has
    passed through the finer level's own cells (a child c with c - e or
    c - 2e an own finer cell), found here by shifting dense masks."""

    def __init__(self, forest, omega0):
        self.n = forest.n
        self.Lmax = forest.max_level
        self.omega = [orc.omega_level(omega0, L) for L in range(self.Lmax + 1)]
        self.e, _ = orc.lattice()
        self.opp = [int(np.nonzero(np.all(self.e == -self.e[a], axis=1))[0][0]) for a in range(19)]
        self.D, self.own, self.coarser = [], [], []
        for L in range(self.Lmax + 1):
            cov = forest.coverage_grid(L)
            cc = np.repeat(np.repeat(np.repeat(cov, self.n, 0), self.n, 1), self.n, 2)
            self.own.append(cc == L)
            self.coarser.append(cc < L)
            self.D.append(np.full(cc.shape + (19,), np.nan))

    def load(self, L, coords, f):
        self.D[L][coords[:, 0], coords[:, 1], coords[:, 2]] = f

    def _pull(self, arr, a, src_mask=None):
        """arr[..., a] streamed one step along e_a with bounce-back at the y ends."""
        e = [int(v) for v in self.e[a]]
        out = np.roll(arr[..., a], shift=e, axis=(0, 1, 2))
        if e[1] == 1:
            out[:, 0, :] = arr[:, 0, :, self.opp[a]]
        elif e[1] == -1:
            out[:, -1, :] = arr[:, -1, :, self.opp[a]]
        return out

    def _stream(self, L):
        old = self.D[L].copy()
        for a in range(19):
            self.D[L][..., a] = self._pull(old, a)

    def _collide(self, L):
        m = self.own[L]
        self.D[L][m] = orc.collide(self.D[L][m], self.omega[L])

    def _explode(self, L):
        up = np.repeat(np.repeat(np.repeat(self.D[L - 1], 2, 0), 2, 1), 2, 2)
        m = self.coarser[L]
        self.D[L][m] = up[m]

    def _through_fine(self, L, a):
        """Own coarse cells X whose (X, a) is coalesced: some child c has
        c - e_a or c - 2 e_a in an own cell of level L+1 (inside the domain)."""
        own = self.own[L + 1]
        e = [int(v) for v in self.e[a]]
        hit = np.zeros_like(own)
        for k in (1, 2):
            src = np.roll(own, shift=[k * v for v in e], axis=(0, 1, 2))  # src[c] = own[c - k e]
            if e[1] != 0:  # sources beyond the y ends are not own cells
                ny = own.shape[1]
                if e[1] > 0:
                    src[:, :k, :] = False
                else:
                    src[:, ny - k:, :] = False
            hit |= src
        s = hit.shape
        return hit.reshape(s[0] // 2, 2, s[1] // 2, 2, s[2] // 2, 2).any(axis=(1, 3, 5)) & self.own[L]

    def _coalesce(self, L):
        fine = self.D[L + 1]
        s = fine.shape
        mean = fine.reshape(s[0] // 2, 2, s[1] // 2, 2, s[2] // 2, 2, 19).mean(axis=(1, 3, 5))
        for a in range(19):
            m = self._through_fine(L, a)
            self.D[L][..., a][m] = mean[..., a][m]

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


@pytest.mark.parametrize("make, omega0", [(two_level_walls, 1.3), (three_level_walls, 1.7), (three_level_walls, 0.8)])
def test_matches_virtual_fine_brute_force_with_walls(make, omega0):
    forest = make(4)
    o = RefinedOracle(forest, omega0)
    vf = VirtualFineWalls(forest, omega0)
    rng = np.random.default_rng(23)
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
