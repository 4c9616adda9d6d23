"""Seeded synthetic workloads: forest shapes and initial fields.

This module holds no lattice Boltzmann arithmetic.  It only says which blocks
to refine and which (rho, u) field to start from; both the library and the
oracle receive the same values from here.

The paper measures on a lid-driven cavity and a vocal-fold geometry that need
walls and geometry data (section 5); the periodic synthetic grids below stand
in for them with the shapes used for the throughput runs: a 4-level
refinement around a sphere, a 4-level slab-plus-sphere grid of about 8.5 M
cells (the size of the paper's strong-scaling case, section 5.2), and a
5-level 16^3-block grid with decaying vortices.

Initial fields are given at cell centres in domain units [0, 1)^3: level-L
cell g has centre (g + 1/2) / (R n 2^L) along each axis.  Noise comes from
SplitMix64 (Steele, Lea & Flood, "Fast splittable pseudorandom number
generators", OOPSLA 2014) used as a counter-based generator: value k of
stream `seed` is mix64(seed + k * GOLDEN_GAMMA), mix64 being the generator's
published output function.
"""

from __future__ import annotations

import dataclasses
import math
from typing import Callable, Optional

import numpy as np

GOLDEN_GAMMA = np.uint64(0x9E3779B97F4A7C15)


def splitmix64(seed: int, counter: np.ndarray) -> np.ndarray:
    """k-th output (k = counter + 1) of the SplitMix64 stream with state `seed`."""
    with np.errstate(over="ignore"):
        z = np.uint64(seed & 0xFFFFFFFFFFFFFFFF) + (counter.astype(np.uint64) + np.uint64(1)) * GOLDEN_GAMMA
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
        z = z ^ (z >> np.uint64(31))
    return z


def uniform01(seed: int, counter: np.ndarray) -> np.ndarray:
    """Top 53 bits of the SplitMix64 output as a double in [0, 1)."""
    return (splitmix64(seed, counter) >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)


# ----------------------------------------------------------------------------
# forest shapes
# ----------------------------------------------------------------------------

def _box(R, level, x, y, z):
    """Domain-unit box [lo, hi] of block (level, x, y, z); the domain is the
    unit cube split into R^3 root blocks."""
    s = 1.0 / (R << level)
    return np.array([x, y, z], dtype=np.float64) * s, np.array([x + 1, y + 1, z + 1], dtype=np.float64) * s


def box_meets_ball(lo, hi, centre, radius) -> bool:
    """Closed box meets the open ball: distance from centre to box < radius."""
    c = np.asarray(centre, dtype=np.float64)
    d = np.maximum(np.maximum(lo - c, c - hi), 0.0)
    return float(np.sqrt((d * d).sum())) < radius


def box_meets_sphere(lo, hi, centre, radius) -> bool:
    """Closed box meets the sphere surface |x - c| = r."""
    c = np.asarray(centre, dtype=np.float64)
    d = np.maximum(np.maximum(lo - c, c - hi), 0.0)
    near = float(np.sqrt((d * d).sum()))
    far_corner = np.maximum(np.abs(lo - c), np.abs(hi - c))
    far = float(np.sqrt((far_corner * far_corner).sum()))
    return near <= radius <= far


def box_meets_plate(lo, hi, plo, phi) -> bool:
    """Closed box meets the closed axis-aligned box [plo, phi]."""
    return bool(np.all(lo <= np.asarray(phi)) and np.all(hi >= np.asarray(plo)))


@dataclasses.dataclass
class Workload:
    name: str
    roots: int                    # root blocks per axis (cube domain)
    n: int                        # cells per block edge
    max_level: int
    omega0: float
    refine: Optional[Callable[[int, int, int, int], bool]]
    field: str                    # "taylor_green" or "vortex_blobs"
    amplitude: float
    noise: float
    seed: int
    coarse_steps: int
    description: str = ""

    @property
    def R(self):
        return (self.roots, self.roots, self.roots)


def config_two_level(n: int = 16) -> Workload:
    """Periodic cube of 2x2x2 coarse blocks, the octant block at the origin
    refined once (8 fine blocks), omega0 = 1.6, Taylor-Green amplitude 0.01
    plus uniform noise of +-1e-4, rho = 1, 100 coarse steps."""
    def refine(level, x, y, z):
        return level == 0 and (x, y, z) == (0, 0, 0)
    return Workload("two_level_61k", 2, n, 1, 1.6, refine, "taylor_green", 0.01, 1e-4, 1, 100,
                    "2x2x2 roots of %d^3, octant refined once" % n)


def config_sphere(n: int = 32, roots: int = 4) -> Workload:
    """Periodic cube, levels 0..3, blocks meeting the surface of a central
    sphere of radius 0.25 refined at every level, omega0 = 1.9, Taylor-Green
    amplitude 0.02 plus noise +-1e-4, 50 coarse steps.  With 4^3 roots of
    32^3 cells this is 121.4 M cells in (0, 352, 984, 2368) blocks: every
    root touches the refined shell, so the 2:1 balance splits all of them."""
    R = roots

    def refine(level, x, y, z):
        lo, hi = _box(R, level, x, y, z)
        return box_meets_sphere(lo, hi, (0.5, 0.5, 0.5), 0.25)
    return Workload("sphere_shell_n%d_R%d" % (n, R), R, n, 3, 1.9, refine, "taylor_green", 0.02, 1e-4, 2, 50,
                    "%d^3 roots of %d^3 cells, sphere r=0.25 surface refined to level 3" % (R, n))


def config_uniform(n: int = 32, roots: int = 16) -> Workload:
    """Periodic cube of roots^3 blocks of n^3 cells on one level (no
    refinement): 512^3 cells with the defaults.  omega0 = 1.9, Taylor-Green
    amplitude 0.02 plus noise +-1e-4.  The grid for comparing two-buffer and
    in-place streaming."""
    return Workload("uniform_n%d_R%d" % (n, roots), roots, n, 0, 1.9, None, "taylor_green", 0.02, 1e-4, 3, 20,
                    "%d^3 roots of %d^3 cells, one level" % (roots, n))


def config_slab_sphere(n: int = 16, roots: int = 5) -> Workload:
    """About 8.5 M cells over 4 levels in 16^3 blocks: refinement along a
    thin plate and a small sphere surface (seeded positions), omega0 = 1.9."""
    R = roots
    rng = np.random.default_rng(4)
    plo = np.array([0.30, 0.28, 0.30]) + rng.uniform(0.0, 0.02, 3)
    phi = plo + np.array([0.40, 0.25, 0.0])
    centre = np.array([0.62, 0.58, 0.70]) + rng.uniform(-0.01, 0.01, 3)
    radius = 0.07

    def refine(level, x, y, z):
        lo, hi = _box(R, level, x, y, z)
        return box_meets_plate(lo, hi, plo, phi) or box_meets_sphere(lo, hi, centre, radius)
    return Workload("slab_sphere_n%d_R%d" % (n, R), R, n, 3, 1.9, refine, "taylor_green", 0.02, 1e-4, 4, 50,
                    "%d^3 roots of %d^3 cells, plate + sphere surface refined to level 3" % (R, n))


def vortex_blobs(seed: int = 5, count: int = 4, sigma: float = 0.06):
    """Seeded blob centres in [0.2, 0.8]^3 and unit rotation axes."""
    rng = np.random.default_rng(seed)
    centres = rng.uniform(0.2, 0.8, (count, 3))
    axes = rng.normal(size=(count, 3))
    axes /= np.linalg.norm(axes, axis=1, keepdims=True)
    return centres, axes, sigma


def config_vortices(n: int = 16, roots: int = 4, max_level: int = 4, seed: int = 5) -> Workload:
    """5 levels (0..4) of 16^3-cell blocks on 4^3 roots, 4 seeded Gaussian
    vortex blobs of peak velocity 0.05 (sigma = 0.06); the initial forest
    refines level-l blocks within (3 - 0.5 l) sigma of a blob centre.  The
    seed places the blobs."""
    R = roots
    centres, axes, sigma = vortex_blobs(seed)
    shifts = np.array(np.meshgrid([-1, 0, 1], [-1, 0, 1], [-1, 0, 1])).T.reshape(-1, 3)
    images = (centres[:, None, :] + shifts[None, :, :]).reshape(-1, 3)  # all periodic images

    def refine(level, x, y, z):
        lo, hi = _box(R, level, x, y, z)
        d = np.maximum(np.maximum(lo[None, :] - images, images - hi[None, :]), 0.0)
        return bool(np.any(np.sqrt((d * d).sum(1)) < (3.0 - 0.5 * level) * sigma))
    return Workload("vortices_n%d_R%d_L%d_s%d" % (n, R, max_level, seed), R, n, max_level, 1.9, refine, "vortex_blobs",
                    0.05, 0.0, seed, 500, "%d^3 roots of %d^3 cells, 4 vortex blobs, levels 0..%d" % (R, n, max_level))


# ----------------------------------------------------------------------------
# initial fields
# ----------------------------------------------------------------------------

def cell_centres(leaves, R, n):
    """Domain-unit centres (N, 3), levels (N,) and per-level global linear
    cell indices (N,) of all cells of `leaves`, in the given leaf order, x
    fastest inside a block."""
    R = np.asarray(R, dtype=np.int64)
    leaves = np.asarray(leaves, dtype=np.int64).reshape(-1, 4)
    i = np.arange(n)
    lz, ly, lx = np.meshgrid(i, i, i, indexing="ij")
    loc = np.stack([lx.ravel(), ly.ravel(), lz.ravel()], -1)  # x fastest
    levels = np.repeat(leaves[:, 0], n ** 3)
    g = (leaves[:, None, 1:] * n + loc[None, :, :]).reshape(-1, 3)
    dims = (R[None, :] * n) << levels[:, None]
    centres = (g + 0.5) / dims
    lin = g[:, 0] + dims[:, 0] * (g[:, 1] + dims[:, 1] * g[:, 2])
    return centres, levels, lin


def _blob_velocity(xyz, centres, axes, sigma, peak):
    """Sum of blobs u = peak sqrt(e) (a x r) / sigma exp(-|r|^2 / (2 sigma^2)),
    r = x - c at the nearest periodic image: divergence-free, speed `peak`
    at distance sigma from the axis in the blob's mid-plane."""
    u = np.zeros_like(xyz)
    for c, a in zip(centres, axes):
        r = xyz - c
        r -= np.round(r)
        ar = np.cross(a[None, :], r)
        g = np.exp(-(r * r).sum(1) / (2.0 * sigma * sigma))
        u += peak * math.sqrt(math.e) / sigma * ar * g[:, None]
    return u


def initial_field(w: Workload, leaves):
    """(rho, u) at every cell of `leaves` (given order)."""
    centres, levels, lin = cell_centres(leaves, w.R, w.n)
    N = len(centres)
    rho = np.ones(N)
    if w.field == "taylor_green":
        x, y, z = (2.0 * math.pi * centres[:, a] for a in range(3))
        u = np.zeros((N, 3))
        u[:, 0] = w.amplitude * np.sin(x) * np.cos(y) * np.cos(z)
        u[:, 1] = -w.amplitude * np.cos(x) * np.sin(y) * np.cos(z)
    elif w.field == "vortex_blobs":
        centres_b, axes_b, sigma = vortex_blobs(w.seed)
        u = _blob_velocity(centres, centres_b, axes_b, sigma, w.amplitude)
    elif w.field == "uniform":
        u = np.tile(np.asarray(w.amplitude, dtype=np.float64).reshape(1, 3), (N, 1))
    else:
        raise ValueError(w.field)
    if w.noise:
        base = (levels.astype(np.uint64) << np.uint64(44)) + lin.astype(np.uint64)
        for a in range(3):
            r = uniform01(w.seed, base * np.uint64(4) + np.uint64(a))
            u[:, a] += w.noise * (2.0 * r - 1.0)
    return rho, u
