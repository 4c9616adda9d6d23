"""Pins of the oracle's single-cell arithmetic (section 2, section 2.3).

Each check is fixed by mathematics the paper relies on, not by re-typing the
oracle's formulas: lattice isotropy of D3Q19, the exact moments of the
incompressible equilibrium, conservation by the collision, and the exact
level relaxation rates that keep the viscosity of eq. viscosity_srt equal on
all levels under acoustic scaling.
"""

from fractions import Fraction

import numpy as np
import pytest

from oracle import refined as orc


def test_lattice_isotropy():
    e, w = orc.lattice()
    e = e.astype(np.float64)
    assert len(w) == 19
    # every non-rest velocity is a face or edge neighbour, never a corner (section 2)
    norms = np.abs(e).sum(1)
    assert norms[0] == 0 and sorted(norms[1:].tolist()) == [1] * 6 + [2] * 12
    assert len({tuple(v) for v in e.astype(int)}) == 19
    # opposite directions adjacent
    for a in range(1, 19, 2):
        assert np.all(e[a] == -e[a + 1])
    d = np.eye(3)
    assert abs(w.sum() - 1.0) < 1e-15
    assert np.allclose(np.einsum("a,ai->i", w, e), 0.0, atol=1e-16)
    assert np.allclose(np.einsum("a,ai,aj->ij", w, e, e), d / 3.0, atol=1e-16)
    assert np.allclose(np.einsum("a,ai,aj,ak->ijk", w, e, e, e), 0.0, atol=1e-16)
    iso4 = (np.einsum("ij,kl->ijkl", d, d) + np.einsum("ik,jl->ijkl", d, d) + np.einsum("il,jk->ijkl", d, d)) / 9.0
    assert np.allclose(np.einsum("a,ai,aj,ak,al->ijkl", w, e, e, e, e), iso4, atol=1e-16)


def test_equilibrium_moments():
    rng = np.random.default_rng(11)
    N = 500
    rho = 1.0 + 0.2 * rng.standard_normal(N)
    u = 0.1 * rng.standard_normal((N, 3))
    feq = orc.equilibrium(rho, u)
    e, _ = orc.lattice()
    e = e.astype(np.float64)
    # zeroth and first moments (eq. fvelocity with rho0 = 1)
    assert np.allclose(feq.sum(1), rho, rtol=0, atol=1e-15)
    assert np.allclose(feq @ e, u, rtol=0, atol=1e-15)
    # second moment of the incompressible equilibrium: rho/3 delta + rho0 u u
    P = np.einsum("na,ai,aj->nij", feq, e, e)
    expect = rho[:, None, None] * np.eye(3)[None] / 3.0 + np.einsum("ni,nj->nij", u, u)
    assert np.allclose(P, expect, rtol=0, atol=1e-14)
    # rest state is the weight vector
    _, w = orc.lattice()
    assert np.allclose(orc.equilibrium(np.ones(1), np.zeros((1, 3)))[0], w, atol=0)


def test_moments_of_pdfs():
    rng = np.random.default_rng(12)
    f = rng.uniform(0.0, 0.1, (64, 19))
    rho, u = orc.moments(f)
    e, _ = orc.lattice()
    assert np.allclose(rho, f.sum(1))
    # brute-force first moment, component by component
    for i in range(64):
        for c in range(3):
            s = sum(f[i, a] * e[a, c] for a in range(19))
            assert abs(u[i, c] - s) < 1e-15


@pytest.mark.parametrize("omega", [0.0, 0.3, 1.0, 1.6, 1.99])
def test_collision_conserves_mass_and_momentum(omega):
    rng = np.random.default_rng(int(omega * 100))
    f = rng.uniform(0.0, 0.12, (200, 19))
    g = orc.collide(f, omega)
    r0, u0 = orc.moments(f)
    r1, u1 = orc.moments(g)
    assert np.allclose(r1, r0, rtol=0, atol=1e-15)
    assert np.allclose(u1, u0, rtol=0, atol=1e-15)


def test_collision_fixed_points():
    rng = np.random.default_rng(13)
    rho = 1.0 + 0.01 * rng.standard_normal(50)
    u = 0.05 * rng.standard_normal((50, 3))
    feq = orc.equilibrium(rho, u)
    # an equilibrium is invariant under collision for any omega
    for om in (0.5, 1.2, 1.9):
        assert np.allclose(orc.collide(feq, om), feq, rtol=0, atol=1e-15)
    # omega = 1 relaxes any state to the equilibrium of its own moments
    f = feq + 1e-3 * rng.standard_normal(feq.shape)
    r, v = orc.moments(f)
    assert np.allclose(orc.collide(f, 1.0), orc.equilibrium(r, v), rtol=0, atol=1e-15)
    # omega = 0 changes nothing
    assert np.array_equal(orc.collide(f, 0.0), f)


@pytest.mark.parametrize("omega0, expect", [
    (Fraction(8, 5), [Fraction(8, 5), Fraction(4, 3), Fraction(1), Fraction(2, 3), Fraction(2, 5)]),
    (Fraction(19, 10), [Fraction(19, 10), Fraction(38, 21), Fraction(38, 23), Fraction(38, 27), Fraction(38, 35)]),
])
def test_level_omega_exact(omega0, expect):
    got = [orc.omega_level(omega0, L) for L in range(5)]
    assert got == expect
    # eq. viscosity_srt with dt_L = dt_0 / 2^L: (1/omega_L - 1/2) / 2^L is the same on every level
    nu = {(1 / w - Fraction(1, 2)) / 2 ** L for L, w in enumerate(got)}
    assert len(nu) == 1
    # recursive form of eq. omega_scaling with K = L, L -> L + 1
    for L in range(4):
        assert got[L + 1] == 2 * got[L] / (4 - got[L])
    # float path agrees with the exact value
    for L in range(5):
        assert abs(orc.omega_level(float(omega0), L) - float(expect[L])) < 1e-15
