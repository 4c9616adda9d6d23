"""Pins of the oracle's TRT collision and body force (section 2: TRT model,
external forces; section 2.3: eq. omega_scaling_0 for lambda_e, eq.
lambda_eo / lambda_oL for lambda_o, eq. force_scaling for the acceleration).

* lambda_o,L from eq. lambda_oL keeps Lambda_eo of eq. lambda_eo exactly on
  every level (rational arithmetic), and lambda_e = 8/5, Lambda = 3/16 gives
  lambda_o = 1/2.
* With lambda_o = lambda_e and no force the TRT operator is the SRT one.
* The even part of f - f^eq relaxes by (1 - lambda_e) whatever lambda_o is,
  the odd part by (1 - lambda_o) whatever lambda_e is (a swap of the two
  rates fails both).
* The force term adds no mass and exactly rho0 a of momentum per collision.
* On a three-level grid the volume-weighted momentum grows by exactly
  rho0 a_0 V per coarse step (level L takes 2^L steps with a_0 / 2^L), mass
  is unchanged.
* A shear wave decays with the viscosity of lambda_e (eq. viscosity_trt).
"""

import math
from fractions import Fraction

import numpy as np
import pytest

from oracle import Forest, RefinedOracle, collide, collide_trt, lambda_o_level, omega_level
from oracle import refined as orc


def test_lambda_o_keeps_lambda_eo_on_every_level():
    le0, lam = Fraction(8, 5), Fraction(3, 16)
    assert lambda_o_level(le0, lam) == Fraction(1, 2)
    for L in range(6):
        le = omega_level(le0, L)
        lo = lambda_o_level(le, lam)
        assert (1 / le - Fraction(1, 2)) * (1 / lo - Fraction(1, 2)) == lam
        assert 0 < lo < 2


def _random_state(n, seed):
    rng = np.random.default_rng(seed)
    _, w = orc.lattice()
    return w[None, :] * (1.0 + 0.3 * rng.uniform(-1, 1, (n, 19)))


def test_trt_with_equal_rates_is_srt():
    f = _random_state(50, 1)
    for om in (0.7, 1.3, 1.9):
        assert np.max(np.abs(collide_trt(f, om, om) - collide(f, om))) < 1e-15


def _opposite():
    e, _ = orc.lattice()
    return np.array([next(b for b in range(19) if np.array_equal(e[b], -e[a])) for a in range(19)])


def test_even_and_odd_parts_relax_with_their_own_rates():
    e, w = orc.lattice()
    opp = _opposite()
    rng = np.random.default_rng(2)
    n = 40
    rho = 1.0 + 0.05 * rng.uniform(-1, 1, n)
    u = 0.05 * rng.uniform(-1, 1, (n, 3))
    feq = orc.equilibrium(rho, u)
    g = rng.uniform(-1, 1, (n, 19)) * w[None, :] * 0.1
    even = 0.5 * (g + g[:, opp])
    even -= (even.sum(1, keepdims=True) / 1.0) * w[None, :]       # no mass (w sums to 1)
    odd = 0.5 * (g - g[:, opp])
    mom = odd @ e.astype(float)
    odd -= 3.0 * w[None, :] * (mom @ e.T.astype(float))          # no momentum
    assert np.max(np.abs(even.sum(1))) < 1e-15 and np.max(np.abs(odd @ e)) < 1e-15
    for lo in (0.3, 1.1):
        out = collide_trt(feq + even, 1.4, lo)
        assert np.max(np.abs(out - (feq + (1 - 1.4) * even))) < 1e-15
    for le in (0.6, 1.7):
        out = collide_trt(feq + odd, le, 0.9)
        assert np.max(np.abs(out - (feq + (1 - 0.9) * odd))) < 1e-15


def test_force_adds_no_mass_and_rho0_a_of_momentum():
    e, _ = orc.lattice()
    f = _random_state(30, 3)
    a = np.array([2e-4, -1e-4, 5e-5])
    out = collide_trt(f, 1.2, 0.7, a)
    r0, u0 = orc.moments(f)
    r1, u1 = orc.moments(out)
    assert np.max(np.abs(r1 - r0)) < 1e-15
    assert np.max(np.abs(u1 - u0 - a[None, :])) < 1e-15


def _three_level():
    def refine(L, x, y, z):
        return (L == 0 and (x, y, z) == (1, 1, 1)) or (L == 1 and (x, y, z) == (3, 3, 2))
    return Forest.build((3, 3, 3), 4, 2, refine)


def test_refined_grid_momentum_grows_by_a0_per_coarse_step():
    forest = _three_level()
    a0 = np.array([1e-4, -2e-5, 3e-5])
    o = RefinedOracle(forest, 1.6, lambda_eo=3 / 16, accel0=a0)
    rng = np.random.default_rng(4)
    N = o.total_cells()
    o.init_pdfs(1.0 + 0.01 * rng.uniform(-1, 1, N), 0.03 * rng.uniform(-1, 1, (N, 3)))
    V = float(o.level_weights().sum())
    M0, J0 = o.mass()
    for k in range(1, 4):
        o.step(1)
        M, J = o.mass()
        assert abs(M - M0) < 1e-11
        assert np.max(np.abs(J - J0 - k * V * a0)) < 1e-11, k
    # the same without the force: momentum is conserved, so the growth is the force's
    o2 = RefinedOracle(forest, 1.6, lambda_eo=3 / 16)
    o2.init_pdfs(1.0 + 0.01 * rng.uniform(-1, 1, N), 0.03 * rng.uniform(-1, 1, (N, 3)))
    _, J0 = o2.mass()
    o2.step(2)
    assert np.max(np.abs(o2.mass()[1] - J0)) < 1e-11


def test_trt_shear_wave_decays_with_the_even_rate():
    N, n = 32, 8
    le = 1.6
    forest = Forest.build((1, N // n, 1), n, 0, None)
    o = RefinedOracle(forest, le, lambda_eo=3 / 16)
    assert abs(o.lambda_o[0] - 0.5) < 1e-15
    c = o.tables[0].cells
    xyz = c.coords[:c.n_int]
    k = 2 * math.pi / N
    u = np.zeros((len(xyz), 3))
    u[:, 0] = 1e-3 * np.sin(k * (xyz[:, 1] + 0.5))
    o.init_pdfs(np.ones(len(xyz)), u)
    basis = np.sin(k * (xyz[:, 1] + 0.5))
    amp = {}
    t = 0
    for target in (40, 240):
        o.step(target - t)
        t = target
        amp[t] = (o.moments()[1][:, 0] @ basis) / (basis @ basis)
    nu_meas = -math.log(amp[240] / amp[40]) / (k * k * 200)
    nu_even = (1 / le - 0.5) / 3
    assert abs(nu_meas / nu_even - 1) < 1e-2
