"""Single-level pins of the oracle.

* A forest with only level-0 blocks is a plain periodic D3Q19 SRT grid; the
  oracle's block-structured tables must reproduce a dense np.roll
  implementation of collide-then-stream (eq. collide, eq. stream).
* A shear wave decays at the rate nu k^2 with nu from eq. viscosity_srt
  (nu = (1/omega - 1/2)/3 in lattice units), up to an O(k^2) lattice error.
* A small-amplitude 3-D Taylor-Green field, u = A (sin kx cos ky cos kz,
  -cos kx sin ky cos kz, 0), is a Stokes mode with |k|^2 = 3 k^2: its
  kinetic energy decays as exp(-6 nu k^2 t), again up to O(k^2).
"""

import math

import numpy as np
import pytest

from oracle import Forest, RefinedOracle
from oracle import refined as orc


def _dense_index(oracle, L=0):
    c = oracle.tables[L].cells
    return c.coords[:c.n_int], tuple(int(v) for v in c.cdims)


@pytest.mark.parametrize("roots, n", [((2, 3, 2), 4), ((1, 2, 3), 8)])
def test_single_level_matches_np_roll(roots, n):
    forest = Forest.build(roots, n, 0, None)
    o = RefinedOracle(forest, 1.3)
    xyz, dims = _dense_index(o)
    rng = np.random.default_rng(7)
    _, w = orc.lattice()
    f0 = w[None, :] * (1.0 + 0.2 * rng.uniform(-1, 1, (len(xyz), 19)))
    o.set_interior_pdfs(0, f0)
    D = np.zeros(dims + (19,))
    D[xyz[:, 0], xyz[:, 1], xyz[:, 2]] = f0
    e, _ = orc.lattice()
    for _ in range(3):
        o.step(1)
        D = orc.collide(D.reshape(-1, 19), 1.3).reshape(D.shape)
        for a in range(19):
            D[..., a] = np.roll(D[..., a], shift=tuple(int(v) for v in e[a]), axis=(0, 1, 2))
        got = o.interior_pdfs(0)
        ref = D[xyz[:, 0], xyz[:, 1], xyz[:, 2]]
        assert np.max(np.abs(got - ref)) <= 1e-15


def _shear_wave_nu(N, omega, steps=(40, 240)):
    n = 8
    forest = Forest.build((1, N // n, 1), n, 0, None)
    o = RefinedOracle(forest, omega)
    xyz, dims = _dense_index(o)
    U = 1e-3
    k = 2 * math.pi / N
    u = np.zeros((len(xyz), 3))
    u[:, 0] = U * np.sin(k * (xyz[:, 1] + 0.5))
    o.init_pdfs(np.ones(len(xyz)), u)
    basis = np.sin(k * (xyz[:, 1] + 0.5))
    amp = {}
    t = 0
    for target in steps:
        o.step(target - t)
        t = target
        _, uu = o.moments()
        amp[t] = (uu[:, 0] @ basis) / (basis @ basis)
    t1, t2 = steps
    return -math.log(amp[t2] / amp[t1]) / (k * k * (t2 - t1))


def test_shear_wave_viscosity():
    omega = 1.6
    nu = (1.0 / omega - 0.5) / 3.0
    err16 = abs(_shear_wave_nu(16, omega) / nu - 1.0)
    err32 = abs(_shear_wave_nu(32, omega) / nu - 1.0)
    assert err32 < 5e-3
    # O(k^2) lattice error: halving k cuts it by about 4
    assert 3.5 < err16 / err32 < 4.5


def _taylor_green_rate(N, omega=1.6, A=1e-3, n=8):
    """Fitted energy decay rate / (6 nu k^2) on a single-level N^3 grid."""
    o = RefinedOracle(Forest.build((N // n,) * 3, n, 0, None), omega)
    xyz, _ = _dense_index(o)
    k = 2 * math.pi / N
    x, y, z = [(xyz[:, i] + 0.5) * k for i in range(3)]
    u = np.zeros((len(xyz), 3))
    u[:, 0] = A * np.sin(x) * np.cos(y) * np.cos(z)
    u[:, 1] = -A * np.cos(x) * np.sin(y) * np.cos(z)
    o.init_pdfs(np.ones(len(xyz)), u)
    steps = (N, 5 * N)
    energy, t = {}, 0
    for target in steps:
        o.step(target - t)
        t = target
        _, uu = o.moments()
        energy[target] = np.sum(uu ** 2)
    nu = (1.0 / omega - 0.5) / 3.0
    return -math.log(energy[steps[1]] / energy[steps[0]]) / (steps[1] - steps[0]) / (6 * nu * k * k)


def test_taylor_green_energy_decay():
    r16 = _taylor_green_rate(16)
    r32 = _taylor_green_rate(32)
    assert abs(r32 - 1.0) < 1.5e-2
    assert 3.5 < abs(r16 - 1.0) / abs(r32 - 1.0) < 4.7
