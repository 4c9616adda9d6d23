"""The interpolated explosion on the GPU against the FP64 oracle's, through
the C ABI (lbm_set_explosion_interpolation; the limited linear
reconstruction inside the coarse parent, read from Algorithm 2's
interpolation of exploded values, section 4.1).

FP64 storage agrees with the oracle to rounding order (1e-12 after 6 steps)
on two- and three-level forests, with walls, and at the benchmark's block
size; FP32 and FP16 storage meet their targets; the launch shapes and the
schedules stay bitwise equal; switching the interpolation off restores the
homogeneous explosion bitwise.
"""

import numpy as np
import pytest

from oracle import Forest, RefinedOracle
from paper_1508_07982_amd import lbm
from paper_1508_07982_amd import workloads as W

pytestmark = pytest.mark.gpu


def say(msg):
    print(msg, flush=True)


def three(L, x, y, z):
    return (L == 0 and (x, y, z) == (1, 1, 1)) or (L == 1 and (x, y, z) == (3, 3, 2))


def corner(L, x, y, z):
    return (L == 0 and (x, y, z) == (0, 0, 0)) or (L == 1 and (x, y, z) == (0, 0, 1))


def octant(L, x, y, z):
    return L == 0 and (x, y, z) == (0, 0, 0)


PERIODIC = (True, True, True)
SPECS = {
    "two4": ((2, 2, 2), 4, 1, octant, PERIODIC),
    "two8": ((2, 2, 2), 8, 1, octant, PERIODIC),
    "three4": ((3, 3, 3), 4, 2, three, PERIODIC),
    "three8": ((3, 3, 3), 8, 2, three, PERIODIC),
    "corner_box8": ((3, 3, 3), 8, 2, corner, (False, False, False)),
    "octant_wall_y8": ((2, 2, 2), 8, 1, octant, (True, False, True)),
    "two32": ((2, 2, 2), 32, 1, octant, PERIODIC),
}


def make_pair(name, storage, omega0=1.45, seed=3, amp=0.03):
    R, n, Lmax, refine, periodic = SPECS[name]
    of = Forest.build(R, n, Lmax, refine, periodic=periodic)
    o = RefinedOracle(of, omega0, interpolation=True)
    g = lbm.Forest(R, n, Lmax, refine=refine, storage=storage, periodic=periodic)
    rng = np.random.default_rng(seed)
    N = o.total_cells()
    rho = 1.0 + 0.01 * rng.uniform(-1, 1, N)
    u = amp * rng.uniform(-1, 1, (N, 3))
    o.init_pdfs(rho, u)
    g.set_level_omega(omega0)
    g.set_explosion_interpolation(True)
    g.init_pdfs(rho, u)
    return o, g


@pytest.mark.parametrize("name", sorted(SPECS))
def test_fp64_interpolated_explosion_matches_oracle(name):
    say(f"fp64 interpolation {name}")
    o, g = make_pair(name, "f64")
    for step in range(6):
        o.step(1)
        g.step_coarse(1)
        r0, u0 = o.moments()
        r1, u1 = g.moments()
        assert np.max(np.abs(u1 - u0)) < 1e-12, step
        assert np.max(np.abs(r1 - r0)) < 1e-12, step
    M0, _ = o.mass()
    M1, _ = g.mass()
    assert abs(M1 - M0) / M0 < 1e-13
    g.close()


@pytest.mark.parametrize("storage, tol", [("f32", 1e-5), ("f16", 1e-3)])
def test_storage_forms_with_interpolation(storage, tol):
    w = W.config_two_level(16)
    say(f"two-level Taylor-Green, interpolated explosion, {storage}")
    of = Forest.build(w.R, w.n, w.max_level, w.refine)
    o = RefinedOracle(of, w.omega0, interpolation=True)
    rho, u = W.initial_field(w, of.canonical_leaves())
    o.init_pdfs(rho, u)
    g = lbm.Forest(w.R, w.n, w.max_level, refine=w.refine, storage=storage)
    g.set_level_omega(w.omega0)
    g.set_explosion_interpolation(True)
    g.init_pdfs(rho, u)
    M0, _ = g.mass()
    o.step(50)
    g.step_coarse(50)
    _, u0 = o.moments()
    _, u1 = g.moments()
    wts = o.level_weights()
    eu = np.sqrt(np.sum(wts[:, None] * (u1 - u0) ** 2) / np.sum(wts[:, None] * u0 ** 2))
    M1, _ = g.mass()
    say(f"  velocity rel-L2 {eu:.3e}, mass drift {abs(M1 - M0) / M0:.3e}")
    assert eu <= tol
    assert abs(M1 - M0) / M0 <= 1e-6
    g.close()


def _run(storage, interp, shape=None, schedule="graph", steps=3, toggle=False):
    R, n, Lmax, refine, periodic = SPECS["three8"]
    g = lbm.Forest(R, n, Lmax, refine=refine, storage=storage, periodic=periodic)
    N = g.num_cells()
    rng = np.random.default_rng(11)
    g.set_level_omega(1.7)
    g.init_pdfs(1.0 + 0.01 * rng.uniform(-1, 1, N), 0.03 * rng.uniform(-1, 1, (N, 3)))
    g.set_schedule(schedule)
    if shape is not None:
        for L in range(g.num_levels):
            g.set_level_launch(L, *shape)
    if toggle:  # the other setting first, then this one
        g.set_explosion_interpolation(not interp)
    g.set_explosion_interpolation(interp)
    g.step_coarse(steps)
    out = g.get_pdfs()
    g.close()
    return out


@pytest.mark.parametrize("storage", ["f32", "f16"])
def test_interpolation_launch_shapes_and_schedules_bitwise(storage):
    say(f"interpolation shapes {storage}")
    ref = _run(storage, True, schedule="direct")
    for shape in [(0, 1, 2), (2, 1, 1), (0, 0, 4)]:
        assert np.array_equal(_run(storage, True, shape=shape), ref), shape
    assert np.array_equal(_run(storage, True, schedule="per_block"), ref)
    plain = _run(storage, False)
    assert not np.array_equal(plain, ref)  # the interpolation changes the ghost values
    assert np.array_equal(_run(storage, False, toggle=True), plain)  # and switching it off restores eq. ctof
