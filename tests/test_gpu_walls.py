"""No-slip walls on the GPU against the FP64 oracle, through the C ABI.

The library's walls (section 2.2: halfway bounce-back on non-periodic axes,
applied in the fine ghost layers too, section 4.1) against the oracle's, on
forests whose refinement touches the walls: interfaces parallel to a wall
(slabs) and meeting it at right angles (octant and corner refinement), walls
along y, along x and z (the x-edge path of the sweep), and a closed box.
Then plane Poiseuille flow (section 5.1) with TRT, Lambda_eo = 3/16 and a
body force on the GPU: the parabola to rounding in FP64 storage, with
refinement at the walls and in the middle.

Tolerances: FP64 storage differs from the oracle only in rounding order
(1e-12 after 6 steps); FP32 / FP16 use the targets of those forms.
"""

import numpy as np
import pytest

from oracle import Forest, RefinedOracle
from paper_1508_07982_amd import lbm

pytestmark = pytest.mark.gpu

WALLS_Y = (True, False, True)


def say(msg):
    print(msg, flush=True)


def corner(L, x, y, z):
    return (L == 0 and (x, y, z) == (0, 0, 0)) or (L == 1 and (x, y, z) == (0, 0, 1))


def octant(L, x, y, z):
    return L == 0 and (x, y, z) == (0, 0, 0)


def slab(L, x, y, z):
    return y == 0


SPECS = {
    "octant_y4": ((2, 2, 2), 4, 1, octant, WALLS_Y),
    "octant_y8": ((2, 2, 2), 8, 1, octant, WALLS_Y),
    "corner_y4": ((3, 3, 3), 4, 2, corner, WALLS_Y),
    "corner_xz8": ((3, 3, 3), 8, 2, corner, (False, True, False)),
    "corner_box8": ((3, 3, 3), 8, 2, corner, (False, False, False)),
    "slab2_y8": ((2, 3, 2), 8, 2, slab, WALLS_Y),
    "slab1_y32": ((2, 2, 1), 32, 1, lambda L, x, y, z: L == 0 and y == 0, WALLS_Y),
    "corner_x32": ((2, 2, 2), 32, 1, octant, (False, True, True)),
}


def make_pair(name, storage, omega0=1.45, seed=3, amp=0.03, trt=None):
    R, n, Lmax, refine, periodic = SPECS[name]
    of = Forest.build(R, n, Lmax, refine, periodic=periodic)
    if trt is None:
        o = RefinedOracle(of, omega0)
    else:
        o = RefinedOracle(of, omega0, lambda_eo=trt[0], accel0=trt[1])
    g = lbm.Forest(R, n, Lmax, refine=refine, storage=storage, periodic=periodic)
    assert g.leaves().tolist() == [list(t) for t in of.canonical_leaves()]
    rng = np.random.default_rng(seed)
    N = o.total_cells()
    rho = 1.0 + 0.01 * rng.uniform(-1, 1, N)
    u = amp * rng.uniform(-1, 1, (N, 3))
    o.init_pdfs(rho, u)
    g.set_level_omega(omega0)
    if trt is not None:
        g.set_trt_force(*trt)
    g.init_pdfs(rho, u)
    return o, g


@pytest.mark.parametrize("name", sorted(SPECS))
def test_fp64_walls_match_oracle(name):
    say(f"fp64 walls {name}")
    o, g = make_pair(name, "f64")
    for step in range(6):
        o.step(1)
        g.step_coarse(1)
        r0, u0 = o.moments()
        r1, u1 = g.moments()
        assert np.max(np.abs(u1 - u0)) < 1e-12, step
        assert np.max(np.abs(r1 - r0)) < 1e-12, step
    M0, J0 = o.mass()
    M1, J1 = g.mass()
    assert abs(M1 - M0) / M0 < 1e-13
    assert np.max(np.abs(J1 - J0)) < 1e-10
    g.close()


@pytest.mark.parametrize("name", ["corner_y4", "corner_box8"])
def test_fp64_walls_trt_force_match_oracle(name):
    say(f"fp64 walls trt {name}")
    o, g = make_pair(name, "f64", omega0=1.2, trt=(3.0 / 16.0, (2e-5, 0.0, -1e-5)))
    o.step(6)
    g.step_coarse(6)
    r0, u0 = o.moments()
    r1, u1 = g.moments()
    assert np.max(np.abs(u1 - u0)) < 1e-12
    assert np.max(np.abs(r1 - r0)) < 1e-12
    g.close()


@pytest.mark.parametrize("storage, tol", [("f32", 1e-5), ("f16", 1e-3)])
@pytest.mark.parametrize("name", ["corner_box8", "slab1_y32"])
def test_storage_forms_with_walls(name, storage, tol):
    say(f"walls {name} {storage}")
    o, g = make_pair(name, storage, omega0=1.6, amp=0.02)
    M0, _ = g.mass()
    o.step(20)
    g.step_coarse(20)
    _, u0 = o.moments()
    _, u1 = g.moments()
    w = o.level_weights()
    eu = np.sqrt(np.sum(w[:, None] * (u1 - u0) ** 2) / np.sum(w[:, None] * u0 ** 2))
    M1, _ = g.mass()
    say(f"  velocity rel-L2 {eu:.3e}, mass drift {abs(M1 - M0) / M0:.3e}")
    assert eu <= tol
    g.close()


@pytest.mark.parametrize("shape", [(0, 1, 1), (0, 0, 4), (2, 1, 2), (4, 0, 1)])
def test_walls_launch_shapes_bitwise(shape):
    say(f"walls launch shape {shape}")
    R, n, Lmax, refine, periodic = SPECS["corner_x32"]
    outs = []
    for sh in (None, shape):
        g = lbm.Forest(R, n, Lmax, refine=refine, storage="f32", periodic=periodic)
        N = g.num_cells()
        rng = np.random.default_rng(9)
        g.set_level_omega(1.7)
        g.init_pdfs(1.0 + 0.01 * rng.uniform(-1, 1, N), 0.03 * rng.uniform(-1, 1, (N, 3)))
        if sh is not None:
            for L in range(g.num_levels):
                g.set_level_launch(L, *sh)
        g.step_coarse(3)
        outs.append(g.get_pdfs())
        g.close()
    assert np.array_equal(outs[0], outs[1])


POISEUILLE = {
    "uniform": ((1, 2, 1), 0, None),
    "bottom_wall": ((1, 2, 1), 1, lambda L, x, y, z: L == 0 and y == 0),
    "both_walls": ((1, 3, 1), 1, lambda L, x, y, z: L == 0 and y != 1),
    "middle": ((1, 3, 1), 1, lambda L, x, y, z: L == 0 and y == 1),
    "bottom_two_levels": ((1, 2, 1), 2, lambda L, x, y, z: y == 0),
}


@pytest.mark.parametrize("layout", sorted(POISEUILLE))
def test_poiseuille_on_the_gpu(layout):
    """Plane Poiseuille flow (section 5.1): walls at y = 0 and y = H, periodic
    x and z, TRT with Lambda_eo = 3/16, acceleration a along x scaled per level
    by eq. force_scaling; the steady profile is the parabola at the cell
    centres to rounding (FP64 storage), and FP32 storage follows it to the
    FP32 form's accuracy."""
    R, Lmax, refine = POISEUILLE[layout]
    n, a0, lam = 8, 1e-6, 1.0
    steps = 4000 if R[1] == 2 else 7000
    nu = (1.0 / lam - 0.5) / 3.0
    H = R[1] * n
    errs = {}
    for storage in ("f64", "f32"):
        g = lbm.Forest(R, n, Lmax, refine=refine, storage=storage, periodic=WALLS_Y)
        lv = g.leaves()
        y = np.concatenate([((lv[lv[:, 0] == L][:, 2:3] * n +
                              np.tile(np.repeat(np.arange(n), n), n)[None, :]).ravel() + 0.5) / 2 ** L
                            for L in range(g.num_levels)])
        exact = a0 / (2.0 * nu) * y * (H - y)
        u = np.zeros((len(y), 3))
        u[:, 0] = exact
        g.set_level_omega(lam)
        g.set_trt_force(3.0 / 16.0, (a0, 0.0, 0.0))
        g.init_pdfs(np.ones(len(y)), u)
        g.step_coarse(steps)
        _, got = g.moments()
        errs[storage] = np.max(np.abs(got[:, 0] - exact)) / np.max(exact)
        g.close()
    say(f"  Poiseuille {layout}: L-inf / u_max FP64 {errs['f64']:.3e}, FP32 {errs['f32']:.3e}")
    assert errs["f64"] < 1e-9
    assert errs["f32"] < 1e-3
