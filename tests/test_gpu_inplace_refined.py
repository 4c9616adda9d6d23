"""In-place streaming of the finest level of a refined forest (lbm_set_inplace
on a forest with more than one level), through the C ABI.

The finest level keeps one PDF buffer; the values its second substep's
back-trace and the coarser level's coalescence need (what the fine cells send
into the fine ghost layers at t and t + 1/2, section 4) are saved by the
in-place launches, and the explosion reads the parent level's current state
(eq. ctof).  Results must equal the two-buffer path's bitwise on two- and
three-level forests, with walls (section 2.2) and TRT with a body force, in
every storage form; FP64 meets the oracle to rounding order; the finest
level's memory shrinks by two buffers less the saves.
"""

import numpy as np
import pytest

from oracle import Forest, RefinedOracle
from paper_1508_07982_amd import lbm

pytestmark = pytest.mark.gpu

PERIODIC = (True, True, True)
WALLS_Y = (True, False, True)


def say(msg):
    print(msg, flush=True)


def three(L, x, y, z):
    return (L == 0 and (x, y, z) == (1, 1, 1)) or (L == 1 and (x, y, z) == (3, 3, 2))


def corner(L, x, y, z):
    return (L == 0 and (x, y, z) == (0, 0, 0)) or (L == 1 and (x, y, z) == (0, 0, 1))


def octant(L, x, y, z):
    return L == 0 and (x, y, z) == (0, 0, 0)


def slab(L, x, y, z):
    return y == 0


SPECS = {
    "two4": ((2, 2, 2), 4, 1, octant, PERIODIC),
    "two8": ((2, 2, 2), 8, 1, octant, PERIODIC),
    "three8": ((3, 3, 3), 8, 2, three, PERIODIC),
    "two32": ((2, 2, 2), 32, 1, octant, PERIODIC),
    "octant_y8": ((2, 2, 2), 8, 1, octant, WALLS_Y),
    "corner_box8": ((3, 3, 3), 8, 2, corner, (False, False, False)),
    "slab2_y8": ((2, 3, 2), 8, 2, slab, WALLS_Y),
    "corner_x32": ((2, 2, 2), 32, 1, octant, (False, True, True)),
}
TRT = (3.0 / 16.0, (2e-5, 0.0, -1e-5))


def make(name, storage, inplace, omega=1.7, trt=None, seed=4):
    R, n, Lmax, refine, per = SPECS[name]
    g = lbm.Forest(R, n, Lmax, refine=refine, storage=storage, periodic=per)
    assert g.num_levels == Lmax + 1
    N = g.num_cells()
    rng = np.random.default_rng(seed)
    g.set_level_omega(omega)
    if trt is not None:
        g.set_trt_force(*trt)
    g.init_pdfs(1.0 + 0.01 * rng.uniform(-1, 1, N), 0.03 * rng.uniform(-1, 1, (N, 3)))
    if inplace:
        g.set_inplace(True)
    return g


def run_pair(name, storage, chunks, trt=None, schedule="graph"):
    a = make(name, storage, False, trt=trt)
    b = make(name, storage, True, trt=trt)
    b.set_schedule(schedule)
    for steps in chunks:
        a.step_coarse(steps)
        b.step_coarse(steps)
        ra, ua = a.moments()
        rb, ub = b.moments()
        assert np.array_equal(ra, rb) and np.array_equal(ua, ub), (name, storage, steps, np.max(np.abs(ua - ub)))
        assert np.array_equal(a.get_pdfs(), b.get_pdfs()), (name, storage, steps)
    ma, ja = a.mass()
    mb, jb = b.mass()
    assert ma == mb and np.array_equal(ja, jb)
    a.close()
    b.close()


@pytest.mark.parametrize("storage", ["f64", "f32", "f16"])
@pytest.mark.parametrize("name", sorted(SPECS))
def test_refined_inplace_equals_two_buffer_bitwise(name, storage):
    say(f"refined in place vs two-buffer {name} {storage}")
    run_pair(name, storage, [1, 1, 2, 3])


@pytest.mark.parametrize("storage", ["f64", "f16"])
@pytest.mark.parametrize("name", ["three8", "corner_box8"])
def test_refined_inplace_trt_force_bitwise(name, storage):
    say(f"refined in place TRT + force {name} {storage}")
    run_pair(name, storage, [2, 3], trt=TRT)


def test_refined_inplace_direct_schedule_bitwise():
    say("refined in place, direct launches")
    run_pair("three8", "f32", [3], schedule="direct")


@pytest.mark.parametrize("name", ["two8", "three8", "corner_box8"])
def test_fp64_refined_inplace_matches_oracle(name):
    R, n, Lmax, refine, per = SPECS[name]
    say(f"refined in place FP64 vs oracle {name}")
    of = Forest.build(R, n, Lmax, refine, periodic=per)
    o = RefinedOracle(of, 1.45)
    g = lbm.Forest(R, n, Lmax, refine=refine, storage="f64", periodic=per)
    N = g.num_cells()
    rng = np.random.default_rng(3)
    rho, u = 1.0 + 0.01 * rng.uniform(-1, 1, N), 0.03 * rng.uniform(-1, 1, (N, 3))
    o.init_pdfs(rho, u)
    g.set_level_omega(1.45)
    g.init_pdfs(rho, u)
    g.set_inplace(True)
    for step in range(5):
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


def test_refined_switching_off_and_on_continues_bitwise():
    say("refined in place on, off, on")
    a = make("three8", "f32", False)
    b = make("three8", "f32", True)
    a.step_coarse(7)
    b.step_coarse(2)
    b.set_inplace(False)
    b.step_coarse(3)
    b.set_inplace(True)
    b.step_coarse(2)
    assert np.array_equal(a.get_pdfs(), b.get_pdfs())
    a.close()
    b.close()


def test_refined_memory():
    R, n, Lmax, refine, per = SPECS["two32"]
    g = lbm.Forest(R, n, Lmax, refine=refine, storage="f32", periodic=per)
    N = g.num_cells()
    g.set_level_omega(1.5)
    g.init_pdfs(np.ones(N), np.zeros((N, 3)))
    g.synchronize()
    free0, _ = lbm.device_memory(0)
    g.set_inplace(True)
    free1, _ = lbm.device_memory(0)
    nf, nb = g.num_cells(1), g.num_blocks(1)
    freed = 2 * nf * 19 * 4 + nb * 10 * n * n * 4 - 3 * nb * 30 * n * n * 4
    say(f"  freed {free1 - free0} bytes, expected {freed}")
    assert free1 - free0 >= 0.95 * freed
    g.close()


def test_refined_refusals():
    g = make("two8", "f32", True)
    with pytest.raises(lbm.LBMError) as e:
        g.set_explosion_interpolation(True)
    assert e.value.name == "LBM_E_STATE"
    g.close()
    g = make("two8", "f32", False)
    g.set_explosion_interpolation(True)
    with pytest.raises(lbm.LBMError) as e:
        g.set_inplace(True)
    assert e.value.name == "LBM_E_STATE"
    g.close()
