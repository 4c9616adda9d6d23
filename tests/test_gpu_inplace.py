"""In-place (AA pattern) streaming on the GPU, through the C ABI
(lbm_set_inplace).

Section 4.1 keeps two grids and names the AA pattern as the in-place
alternative.  This file covers forests whose leaves all lie on level 0
(test_gpu_inplace_refined.py the finest level of refined forests).  Results
must equal the two-buffer path's bitwise, for every
storage form, SRT and TRT with a body force, periodic axes and no-slip walls
(section 2.2), whatever layout the buffer holds when a query reads it (odd
and even step counts); FP64 storage must meet the FP64 oracle to rounding
order.  The PDF memory of the level halves.
"""

import numpy as np
import pytest

from oracle import Forest, RefinedOracle
from paper_1508_07982_amd import lbm

pytestmark = pytest.mark.gpu


def say(msg):
    print(msg, flush=True)


SPECS = {
    "periodic4": ((2, 2, 2), 4, (True, True, True)),
    "periodic8_x_self": ((1, 2, 2), 8, (True, True, True)),  # a block is its own x neighbour
    "walls_y16": ((2, 2, 2), 16, (True, False, True)),
    "box32": ((2, 1, 2), 32, (False, False, False)),
    "x_walls32": ((2, 2, 1), 32, (False, True, True)),
}
TRT = (3.0 / 16.0, (2e-5, -1e-5, 5e-6))


def make(name, storage, inplace, omega=1.7, trt=None, seed=5, schedule="graph"):
    R, n, per = SPECS[name]
    g = lbm.Forest(R, n, 0, storage=storage, periodic=per)
    assert g.num_levels == 1
    N = g.num_cells()
    rng = np.random.default_rng(seed)
    g.set_level_omega(omega)
    if trt is not None:
        g.set_trt_force(*trt)
    g.init_pdfs(1.0 + 0.01 * rng.uniform(-1, 1, N), 0.03 * rng.uniform(-1, 1, (N, 3)))
    g.set_schedule(schedule)
    if inplace:
        g.set_inplace(True)
        assert g.inplace()
    return g


def run_pair(name, storage, chunks, trt=None, schedule="graph"):
    """Both paths through the same chunks of steps; after each chunk the
    moments and raw PDFs (the in-place buffer brought back to the natural
    layout) must be equal bitwise."""
    a = make(name, storage, False, trt=trt)
    b = make(name, storage, True, trt=trt, schedule=schedule)
    for steps in chunks:
        a.step_coarse(steps)
        b.step_coarse(steps)
        ra, ua = a.moments()
        rb, ub = b.moments()
        assert np.array_equal(ra, rb) and np.array_equal(ua, ub), (name, storage, steps)
        assert np.array_equal(a.get_pdfs(), b.get_pdfs()), (name, storage, steps)
    ma, ja = a.mass()
    mb, jb = b.mass()
    assert ma == mb and np.array_equal(ja, jb)
    a.close()
    b.close()


@pytest.mark.parametrize("storage", ["f64", "f32", "f16"])
@pytest.mark.parametrize("name", sorted(SPECS))
def test_inplace_equals_two_buffer_bitwise(name, storage):
    say(f"in-place vs two-buffer {name} {storage}")
    run_pair(name, storage, [1, 1, 2, 3])  # queries after odd and even launches


@pytest.mark.parametrize("storage", ["f64", "f32", "f16"])
@pytest.mark.parametrize("name", ["walls_y16", "box32"])
def test_inplace_trt_force_bitwise(name, storage):
    say(f"in-place TRT + force {name} {storage}")
    run_pair(name, storage, [3, 2], trt=TRT)


@pytest.mark.parametrize("schedule", ["direct", "per_block"])
def test_inplace_schedules_bitwise(schedule):
    say(f"in-place schedule {schedule}")
    run_pair("x_walls32", "f32", [2, 3], schedule=schedule)


@pytest.mark.parametrize("name", ["periodic4", "walls_y16", "box32"])
def test_fp64_inplace_matches_oracle(name):
    R, n, per = SPECS[name]
    say(f"in-place FP64 vs oracle {name}")
    of = Forest.build(R, n, 0, lambda L, x, y, z: False, periodic=per)
    o = RefinedOracle(of, 1.7)
    g = lbm.Forest(R, n, 0, storage="f64", periodic=per)
    assert g.leaves().tolist() == [list(t) for t in of.canonical_leaves()]
    N = g.num_cells()
    rng = np.random.default_rng(8)
    rho, u = 1.0 + 0.01 * rng.uniform(-1, 1, N), 0.03 * rng.uniform(-1, 1, (N, 3))
    o.init_pdfs(rho, u)
    g.set_level_omega(1.7)
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


def test_switching_off_and_on_continues_bitwise():
    say("in-place on, off, on")
    a = make("walls_y16", "f32", False)
    b = make("walls_y16", "f32", True)
    a.step_coarse(9)
    b.step_coarse(3)
    b.set_inplace(False)
    assert not b.inplace()
    b.step_coarse(3)
    b.set_inplace(True)
    b.step_coarse(3)
    assert np.array_equal(a.get_pdfs(), b.get_pdfs())
    a.close()
    b.close()


def test_set_pdfs_in_place():
    say("set_pdfs on an in-place forest")
    a = make("box32", "f64", False)
    b = make("box32", "f64", True)
    b.step_coarse(1)  # the buffer holds the pushed layout
    h = a.get_pdfs()
    b.set_pdfs(h)
    a.step_coarse(3)
    b.step_coarse(3)
    assert np.array_equal(a.get_pdfs(), b.get_pdfs())
    a.close()
    b.close()


def test_timing_reports_both_launches():
    g = make("x_walls32", "f32", True)
    t = g.time_sweeps(4)
    assert set(t) == {(0, 1), (0, 2)} and t[(0, 1)][1] == 2 and t[(0, 2)][1] == 2
    a = make("x_walls32", "f32", False)
    a.step_coarse(4)
    assert np.array_equal(a.get_pdfs(), g.get_pdfs())
    a.close()
    g.close()


def test_memory_footprint_halves():
    R, n = (4, 4, 4), 32
    g = lbm.Forest(R, n, 0, storage="f32")
    N = g.num_cells()
    g.set_level_omega(1.5)
    g.init_pdfs(np.ones(N), np.zeros((N, 3)))
    g.synchronize()
    free0, _ = lbm.device_memory(0)
    g.set_inplace(True)
    free1, _ = lbm.device_memory(0)
    pdf_bytes = N * 19 * 4 + 64 * 10 * n * n * 4  # one buffer and its x-face copy
    say(f"  freed {free1 - free0} bytes, one buffer {pdf_bytes}")
    assert free1 - free0 >= 0.95 * pdf_bytes
    g.step_coarse(2)
    g.set_inplace(False)
    free2, _ = lbm.device_memory(0)
    assert free1 - free2 >= 0.95 * pdf_bytes
    g.close()


def test_refusals():
    g = make("periodic4", "f32", True)
    g.step_coarse(1)
    with pytest.raises(lbm.LBMError) as e:
        g.autotune(1)
    assert e.value.name == "LBM_E_STATE"
    with pytest.raises(lbm.LBMError) as e:
        g.regrid(np.zeros(g.num_blocks(-1), dtype=np.int8))
    assert e.value.name == "LBM_E_STATE"
    g.set_inplace(False)
    with pytest.raises(lbm.LBMError) as e:  # the last step's start state is gone
        g.regrid(np.zeros(g.num_blocks(-1), dtype=np.int8))
    assert e.value.name == "LBM_E_STATE"
    g.step_coarse(1)
    g.regrid(np.zeros(g.num_blocks(-1), dtype=np.int8))
    g.close()
