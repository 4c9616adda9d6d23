"""The coalescence run inside the finer level's second-substep launch,
through the C ABI (lbm_set_coalescence_fusion).

Algorithm 1 coalesces level L after level L+1's two substeps and before
level L's next stream (eq. ftoc).  By default the library runs those chunks
in the launch of level L+1's second substep, interleaved with its work
units; switched off, each coalescence is a launch of its own.  Both must
give bitwise the same state for every storage form, block size, launch
shape (workgroup splits, XCD order, persistent grids, which keep their own
launch), walls, TRT with a body force and the FP64 accumulation check.
"""

import numpy as np
import pytest

from paper_1508_07982_amd import lbm

pytestmark = pytest.mark.gpu


def say(msg):
    print(msg, flush=True)


def three_levels(L, x, y, z):
    return (L == 0 and (x, y, z) == (1, 1, 1)) or (L == 1 and (x, y, z) == (3, 3, 2))


def make(storage, n, fuse, periodic=(True, True, True), trt=None, seed=3, schedule="graph"):
    g = lbm.Forest((3, 3, 3), n, 3, refine=three_levels, storage=storage, periodic=periodic)
    assert g.num_levels == 3
    N = g.num_cells()
    rng = np.random.default_rng(seed)
    g.set_level_omega(1.7)
    if trt is not None:
        g.set_trt_force(*trt)
    g.init_pdfs(1.0 + 0.01 * rng.uniform(-1, 1, N), 0.03 * rng.uniform(-1, 1, (N, 3)))
    g.set_schedule(schedule)
    g.set_coalescence_fusion(fuse)
    return g


def compare(a, b, chunks=(1, 2)):
    for steps in chunks:
        a.step_coarse(steps)
        b.step_coarse(steps)
        ra, ua = a.moments()
        rb, ub = b.moments()
        assert np.array_equal(ra, rb) and np.array_equal(ua, ub), steps
        assert np.array_equal(a.get_pdfs(), b.get_pdfs()), steps


@pytest.mark.parametrize("storage, n", [("f64", 8), ("f32", 8), ("f16", 8), ("f32", 16), ("f16", 16),
                                        ("f64", 32), ("f32", 32), ("f16", 32)])
def test_fused_equals_separate_bitwise(storage, n):
    say(f"fused vs separate coalescence {storage} n={n}")
    a = make(storage, n, True)
    b = make(storage, n, False)
    compare(a, b)
    a.close()
    b.close()


@pytest.mark.parametrize("storage, n", [("f64", 8), ("f32", 16), ("f16", 16)])
def test_fused_with_walls_bitwise(storage, n):
    say(f"fused vs separate, no-slip walls {storage} n={n}")
    a = make(storage, n, True, periodic=(False, True, False))
    b = make(storage, n, False, periodic=(False, True, False))
    compare(a, b)
    a.close()
    b.close()


def test_fused_trt_force_bitwise():
    say("fused vs separate, TRT + force")
    trt = (3.0 / 16.0, (2e-5, -1e-5, 5e-6))
    a = make("f32", 16, True, trt=trt)
    b = make("f32", 16, False, trt=trt)
    compare(a, b)
    a.close()
    b.close()


@pytest.mark.parametrize("shape", [[(0, 0, 1), (0, 1, 2), (0, 1, 4)], [(0, 1, 1), (2, 0, 1), (0, 0, 2)],
                                   [(4, 1, 1), (0, 0, 4), (1, 0, 1)]])
def test_fused_launch_shapes_bitwise(shape):
    """Workgroup splits and XCD order change the spacing of the chunks in the
    grid; a persistent level keeps a separate coalescence launch."""
    say(f"fused launch shapes {shape}")
    a = make("f32", 16, True)
    for L, (p, o, s) in enumerate(shape):
        a.set_level_launch(L, p, o, s)
    b = make("f32", 16, False, schedule="per_block")
    compare(a, b)
    a.close()
    b.close()


def test_direct_schedule_fused_bitwise():
    say("fused direct launches vs per-block launches")
    a = make("f16", 16, True, schedule="direct")
    b = make("f16", 16, True, schedule="per_block")  # the per-block schedule never fuses
    compare(a, b)
    a.close()
    b.close()


def test_fused_coalescence_check_counts_every_pair():
    say("FP64 accumulation check inside the fused launch")
    figs = []
    for fuse in (True, False):
        g = make("f32", 16, fuse)
        g.set_coalescence_check(True)
        g.step_coarse(2)
        figs.append(g.coalescence_check())
        g.close()
    assert figs[0]["pairs"] == figs[1]["pairs"] > 0
    assert figs[0]["max_abs_dev"] == figs[1]["max_abs_dev"]
    assert figs[0]["max_bound_ratio"] == figs[1]["max_bound_ratio"] <= 1.0


def test_timing_shows_where_the_coalescence_runs():
    a = make("f32", 16, True)
    sweeps, coal = a.time_launches(2)
    assert coal == {}  # every level's finer neighbour runs one workgroup per tile
    assert set(sweeps) == {(0, 1), (1, 1), (1, 2), (2, 1), (2, 2)}
    b = make("f32", 16, False)
    sweeps, coal = b.time_launches(2)
    assert set(coal) == {0, 1} and coal[0][1] == 2 and coal[1][1] == 4
    assert np.array_equal(a.get_pdfs(), b.get_pdfs())
    a.close()
    b.close()


def test_persistent_finer_level_keeps_its_own_coalescence_launch():
    """A finer level whose grid is smaller than its work units (persistent)
    leaves the coarser coalescence as a launch of its own, bitwise equal."""
    def half(L, x, y, z):
        return L == 0 and x < 2

    def make2(fuse, persistent):
        g = lbm.Forest((4, 4, 4), 16, 1, refine=half, storage="f32")
        N = g.num_cells()
        rng = np.random.default_rng(9)
        g.set_level_omega(1.7)
        g.init_pdfs(1.0 + 0.01 * rng.uniform(-1, 1, N), 0.03 * rng.uniform(-1, 1, (N, 3)))
        g.set_coalescence_fusion(fuse)
        g.set_level_launch(1, persistent, 0, 1)
        return g

    a = make2(True, 1)  # one workgroup per compute unit looping over the tiles
    assert a.level_stats(1)["work_tiles"] > 256  # more tiles than compute units
    _, coal = a.time_launches(1)
    assert set(coal) == {0} and coal[0][1] == 1
    b = make2(True, 0)
    _, coal = b.time_launches(1)
    assert coal == {}
    c = make2(False, 0)
    c.step_coarse(1)
    want = c.get_pdfs()
    assert np.array_equal(a.get_pdfs(), want) and np.array_equal(b.get_pdfs(), want)
    compare(a, c)
    for g in (a, b, c):
        g.close()


def test_fusion_switch_rejects_other_values():
    g = make("f32", 8, True)
    with pytest.raises(lbm.LBMError) as e:
        lbm._check(g._lib.lbm_set_coalescence_fusion(g._h, 2))
    assert e.value.name == "LBM_E_INVALID"
    g.close()


def test_per_level_fusion_bitwise():
    """Fusion on one level and off on another, against all separate."""
    say("per-level fusion")
    a = make("f16", 16, True)
    a.set_level_fusion(1, 1)
    a.set_level_fusion(2, 0)
    assert a.get_level_fusion(1) and not a.get_level_fusion(2)
    _, coal = a.time_launches(1)
    assert set(coal) == {1}  # level 2 leaves level 1's coalescence on its own
    b = make("f16", 16, False)
    b.step_coarse(1)
    assert np.array_equal(a.get_pdfs(), b.get_pdfs())
    compare(a, b)
    a.set_level_fusion(2, -1)  # back to the forest-wide setting (on)
    assert a.get_level_fusion(2)
    a.set_coalescence_fusion(False)
    assert not a.get_level_fusion(1) and not a.get_level_fusion(2)
    compare(a, b, chunks=(1,))
    a.close()
    b.close()
