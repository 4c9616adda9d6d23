"""Parity at 32^3-cell blocks, the block size of the throughput benchmark.

At n = 32 the sweep runs its own lane layouts: FP32 keeps 4 cells per lane
(8 lanes per cell row, two rows per 16-lane DPP row, 32 work tiles per
block), FP64 2 cells per lane (a cell row fills a DPP row) and packed FP16 8
cells per lane (4 lanes per row, 16 tiles per block).  Every launch shape
the autotuner can choose (one workgroup per work unit with split 1, 2 or 4,
persistent grids of 1..8 workgroups per CU, canonical or XCD-grouped tile
order) is compared here with the FP64 oracle or, for the reduced-precision
forms, bitwise with the default shape.

Tolerances: FP64 storage differs from the oracle only in rounding order
(shifted form, fused collision), a few ulp per step, so moments agree to
1e-12 after 6 steps; FP32 / FP16 use the targets of those storage forms
(velocity relative L2 <= 1e-5 / 1e-3, mass drift <= 1e-6).
"""

import numpy as np
import pytest

from oracle import Forest, RefinedOracle
from paper_1508_07982_amd import lbm
from paper_1508_07982_amd import workloads as W

pytestmark = pytest.mark.gpu

N32 = 32
# (persistent workgroups per CU, tile order, split): the autotuner's 14
# candidates, and persistent grids with a split
SHAPES = [(0, 0, 1), (0, 1, 1), (0, 0, 2), (0, 1, 2), (0, 0, 4), (0, 1, 4), (1, 0, 1), (1, 1, 1), (2, 0, 1),
          (2, 1, 1), (4, 0, 1), (4, 1, 1), (8, 0, 1), (8, 1, 1), (2, 1, 4), (2, 0, 2)]
SHAPE_IDS = ["p%d_o%d_s%d" % s for s in SHAPES]


def say(msg):
    print(msg, flush=True)


def spec_two():
    return (2, 2, 2), N32, 1, lambda L, x, y, z: L == 0 and (x, y, z) == (0, 0, 0)


def spec_three():
    def refine(L, x, y, z):
        return (L == 0 and (x, y, z) == (1, 1, 1)) or (L == 1 and (x, y, z) == (3, 3, 2))
    return (3, 3, 3), N32, 2, refine


def random_field(N, seed=3, amp=0.03):
    rng = np.random.default_rng(seed)
    return 1.0 + 0.01 * rng.uniform(-1, 1, N), amp * rng.uniform(-1, 1, (N, 3))


def oracle_run(spec, omega0, checkpoints):
    """FP64 oracle moments at the given coarse step counts, and its mass."""
    R, n, Lmax, refine = spec
    of = Forest.build(R, n, Lmax, refine)
    o = RefinedOracle(of, omega0)
    rho, u = random_field(o.total_cells())
    o.init_pdfs(rho, u)
    out, done = {}, 0
    for s in checkpoints:
        o.step(s - done)
        done = s
        out[s] = o.moments()
    return {"leaves": of.canonical_leaves(), "rho": rho, "u": u, "moments": out, "mass": o.mass()}


@pytest.fixture(scope="module")
def two_ref():
    say("oracle: two-level n=32")
    return oracle_run(spec_two(), 1.45, (1, 3, 6))


@pytest.fixture(scope="module")
def three_ref():
    say("oracle: three-level n=32")
    return oracle_run(spec_three(), 1.45, (1, 3, 6))


def gpu_forest(spec, storage, ref=None, shape=None, seed=3):
    R, n, Lmax, refine = spec
    g = lbm.Forest(R, n, Lmax, refine=refine, storage=storage)
    if ref is not None:
        assert g.leaves().tolist() == [list(t) for t in ref["leaves"]]
        rho, u = ref["rho"], ref["u"]
    else:
        rho, u = random_field(g.num_cells(), seed)
    g.set_level_omega(1.45)
    g.init_pdfs(rho, u)
    if shape is not None:
        for L in range(g.num_levels):
            g.set_level_launch(L, *shape)
    return g


def check_fp64(g, ref):
    done = 0
    for s, (r0, u0) in ref["moments"].items():
        g.step_coarse(s - done)
        done = s
        r1, u1 = g.moments()
        assert np.max(np.abs(u1 - u0)) < 1e-12, s
        assert np.max(np.abs(r1 - r0)) < 1e-12, s
    M0, J0 = ref["mass"]
    M1, J1 = g.mass()
    assert abs(M1 - M0) / M0 < 1e-13
    assert np.max(np.abs(J1 - J0)) < 1e-10


@pytest.mark.parametrize("shape", SHAPES, ids=SHAPE_IDS)
def test_fp64_two_level_n32_every_launch_shape(two_ref, shape):
    say(f"fp64 two-level n=32 shape {shape}")
    g = gpu_forest(spec_two(), "f64", two_ref, shape)
    check_fp64(g, two_ref)
    g.close()


@pytest.mark.parametrize("shape", [(0, 0, 1), (0, 1, 1), (0, 1, 2), (0, 0, 4), (2, 1, 1), (8, 0, 1)],
                         ids=["p0_o0_s1", "p0_o1_s1", "p0_o1_s2", "p0_o0_s4", "p2_o1_s1", "p8_o0_s1"])
def test_fp64_three_level_n32(three_ref, shape):
    say(f"fp64 three-level n=32 shape {shape}")
    g = gpu_forest(spec_three(), "f64", three_ref, shape)
    check_fp64(g, three_ref)
    g.close()


@pytest.mark.parametrize("storage", ["f32", "f16"])
@pytest.mark.parametrize("shape", SHAPES[1:], ids=SHAPE_IDS[1:])
def test_launch_shapes_bitwise_n32(storage, shape):
    say(f"bitwise n=32 {storage} shape {shape}")
    ref = gpu_forest(spec_three(), storage, shape=SHAPES[0], seed=5)
    ref.set_schedule("direct")
    ref.step_coarse(3)
    want = ref.get_pdfs()
    ref.close()
    g = gpu_forest(spec_three(), storage, shape=shape, seed=5)
    g.step_coarse(3)
    assert np.array_equal(g.get_pdfs(), want)
    g.close()


def rel_l2(a, b, w):
    num = np.sqrt(np.sum(w[:, None] * (a - b).reshape(len(w), -1) ** 2))
    den = np.sqrt(np.sum(w[:, None] * b.reshape(len(w), -1) ** 2))
    return num / den


@pytest.fixture(scope="module")
def tg_ref():
    """Two-level Taylor-Green at n = 32 (491,520 cells): omega0 = 1.6,
    amplitude 0.01 plus noise, 100 coarse steps of the FP64 oracle."""
    w = W.config_two_level(N32)
    say("oracle: two-level Taylor-Green n=32, 100 steps")
    of = Forest.build(w.R, w.n, w.max_level, w.refine)
    o = RefinedOracle(of, w.omega0)
    rho, u = W.initial_field(w, of.canonical_leaves())
    o.init_pdfs(rho, u)
    o.step(w.coarse_steps)
    r0, u0 = o.moments()
    return w, rho, u, r0, u0, o.level_weights()


@pytest.mark.parametrize("storage, tol_u", [("f32", 1e-5), ("f16", 1e-3), ("f64", 1e-11)])
def test_storage_forms_n32_autotuned(tg_ref, storage, tol_u):
    """The storage forms at n = 32 with the launch shapes the autotuner picks
    (the benchmark's path) against the FP64 oracle."""
    w, rho, u, r0, u0, wts = tg_ref
    say(f"two-level Taylor-Green n=32 {storage}, autotuned")
    g = lbm.Forest(w.R, w.n, w.max_level, refine=w.refine, storage=storage)
    g.set_level_omega(w.omega0)
    g.init_pdfs(rho, u)
    shapes = g.autotune(1)
    say(f"  launch shapes {[(r['persistent'], r['order'], r['split']) for r in shapes]}")
    M0, _ = g.mass()
    g.step_coarse(w.coarse_steps)
    M1, _ = g.mass()
    r1, u1 = g.moments()
    eu = rel_l2(u1, u0, wts)
    er = rel_l2(r1, r0, wts)
    drift = abs(M1 - M0) / M0
    say(f"  velocity rel-L2 {eu:.3e}  density rel-L2 {er:.3e}  mass drift {drift:.3e}")
    assert eu <= tol_u
    assert er <= tol_u
    assert drift <= 1e-6
    g.close()
