"""GPU regrid against the oracle's regrid, through the C ABI (FP64 storage:
same operators, rounding-order differences only), and FP32 conservation."""

import numpy as np
import pytest

from oracle import Forest, RefinedOracle
from paper_1508_07982_amd import lbm

pytestmark = pytest.mark.gpu


def three_level_spec(n):
    def refine(L, x, y, z):
        return (L == 0 and (x, y, z) == (1, 1, 1)) or (L == 1 and (x, y, z) == (3, 3, 2))
    return (3, 3, 3), n, refine


@pytest.mark.parametrize("n, steps_before, seed", [(4, 2, 0), (8, 3, 1), (8, 0, 2)])
def test_regrid_matches_oracle_fp64(n, steps_before, seed):
    print(f"regrid parity n={n} steps_before={steps_before} seed={seed}", flush=True)
    R, _, refine = three_level_spec(n)
    Lmax = 3
    of = Forest.build(R, n, 2, refine)
    o = RefinedOracle(of, 1.35)
    g = lbm.Forest(R, n, Lmax, refine=refine, storage="f64")
    assert g.leaves().tolist() == [list(t) for t in of.canonical_leaves()]
    rng = np.random.default_rng(seed)
    N = o.total_cells()
    rho = 1.0 + 0.01 * rng.uniform(-1, 1, N)
    u = 0.04 * rng.uniform(-1, 1, (N, 3))
    o.init_pdfs(rho, u)
    g.set_level_omega(1.35)
    g.init_pdfs(rho, u)
    o.step(steps_before)
    g.step_coarse(steps_before)
    flags = rng.choice([-1, 0, 1], size=len(of.leaves), p=[0.5, 0.3, 0.2]).astype(np.int8)
    o2 = o.regrid(flags, Lmax)
    g.regrid(flags)
    assert g.leaves().tolist() == [list(t) for t in o2.forest.canonical_leaves()]
    r0, u0 = o2.moments()
    r1, u1 = g.moments()
    assert np.max(np.abs(u1 - u0)) < 1e-12
    assert np.max(np.abs(r1 - r0)) < 1e-12
    for _ in range(3):
        o2.step(1)
        g.step_coarse(1)
    r0, u0 = o2.moments()
    r1, u1 = g.moments()
    assert np.max(np.abs(u1 - u0)) < 1e-12
    assert np.max(np.abs(r1 - r0)) < 1e-12
    M0, _ = o2.mass()
    M1, _ = g.mass()
    assert abs(M1 - M0) / M0 < 1e-13


def test_regrid_twice_fp32_conserves_mass():
    R, n, refine = three_level_spec(8)
    g = lbm.Forest(R, n, 3, refine=refine, storage="f32")
    N = g.num_cells()
    rng = np.random.default_rng(3)
    g.set_level_omega(1.7)
    g.init_pdfs(1.0 + 0.01 * rng.uniform(-1, 1, N), 0.03 * rng.uniform(-1, 1, (N, 3)))
    g.step_coarse(2)
    M0, _ = g.mass()
    for k in range(2):
        flags = rng.choice([-1, 0, 1], size=g.num_blocks(), p=[0.4, 0.4, 0.2]).astype(np.int8)
        g.regrid(flags)
        g.step_coarse(2)
    M1, _ = g.mass()
    assert abs(M1 - M0) / M0 < 1e-6
