"""lbm_get_moments_static (the entry point for callers that cannot allocate)
against lbm_get_moments through the C ABI: two calls in a row on the same
device, the second on a smaller forest, each bitwise equal to the
allocating entry point (same kernel, same arithmetic).  The first forest
holds more cells than one staging chunk (524,288), so the chunked path and
its ragged last chunk are covered; the second fits in one chunk, and the
array then still holds the first call's values beyond it."""

import numpy as np
import pytest

from paper_1508_07982_amd import lbm

pytestmark = pytest.mark.gpu

STAGE_CELLS = 1 << 19


def _forest(R, n, Lmax, refine, storage, seed, trt=False):
    g = lbm.Forest(R, n, Lmax, refine=refine, storage=storage)
    N = g.num_cells()
    rng = np.random.default_rng(seed)
    g.set_level_omega(1.6)
    if trt:
        g.set_trt_force(3.0 / 16.0, (2e-5, -1e-5, 0.0))
    g.init_pdfs(1.0 + 0.01 * rng.uniform(-1, 1, N), 0.03 * rng.uniform(-1, 1, (N, 3)))
    g.step_coarse(2)
    return g


@pytest.mark.parametrize("storage", ["f32", "f64", "f16"])
def test_moments_static_matches_allocating_entry_point(storage):
    print(f"moments_static {storage}", flush=True)
    big = _forest((3, 3, 3), 32, 2, lambda L, x, y, z: (L == 0 and (x, y, z) == (1, 1, 1)) or
                  (L == 1 and (x, y, z) == (3, 3, 2)), storage, 1, trt=storage == "f32")
    assert big.num_cells() > 2 * STAGE_CELLS and big.num_cells() % STAGE_CELLS != 0
    small = _forest((2, 2, 2), 8, 1, lambda L, x, y, z: L == 0 and (x, y, z) == (0, 0, 0), storage, 2)
    assert small.num_cells() < STAGE_CELLS
    for g in (big, small):
        r_ref, u_ref = g.moments()
        r, u = g.moments_static()
        assert np.array_equal(r, r_ref)
        assert np.array_equal(u, u_ref)
        assert np.all(np.isfinite(r)) and np.all(r > 0.5)
    big.close()
    small.close()
