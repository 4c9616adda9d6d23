"""Storage forms on the benchmark geometry against the FP64 oracle.

The sphere-shell grid of the throughput benchmark (4^3 roots, blocks meeting
the sphere surface of radius 0.25 refined to level 3) with 8^3-cell blocks
(1.9 M cells, 1/64 of the benchmark's cells), omega_0 = 1.9, Taylor-Green
0.02 plus noise, 20 coarse steps.  Targets: velocity rel-L2 <= 1e-5 (FP32),
<= 1e-3 (FP16), mass drift <= 1e-6 (both), volume-weighted over all cells.
"""

import numpy as np
import pytest

from oracle import Forest, RefinedOracle
from paper_1508_07982_amd import lbm
from paper_1508_07982_amd import workloads as W

pytestmark = pytest.mark.gpu

STEPS = 20


def rel_l2(a, b, w):
    num = np.sqrt(np.sum(w[:, None] * (a - b).reshape(len(w), -1) ** 2))
    den = np.sqrt(np.sum(w[:, None] * b.reshape(len(w), -1) ** 2))
    return num / den


@pytest.fixture(scope="module")
def reference():
    w = W.config_sphere(8, 4)
    print(f"oracle on {w.name}: building tables", flush=True)
    of = Forest.build(w.R, w.n, w.max_level, w.refine)
    o = RefinedOracle(of, w.omega0)
    rho, u = W.initial_field(w, of.canonical_leaves())
    o.init_pdfs(rho, u)
    print(f"oracle: {o.total_cells()} cells, {STEPS} coarse steps", flush=True)
    o.step(STEPS)
    r0, u0 = o.moments()
    return w, rho, u, r0, u0, o.level_weights()


@pytest.mark.parametrize("storage, tol_u", [("f32", 1e-5), ("f16", 1e-3)])
def test_sphere_shell_storage_form(reference, storage, tol_u):
    w, rho, u, r0, u0, wts = reference
    print(f"sphere shell n=8 {storage}", flush=True)
    g = lbm.Forest(w.R, w.n, w.max_level, refine=w.refine, storage=storage)
    g.set_level_omega(w.omega0)
    g.init_pdfs(rho, u)
    g.autotune(1)
    M0, _ = g.mass()
    g.step_coarse(STEPS)
    M1, _ = g.mass()
    r1, u1 = g.moments()
    eu = rel_l2(u1, u0, wts)
    er = rel_l2(r1, r0, wts)
    drift = abs(M1 - M0) / M0
    print(f"  velocity rel-L2 {eu:.3e}  density rel-L2 {er:.3e}  mass drift {drift:.3e}", flush=True)
    assert eu <= tol_u
    assert er <= tol_u
    assert drift <= 1e-6
    g.close()
