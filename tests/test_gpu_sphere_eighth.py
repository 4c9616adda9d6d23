"""Storage forms against the FP64 oracle on the benchmark geometry at 1/8 of
its cells.

The sphere-shell grid of the throughput benchmark (4^3 roots, blocks meeting
the surface of the central sphere of radius 0.25 refined at every level up to
level 3) with 16^3-cell blocks instead of 32^3: 15.2 M cells, exactly 1/8 of
the benchmark's 121.4 M.  omega_0 = 1.9, Taylor-Green amplitude 0.02 plus
noise of +-1e-4, 50 coarse steps (400 finest-level substeps).

Targets of the storage forms: velocity and density relative L2 (volume
weighted over all cells) <= 1e-5 for FP32 and <= 1e-3 for FP16 shifted
storage, mass drift <= 1e-6; FP64 storage agrees to rounding order.
The oracle needs about a minute of host time on 16 cores here.
"""

import time

import numpy as np
import pytest

from oracle import Forest, RefinedOracle
from paper_1508_07982_amd import lbm
from paper_1508_07982_amd import workloads as W

pytestmark = [pytest.mark.gpu, pytest.mark.timeout(900)]

STEPS = 50


def say(msg):
    print(msg, flush=True)


def rel_l2(a, b, w):
    num = np.sqrt(np.sum(w[:, None] * (a - b).reshape(len(w), -1) ** 2))
    den = np.sqrt(np.sum(w[:, None] * b.reshape(len(w), -1) ** 2))
    return num / den


@pytest.fixture(scope="module")
def reference():
    w = W.config_sphere(16, 4)
    t0 = time.time()
    say(f"oracle on {w.name}: building tables")
    of = Forest.build(w.R, w.n, w.max_level, w.refine)
    o = RefinedOracle(of, w.omega0)
    rho, u = W.initial_field(w, of.canonical_leaves())
    o.init_pdfs(rho, u)
    say(f"oracle: {o.total_cells()} cells, tables in {time.time() - t0:.0f} s")
    for s in range(0, STEPS, 10):
        o.step(10)
        say(f"  oracle step {s + 10}/{STEPS}: {time.time() - t0:.0f} s")
    r0, u0 = o.moments()
    wts = o.level_weights()
    leaves = of.canonical_leaves()
    del o, of
    return w, leaves, rho, u, r0, u0, wts


@pytest.mark.parametrize("storage, tol", [("f32", 1e-5), ("f16", 1e-3), ("f64", 1e-11)])
def test_sphere_shell_eighth_storage_form(reference, storage, tol):
    w, leaves, rho, u, r0, u0, wts = reference
    say(f"sphere shell n=16 (1/8 of the benchmark grid) {storage}, {STEPS} coarse steps")
    g = lbm.Forest(w.R, w.n, w.max_level, refine=w.refine, storage=storage)
    assert g.leaves().tolist() == [list(t) for t in leaves]
    assert g.num_cells() * 8 == 121372672
    g.set_level_omega(w.omega0)
    g.init_pdfs(rho, u)
    g.autotune(1)
    M0, _ = g.mass()
    g.step_coarse(STEPS)
    M1, _ = g.mass()
    r1, u1 = g.moments()
    eu = rel_l2(u1, u0, wts)
    er = rel_l2(r1, r0, wts)
    edr = rel_l2(r1 - 1.0, r0 - 1.0, wts)
    drift = abs(M1 - M0) / M0
    say(f"  velocity rel-L2 {eu:.3e}  density rel-L2 {er:.3e}  density-deviation rel-L2 {edr:.3e}  "
        f"mass drift {drift:.3e}")
    assert eu <= tol
    assert er <= tol
    assert drift <= 1e-6
    g.close()
