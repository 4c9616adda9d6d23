"""TRT collision with a constant body force (section 2: TRT model, external
forces; eq. lambda_oL, eq. force_scaling) through the C ABI, against the
FP64 oracle.

* FP64 storage: moments (with the a_L / 2 velocity term) agree with the
  oracle to 1e-12 after 6 coarse steps on 3-level forests.
* The volume-weighted momentum grows by exactly a_0 V per coarse step on the
  GPU as well (independent of the oracle), mass stays put.
* FP32 / FP16: velocity rel-L2 against the oracle within the storage forms'
  targets (1e-5, 1e-3).
* lambda_eo = 0 without acceleration is SRT again (bitwise); regrid and bad
  arguments are refused.
"""

import numpy as np
import pytest

from oracle import Forest, RefinedOracle
from paper_1508_07982_amd import lbm

pytestmark = pytest.mark.gpu

A0 = (2e-5, -1e-5, 5e-6)
LAMBDA_EO = 3 / 16


def say(msg):
    print(msg, flush=True)


def three_level(n):
    def refine(L, x, y, z):
        return (L == 0 and (x, y, z) == (1, 1, 1)) or (L == 1 and (x, y, z) == (3, 3, 2))
    return (3, 3, 3), n, 2, refine


def make_pair(n, storage, omega0=1.45, seed=3):
    R, n, Lmax, refine = three_level(n)
    of = Forest.build(R, n, Lmax, refine)
    o = RefinedOracle(of, omega0, lambda_eo=LAMBDA_EO, accel0=A0)
    g = lbm.Forest(R, n, Lmax, refine=refine, storage=storage)
    rng = np.random.default_rng(seed)
    N = o.total_cells()
    rho = 1.0 + 0.01 * rng.uniform(-1, 1, N)
    u = 0.03 * rng.uniform(-1, 1, (N, 3))
    o.init_pdfs(rho, u)
    g.set_level_omega(omega0)
    g.set_trt_force(LAMBDA_EO, A0)
    g.init_pdfs(rho, u)
    return o, g


def rel_l2(a, b, w):
    num = np.sqrt(np.sum(w[:, None] * (a - b).reshape(len(w), -1) ** 2))
    den = np.sqrt(np.sum(w[:, None] * b.reshape(len(w), -1) ** 2))
    return num / den


@pytest.mark.parametrize("n", [4, 8])
def test_trt_force_fp64_matches_oracle(n):
    say(f"trt+force fp64 n={n}")
    o, g = make_pair(n, "f64")
    r0, u0 = o.moments()
    r1, u1 = g.moments()
    assert np.max(np.abs(u1 - u0)) < 1e-14
    for step in range(6):
        o.step(1)
        g.step_coarse(1)
        r0, u0 = o.moments()
        r1, u1 = g.moments()
        assert np.max(np.abs(u1 - u0)) < 1e-12, step
        assert np.max(np.abs(r1 - r0)) < 1e-12, step
    g.close()


def test_trt_force_momentum_growth_on_gpu():
    say("trt+force momentum growth fp64")
    _, g = make_pair(8, "f64", seed=5)
    V = sum(g.num_cells(L) * 8.0 ** (-L) for L in range(g.num_levels))
    M0, J0 = g.mass()
    for k in range(1, 4):
        g.step_coarse(1)
        M, J = g.mass()
        assert abs(M - M0) / M0 < 1e-13
        assert np.max(np.abs(J - J0 - k * V * np.array(A0))) < 1e-11, k
    g.close()


@pytest.mark.parametrize("storage, n, tol", [("f32", 8, 1e-5), ("f16", 8, 1e-3), ("f32", 4, 1e-5), ("f16", 4, 1e-3)])
def test_trt_force_storage_forms(storage, n, tol):
    say(f"trt+force {storage} n={n}")
    o, g = make_pair(n, storage)
    w = o.level_weights()
    o.step(10)
    g.step_coarse(10)
    _, u0 = o.moments()
    _, u1 = g.moments()
    assert rel_l2(u1, u0, w) < tol
    g.close()


def test_trt_off_is_srt_and_refusals():
    say("trt off / refusals")
    R, n, Lmax, refine = three_level(4)
    outs = []
    for switch in (False, True):
        g = lbm.Forest(R, n, Lmax, refine=refine, storage="f32")
        N = g.num_cells()
        rng = np.random.default_rng(9)
        g.set_level_omega(1.7)
        if switch:
            g.set_trt_force(LAMBDA_EO, A0)
            g.set_trt_force(0.0, None)
        g.init_pdfs(1.0 + 0.01 * rng.uniform(-1, 1, N), 0.02 * rng.uniform(-1, 1, (N, 3)))
        g.step_coarse(3)
        outs.append(g.get_pdfs())
        if switch:
            # the acceleration is part of the stored state: refused once set
            with pytest.raises(lbm.LBMError) as e:
                g.set_trt_force(LAMBDA_EO, A0)
            assert e.value.name == "LBM_E_STATE"
            g.set_trt_force(LAMBDA_EO, None)  # the TRT rates alone may change
            with pytest.raises(lbm.LBMError):
                g.regrid(np.zeros(len(g.leaves()), dtype=np.int8))
            with pytest.raises(lbm.LBMError):
                g.set_trt_force(-1.0, None)
            with pytest.raises(lbm.LBMError):
                g.set_trt_force(0.1, (np.nan, 0.0, 0.0))
        g.close()
    assert np.array_equal(outs[0], outs[1])


def _trt_forest(schedule="graph"):
    R, n, Lmax, refine = three_level(8)
    g = lbm.Forest(R, n, Lmax, refine=refine, storage="f32")
    N = g.num_cells()
    rng = np.random.default_rng(11)
    g.set_level_omega(1.7)
    g.set_trt_force(LAMBDA_EO, A0)
    g.set_schedule(schedule)
    g.init_pdfs(1.0 + 0.01 * rng.uniform(-1, 1, N), 0.02 * rng.uniform(-1, 1, (N, 3)))
    return g


def test_trt_schedules_and_autotune_bitwise():
    """Graph, direct and per-block launches give the same TRT state, and the
    autotuner leaves it where it was."""
    say("trt schedules / autotune")
    outs = {}
    for schedule in ("graph", "direct", "per_block"):
        g = _trt_forest(schedule)
        g.step_coarse(3)
        outs[schedule] = g.get_pdfs()
        g.close()
    assert np.array_equal(outs["graph"], outs["direct"])
    assert np.array_equal(outs["graph"], outs["per_block"])
    g = _trt_forest()
    g.step_coarse(1)
    g.autotune(n_steps=1)
    g.step_coarse(2)
    assert np.array_equal(g.get_pdfs(), outs["graph"])
    g.close()
