"""GPU parity: the HIP library against the FP64 oracle, through the C ABI.

Tolerances:
* FP64 storage (shifted, FP64 arithmetic): the two sides differ only in
  rounding order (the library works on h = f - w and fuses the collision of
  the next step into this one), so PDFs and moments agree to ~1e-13 after
  tens of steps; the test uses 1e-11 relative to the velocity scale.
* FP32 form: volume-weighted relative L2 error of the velocity <= 1e-5, of
  the density deviation <= 1e-5, mass drift <= 1e-6.
* FP16 shifted form: velocity relative L2 <= 1e-3, mass drift <= 1e-6.
These are the targets stated for the storage forms; the FP64 bound is set
from the arithmetic (a few ulp per step).
"""

import numpy as np
import pytest

from oracle import Forest, RefinedOracle
from paper_1508_07982_amd import lbm
from paper_1508_07982_amd import workloads as W

pytestmark = pytest.mark.gpu


def say(msg):
    print(msg, flush=True)


def forest_three(n):
    def refine(L, x, y, z):
        return (L == 0 and (x, y, z) == (1, 1, 1)) or (L == 1 and (x, y, z) == (3, 3, 2))
    return (3, 3, 3), n, 2, refine


def forest_three_empty0(n):
    def refine(L, x, y, z):
        return (L == 0 and (x, y, z) == (0, 0, 0)) or (L == 1 and (x, y, z) == (1, 1, 0))
    return (2, 2, 2), n, 2, refine


def forest_two(n):
    return (2, 2, 2), n, 1, lambda L, x, y, z: L == 0 and (x, y, z) == (0, 0, 0)


def forest_single(n):
    return (2, 3, 2), n, 0, None


def forest_narrow(n):
    """One root wide in x and z (periodic): a level-0 block is its own x
    neighbour, and the two level-1 blocks of a row are each other's on both
    sides."""
    return (1, 3, 1), n, 1, lambda L, x, y, z: L == 0 and (x, y, z) == (0, 0, 0)


def rel_l2(a, b, w):
    num = np.sqrt(np.sum(w[:, None] * (a - b).reshape(len(w), -1) ** 2))
    den = np.sqrt(np.sum(w[:, None] * b.reshape(len(w), -1) ** 2))
    return num / den


def make_pair(spec, storage, omega0, field_seed=3, amp=0.03):
    R, n, Lmax, refine = spec
    of = Forest.build(R, n, Lmax, refine)
    o = RefinedOracle(of, omega0)
    g = lbm.Forest(R, n, Lmax, refine=refine, storage=storage)
    assert g.leaves().tolist() == [list(t) for t in of.canonical_leaves()]
    rng = np.random.default_rng(field_seed)
    N = o.total_cells()
    rho = 1.0 + 0.01 * rng.uniform(-1, 1, N)
    u = amp * rng.uniform(-1, 1, (N, 3))
    o.init_pdfs(rho, u)
    g.set_level_omega(omega0)
    g.init_pdfs(rho, u)
    return o, g


@pytest.mark.parametrize("spec", [forest_single(8), forest_two(4), forest_two(8), forest_three(4), forest_three(8),
                                  forest_three_empty0(4), forest_narrow(4), forest_narrow(8)],
                         ids=["single8", "two4", "two8", "three4", "three8", "three4_empty0", "narrow4", "narrow8"])
def test_fp64_matches_oracle(spec):
    say(f"fp64 parity {spec[:3]}")
    o, g = make_pair(spec, "f64", 1.45)
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
    assert np.max(np.abs(J1 - J0)) < 1e-11


@pytest.mark.parametrize("schedule", ["graph", "direct", "per_block"])
@pytest.mark.parametrize("persistent", [0, 2])
def test_schedules_bitwise_equal(schedule, persistent):
    say(f"schedule {schedule} persistent {persistent}")
    spec = forest_three(8)
    ref = None
    R, n, Lmax, refine = spec
    g = lbm.Forest(R, n, Lmax, refine=refine, storage="f32")
    N = g.num_cells()
    rng = np.random.default_rng(1)
    rho = 1.0 + 0.01 * rng.uniform(-1, 1, N)
    u = 0.03 * rng.uniform(-1, 1, (N, 3))
    g.set_level_omega(1.7)
    g.set_schedule(schedule)
    g.set_launch(persistent)
    g.init_pdfs(rho, u)
    g.step_coarse(3)
    h = g.get_pdfs()
    g2 = lbm.Forest(R, n, Lmax, refine=refine, storage="f32")
    g2.set_level_omega(1.7)
    g2.set_schedule("direct")
    g2.init_pdfs(rho, u)
    g2.step_coarse(3)
    ref = g2.get_pdfs()
    assert np.array_equal(h, ref)


def _tg_pair(w, storage, n_override=None):
    n = n_override or w.n
    of = Forest.build(w.R, n, w.max_level, w.refine)
    leaves = of.canonical_leaves()
    o = RefinedOracle(of, w.omega0)
    rho, u = W.initial_field(w, leaves)
    o.init_pdfs(rho, u)
    g = lbm.Forest(w.R, n, w.max_level, refine=w.refine, storage=storage)
    g.set_level_omega(w.omega0)
    g.init_pdfs(rho, u)
    return o, g


# rho - 1 is O(u^2) ~ 1e-4 here while FP16 stores h = f - w (|h| ~ 1e-3) with a
# spacing of ~1e-6: the density deviation of a cell carries a relative
# rounding error of ~1e-2 in FP16 storage (measured 1.5e-2 after 100 steps)
@pytest.mark.parametrize("storage, tol_u, tol_drho", [("f64", 1e-11, 1e-9), ("f32", 1e-5, 1e-4), ("f16", 1e-3, 5e-2)])
def test_two_level_taylor_green_100_steps(storage, tol_u, tol_drho):
    """2x2x2 roots of 16^3, one octant refined (61,440 cells), omega0 = 1.6,
    Taylor-Green 0.01 + noise, 100 coarse steps (200 fine substeps)."""
    w = W.config_two_level()
    say(f"two-level TG {storage}")
    o, g = _tg_pair(w, storage)
    M0o, _ = o.mass()
    M0g, _ = g.mass()
    o.step(w.coarse_steps)
    g.step_coarse(w.coarse_steps)
    r0, u0 = o.moments()
    r1, u1 = g.moments()
    wts = o.level_weights()
    eu = rel_l2(u1, u0, wts)
    erho = rel_l2(r1, r0, wts)
    edrho = rel_l2(r1 - 1.0, r0 - 1.0, wts)
    M1g, _ = g.mass()
    say(f"  velocity rel-L2 {eu:.3e}  density rel-L2 {erho:.3e}  density-deviation rel-L2 {edrho:.3e}"
        f"  mass drift {abs(M1g - M0g) / M0g:.3e}")
    assert eu <= tol_u
    assert erho <= tol_u
    # rho - 1 is O(u^2) ~ 1e-4 here, so its relative error is the harsher figure
    assert edrho <= tol_drho
    assert abs(M1g - M0g) / M0g <= 1e-6


def test_uniform_flow_and_mass_on_gpu():
    spec = forest_three(8)
    R, n, Lmax, refine = spec
    say("uniform flow fp32")
    g = lbm.Forest(R, n, Lmax, refine=refine, storage="f32")
    N = g.num_cells()
    U = np.array([0.03, -0.02, 0.01])
    g.set_level_omega(1.8)
    g.init_pdfs(np.ones(N), np.tile(U, (N, 1)))
    g.step_coarse(20)
    rho, u = g.moments()
    assert np.max(np.abs(u - U)) < 2e-7
    assert np.max(np.abs(rho - 1.0)) < 2e-7


def test_raw_pdf_roundtrip_and_packet_trace():
    """omega = 0: a coarse packet entering the refined octant ends in the
    2x2x2 fine cells of the two layers next to the face."""
    n = 4
    R, _, Lmax, refine = forest_two(n)
    say("packet trace fp64")
    g = lbm.Forest(R, n, Lmax, refine=refine, storage="f64")
    g.set_level_omega(0.0)
    N = g.num_cells()
    e, w = lbm.lattice()
    of = Forest.build(R, n, Lmax, refine)
    o = RefinedOracle(of, 0.0)
    c0 = o.tables[0].cells.coords[:o.n_int(0)]
    c1 = o.tables[1].cells.coords[:o.n_int(1)]
    f = np.zeros((N, 19))
    X = int(np.nonzero(np.all(c0 == (n, 1, 1), axis=1))[0][0])
    f[X, 2] = 1.0
    g.set_pdfs(f - w[None, :])
    back = g.get_pdfs() + w[None, :]
    assert np.array_equal(back, f)
    g.step_coarse(1)
    out = g.get_pdfs() + w[None, :]
    nz = {(int(i), int(a)) for i, a in zip(*np.nonzero(np.abs(out) > 1e-15))}
    off = o.n_int(0)
    expect = set()
    for x in (2 * n - 2, 2 * n - 1):
        for y in (2, 3):
            for z in (2, 3):
                i = int(np.nonzero(np.all(c1 == (x, y, z), axis=1))[0][0])
                expect.add((off + i, 2))
    assert nz == expect
    for (i, a) in expect:
        assert abs(out[i, a] - 1.0) < 1e-15


@pytest.mark.parametrize("storage, n, tol", [("f64", 8, 1e-15), ("f32", 4, 1e-7), ("f16", 8, 1e-4)])
def test_set_pdfs_then_streaming_matches_oracle(storage, n, tol):
    """omega = 0 (streaming, explosion and coalescence only) from random PDFs
    written with set_pdfs over an already stepped state: every value the
    coalescence reads, the x-face values of the fine blocks included, must
    come from the state that was set."""
    R, n, Lmax, refine = forest_three(n)
    say(f"set_pdfs + streaming {storage} n={n}")
    of = Forest.build(R, n, Lmax, refine)
    o = RefinedOracle(of, 0.0)
    g = lbm.Forest(R, n, Lmax, refine=refine, storage=storage)
    g.set_level_omega(0.0)
    N = g.num_cells()
    _, w = lbm.lattice()
    g.init_pdfs(np.ones(N), np.zeros((N, 3)))
    g.step_coarse(1)
    rng = np.random.default_rng(7)
    f = w[None, :] * (1.0 + 0.1 * rng.uniform(-1, 1, (N, 19)))
    g.set_pdfs(f - w[None, :])
    f = g.get_pdfs() + w[None, :]  # as stored (rounded to the storage form)
    off = 0
    for L in range(o.num_levels):
        m = o.n_int(L)
        o.set_interior_pdfs(L, f[off:off + m])
        off += m
    o.step(2)
    g.step_coarse(2)
    got = g.get_pdfs() + w[None, :]
    want = np.concatenate([o.interior_pdfs(L) for L in range(o.num_levels)])
    assert np.max(np.abs(got - want)) < tol
    g.close()


def test_nonfinite_detected():
    R, n, Lmax, refine = forest_two(4)
    say("nonfinite")
    g = lbm.Forest(R, n, Lmax, refine=refine, storage="f32")
    g.set_level_omega(1.2)
    N = g.num_cells()
    rho = np.ones(N)
    u = np.zeros((N, 3))
    rho[5] = np.nan
    g.init_pdfs(rho, u)
    with pytest.raises(lbm.LBMError) as e:
        g.mass()
    assert e.value.name == "LBM_E_NONFINITE"


@pytest.mark.parametrize("storage", ["f32", "f16", "f64"])
def test_coalescence_accumulation_check(storage):
    """FP64 accumulation check of the 8-child means (eq. ftoc): the state is
    bitwise the same with the check on; every coalesced pair of every launch
    is checked; the FP32 sums of FP32-stored values stay within the
    recursive-summation bound gamma_7 sum |v| and differ from the FP64 sums
    (so the check really sums in another precision).  FP16-stored values have
    11 significant bits: 8 of them within a factor 2^13 of each other add up
    exactly in FP32's 24, which the check confirms (deviation 0 here); FP64
    storage sums in FP64 already (deviation 0)."""
    w = W.config_two_level(16)
    say(f"coalescence check {storage}")
    runs = []
    for check in (False, True):
        g = lbm.Forest(w.R, w.n, w.max_level, refine=w.refine, storage=storage)
        rho, u = W.initial_field(w, g.leaves())
        g.set_level_omega(w.omega0)
        g.init_pdfs(rho, u)
        g.set_coalescence_check(check)
        g.step_coarse(5)
        fig = g.coalescence_check()
        runs.append((g.get_pdfs(), fig, g.level_stats(0)["coalesced_pairs"]))
        g.close()
    (h0, fig0, _), (h1, fig1, pairs) = runs
    say(f"  {fig1}")
    assert np.array_equal(h0, h1)
    assert fig0 == {"max_abs_dev": 0.0, "max_bound_ratio": 0.0, "pairs": 0}
    assert fig1["pairs"] == 5 * pairs  # one coalescence launch of level 0 per coarse step
    assert fig1["max_bound_ratio"] <= 1.0
    if storage == "f32":
        assert 0.0 < fig1["max_abs_dev"] < 1e-9
    else:
        assert fig1["max_abs_dev"] == 0.0
