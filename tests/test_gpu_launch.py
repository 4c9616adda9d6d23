"""Launch shapes and the autotuner through the C ABI: per-level persistent
grids, XCD-grouped tile orders and workgroup splits give bitwise the same
state as the default launch, the autotuner leaves the simulation state
exactly where it was (and its JSON cache reproduces its choice), and
per-level settings survive a regrid."""

import numpy as np
import pytest

from paper_1508_07982_amd import lbm

pytestmark = pytest.mark.gpu


def spec_three(n):
    def refine(L, x, y, z):
        return (L == 0 and (x, y, z) == (1, 1, 1)) or (L == 1 and (x, y, z) == (3, 3, 2))
    return (3, 3, 3), n, 3, refine


def make(storage="f32", n=8, seed=1):
    R, n, Lmax, refine = spec_three(n)
    g = lbm.Forest(R, n, Lmax, refine=refine, storage=storage)
    N = g.num_cells()
    rng = np.random.default_rng(seed)
    g.set_level_omega(1.7)
    g.init_pdfs(1.0 + 0.01 * rng.uniform(-1, 1, N), 0.03 * rng.uniform(-1, 1, (N, 3)))
    return g


@pytest.mark.parametrize("storage, n", [("f32", 8), ("f16", 8), ("f64", 8), ("f32", 16), ("f16", 16)])
@pytest.mark.parametrize("shape", [[(0, 1, 1), (2, 0, 2), (1, 1, 4)], [(4, 1, 2), (0, 1, 4), (8, 0, 1)],
                                   [(-1, 1, 2), (-1, 1, 1), (-1, 0, 4)]])
def test_level_launch_shapes_bitwise_equal(storage, n, shape):
    print(f"level launch {storage} n={n} {shape}", flush=True)
    ref = make(storage, n)
    ref.set_schedule("direct")
    ref.step_coarse(3)
    want = ref.get_pdfs()
    ref.close()
    g = make(storage, n)
    for L, (p, o, s) in enumerate(shape):
        g.set_level_launch(L, p, o, s)
        got = g.get_level_launch(L)
        assert got[:2] == (p, o) and got[2] in (1, 2, 4) and got[2] <= s
    g.step_coarse(3)
    assert np.array_equal(g.get_pdfs(), want)
    g.close()


def test_autotune_restores_state_and_applies_choice():
    ref = make("f32", seed=4)
    ref.step_coarse(2)
    ref.step_coarse(2)
    want = ref.get_pdfs()
    ref.close()
    g = make("f32", seed=4)
    g.step_coarse(2)
    res = g.autotune(n_steps=1)
    assert len(res) == g.num_levels
    for r in res:
        assert r["persistent"] in (0, 1, 2, 4, 8) and r["order"] in (0, 1) and r["split"] in (1, 2, 4)
        assert r["fuse"] in (0, 1) and g.get_level_fusion(r["level"]) == bool(r["fuse"])
        assert r["ms_per_level_step"] > 0
        assert g.get_level_launch(r["level"]) == (r["persistent"], r["order"], r["split"])
    g.step_coarse(2)
    assert np.array_equal(g.get_pdfs(), want)
    g.close()


def test_autotune_cache_reproduces_choice(tmp_path):
    cache = str(tmp_path / "launch.json")
    g = make("f32", seed=7)
    first = g.autotune(n_steps=1, cache=cache)
    g.close()
    g = make("f32", seed=7)
    again = g.autotune(n_steps=1, cache=cache)
    assert all(r.get("cached") for r in again)
    for a, b in zip(first, again):
        assert (a["persistent"], a["order"], a["split"], a["fuse"]) == (b["persistent"], b["order"], b["split"], b["fuse"])
        assert g.get_level_launch(a["level"]) == (a["persistent"], a["order"], a["split"])
        assert g.get_level_fusion(a["level"]) == bool(a["fuse"])
    g.close()


def test_autotune_with_empty_level():
    # level 0 holds no blocks: the 2:1 balance splits every root
    def refine(L, x, y, z):
        return L == 0 or (L == 1 and (x, y, z) == (1, 1, 0))
    want = None
    for tune in (False, True):
        g = lbm.Forest((2, 2, 2), 8, 2, refine=refine, storage="f32")
        assert g.num_cells(0) == 0
        N = g.num_cells()
        rng = np.random.default_rng(6)
        g.set_level_omega(1.6)
        g.init_pdfs(1.0 + 0.01 * rng.uniform(-1, 1, N), 0.03 * rng.uniform(-1, 1, (N, 3)))
        g.step_coarse(1)
        if tune:
            res = g.autotune(n_steps=1)
            assert res[0]["ms_per_level_step"] == 0.0
        g.step_coarse(2)
        if want is None:
            want = g.get_pdfs()
        else:
            assert np.array_equal(g.get_pdfs(), want)
        g.close()


def test_level_launch_kept_across_regrid():
    a = make("f32", seed=5)
    b = make("f32", seed=5)
    for L in range(b.num_levels):
        b.set_level_launch(L, 2, 1, 2)
    a.step_coarse(1)
    b.step_coarse(1)
    rng = np.random.default_rng(9)
    flags = rng.choice([-1, 0, 1], size=a.num_blocks(), p=[0.4, 0.4, 0.2]).astype(np.int8)
    nl = b.num_levels
    a.regrid(flags)
    b.regrid(flags)
    for L in range(min(nl, b.num_levels)):
        assert b.get_level_launch(L)[:2] == (2, 1)
    a.step_coarse(2)
    b.step_coarse(2)
    assert np.array_equal(a.get_pdfs(), b.get_pdfs())
    a.close()
    b.close()


def test_level_launch_rejects_bad_arguments():
    g = make("f32")
    with pytest.raises(lbm.LBMError):
        g.set_level_launch(g.num_levels, 0, 0)
    with pytest.raises(lbm.LBMError):
        g.set_level_launch(0, 0, 2)
    with pytest.raises(lbm.LBMError):
        g.set_level_launch(0, 65, 0)
    with pytest.raises(lbm.LBMError):
        g.set_level_launch(0, 0, 0, 3)
    g.close()
