"""Refinement indicators and the MLP on the GPU against the FP64 oracle
(oracle/indicator.py), through the C ABI.

* criterion values and features of every block (FP64 storage: rounding
  order only) and the fused single-pass features against the two-pass ones;
* MLP forward and gradient (FP32 kernels) against the FP64 oracle with the
  same parameters; training lowers the loss, and the reported epoch loss is
  the oracle's loss of the trained parameters;
* regrid flags: the criterion path against the oracle's decision, the MLP
  path with every block sent to the fallback, and with none.
"""

import numpy as np
import pytest

from oracle import Forest, RefinedOracle
from oracle import indicator as ind
from paper_1508_07982_amd import lbm

pytestmark = pytest.mark.gpu

MAX_LEVEL = 3


def three_level_spec(n):
    def refine(L, x, y, z):
        return (L == 0 and (x, y, z) == (1, 1, 1)) or (L == 1 and (x, y, z) == (3, 3, 2))
    return (3, 3, 3), n, refine


def _pair(n, storage, seed, steps):
    R, _, refine = three_level_spec(n)
    of = Forest.build(R, n, 2, refine)
    o = RefinedOracle(of, 1.45)
    g = lbm.Forest(R, n, MAX_LEVEL, refine=refine, storage=storage)
    rng = np.random.default_rng(seed)
    N = o.total_cells()
    rho = 1.0 + 0.01 * rng.uniform(-1, 1, N)
    u = 0.04 * rng.uniform(-1, 1, (N, 3))
    o.init_pdfs(rho, u)
    g.set_level_omega(1.45)
    g.init_pdfs(rho, u)
    o.step(steps)
    g.step_coarse(steps)
    return o, g


@pytest.mark.parametrize("n, seed, steps", [(8, 0, 2), (4, 1, 1), (16, 2, 1)])
def test_indicators_match_oracle_fp64(n, seed, steps):
    print(f"indicators n={n} seed={seed} steps={steps}", flush=True)
    o, g = _pair(n, "f64", seed, steps)
    f0, c0 = ind.block_indicators(o)
    f1, c1 = g.block_indicators()
    assert f1.shape == f0.shape and c1.shape == c0.shape
    assert np.max(np.abs(c1 - c0) / np.abs(c0)) < 1e-10
    assert np.max(np.abs(f1 - f0)) < 1e-8
    g.close()


@pytest.mark.parametrize("storage", ["f64", "f32", "f16"])
def test_fused_features_equal_two_pass(storage):
    print(f"fused features {storage}", flush=True)
    _, g = _pair(8, storage, 3, 1)
    f_two, _ = g.block_indicators()
    f_one = g.block_features()
    assert np.max(np.abs(f_one - f_two)) < 1e-9
    g.close()


def _mlp_inputs(seed, B=300):
    rng = np.random.default_rng(seed)
    X = rng.normal(size=(B, ind.NFEAT)) * rng.uniform(0.5, 3, ind.NFEAT) + rng.normal(size=ind.NFEAT)
    t = rng.choice([0.0, 0.5, 1.0], size=B)
    return X, t


def test_mlp_forward_matches_oracle():
    X, _ = _mlp_inputs(4)
    m = lbm.MLP(seed=11)
    m.fit_normalization(X)
    p = m.params().astype(np.float64)
    mean, std = X.mean(0), np.maximum(X.std(0), 1e-6)
    want, _ = ind.forward(p, X, mean, std)
    got = m.predict(X)
    assert np.max(np.abs(got - want)) < 2e-6
    m.close()


def test_mlp_gradient_matches_oracle():
    X, t = _mlp_inputs(5)
    m = lbm.MLP(seed=12)
    m.fit_normalization(X)
    p = m.params().astype(np.float64)
    mean, std = X.mean(0), np.maximum(X.std(0), 1e-6)
    want = ind.gradient(p, X, t, mean, std)
    got = m.gradient(X, t).astype(np.float64)
    assert np.linalg.norm(got - want) / np.linalg.norm(want) < 1e-4
    m.close()


def test_mlp_adam_steps_match_oracle():
    """Three full-batch training steps (batch = n, so the shuffle does not
    change the mean gradient) against the FP64 Adam of the oracle from the
    same initial parameters: the parameter changes agree to FP32 accuracy."""
    X, t = _mlp_inputs(7)
    m = lbm.MLP(seed=3)
    m.fit_normalization(X)
    p0 = m.params().astype(np.float64)
    mean, std = X.mean(0), np.maximum(X.std(0), 1e-6)
    lr = 1e-3
    want = ind.adam(p0, lambda p: ind.gradient(p, X, t, mean, std), 3, lr)
    g0 = np.abs(ind.gradient(p0, X, t, mean, std))
    # parameters whose gradient is far above FP32 rounding of the sums: Adam
    # moves them by about lr per step whatever the gradient's size, so a
    # gradient at rounding level would decide a sign
    live = g0 > 1e-5 * g0.max()
    for step in range(3):
        m.train(X, t, epochs=1, batch=len(X), lr=lr, seed=step)
        got = m.params().astype(np.float64)
        d_got, d_want = got - p0, want[step] - p0
        assert np.max(np.abs(d_got[live] - d_want[live])) < 2e-2 * lr * (step + 1), step
        assert np.max(np.abs(d_got)) <= 1.1 * lr * (step + 1)
    m.close()


def test_mlp_training_lowers_loss():
    rng = np.random.default_rng(6)
    X = rng.normal(size=(2048, ind.NFEAT))
    s = X[:, 0] + 0.5 * X[:, 3] - X[:, 7]
    t = np.where(s > 0.5, 1.0, np.where(s < -0.5, 0.0, 0.5))
    m = lbm.MLP(seed=1)
    m.fit_normalization(X)
    mean, std = X.mean(0), np.maximum(X.std(0), 1e-6)
    l0 = ind.loss(m.params().astype(np.float64), X, t, mean, std)
    losses = m.train(X, t, epochs=20, batch=128, lr=3e-3, seed=2)
    l1 = ind.loss(m.params().astype(np.float64), X, t, mean, std)
    assert abs(losses[-1] - l1) < 1e-4
    assert losses[-1] < losses[0] and l1 < 0.75 * l0
    # entropy floor of the soft targets: 0.5 labels cost log 2 at best
    floor = np.mean(t == 0.5) * np.log(2.0)
    assert l1 - floor < 0.15
    m.close()


def _oracle_flags(o, crit, th_w, th_n):
    t = ind.plain_targets(crit, th_w, th_n)
    levels = np.concatenate([np.full(o.n_int(L) // o.n ** 3, L) for L in range(o.num_levels)])
    d = np.where(t == 1.0, 1, np.where(t == 0.0, -1, 0))
    d[(d > 0) & (levels >= MAX_LEVEL)] = 0
    d[(d < 0) & (levels == 0)] = 0
    return d.astype(np.int8)


def _thresholds(crit):
    """Thresholds at the medians, moved off any value within 1e-6 relative."""
    th = []
    for k in range(2):
        v = np.sort(crit[:, k])
        x = float(np.median(v))
        while np.any(np.abs(v - x) < 1e-6 * x) or np.any(np.abs(v - 0.5 * x) < 1e-6 * x):
            x *= 1.001
        th.append(x)
    return th


def test_plain_flags_match_oracle():
    o, g = _pair(8, "f64", 7, 2)
    _, crit = ind.block_indicators(o)
    th_w, th_n = _thresholds(crit)
    flags, nfb = g.refinement_flags(th_w, th_n)
    assert nfb == 0
    want = _oracle_flags(o, crit, th_w, th_n)
    assert np.array_equal(flags, want)
    assert np.any(flags > 0) and np.any(flags < 0)
    g.close()


def test_mlp_flags_fallback_and_direct():
    o, g = _pair(8, "f32", 8, 2)
    feat, crit = g.block_indicators()
    th_w, th_n = _thresholds(crit)
    plain, _ = g.refinement_flags(th_w, th_n)
    m = lbm.MLP(seed=3)
    m.fit_normalization(feat)
    # delta 0.5: every probability is within 0.5 of 0.25 or 0.75
    flags, nfb = g.refinement_flags(th_w, th_n, mlp=m, delta=0.5)
    assert nfb == g.num_blocks()
    assert np.array_equal(flags, plain)
    # delta 0 and a training range that covers the features: the MLP decides
    flags, nfb = g.refinement_flags(th_w, th_n, mlp=m, delta=0.0)
    assert nfb == 0
    p = m.predict(g.block_features())
    levels = g.leaves()[:, 0]
    want = np.where(p > 0.75, 1, np.where(p < 0.25, -1, 0))
    want[(want > 0) & (levels >= MAX_LEVEL)] = 0
    want[(want < 0) & (levels == 0)] = 0
    clear = (np.abs(p - 0.75) > 1e-5) & (np.abs(p - 0.25) > 1e-5)
    assert np.array_equal(flags[clear], want[clear].astype(np.int8))
    # features outside the training range go to the fallback
    m.set_normalization(feat.mean(0), np.maximum(feat.std(0), 1e-6), feat.min(0) + 1e-9, feat.max(0))
    flags, nfb = g.refinement_flags(th_w, th_n, mlp=m, delta=0.0)
    assert nfb >= 1
    m.close()
    g.close()
