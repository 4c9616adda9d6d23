"""Pins of the oracle's refinement indicators and MLP (oracle/indicator.py).

The criterion and the surrogate are this project's definitions (the paper
refines statically, section 3.3); each pin fixes a value by a closed form
that the definitions imply, not by re-running the oracle's formulas:

* an equilibrium state with a velocity field linear inside every block has
  exact block-local differences, so max |curl u| and the octant-mean curl
  are the constant curl of the field, the octant jumps are slope * n / 2,
  and the non-equilibrium norm vanishes;
* a non-hydrodynamic perturbation g (zero mass and momentum) added to the
  equilibrium leaves f_eq unchanged and is scaled by (1 - omega) by the
  collision, so mean neq = |1 - omega| delta ||g|| / rho;
* density linear along x gives mean and std of rho in closed form;
* the MLP with identity hidden layers computes sigmoid(sum relu(x_hat));
* the analytic gradient matches central differences of the loss;
* Adam with a constant gradient moves every parameter by lr g / (|g| + eps)
  per step, and its moment recursion written out by hand for two steps on a
  quadratic gives the same path.
"""

import numpy as np

from oracle import Forest, RefinedOracle
from oracle import indicator as ind
from oracle import refined as orc


def two_level(n=8):
    return Forest.build((2, 2, 2), n, 1, lambda L, x, y, z: (x, y, z) == (1, 0, 1))


def local_index(n):
    c = np.arange(n ** 3)
    return c % n, (c // n) % n, c // (n * n)


def set_equilibrium(o, rho_fn, u_fn):
    """Interior PDFs = f_eq(rho, u) with rho, u functions of the local index."""
    n = o.n
    i, j, k = local_index(n)
    for L in range(o.num_levels):
        B = o.n_int(L) // n ** 3
        rho = np.tile(rho_fn(i, j, k), B)
        u = np.tile(u_fn(i, j, k), (B, 1))
        o.set_interior_pdfs(L, orc.equilibrium(rho, u))


def test_linear_field_curl_jumps_and_zero_neq():
    n = 8
    o = RefinedOracle(two_level(n), 1.4)
    a, b, c = 2e-3, -1.5e-3, 7e-4
    # u = (a j, b i, c j): curl = (c, 0, b - a)
    set_equilibrium(o, lambda i, j, k: np.ones(n ** 3),
                    lambda i, j, k: np.stack([a * j, b * i, c * j], -1).astype(float))
    feat, crit = ind.block_indicators(o)
    curl = np.hypot(c, b - a)
    assert np.allclose(crit[:, 0], curl, rtol=0, atol=1e-15)
    assert np.all(crit[:, 1] < 1e-15)
    # octant means: jumps along x = |b| n/2 (u_y), along y = hypot(a, c) n/2, along z = 0
    assert np.allclose(feat[:, 6], np.log10(abs(b) * n / 2 + 1e-12), atol=1e-12)
    assert np.allclose(feat[:, 7], np.log10(np.hypot(a, c) * n / 2 + 1e-12), atol=1e-12)
    assert np.allclose(feat[:, 8], -12.0, atol=1e-3)
    assert np.allclose(feat[:, 9], np.log10(curl + 1e-12), atol=1e-12)
    # rms |u - mean u|: each component is linear in one index, whose
    # variance over 0..n-1 is (n^2 - 1) / 12
    rms = np.sqrt((a * a + b * b + c * c) * (n * n - 1) / 12.0)
    assert np.allclose(feat[:, 4], np.log10(rms + 1e-12), atol=1e-12)
    # level / Lmax and the density features of rho = 1
    levels = np.concatenate([np.full(o.n_int(L) // n ** 3, L) for L in range(o.num_levels)])
    assert np.array_equal(feat[:, 0], levels / 1.0)
    assert np.allclose(feat[:, 1], 0.0, atol=1e-12)
    assert np.allclose(feat[:, 2], -12.0, atol=1e-3)


def test_uniform_flow_features():
    n = 8
    o = RefinedOracle(two_level(n), 1.2)
    u0 = np.array([0.03, -0.01, 0.02])
    set_equilibrium(o, lambda i, j, k: np.full(n ** 3, 1.0), lambda i, j, k: np.tile(u0, (n ** 3, 1)))
    feat, crit = ind.block_indicators(o)
    assert np.all(crit < 1e-15)
    un = np.linalg.norm(u0)
    assert np.allclose(feat[:, 3], np.log10(un + 1e-12), atol=1e-12)   # |mean u|
    assert np.allclose(feat[:, 5], np.log10(un + 1e-12), atol=1e-12)   # max |u|
    assert np.all(feat[:, 4] < -7)                                       # rms |u - mean u| ~ roundoff


def test_density_ramp_mean_and_std():
    n = 8
    o = RefinedOracle(two_level(n), 1.0)  # omega = 1 on level 0: collision maps to f_eq
    eps = 1e-3
    set_equilibrium(o, lambda i, j, k: 1.0 + eps * i, lambda i, j, k: np.zeros((n ** 3, 3)))
    feat, _ = ind.block_indicators(o)
    assert np.allclose(feat[:, 1], 1e3 * eps * (n - 1) / 2, atol=1e-10)
    assert np.allclose(feat[:, 2], np.log10(eps * np.sqrt((n * n - 1) / 12.0) + 1e-12), atol=1e-10)


def test_non_equilibrium_norm_of_ghost_mode():
    n = 8
    omega0 = 1.3
    o = RefinedOracle(two_level(n), omega0)
    e, _ = orc.lattice()
    # g: +1 on the x faces, -1 on the y faces: zero mass and momentum, ||g|| = 2
    g = np.zeros(19)
    for a in range(19):
        if abs(e[a, 0]) == 1 and e[a, 1] == 0 and e[a, 2] == 0:
            g[a] = 1.0
        if abs(e[a, 1]) == 1 and e[a, 0] == 0 and e[a, 2] == 0:
            g[a] = -1.0
    assert g.sum() == 0 and np.all(g @ e == 0) and np.linalg.norm(g) == 2.0
    delta = 1e-3
    rho0 = 1.01
    for L in range(o.num_levels):
        m = o.n_int(L)
        f = orc.equilibrium(np.full(m, rho0), np.tile([0.01, 0.0, -0.02], (m, 1))) + delta * g
        o.set_interior_pdfs(L, f)
    _, crit = ind.block_indicators(o)
    nb0 = o.n_int(0) // n ** 3
    for L in range(o.num_levels):
        want = abs(1.0 - o.omega[L]) * delta * 2.0 / rho0
        sl = slice(0, nb0) if L == 0 else slice(nb0, None)
        assert np.allclose(crit[sl, 1], want, rtol=1e-10, atol=0)


def test_non_equilibrium_of_one_cell_mean_and_max():
    """The ghost mode g on one cell of every block: the block's mean
    non-equilibrium norm is |1 - omega| delta ||g|| / rho / n^3 and its
    maximum (feature 11) |1 - omega| delta ||g|| / rho."""
    n = 8
    o = RefinedOracle(two_level(n), 1.3)
    e, _ = orc.lattice()
    g = np.zeros(19)
    g[[1, 2]] = 1.0   # the two x faces
    g[[5, 6]] = -1.0  # the two z faces
    assert g.sum() == 0 and np.all(g @ e == 0)
    delta, rho0, cell = 2e-3, 0.99, 37
    for L in range(o.num_levels):
        m = o.n_int(L)
        f = orc.equilibrium(np.full(m, rho0), np.tile([-0.01, 0.02, 0.005], (m, 1)))
        f[cell::n ** 3] += delta * g
        o.set_interior_pdfs(L, f)
    feat, crit = ind.block_indicators(o)
    nb0 = o.n_int(0) // n ** 3
    for L in range(o.num_levels):
        peak = abs(1.0 - o.omega[L]) * delta * 2.0 / rho0
        sl = slice(0, nb0) if L == 0 else slice(nb0, None)
        assert np.allclose(crit[sl, 1], peak / n ** 3, rtol=1e-9, atol=0)
        assert np.allclose(feat[sl, 10], np.log10(peak / n ** 3 + 1e-12), atol=1e-9)
        assert np.allclose(feat[sl, 11], np.log10(peak + 1e-12), atol=1e-9)


def test_adam_constant_gradient_closed_form():
    """With a constant gradient g the bias-corrected moments are g and g^2
    at every step, so each Adam step moves p by -lr g / (|g| + eps)."""
    g = np.array([3.0, -0.5, 0.0, 2e-9, -1e4])
    p0 = np.array([1.0, 2.0, 3.0, 4.0, 5.0])
    lr = 1e-2
    path = ind.adam(p0, lambda p: g, 4, lr)
    step = -lr * g / (np.abs(g) + 1e-8)
    for t in range(4):
        assert np.allclose(path[t], p0 + (t + 1) * step, rtol=0, atol=1e-14)


def test_adam_on_quadratic_descends_and_follows_the_moments():
    """On f(p) = |p|^2 / 2 (gradient p) Adam's first step is lr sign(p), and
    the recursion of m and v written out for two steps gives the second."""
    p0 = np.array([0.5, -2.0, 1e-3])
    lr = 0.1
    path = ind.adam(p0, lambda p: p, 2, lr)
    p1 = p0 - lr * p0 / (np.abs(p0) + 1e-8)
    assert np.allclose(path[0], p1, rtol=0, atol=1e-15)
    m = 0.9 * 0.1 * p0 + 0.1 * p1
    v = 0.999 * 0.001 * p0 ** 2 + 0.001 * p1 ** 2
    p2 = p1 - lr * (m / (1 - 0.81)) / (np.sqrt(v / (1 - 0.999 ** 2)) + 1e-8)
    assert np.allclose(path[1], p2, rtol=0, atol=1e-15)


def test_plain_targets_cases():
    crit = np.array([[2.0, 0.0], [0.0, 2.0], [0.4, 0.4], [0.4, 0.6], [0.6, 0.4], [1.0, 1.0]])
    t = ind.plain_targets(crit, 1.0, 1.0)
    assert t.tolist() == [1.0, 1.0, 0.0, 0.5, 0.5, 0.5]


def test_mlp_identity_network():
    H, F = ind.H, ind.NFEAT
    p = np.zeros(ind.NPARAM)
    W1 = np.zeros((H, F))
    W1[:F, :F] = np.eye(F)
    W2 = np.zeros((H, H))
    W2[:F, :F] = np.eye(F)
    w3 = np.zeros(H)
    w3[:F] = 1.0
    b3 = -0.5
    p[:H * F] = W1.ravel()
    o = H * F + H
    p[o:o + H * H] = W2.ravel()
    o += H * H + H
    p[o:o + H] = w3
    p[o + H] = b3
    rng = np.random.default_rng(3)
    X = rng.normal(size=(20, F))
    mean, std = rng.normal(size=F), rng.uniform(0.5, 2.0, F)
    xh = (X - mean) / std
    want = 1.0 / (1.0 + np.exp(-(np.maximum(xh, 0).sum(1) + b3)))
    got, _ = ind.forward(p, X, mean, std)
    assert np.allclose(got, want, rtol=0, atol=1e-15)


def test_mlp_gradient_matches_central_differences():
    rng = np.random.default_rng(7)
    p = rng.normal(scale=0.3, size=ind.NPARAM)
    X = rng.normal(size=(16, ind.NFEAT))
    t = rng.choice([0.0, 0.5, 1.0], size=16)
    mean, std = rng.normal(size=ind.NFEAT), rng.uniform(0.5, 2.0, ind.NFEAT)
    g = ind.gradient(p, X, t, mean, std)
    idx = rng.choice(ind.NPARAM, 60, replace=False)
    idx = np.concatenate([idx, [ind.NPARAM - 1, 0, ind.H * ind.NFEAT]])  # b3, W1[0][0], b1[0]
    h = 1e-6
    for q in idx:
        pp, pm = p.copy(), p.copy()
        pp[q] += h
        pm[q] -= h
        fd = (ind.loss(pp, X, t, mean, std) - ind.loss(pm, X, t, mean, std)) / (2 * h)
        assert abs(fd - g[q]) <= 1e-7 + 1e-5 * abs(fd), (q, fd, g[q])
