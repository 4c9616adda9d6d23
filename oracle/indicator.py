"""FP64 oracle of the refinement indicators and of the MLP (test infrastructure).

The paper refines statically and leaves the refinement criterion to the user
(section 3.3); the criterion and the learned surrogate below are this
project's definitions, written out plainly so that the HIP kernels can be
checked against them.

Per block, from the post-collision state (the state the library stores
between coarse steps; from the oracle's post-streaming state it is one
collision away):

  rho, u per cell (eq. fvelocity), f_eq (eq. fequ),
  neq(x)   = ||f(x) - f_eq(x)||_2 / rho(x)
  curl(x)  = |curl u| with block-local differences in lattice units of the
             block's level: central (u[i+1] - u[i-1]) / 2 inside, one-sided
             u[1] - u[0] and u[n-1] - u[n-2] on the block faces
  I_omega  = max_x curl(x),  I_neq = mean_x neq(x)

Plain decision: refine-worthy (target 1) if I_omega > theta_omega or
I_neq > theta_neq; coarsen-worthy (target 0) if I_omega < theta_omega / 2 and
I_neq < theta_neq / 2; keep (target 0.5) otherwise.

Features (12): level / Lmax, 1e3 * mean(rho - 1), then log10(x + 1e-12) of
std(rho), |mean u|, rms |u - mean u|, max |u|, the three octant-mean jumps
|mean over the upper half - mean over the lower half| of u along x, y, z,
|curl| of the 2x2x2 octant-mean field (spacing n/2), mean neq and max neq.

MLP 12 -> 64 -> 64 -> 1: x_hat = (x - mean) / std, h1 = relu(W1 x_hat + b1),
h2 = relu(W2 h1 + b2), p = sigmoid(w3 . h2 + b3); loss = mean binary cross
entropy against the soft targets.  Parameters packed as
W1[64][12], b1[64], W2[64][64], b2[64], w3[64], b3.
"""

from __future__ import annotations

import numpy as np

from . import refined as orc

NFEAT = 12
H = 64
NPARAM = H * NFEAT + H + H * H + H + H + 1


def block_moments_post_collision(o, L):
    """(f post-collision (B, n^3, 19), rho, u) of level L of oracle `o`."""
    n = o.n
    f = orc.collide(o.interior_pdfs(L), o.omega[L])
    rho, u = orc.moments(f)
    B = len(f) // n ** 3
    return f.reshape(B, n ** 3, 19), rho.reshape(B, n ** 3), u.reshape(B, n ** 3, 3)


def _curl_block(u, n):
    """|curl u| per cell of one block, u (n^3, 3) x-fastest."""
    U = u.reshape(n, n, n, 3)  # [z][y][x][c]

    def d(axis_arr, ax):
        g = np.empty_like(axis_arr)
        sl = [slice(None)] * 3
        # central inside
        a = np.moveaxis(axis_arr, ax, 0)
        gm = np.moveaxis(g, ax, 0)
        gm[1:-1] = (a[2:] - a[:-2]) / 2.0
        gm[0] = a[1] - a[0]
        gm[-1] = a[-1] - a[-2]
        return g

    # axes of U: 0 = z, 1 = y, 2 = x
    dux_dy = d(U[..., 0], 1)
    dux_dz = d(U[..., 0], 0)
    duy_dx = d(U[..., 1], 2)
    duy_dz = d(U[..., 1], 0)
    duz_dx = d(U[..., 2], 2)
    duz_dy = d(U[..., 2], 1)
    cx = duz_dy - duy_dz
    cy = dux_dz - duz_dx
    cz = duy_dx - dux_dy
    return np.sqrt(cx * cx + cy * cy + cz * cz).ravel()


def block_indicators(o):
    """Per block, canonical order: features (B, 12) and (I_omega, I_neq) (B, 2)."""
    n = o.n
    Lmax = o.num_levels - 1
    _, w = orc.lattice()
    feats, crit = [], []
    loc = np.stack(np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij"), -1)
    loc = loc.transpose(2, 1, 0, 3).reshape(-1, 3)
    half = (loc >= n // 2).astype(int)
    octant = half[:, 0] + 2 * half[:, 1] + 4 * half[:, 2]
    for L in range(o.num_levels):
        if o.n_int(L) == 0:
            continue
        f, rho, u = block_moments_post_collision(o, L)
        for b in range(len(rho)):
            r, v, fb = rho[b], u[b], f[b]
            feq = orc.equilibrium(r, v)
            neq = np.sqrt(((fb - feq) ** 2).sum(1)) / r
            curl = _curl_block(v, n)
            ubar = v.mean(0)
            rms = np.sqrt(max(((v - ubar) ** 2).sum(1).mean(), 0.0))
            oct_mean = np.array([v[octant == q].mean(0) for q in range(8)])
            jumps = []
            grads = []
            for ax in range(3):
                hi = oct_mean[[q for q in range(8) if (q >> ax) & 1]].mean(0)
                lo = oct_mean[[q for q in range(8) if not (q >> ax) & 1]].mean(0)
                jumps.append(np.linalg.norm(hi - lo))
                grads.append((hi - lo) / (n / 2.0))
            gx, gy, gz = grads  # d/dx, d/dy, d/dz of the octant-mean field (vectors)
            curl_oct = np.array([gy[2] - gz[1], gz[0] - gx[2], gx[1] - gy[0]])
            raw = [np.std(r), np.linalg.norm(ubar), rms, np.sqrt((v ** 2).sum(1)).max(),
                   jumps[0], jumps[1], jumps[2], np.linalg.norm(curl_oct), neq.mean(), neq.max()]
            feats.append([L / max(Lmax, 1), 1e3 * (r - 1.0).mean()] + [np.log10(x + 1e-12) for x in raw])
            crit.append([curl.max(), neq.mean()])
    return np.array(feats), np.array(crit)


def plain_targets(crit, theta_omega, theta_neq):
    Iw, In = crit[:, 0], crit[:, 1]
    t = np.full(len(crit), 0.5)
    t[(Iw < theta_omega / 2) & (In < theta_neq / 2)] = 0.0
    t[(Iw > theta_omega) | (In > theta_neq)] = 1.0
    return t


# ---------------------------------------------------------------------------
# MLP in FP64
# ---------------------------------------------------------------------------

def unpack(params):
    p = np.asarray(params, dtype=np.float64)
    i = 0
    W1 = p[i:i + H * NFEAT].reshape(H, NFEAT); i += H * NFEAT
    b1 = p[i:i + H]; i += H
    W2 = p[i:i + H * H].reshape(H, H); i += H * H
    b2 = p[i:i + H]; i += H
    w3 = p[i:i + H]; i += H
    b3 = p[i]
    return W1, b1, W2, b2, w3, b3


def forward(params, X, mean, std):
    W1, b1, W2, b2, w3, b3 = unpack(params)
    Xh = (np.asarray(X, dtype=np.float64) - mean) / std
    a1 = Xh @ W1.T + b1
    h1 = np.maximum(a1, 0.0)
    a2 = h1 @ W2.T + b2
    h2 = np.maximum(a2, 0.0)
    z = h2 @ w3 + b3
    p = 1.0 / (1.0 + np.exp(-z))
    return p, (Xh, a1, h1, a2, h2, z)


def loss(params, X, t, mean, std):
    p, _ = forward(params, X, mean, std)
    p = np.clip(p, 1e-12, 1 - 1e-12)
    return float(np.mean(-(t * np.log(p) + (1 - t) * np.log(1 - p))))


def gradient(params, X, t, mean, std):
    """Analytic gradient of the mean BCE loss (chain rule, layer by layer)."""
    W1, b1, W2, b2, w3, b3 = unpack(params)
    p, (Xh, a1, h1, a2, h2, z) = forward(params, X, mean, std)
    B = len(X)
    dz = (p - t) / B
    gw3 = h2.T @ dz
    gb3 = dz.sum()
    dA2 = np.outer(dz, w3) * (a2 > 0)
    gW2 = dA2.T @ h1
    gb2 = dA2.sum(0)
    dA1 = (dA2 @ W2) * (a1 > 0)
    gW1 = dA1.T @ Xh
    gb1 = dA1.sum(0)
    return np.concatenate([gW1.ravel(), gb1, gW2.ravel(), gb2, gw3, [gb3]])


def adam(params, grad_fn, steps, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """`steps` Adam updates (Kingma & Ba, "Adam: a method for stochastic
    optimization", 2015, Algorithm 1) of params with the gradient grad_fn(p):
    first and second moment estimates m, v with bias corrections
    1 - beta^t, p <- p - lr m_hat / (sqrt(v_hat) + eps).  Returns the
    parameters after every step, (steps, P)."""
    p = np.array(params, dtype=np.float64)
    m = np.zeros_like(p)
    v = np.zeros_like(p)
    out = []
    for t in range(1, steps + 1):
        g = grad_fn(p)
        m = beta1 * m + (1.0 - beta1) * g
        v = beta2 * v + (1.0 - beta2) * g * g
        m_hat = m / (1.0 - beta1 ** t)
        v_hat = v / (1.0 - beta2 ** t)
        p = p - lr * m_hat / (np.sqrt(v_hat) + eps)
        out.append(p.copy())
    return np.array(out)
