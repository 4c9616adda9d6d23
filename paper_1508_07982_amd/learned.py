"""Learned refinement indicator: snapshot collection, training and the gain
experiment on the decaying-vortex workload.

The paper refines statically (section 3.3) and names dynamic refinement as
future work (section 6).  This driver runs the library's dynamic regrid with
two indicators, both evaluated on the GPU by the library:

* the plain criterion (max |curl u| and mean non-equilibrium norm per block,
  two passes over the cells), which also labels the training data;
* the MLP surrogate over 12 per-block features from one fused pass, with the
  criterion as fallback for blocks near a decision boundary or outside the
  training range.

Thresholds follow one calibration rule: after the first coarse step, each
criterion's largest block value expressed in lattice units of the finest
level, I * 2^(L - Lmax).  A level-L block is then refine-worthy where the
physical vorticity (or strain measure) exceeds 2^(L - Lmax) of that peak, so
the initial blob cores reach the finest level.

    python -m paper_1508_07982_amd.learned [--n 16] [--max-level 4] [--steps 500]
        [--every 50] [--train-seeds 11 12] [--test-seed 5] [--snapshots 20000]
        [--out learned_report.json]
"""

from __future__ import annotations

import argparse
import json
import sys
import time

import numpy as np

from . import lbm
from . import workloads as W

CLASSES = ("coarsen", "keep", "refine")


def make_forest(w: W.Workload, storage: str = "f32") -> lbm.Forest:
    g = lbm.Forest(w.R, w.n, w.max_level, refine=w.refine, storage=storage)
    rho, u = W.initial_field(w, g.leaves())
    g.set_level_omega(w.omega0)
    g.init_pdfs(rho, u)
    return g


def updates_per_coarse_step(g: lbm.Forest) -> int:
    return sum((1 << L) * g.num_cells(L) for L in range(g.num_levels))


def calibrate(w: W.Workload, storage: str = "f32"):
    """(theta_omega, theta_neq): the largest block value of each criterion after
    one coarse step, in lattice units of the finest level."""
    g = make_forest(w, storage)
    g.step_coarse(1)
    _, crit = g.block_indicators()
    levels = g.leaves()[:, 0]
    scale = np.exp2(levels - w.max_level)
    th = (float(np.max(crit[:, 0] * scale)), float(np.max(crit[:, 1] * scale)))
    g.close()
    return th


def target_class(t):
    """0 coarsen, 1 keep, 2 refine from the soft targets 0 / 0.5 / 1."""
    return np.rint(np.asarray(t) * 2).astype(int)


def predicted_class(p):
    p = np.asarray(p)
    return np.where(p > 0.75, 2, np.where(p < 0.25, 0, 1))


def level_moments_on_root_grid(g: lbm.Forest, w: W.Workload):
    """Velocity averaged (volume-weighted) onto the level-0 cells, (R n)^3 x 3."""
    rho, u = g.moments()
    centres, levels, _ = W.cell_centres(g.leaves(), w.R, w.n)
    m = w.roots * w.n
    idx = np.floor(centres * m).astype(np.int64)
    lin = idx[:, 0] + m * (idx[:, 1] + m * idx[:, 2])
    wt = np.exp2(-3.0 * levels)
    out = np.zeros((m ** 3, 3))
    for a in range(3):
        out[:, a] = np.bincount(lin, weights=wt * u[:, a], minlength=m ** 3)
    vol = np.bincount(lin, weights=wt, minlength=m ** 3)
    return out / vol[:, None]


def trajectory(w: W.Workload, mode: str, steps: int, every: int, th, mlp=None, storage: str = "f32",
               collect: bool = False, delta: float = 0.05, log=None):
    """Run `steps` coarse steps; mode 'static' never regrids, 'plain' and
    'mlp' regrid every `every` steps with that indicator.  Returns a report
    dict (and the forest, still open)."""
    g = make_forest(w, storage)
    rep = {"mode": mode, "steps": steps, "every": every, "cell_updates": 0, "indicator_s": 0.0, "regrid_s": 0.0,
           "fallback_blocks": 0, "decided_blocks": 0, "regrids": 0, "blocks": [], "cells": []}
    X, C = [], []
    done = 0
    while done < steps:
        k = min(every, steps - done)
        rep["cell_updates"] += updates_per_coarse_step(g) * k
        g.step_coarse(k)
        done += k
        rep["blocks"].append(g.num_blocks())
        rep["cells"].append(g.num_cells())
        if collect:
            feat, crit = g.block_indicators()
            X.append(feat)
            C.append(crit)
        if mode == "static" or done >= steps:
            continue
        g.synchronize()
        t0 = time.perf_counter()
        flags, nfb = g.refinement_flags(th[0], th[1], mlp=mlp if mode == "mlp" else None, delta=delta)
        t1 = time.perf_counter()
        g.regrid(flags)
        g.synchronize()
        t2 = time.perf_counter()
        rep["indicator_s"] += t1 - t0
        rep["regrid_s"] += t2 - t1
        rep["fallback_blocks"] += int(nfb)
        rep["decided_blocks"] += len(flags)
        rep["regrids"] += 1
        if log:
            log(f"{w.name} {mode}: step {done}, {g.num_blocks()} blocks, {g.num_cells()} cells, "
                f"split {int(np.sum(flags > 0))} merge-candidates {int(np.sum(flags < 0))} fallback {nfb}")
    if collect:
        rep["X"] = np.concatenate(X)
        rep["crit"] = np.concatenate(C)
    return rep, g


def split_indices(n: int, seed: int):
    """Seeded 80/10/10 split."""
    perm = np.random.default_rng(seed).permutation(n)
    a, b = int(0.8 * n), int(0.9 * n)
    return perm[:a], perm[a:b], perm[b:]


def train_surrogate(X, crit, th, seed: int = 0, epochs: int = 60, batch: int = 256, lr: float = 2e-3):
    """Train the MLP on the criterion's soft targets; returns (mlp, report)."""
    t = lbm.plain_targets(crit, th[0], th[1])
    tr, va, te = split_indices(len(X), seed)
    m = lbm.MLP(seed=seed)
    m.fit_normalization(X[tr])
    t0 = time.perf_counter()
    losses = m.train(X[tr], t[tr], epochs=epochs, batch=batch, lr=lr, seed=seed + 1)
    train_s = time.perf_counter() - t0
    rep = {"samples": len(X), "train": len(tr), "val": len(va), "test": len(te), "epochs": epochs,
           "batch": batch, "lr": lr, "train_seconds": train_s, "loss_first_epoch": float(losses[0]),
           "loss_last_epoch": float(losses[-1]),
           "target_mix": {c: float(np.mean(target_class(t) == k)) for k, c in enumerate(CLASSES)}}
    for name, idx in (("val", va), ("test", te)):
        p = m.predict(X[idx])
        pc, tc = predicted_class(p), target_class(t[idx])
        rep[f"{name}_misclassification"] = float(np.mean(pc != tc))
        # refine / coarsen decisions that would flip a block the wrong way
        rep[f"{name}_opposite_decisions"] = float(np.mean(np.abs(pc - tc) == 2))
    return m, rep


def compare(g_a, g_b, w):
    """Relative L2 difference of the root-grid velocity of two runs."""
    ua = level_moments_on_root_grid(g_a, w)
    ub = level_moments_on_root_grid(g_b, w)
    return float(np.linalg.norm(ua - ub) / np.linalg.norm(ub))


def indicator_cost(g: lbm.Forest, th, mlp, repeats: int = 5):
    """Seconds per call of the criterion path and of the MLP path (delta 0, so
    no fallback) on the same state."""
    out = {}
    for name, model in (("plain", None), ("mlp", mlp)):
        g.refinement_flags(th[0], th[1], mlp=model, delta=0.0)  # warm-up
        t0 = time.perf_counter()
        for _ in range(repeats):
            g.refinement_flags(th[0], th[1], mlp=model, delta=0.0)
        out[name + "_s"] = (time.perf_counter() - t0) / repeats
    return out


def gain_experiment(n=16, roots=4, max_level=4, steps=500, every=50, train_seeds=(11, 12), test_seed=5,
                    snapshots=20000, epochs=60, storage="f32", delta=0.05, log=print):
    """Static vs plain-criterion regrid vs MLP regrid on the test blobs; the
    MLP is trained on snapshots of plain-criterion runs with other blobs."""
    report = {"workload": dict(n=n, roots=roots, max_level=max_level, steps=steps, every=every,
                               train_seeds=list(train_seeds), test_seed=test_seed, storage=storage, delta=delta)}
    w_test = W.config_vortices(n, roots, max_level, seed=test_seed)
    th = calibrate(w_test, storage)
    report["theta_omega"], report["theta_neq"] = th
    log(f"thresholds: omega {th[0]:.4e} neq {th[1]:.4e}")

    Xs, Cs = [], []
    for s in train_seeds:
        rep, g = trajectory(W.config_vortices(n, roots, max_level, seed=s), "plain", steps, every, th,
                            storage=storage, collect=True, log=log)
        g.close()
        Xs.append(rep["X"])
        Cs.append(rep["crit"])
        log(f"seed {s}: {len(rep['X'])} block snapshots")
    X, C = np.concatenate(Xs), np.concatenate(Cs)
    pick = np.random.default_rng(0).permutation(len(X))[:snapshots]
    mlp, trep = train_surrogate(X[pick], C[pick], th, seed=1, epochs=epochs)
    report["training"] = trep
    log(f"training: {json.dumps(trep)}")

    runs = {}
    for mode in ("plain", "mlp", "static"):
        rep, g = trajectory(w_test, mode, steps, every, th, mlp=mlp, storage=storage, delta=delta, log=log)
        runs[mode] = (rep, g)
        log(f"{mode}: {rep['cell_updates']:.4e} cell updates, regrid {rep['regrid_s']:.3f} s, "
            f"indicator {rep['indicator_s']:.3f} s")
    g_plain = runs["plain"][1]
    report["indicator_cost"] = indicator_cost(g_plain, th, mlp)
    for mode, (rep, g) in runs.items():
        r = {k: v for k, v in rep.items() if k not in ("X", "crit")}
        r["rel_l2_velocity_vs_plain"] = compare(g, g_plain, w_test) if mode != "plain" else 0.0
        report[mode] = r
    for rep, g in runs.values():
        g.close()
    mlp.close()
    return report


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--n", type=int, default=16)
    ap.add_argument("--roots", type=int, default=4)
    ap.add_argument("--max-level", type=int, default=4)
    ap.add_argument("--steps", type=int, default=500)
    ap.add_argument("--every", type=int, default=50)
    ap.add_argument("--train-seeds", type=int, nargs="+", default=[11, 12])
    ap.add_argument("--test-seed", type=int, default=5)
    ap.add_argument("--snapshots", type=int, default=20000)
    ap.add_argument("--epochs", type=int, default=60)
    ap.add_argument("--storage", default="f32")
    ap.add_argument("--delta", type=float, default=0.05)
    ap.add_argument("--out", default=None)
    a = ap.parse_args(argv)

    def log(msg):
        print(msg, flush=True)

    rep = gain_experiment(a.n, a.roots, a.max_level, a.steps, a.every, tuple(a.train_seeds), a.test_seed,
                          a.snapshots, a.epochs, a.storage, a.delta, log)
    text = json.dumps(rep, indent=1)
    print(text, flush=True)
    if a.out:
        with open(a.out, "w") as fh:
            fh.write(text + "\n")
    return 0


if __name__ == "__main__":
    sys.exit(main())
