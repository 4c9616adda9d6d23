"""Storage forms against the FP64 oracle on the benchmark geometry at 1/8 of
its cells: the sphere-shell grid (4^3 roots, sphere surface of radius 0.25
refined to level 3) with 16^3-cell blocks, 15.2 M cells, omega_0 = 1.9,
Taylor-Green 0.02 plus noise.  Too slow for the test suite (the oracle's
tables take minutes); run on a GPU machine as

    python tests/precision_sphere_eighth.py [--steps 10] [--out report.json]

and it prints volume-weighted velocity and density rel-L2 and the mass drift
of the FP32 and FP16 forms after the given number of coarse steps.
"""

import argparse
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(HERE))

from oracle import Forest, RefinedOracle  # noqa: E402
from oracle import refined as oracle_refined  # noqa: E402
from oracle.tables import LevelCells, LevelTables  # noqa: E402
from paper_1508_07982_amd import lbm  # noqa: E402
from paper_1508_07982_amd import workloads as W  # noqa: E402


def say(msg):
    print(msg, flush=True)


def build_tables_with_progress(forest, coalescence="virtual"):
    t0 = time.time()
    cells = []
    for L in range(forest.max_level + 1):
        cells.append(LevelCells(forest, L))
        say(f"  cell sets of level {L}: {time.time() - t0:.0f} s")
    tabs = []
    for L, c in enumerate(cells):
        coarser = cells[L - 1] if L > 0 else None
        finer = cells[L + 1] if L < forest.max_level else None
        tabs.append(LevelTables(c, coarser, finer, coalescence))
        say(f"  tables of level {L}: {time.time() - t0:.0f} s")
    return tabs


def rel_l2(a, b, w):
    num = np.sqrt(np.sum(w[:, None] * (a - b).reshape(len(w), -1) ** 2))
    den = np.sqrt(np.sum(w[:, None] * b.reshape(len(w), -1) ** 2))
    return float(num / den)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--out", default=None)
    a = ap.parse_args()
    w = W.config_sphere(16, 4)
    say(f"{w.name}: oracle tables")
    oracle_refined.build_tables = build_tables_with_progress
    of = Forest.build(w.R, w.n, w.max_level, w.refine)
    o = RefinedOracle(of, w.omega0)
    rho, u = W.initial_field(w, of.canonical_leaves())
    o.init_pdfs(rho, u)
    say(f"oracle: {o.total_cells()} cells")
    t0 = time.time()
    for s in range(a.steps):
        o.step(1)
        say(f"  oracle step {s + 1}/{a.steps}: {time.time() - t0:.0f} s")
    r0, u0 = o.moments()
    wts = o.level_weights()
    report = {"workload": w.name, "cells": int(o.total_cells()), "coarse_steps": a.steps}
    for storage in ("f32", "f16"):
        g = lbm.Forest(w.R, w.n, w.max_level, refine=w.refine, storage=storage)
        g.set_level_omega(w.omega0)
        g.init_pdfs(rho, u)
        M0, _ = g.mass()
        g.step_coarse(a.steps)
        M1, _ = g.mass()
        r1, u1 = g.moments()
        report[storage] = {"velocity_rel_l2": rel_l2(u1, u0, wts), "density_rel_l2": rel_l2(r1, r0, wts),
                           "mass_drift": abs(M1 - M0) / M0}
        say(f"{storage}: {report[storage]}")
        g.close()
    text = json.dumps(report)
    say(text)
    if a.out:
        with open(a.out, "w") as fh:
            fh.write(text + "\n")


if __name__ == "__main__":
    main()
