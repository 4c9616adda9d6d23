"""Throughput of the refined lattice Boltzmann step on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W]

Workload: a periodic cube of 4^3 root blocks of 32^3 cells, blocks meeting
the surface of a central sphere of radius 0.25 refined at every level up to
level 3 (121.4 M cells in (0, 352, 984, 2368) blocks), D3Q19 SRT with
omega_0 = 1.9, Taylor-Green amplitude 0.02 plus seeded noise.  One "step" is
one coarse time step (Algorithm 1 from level 0: sum_L 2^L N_L = 773 M cell
updates), FP32 PDFs, whole step captured as a HIP graph with the launch
shape of every level picked by the library's autotuner; inputs are resident
in HBM before timing starts.

Prints one JSON line: MLUPS across all levels, the roofline of the dominant
kernel (the finest-level sweep), the FP16-shifted and plain per-block-launch
forms on the same grid, and the FP64 CPU oracle timed on the host cores on a
bounded sample of the same workload.
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, HERE)

HBM_PEAK_GBS = 8000.0  # MI355X published HBM3E bandwidth
METRIC = "MLUPS across all levels + % of HBM roofline, FP16/FP32 vs plain form"
TRAFFIC_FILE = os.path.join(HERE, "profiles", "sweep_traffic_sphere_shell_n32.txt")


def measured_traffic(storage: str, level_cells: int, launches_ms: float):
    """HBM bytes per finest-level sweep launch from the committed rocprofv3
    counter summary, or None if absent or taken on another kernel source."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    vals = {}
    with open(TRAFFIC_FILE) as fh:
        for line in fh:
            if ":" in line and not line.startswith("#"):
                k, v = line.split(":", 1)
                vals[k.strip()] = v.strip()
    from paper_1508_07982_amd.profiling import sweep_sources_hash
    if vals.get("kernel_sha256_16") != sweep_sources_hash(storage) or vals.get("storage") != storage:
        return None
    try:
        return float(vals["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def make_forest(lbm, W, w, storage, stream, trt=None):
    """trt: (Lambda_eo, level-0 acceleration) for the TRT collision with a
    body force, None for SRT."""
    g = lbm.Forest(w.R, w.n, w.max_level, refine=w.refine, storage=storage, stream=stream)
    rho, u = W.initial_field(w, g.leaves())
    g.set_level_omega(w.omega0)
    if trt is not None:
        g.set_trt_force(*trt)
    g.init_pdfs(rho, u)
    del rho, u
    return g


def timed_steps(torch, g, stream, steps):
    start = torch.cuda.Event(enable_timing=True)
    end = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    start.record(stream)
    g.step_coarse(steps)
    end.record(stream)
    torch.cuda.synchronize()
    return start.elapsed_time(end) / steps


def level_table(g, sweeps, s_bytes, coal=None):
    """Mean launch time and algorithmic GB/s of every (level, substep), and
    the mean time of each level's coalescence launch."""
    out = {f"L{L}s{s}": {"ms": round(m, 4), "launches": c, "cells": g.num_cells(L),
                         "GBps": round(38 * s_bytes * g.num_cells(L) / (m * 1e-3) / 1e9, 1)}
           for (L, s), (m, c) in sorted(sweeps.items())}
    for L, (m, c) in sorted((coal or {}).items()):
        out[f"L{L}coalesce"] = {"ms": round(m, 4), "launches": c}
    return out


def launch_table(res):
    """Autotuner choice per level: [persistent workgroups per CU (0: one
    per work unit), tile order (1: grouped by XCD), workgroups per tile]."""
    return {f"L{r['level']}": [r["persistent"], r["order"], r["split"]] for r in res}


def batching_form(torch, lbm, W, stream):
    """Time per coarse step on the 8.57 M-cell slab + sphere grid of 16^3
    blocks (uneven block counts per level): the whole step as one graph with
    autotuned launch shapes, direct launches, and one launch per block."""
    wb = W.config_slab_sphere(16, 5)
    out = {"workload": wb.name, "description": wb.description}
    for label, schedule, tune in (("graph_autotuned", "graph", True), ("direct", "direct", False),
                                  ("per_block", "per_block", False)):
        g = make_forest(lbm, W, wb, "f32", stream.cuda_stream)
        if label == "graph_autotuned":
            out["cells"] = g.num_cells()
            out["blocks_per_level"] = [g.num_blocks(L) for L in range(g.num_levels)]
            out["launch"] = launch_table(g.autotune(2))
        g.set_schedule(schedule)
        g.step_coarse(2)
        ms = timed_steps(torch, g, stream, 20 if label != "per_block" else 3)
        out[f"{label}_ms_per_step"] = round(ms, 4)
        out[f"{label}_MLUPS"] = round(g.updates_per_coarse_step() / (ms * 1e-3) / 1e6, 1)
        g.close()
        del g
    return out


def cpu_baseline(W, budget_s: float = 12.0):
    """The FP64 oracle on the same sphere-shell geometry with 8^3-cell
    blocks (1/64 of the cells), timed over as many coarse steps as fit in
    about `budget_s` seconds (two untimed steps estimate the rate)."""
    from oracle import Forest as OForest, RefinedOracle
    w = W.config_sphere(8, 4)
    f = OForest.build(w.R, w.n, w.max_level, w.refine)
    o = RefinedOracle(f, w.omega0)
    rho, u = W.initial_field(w, f.canonical_leaves())
    o.init_pdfs(rho, u)
    t = time.perf_counter()
    o.step(2)
    per_step = (time.perf_counter() - t) / 2
    budget_steps = int(min(200, max(2, budget_s / max(per_step, 1e-3))))
    t = time.perf_counter()
    o.step(budget_steps)
    dt = time.perf_counter() - t
    cores = int(os.environ.get("OMP_NUM_THREADS", "0")) or os.cpu_count()
    return {
        "value": round(o.updates_per_coarse_step() * budget_steps / dt / 1e6, 3),
        "unit": "MLUPS",
        "cores": cores,
        "kind": "oracle",
        "sample": f"FP64 oracle, sphere-shell geometry with 8^3-cell blocks ({o.total_cells()} cells, "
                  f"1/64 of the benchmark grid), {budget_steps} coarse steps, {dt:.1f} s",
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-forms", action="store_true", help="skip the FP16, FP64 and per-block comparison runs")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU: the refined grid lives in one GPU's HBM and the library has no "
              f"multi-GPU path (asked for --gpus {args.gpus})", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1508_07982_amd import lbm
    from paper_1508_07982_amd import workloads as W

    stream = torch.cuda.Stream()
    w = W.config_sphere(32, 4)
    g = make_forest(lbm, W, w, "f32", stream.cuda_stream)
    upd = g.updates_per_coarse_step()
    cells = g.num_cells()
    launch = g.autotune(2)  # per-level launch shape, state restored afterwards
    g.step_coarse(args.warmup)
    M0, _ = g.mass()
    ms = timed_steps(torch, g, stream, args.steps)
    M1, _ = g.mass()
    value = upd / (ms * 1e-3) / 1e6

    # dominant kernel: the finest-level sweep (77.6 M cells, 8 launches per step)
    sweeps, coal = g.time_launches(2)
    Lf = g.num_levels - 1
    fin = [sweeps[k] for k in sweeps if k[0] == Lf]
    fin_ms = sum(m * c for m, c in fin) / sum(c for _, c in fin)
    s_bytes = lbm.STORAGE_BYTES["f32"]
    nf = g.num_cells(Lf)
    alg_bytes = 38 * s_bytes * nf          # 19 PDFs read + 19 written per interior cell
    achieved = alg_bytes / (fin_ms * 1e-3) / 1e9
    traffic = measured_traffic("f32", nf, fin_ms)
    per_level = level_table(g, sweeps, s_bytes, coal)
    g.close()
    del g
    torch.cuda.synchronize()

    forms = {"f32_graph": {"MLUPS": round(value, 1), "ms_per_step": round(ms, 3),
                           "roofline_MLUPS": round(HBM_PEAK_GBS * 1e9 / (38 * 4) / 1e6, 1)}}
    if not args.no_forms:
        g16 = make_forest(lbm, W, w, "f16", stream.cuda_stream)
        launch16 = g16.autotune(2)
        g16.step_coarse(2)
        M16a, _ = g16.mass()
        ms16 = timed_steps(torch, g16, stream, max(3, args.steps // 2))
        M16b, _ = g16.mass()
        sw16, co16 = g16.time_launches(2)
        forms["f16_graph"] = {"MLUPS": round(upd / (ms16 * 1e-3) / 1e6, 1), "ms_per_step": round(ms16, 3),
                              "roofline_MLUPS": round(HBM_PEAK_GBS * 1e9 / (38 * 2) / 1e6, 1),
                              "per_level": level_table(g16, sw16, 2, co16),
                              "launch": launch_table(launch16), "mass_drift": abs(M16b - M16a) / M16a}
        g16.close()
        del g16
        g64 = make_forest(lbm, W, w, "f64", stream.cuda_stream)
        launch64 = g64.autotune(1)
        g64.step_coarse(1)
        M64a, _ = g64.mass()
        ms64 = timed_steps(torch, g64, stream, 3)
        M64b, _ = g64.mass()
        sw64, co64 = g64.time_launches(1)
        forms["f64_graph"] = {"MLUPS": round(upd / (ms64 * 1e-3) / 1e6, 1), "ms_per_step": round(ms64, 3),
                              "roofline_MLUPS": round(HBM_PEAK_GBS * 1e9 / (38 * 8) / 1e6, 1),
                              "per_level": level_table(g64, sw64, 8, co64),
                              "launch": launch_table(launch64), "mass_drift": abs(M64b - M64a) / M64a}
        g64.close()
        del g64
        # TRT with Lambda_eo = 3/16 and a body force along x (section 2), FP32
        gt = make_forest(lbm, W, w, "f32", stream.cuda_stream, trt=(3.0 / 16.0, (1e-6, 0.0, 0.0)))
        launcht = gt.autotune(1)
        gt.step_coarse(1)
        Mta, _ = gt.mass()
        mst = timed_steps(torch, gt, stream, 5)
        Mtb, _ = gt.mass()
        swt, cot = gt.time_launches(1)
        forms["f32_trt_force_graph"] = {"MLUPS": round(upd / (mst * 1e-3) / 1e6, 1), "ms_per_step": round(mst, 3),
                                        "lambda_eo": 3.0 / 16.0, "accel0": [1e-6, 0.0, 0.0],
                                        "per_level": level_table(gt, swt, 4, cot),
                                        "launch": launch_table(launcht), "mass_drift": abs(Mtb - Mta) / Mta}
        gt.close()
        del gt
        forms["batching_slab_sphere"] = batching_form(torch, lbm, W, stream)
        gp = make_forest(lbm, W, w, "f32", stream.cuda_stream)
        gp.set_schedule("per_block")
        gp.step_coarse(1)
        msp = timed_steps(torch, gp, stream, 2)
        forms["f32_per_block_launch"] = {"MLUPS": round(upd / (msp * 1e-3) / 1e6, 1), "ms_per_step": round(msp, 3)}
        gp.close()
        del gp
        torch.cuda.synchronize()

    out = {
        "metric": METRIC,
        "value": round(value, 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": w.name,
            "description": w.description,
            "cells": cells,
            "levels": [lv for lv in range(Lf + 1)],
            "updates_per_coarse_step": upd,
            "omega0": w.omega0,
            "schedule": "hipGraph of the whole coarse step",
            "launch": launch_table(launch),
            "mass_drift": abs(M1 - M0) / M0,
        },
        "roofline": {
            "bound": "hbm",
            "achieved": round(achieved, 1),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": traffic,
            "kernel": f"sweep_kernel<float,32> on level {Lf}",
            "algorithmic_bytes_per_launch": alg_bytes,
            "mean_launch_ms": round(fin_ms, 4),
        },
        "per_level": per_level,
        "forms": forms,
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(W)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
