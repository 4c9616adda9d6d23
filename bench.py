"""Throughput of the refined lattice Boltzmann step on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W]

Workload: a periodic cube of 4^3 root blocks of 32^3 cells, blocks meeting
the surface of a central sphere of radius 0.25 refined at every level up to
level 3 (121.4 M cells in (0, 352, 984, 2368) blocks), D3Q19 SRT with
omega_0 = 1.9, Taylor-Green amplitude 0.02 plus seeded noise.  One "step" is
one coarse time step (Algorithm 1 from level 0: sum_L 2^L N_L = 773 M cell
updates), whole step captured as a HIP graph with the launch shape of every
level picked by the library's autotuner; inputs are resident in HBM before
timing starts.

The headline (`value`) is the FP64 storage form: the paper measures its
throughput in double precision.  The FP32 and FP16-shifted storage forms,
each with its own roofline block, the TRT + body-force form, the batching
grid (slab + sphere, 16^3 blocks) and the plain per-block-launch form follow
under `forms`; `ceilings` holds the copy and sweep-shape probes measured in
the same run, and `cpu_baseline` the FP64 oracle timed on the host cores on
a bounded sample of the same workload (all cores and one core).
"""

from __future__ import annotations

import argparse
import json
import os
import platform
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, HERE)

HBM_PEAK_GBS = 8000.0  # MI355X published HBM3E bandwidth
METRIC = "MLUPS across all levels + % of HBM roofline, FP16/FP32 vs plain form"
BYTES = {"f64": 8, "f32": 4, "f16": 2}


def traffic_file(storage: str) -> str:
    suffix = "" if storage == "f32" else "_" + storage
    return os.path.join(HERE, "profiles", f"sweep_traffic_sphere_shell_n32{suffix}.txt")


def measured_traffic(storage: str):
    """HBM bytes per finest-level sweep launch from the committed rocprofv3
    counter summary, or None if absent or taken on another kernel source."""
    path = traffic_file(storage)
    if not os.path.exists(path):
        return None
    vals = {}
    with open(path) as fh:
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
    the mean time of each level's coalescence launch with the algorithmic
    GB/s of its pairs (8 child reads, the regular source and the write)."""
    out = {f"L{L}s{s}": {"ms": round(m, 4), "launches": c, "cells": g.num_cells(L),
                         "GBps": round(38 * s_bytes * g.num_cells(L) / (m * 1e-3) / 1e9, 1)}
           for (L, s), (m, c) in sorted(sweeps.items())}
    for L, (m, c) in sorted((coal or {}).items()):
        pairs = g.level_stats(L)["coalesced_pairs"]
        out[f"L{L}coalesce"] = {"ms": round(m, 4), "launches": c, "pairs": pairs,
                                "GBps": round(10 * s_bytes * pairs / (m * 1e-3) / 1e9, 1)}
    return out


def launch_table(res):
    """Autotuner choice per level: [persistent workgroups per CU (0: one
    per work unit), tile order (1: grouped by XCD), workgroups per tile]."""
    return {f"L{r['level']}": [r["persistent"], r["order"], r["split"], r["fuse"]] for r in res}


def roofline_block(g, storage, sweeps):
    """Roofline of the dominant kernel, the finest-level sweep: algorithmic
    bytes per launch (19 PDFs read and 19 written per interior cell) over
    its mean launch time from HIP events on the library's stream.  Where the
    finest level's second substep also runs the coarser coalescence (its
    fusion on), only the first substeps enter."""
    Lf = g.num_levels - 1
    fused = Lf > 0 and g.get_level_fusion(Lf) and g.level_stats(Lf - 1)["coalesced_pairs"] > 0
    fin = [sweeps[k] for k in sweeps if k[0] == Lf and (k[1] == 1 or not fused)]
    fin_ms = sum(m * c for m, c in fin) / sum(c for _, c in fin)
    nf = g.num_cells(Lf)
    alg = 38 * BYTES[storage] * nf
    achieved = alg / (fin_ms * 1e-3) / 1e9
    return {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": measured_traffic(storage),
            "kernel": f"sweep_kernel<{ {'f64': 'double', 'f32': 'float', 'f16': '__half'}[storage]},32> on level {Lf}",
            "algorithmic_bytes_per_launch": alg, "cells_per_launch": nf, "bytes_per_cell_update": 38 * BYTES[storage],
            "mean_launch_ms": round(fin_ms, 4), "substeps": [1] if fused else [1, 2]}


def storage_form(torch, lbm, W, w, storage, stream, steps, warmup):
    """MLUPS, roofline and per-level table of one storage form on the
    benchmark grid (graph schedule, autotuned launch shapes)."""
    g = make_forest(lbm, W, w, storage, stream.cuda_stream)
    upd = g.updates_per_coarse_step()
    launch = g.autotune(1 if storage == "f64" else 2)  # state restored afterwards
    g.step_coarse(warmup)
    M0, _ = g.mass()
    ms = timed_steps(torch, g, stream, steps)
    M1, _ = g.mass()
    sweeps, coal = g.time_launches(1 if storage == "f64" else 2)
    value = upd / (ms * 1e-3) / 1e6
    roof_mlups = HBM_PEAK_GBS * 1e9 / (38 * BYTES[storage]) / 1e6
    out = {"MLUPS": round(value, 1), "ms_per_step": round(ms, 4), "steps": steps,
           "roofline_MLUPS": round(roof_mlups, 1), "frac_of_roofline_MLUPS": round(value / roof_mlups, 4),
           "roofline": roofline_block(g, storage, sweeps), "per_level": level_table(g, sweeps, BYTES[storage], coal),
           "launch": launch_table(launch), "mass_drift": abs(M1 - M0) / M0,
           "cells": g.num_cells(), "updates_per_coarse_step": upd}
    g.close()
    del g
    torch.cuda.synchronize()
    return out


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
        if label == "graph_autotuned":
            sweeps, coal = g.time_launches(3)
            out["per_level"] = level_table(g, sweeps, 4, coal)
            busy = sum(m * c for m, c in sweeps.values()) / 3 + sum(m * c for m, c in coal.values()) / 3
            out["kernel_busy_ms_per_step"] = round(busy, 4)
            out["algorithmic_GBps"] = round(g.updates_per_coarse_step() * 152 / (ms * 1e-3) / 1e9, 1)
        g.close()
        del g
    return out


def inplace_form(torch, lbm, W, stream, storage):
    """Two-buffer against in-place (AA pattern) streaming on the uniform
    periodic grid of 16^3 roots of 32^3 cells (512^3 cells, one level):
    MLUPS, mean time and algorithmic GB/s of each launch kind, and the
    device memory the forest holds (free memory before creating it and
    after switching in-place streaming on)."""
    wu = W.config_uniform(32, 16)
    s = BYTES[storage]
    out = {"workload": wu.name, "description": wu.description, "storage": storage}
    rho = u = None
    for label in ("two_buffer", "in_place"):
        torch.cuda.synchronize()
        free0, _ = lbm.device_memory(0)
        g = lbm.Forest(wu.R, wu.n, 0, storage=storage, stream=stream.cuda_stream)
        if rho is None:
            rho, u = W.initial_field(wu, g.leaves())
        g.set_level_omega(wu.omega0)
        g.init_pdfs(rho, u)
        if label == "in_place":
            g.set_inplace(True)
        g.synchronize()
        free1, _ = lbm.device_memory(0)
        N = g.num_cells()
        g.step_coarse(2)
        ms = timed_steps(torch, g, stream, 10)
        sweeps = g.time_sweeps(2)
        launches = {}
        for (L, sub), (m, c) in sorted(sweeps.items()):
            key = ("odd" if sub == 1 else "even") if label == "in_place" else "sweep"
            launches[key] = {"ms": round(m, 4), "launches": c, "GBps": round(38 * s * N / (m * 1e-3) / 1e9, 1)}
        out["cells"] = N
        out[label] = {"MLUPS": round(N / (ms * 1e-3) / 1e6, 1), "ms_per_step": round(ms, 4),
                      "device_bytes": int(free0 - free1), "pdf_buffer_bytes": N * 19 * s, "launches": launches}
        g.close()
        del g
    out["device_bytes_ratio"] = round(out["in_place"]["device_bytes"] / out["two_buffer"]["device_bytes"], 4)
    return out


def inplace_refined_form(torch, lbm, W, w, stream, storage, steps):
    """The benchmark grid with its finest level streamed in place: MLUPS,
    per-level table and the device memory of the forest before and after
    switching in-place streaming on."""
    torch.cuda.synchronize()
    free0, _ = lbm.device_memory(0)
    g = make_forest(lbm, W, w, storage, stream.cuda_stream)
    g.synchronize()
    free1, _ = lbm.device_memory(0)
    g.set_inplace(True)
    free2, _ = lbm.device_memory(0)
    g.step_coarse(2)
    ms = timed_steps(torch, g, stream, steps)
    sweeps, coal = g.time_launches(1)
    upd = g.updates_per_coarse_step()
    out = {"MLUPS": round(upd / (ms * 1e-3) / 1e6, 1), "ms_per_step": round(ms, 4), "steps": steps,
           "device_bytes_two_buffer": int(free0 - free1), "device_bytes_in_place": int(free0 - free2),
           "device_bytes_ratio": round((free0 - free2) / (free0 - free1), 4),
           "per_level": level_table(g, sweeps, BYTES[storage], coal)}
    g.close()
    del g
    torch.cuda.synchronize()
    return out


def ceilings_now(torch, lbm):
    """The copy probe and the sweep-shape probe at the finest level's size
    (FP64 elements, 2368 blocks of 32^3 cells), measured in this run."""
    from paper_1508_07982_amd import profiling
    rows = profiling.ceilings(blocks=2368, n=32, iters=5)
    best = {}
    for r in rows:
        key = "copy" if r["probe"] == "copy" else f"sweep_shape_{r['elem_bytes']}B"
        if r["GBps"] > best.get(key, {"GBps": 0})["GBps"]:
            best[key] = {k: (round(v, 4) if isinstance(v, float) else v) for k, v in r.items()}
    return best


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or "unknown"


def cpu_baseline(W, budget_s: float = 10.0):
    """The FP64 oracle on the same sphere-shell geometry with 8^3-cell
    blocks (1/64 of the cells), timed over as many coarse steps as fit in
    about `budget_s` seconds (one untimed step estimates the rate), first on
    every host core the process may use, then on one core."""
    from oracle import Forest as OForest, RefinedOracle
    from oracle.refined import set_threads
    w = W.config_sphere(8, 4)
    f = OForest.build(w.R, w.n, w.max_level, w.refine)
    o = RefinedOracle(f, w.omega0)
    rho, u = W.initial_field(w, f.canonical_leaves())
    o.init_pdfs(rho, u)
    upd = o.updates_per_coarse_step()

    def run(threads):
        prev = set_threads(threads)
        try:
            t = time.perf_counter()
            o.step(1)
            per_step = time.perf_counter() - t
            steps = int(min(200, max(1, budget_s / max(per_step, 1e-3))))
            t = time.perf_counter()
            o.step(steps)
            dt = time.perf_counter() - t
        finally:
            set_threads(prev)
        return upd * steps / dt / 1e6, steps, dt

    cores = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    cores = min(cores, int(os.environ.get("OMP_NUM_THREADS", "0")) or cores)
    v_all, s_all, t_all = run(cores)
    v_one, s_one, t_one = run(1)
    return {
        "value": round(v_all, 3),
        "unit": "MLUPS",
        "cores": cores,
        "kind": "oracle",
        "sample": f"FP64 oracle (gcc -O3, OpenMP), sphere-shell geometry with 8^3-cell blocks "
                  f"({o.total_cells()} cells, 1/64 of the benchmark grid), {s_all} coarse steps in {t_all:.1f} s "
                  f"on {cores} threads",
        "single_core": {"value": round(v_one, 3), "unit": "MLUPS", "cores": 1,
                        "sample": f"the same, {s_one} coarse steps in {t_one:.1f} s on 1 thread"},
        "cpu_model": cpu_model(),
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-forms", action="store_true",
                    help="skip the FP32/FP16, TRT, interpolation, batching, per-block and in-place comparison runs")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-ceilings", action="store_true")
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
    head = storage_form(torch, lbm, W, w, "f64", stream, args.steps, args.warmup)
    print(f"f64: {head['MLUPS']} MLUPS", file=sys.stderr, flush=True)

    forms = {}
    if not args.no_forms:
        for storage in ("f32", "f16"):
            forms[f"{storage}_graph"] = storage_form(torch, lbm, W, w, storage, stream, args.steps, args.warmup)
            print(f"{storage}: {forms[storage + '_graph']['MLUPS']} MLUPS", file=sys.stderr, flush=True)
        # TRT with Lambda_eo = 3/16 and a body force along x (section 2), FP32
        gt = make_forest(lbm, W, w, "f32", stream.cuda_stream, trt=(3.0 / 16.0, (1e-6, 0.0, 0.0)))
        launcht = gt.autotune(1)
        gt.step_coarse(1)
        Mta, _ = gt.mass()
        mst = timed_steps(torch, gt, stream, 5)
        Mtb, _ = gt.mass()
        swt, cot = gt.time_launches(1)
        forms["f32_trt_force_graph"] = {"MLUPS": round(head["updates_per_coarse_step"] / (mst * 1e-3) / 1e6, 1),
                                        "ms_per_step": round(mst, 3), "lambda_eo": 3.0 / 16.0,
                                        "accel0": [1e-6, 0.0, 0.0], "per_level": level_table(gt, swt, 4, cot),
                                        "launch": launch_table(launcht), "mass_drift": abs(Mtb - Mta) / Mta}
        gt.close()
        del gt
        # the interpolated explosion (limited linear reconstruction of the
        # exploded values) instead of eq. ctof, FP32
        gi = make_forest(lbm, W, w, "f32", stream.cuda_stream)
        gi.set_explosion_interpolation(True)
        gi.step_coarse(1)
        msi = timed_steps(torch, gi, stream, 5)
        swi, coi = gi.time_launches(1)
        forms["f32_interpolated_explosion_graph"] = {
            "MLUPS": round(head["updates_per_coarse_step"] / (msi * 1e-3) / 1e6, 1), "ms_per_step": round(msi, 3),
            "per_level": level_table(gi, swi, 4, coi)}
        gi.close()
        del gi
        forms["batching_slab_sphere"] = batching_form(torch, lbm, W, stream)
        gp = make_forest(lbm, W, w, "f32", stream.cuda_stream)
        gp.set_schedule("per_block")
        gp.step_coarse(1)
        msp = timed_steps(torch, gp, stream, 2)
        forms["f32_per_block_launch"] = {"MLUPS": round(head["updates_per_coarse_step"] / (msp * 1e-3) / 1e6, 1),
                                         "ms_per_step": round(msp, 3)}
        gp.close()
        del gp
        for storage in ("f64", "f32", "f16"):
            forms[f"{storage}_inplace_finest_graph"] = inplace_refined_form(torch, lbm, W, w, stream, storage, 5)
            print(f"{storage} finest level in place: {forms[storage + '_inplace_finest_graph']['MLUPS']} MLUPS",
                  file=sys.stderr, flush=True)
        for storage in ("f64", "f32", "f16"):
            forms[f"{storage}_inplace_uniform"] = inplace_form(torch, lbm, W, stream, storage)
            print(f"{storage} in place: {forms[storage + '_inplace_uniform']['in_place']['MLUPS']} MLUPS",
                  file=sys.stderr, flush=True)
        torch.cuda.synchronize()

    out = {
        "metric": METRIC,
        "value": head["MLUPS"],
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": w.name,
            "description": w.description + " (level 0 holds no leaves: the 2:1 balance splits every root)",
            "cells": head["cells"],
            "blocks_per_level": [lbm.plan_level_stats(w.R, w.n, w.max_level, L, refine=w.refine)["blocks"]
                                 for L in range(w.max_level + 1)],
            "updates_per_coarse_step": head["updates_per_coarse_step"],
            "omega0": w.omega0,
            "storage": "f64 (PDFs stored as f - w in FP64, FP64 arithmetic)",
            "schedule": "hipGraph of the whole coarse step",
            "launch": head["launch"],
            "mass_drift": head["mass_drift"],
            "roofline_MLUPS": head["roofline_MLUPS"],
            "frac_of_roofline_MLUPS": head["frac_of_roofline_MLUPS"],
        },
        "roofline": head["roofline"],
        "per_level": head["per_level"],
        "forms": forms,
    }
    if not args.no_ceilings:
        out["ceilings"] = ceilings_now(torch, lbm)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(W)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
