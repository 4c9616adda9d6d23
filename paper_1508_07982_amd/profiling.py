"""Profiling helpers: workloads to run under rocprofv3 and summaries of its output.

    python -m paper_1508_07982_amd.profiling copy                 # 1 GiB device copy x 3 (counter scale)
    python -m paper_1508_07982_amd.profiling ceiling OUT.txt       # copy and sweep-shape probes
    python -m paper_1508_07982_amd.profiling sweep [--storage f32] [--workload sphere|slab] [--steps 2]
            [--separate-coalescence]
    python -m paper_1508_07982_amd.profiling trace-summary  RESULTS_DIR OUT.txt --command "..."
            [--storage f32] [--workload sphere|slab]
    python -m paper_1508_07982_amd.profiling traffic-summary COPY_FETCH COPY_WRITE SWEEP_FETCH SWEEP_WRITE OUT.txt
            --command "..." [--storage f32]

The sweep workload is the benchmark grid (sphere shell, 4^3 roots of 32^3
cells, 121.4 M cells) or the slab + sphere grid of the batching form
(5^3 roots of 16^3 cells, 8.57 M cells) with the launch shape chosen by the
autotuner, as in bench.py, stepped with one launch per level substep, so
every sweep dispatch shows up in the trace (a level whose second substep
runs the coarser coalescence shows that launch as "fused"; with
--separate-coalescence every coalescence is a launch of its own, as the
counter passes use it).  FETCH_SIZE and WRITE_SIZE (KiB
per dispatch) are scaled by what the same counters read for the library's
copy probe (lbm_probe_copy) of a known byte count; the result is the HBM
traffic of one finest-level sweep launch.

Both workloads run the autotuner first and then a mass reduction; only
sweep dispatches after the first reduction kernel (the measured phase) enter
the per-level figures.
"""

from __future__ import annotations

import argparse
import csv
import glob
import hashlib
import os
import re
import sqlite3
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
COPY_BYTES = 1 << 30


def sweep_sources_hash(storage: str = "f32") -> str:
    """Hash of the sweep kernel's sources with comments and blank space
    removed, so that a counter summary stays valid across comment edits."""
    h = hashlib.sha256()
    for f in ("sweep.hpp", "coalesce.hpp", "lattice.hpp", "kernels.hpp", f"sweep_{storage}.hip"):
        with open(os.path.join(HERE, "csrc", f)) as fh:
            text = re.sub(r"/\*.*?\*/", " ", fh.read(), flags=re.S)
        code = [" ".join(line.split("//", 1)[0].split()) for line in text.splitlines()]
        h.update("\n".join(c for c in code if c).encode())
    return h.hexdigest()[:16]


def run_copy():
    import torch
    sys.path.insert(0, ROOT)
    from paper_1508_07982_amd import lbm
    a = torch.zeros(COPY_BYTES // 4, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    ms = lbm.probe_copy(b.data_ptr(), a.data_ptr(), COPY_BYTES, iters=2)  # warm-up + 2 copies
    print(f"copied {COPY_BYTES} bytes x 3 with lbm_probe_copy: {COPY_BYTES / ms / 1e6:.1f} GB/s", flush=True)


def _workload(name: str):
    from paper_1508_07982_amd import workloads as W
    return W.config_sphere(32, 4) if name == "sphere" else W.config_slab_sphere(16, 5)


def ceilings(blocks: int = 2368, n: int = 32, iters: int = 10):
    """Bandwidth ceilings measured with the library's probes: a 1 GiB copy
    (plain and nontemporal stores), and the sweep's access shape without
    arithmetic (19 rows read and written per tile) over `blocks` blocks of
    n^3 cells -- the finest level of the benchmark grid -- for every storage
    width, workgroup size and tile order.  Returns a list of dicts."""
    import torch
    sys.path.insert(0, ROOT)
    from paper_1508_07982_amd import lbm
    out = []
    a = torch.zeros(COPY_BYTES // 4, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    for nt in (True, False):
        ms = lbm.probe_copy(b.data_ptr(), a.data_ptr(), COPY_BYTES, iters=iters, nontemporal=nt)
        out.append({"probe": "copy", "bytes": COPY_BYTES, "nontemporal": nt, "ms": ms,
                    "GBps": 2 * COPY_BYTES / ms / 1e6})
    del a, b
    for s in (8, 4, 2):
        nbytes = blocks * 19 * n ** 3 * s
        src = torch.zeros(nbytes // 4, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        for lanes in (64, 128, 256):
            for xcd in (False, True):
                ms = lbm.probe_streams(dst.data_ptr(), src.data_ptr(), blocks, n, s, lanes, xcd, iters)
                out.append({"probe": "sweep_shape", "elem_bytes": s, "blocks": blocks, "n": n, "lanes": lanes,
                            "xcd": xcd, "ms": ms, "GBps": 2 * nbytes / ms / 1e6})
        del src, dst
    torch.cuda.synchronize()
    return out


def write_ceilings(out_path: str, command: str):
    rows = ceilings()
    with open(out_path, "w") as fh:
        fh.write("# bandwidth ceilings from the library's probes (lbm_probe.h), HIP events, mean of 10 launches\n")
        fh.write(f"# command: {command}\n")
        fh.write("# GB/s = bytes read + bytes written per launch / mean launch time\n\n")
        for r in rows:
            if r["probe"] == "copy":
                fh.write(f"copy {r['bytes']} B, {'nontemporal' if r['nontemporal'] else 'plain'} stores: "
                         f"{r['ms']:.3f} ms, {r['GBps']:.1f} GB/s\n")
            else:
                fh.write(f"sweep shape, {r['elem_bytes']}-byte elements, {r['blocks']} blocks of {r['n']}^3, "
                         f"{r['lanes']} lanes, {'XCD-grouped' if r['xcd'] else 'canonical'} order: "
                         f"{r['ms']:.3f} ms, {r['GBps']:.1f} GB/s\n")
    print(open(out_path).read(), flush=True)


def run_sweep(storage: str, steps: int, workload: str = "sphere", separate: bool = False):
    sys.path.insert(0, ROOT)
    from paper_1508_07982_amd import lbm
    from paper_1508_07982_amd import workloads as W
    w = _workload(workload)
    g = lbm.Forest(w.R, w.n, w.max_level, refine=w.refine, storage=storage)
    rho, u = W.initial_field(w, g.leaves())
    g.set_level_omega(w.omega0)
    g.set_schedule("direct")
    g.init_pdfs(rho, u)
    del rho, u
    launch = g.autotune(2)
    if separate:  # every coalescence in a launch of its own (counter passes)
        g.set_coalescence_fusion(False)
    print("launch per level (persistent, order, split, fuse)",
          [(r["persistent"], r["order"], r["split"], 0 if separate else r["fuse"]) for r in launch], flush=True)
    g.mass()  # marks the start of the measured phase in the dispatch list
    g.step_coarse(steps)
    g.synchronize()
    tiles = {L: g.level_stats(L)["work_tiles"] for L in range(g.num_levels)}
    print("work tiles per level", tiles, flush=True)
    g.close()


def _finest_tiles(storage: str = "f32", workload: str = "sphere"):
    sys.path.insert(0, ROOT)
    from paper_1508_07982_amd import lbm
    w = _workload(workload)
    return {L: lbm.plan_level_stats(w.R, w.n, w.max_level, L, refine=w.refine, storage=storage)["work_tiles"]
            for L in range(w.max_level + 1)}


def _db(path):
    if os.path.isdir(path):
        hits = glob.glob(os.path.join(path, "**", "*_results.db"), recursive=True)
        if not hits:
            raise FileNotFoundError(f"no *_results.db under {path}")
        path = hits[0]
    return sqlite3.connect(path)


def _units_per_tile(name):
    """Workgroups per work tile of a sweep dispatch: the kernel's last
    template argument (its split), 1 if absent."""
    inner = name.split("<", 1)[1].split(">", 1)[0] if "<" in name else ""
    parts = [p.strip() for p in inner.split(",")]
    return int(parts[3]) if len(parts) >= 4 and parts[3].isdigit() else 1


def _fused(name):
    """Whether a sweep dispatch also runs coalescence chunks (its last
    template argument)."""
    inner = name.split("<", 1)[1].split(">", 1)[0] if "<" in name else ""
    parts = [p.strip() for p in inner.split(",")]
    return len(parts) >= 7 and parts[6] == "true"


def _measured_from(db):
    """Dispatch id of the first reduction kernel (the start of the measured
    phase), or 0 if there is none."""
    rows = [d for n, d in db.execute("select name, dispatch_id from kernels") if "reduce_kernel" in n]
    return min(rows) if rows else 0


def trace_summary(results: str, out: str, command: str, storage: str = "f32", workload: str = "sphere"):
    db = _db(results)
    first = _measured_from(db)
    rows = list(db.execute("select name, duration, grid_x, workgroup_x, dispatch_id from kernels"))
    tiles = _finest_tiles(storage, workload)
    level_of_grid = {}
    for L, t in tiles.items():
        level_of_grid.setdefault(t, L)
    stats = {}
    for name, dur, gx, wx, did in rows:
        key = name.rsplit("(", 1)[0]
        stats.setdefault(key, []).append(dur)
    per_level = {}
    for name, dur, gx, wx, did in rows:
        if "sweep_kernel" in name and did > first:
            # a launch that also runs coalescence chunks has a grid of its
            # own size: "fused" instead of a level
            L = "fused" if _fused(name) else level_of_grid.get(gx // max(wx, 1) // _units_per_tile(name))
            per_level.setdefault((name.rsplit("(", 1)[0], L), []).append(dur)
    with open(out, "w") as fh:
        fh.write(f"# rocprofv3 --kernel-trace --stats summary\n# command: {command}\n")
        fh.write("# durations in microseconds; all dispatches of the run (autotuner candidates included)\n\n")
        fh.write(f"{'kernel':70s} {'calls':>6s} {'total_us':>12s} {'avg_us':>10s} {'min_us':>10s} {'max_us':>10s}\n")
        for k, v in sorted(stats.items(), key=lambda kv: -sum(kv[1])):
            fh.write(f"{k[:70]:70s} {len(v):6d} {sum(v) / 1e3:12.1f} {sum(v) / len(v) / 1e3:10.2f} "
                     f"{min(v) / 1e3:10.2f} {max(v) / 1e3:10.2f}\n")
        fh.write(f"\n# measured phase (dispatches after the first reduce_kernel, id {first}): sweep launches by\n"
                 "# level (level from the grid size = work tiles of that level times the workgroups per tile;\n"
                 "# None = persistent grid)\n")
        for (k, L), v in sorted(per_level.items(), key=lambda kv: (kv[0][0], str(kv[0][1]))):
            fh.write(f"{k[:60]:60s} level {L}: {len(v):5d} launches, avg {sum(v) / len(v) / 1e3:10.2f} us\n")
    print(open(out).read())


def _counter(path, counter):
    db = _db(path)
    return list(db.execute("select name, counter_value from pmc_events where counter_name = ?", (counter,)))


def traffic_summary(copy_fetch, copy_write, sweep_fetch, sweep_write, out, command, storage="f32"):
    cf = [v for n, v in _counter(copy_fetch, "FETCH_SIZE") if "copy" in n.lower() or "elementwise" in n.lower()]
    cw = [v for n, v in _counter(copy_write, "WRITE_SIZE") if "copy" in n.lower() or "elementwise" in n.lower()]
    if not cf or not cw:
        raise RuntimeError("copy kernel not found in the copy profiles")
    fetch_scale = COPY_BYTES / (max(cf) * 1024.0)
    write_scale = COPY_BYTES / (max(cw) * 1024.0)
    tiles = _finest_tiles(storage)
    Lf = max(tiles)
    sys.path.insert(0, ROOT)
    def finest(path, counter):
        db = _db(path)
        first = _measured_from(db)
        return [v for n, v, g, w, d in db.execute(
            "select p.name, p.counter_value, k.grid_x, k.workgroup_x, k.dispatch_id from pmc_events p join kernels k "
            "on p.dispatch_id = k.dispatch_id where p.counter_name = ?", (counter,)) if "sweep_kernel" in n
            and not _fused(n) and g // max(w, 1) // _units_per_tile(n) == tiles[Lf] and d > first]
    fin_f = finest(sweep_fetch, "FETCH_SIZE")
    fin_w = finest(sweep_write, "WRITE_SIZE")
    if not fin_f or not fin_w:
        raise RuntimeError("finest-level sweep dispatches not found")
    fetch = sum(fin_f) / len(fin_f) * 1024.0 * fetch_scale
    write = sum(fin_w) / len(fin_w) * 1024.0 * write_scale
    from paper_1508_07982_amd import workloads as W
    from paper_1508_07982_amd import lbm
    w = W.config_sphere(32, 4)
    cells = lbm.plan_level_stats(w.R, w.n, w.max_level, Lf, refine=w.refine)["interior_cells"]
    s = lbm.STORAGE_BYTES[storage]
    alg = 38 * s * cells
    with open(out, "w") as fh:
        fh.write("# HBM traffic of one finest-level sweep launch, from rocprofv3 --pmc passes\n")
        fh.write(f"# command: {command}\n")
        fh.write(f"# copy of {COPY_BYTES} bytes: FETCH_SIZE {max(cf):.0f} KiB, WRITE_SIZE {max(cw):.0f} KiB\n")
        fh.write(f"storage: {storage}\n")
        fh.write(f"kernel_sha256_16: {sweep_sources_hash(storage)}\n")
        fh.write(f"level: {Lf}\n")
        fh.write(f"interior_cells: {cells}\n")
        fh.write(f"fetch_scale: {fetch_scale:.4f}\n")
        fh.write(f"write_scale: {write_scale:.4f}\n")
        fh.write(f"fetch_bytes_per_launch: {fetch:.0f}\n")
        fh.write(f"write_bytes_per_launch: {write:.0f}\n")
        fh.write(f"hbm_bytes_per_launch: {fetch + write:.0f}\n")
        fh.write(f"algorithmic_bytes_per_launch: {alg}\n")
        fh.write(f"traffic_over_algorithmic: {(fetch + write) / alg:.4f}\n")
        fh.write(f"launches_averaged: {len(fin_f)}\n")
        # the coalescence launches, one group per level (grid = that level's
        # pair chunks; more pairs, more chunks); algorithmic bytes per pair:
        # 8 child reads, the regular source and the write
        lv = [(st["coalesced_pairs"], L) for L in range(w.max_level + 1)
              for st in [lbm.plan_level_stats(w.R, w.n, w.max_level, L, refine=w.refine)] if st["coalesced_pairs"]]
        groups = {}
        for path, counter, key in ((sweep_fetch, "FETCH_SIZE", 0), (sweep_write, "WRITE_SIZE", 1)):
            db = _db(path)
            first = _measured_from(db)
            for n, v, g, d in db.execute(
                    "select p.name, p.counter_value, k.grid_x, k.dispatch_id from pmc_events p join kernels k "
                    "on p.dispatch_id = k.dispatch_id where p.counter_name = ?", (counter,)):
                if "coalesce_kernel" in n and d > first:
                    groups.setdefault(g, ([], []))[key].append(v)
        for (pairs, L), g in zip(sorted(lv), sorted(groups)):
            f_, w_ = groups[g]
            if not f_ or not w_:
                continue
            fb = sum(f_) / len(f_) * 1024.0 * fetch_scale
            wb = sum(w_) / len(w_) * 1024.0 * write_scale
            fh.write(f"coalesce_level_{L}: pairs {pairs}, fetch_bytes_per_launch {fb:.0f}, "
                     f"write_bytes_per_launch {wb:.0f}, algorithmic_bytes_per_launch {10 * s * pairs}, "
                     f"traffic_over_algorithmic {(fb + wb) / (10 * s * pairs):.3f}, launches_averaged {len(f_)}\n")
    print(open(out).read())


def main():
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    sub.add_parser("copy")
    c = sub.add_parser("ceiling")
    c.add_argument("out")
    c.add_argument("--command", default="python3 -m paper_1508_07982_amd.profiling ceiling OUT")
    s = sub.add_parser("sweep")
    s.add_argument("--storage", default="f32")
    s.add_argument("--steps", type=int, default=2)
    s.add_argument("--workload", default="sphere", choices=["sphere", "slab"])
    s.add_argument("--separate-coalescence", action="store_true")
    t = sub.add_parser("trace-summary")
    t.add_argument("results")
    t.add_argument("out")
    t.add_argument("--command", required=True)
    t.add_argument("--storage", default="f32")
    t.add_argument("--workload", default="sphere", choices=["sphere", "slab"])
    tr = sub.add_parser("traffic-summary")
    for k in ("copy_fetch", "copy_write", "sweep_fetch", "sweep_write", "out"):
        tr.add_argument(k)
    tr.add_argument("--command", required=True)
    tr.add_argument("--storage", default="f32")
    a = ap.parse_args()
    if a.cmd == "copy":
        run_copy()
    elif a.cmd == "ceiling":
        write_ceilings(a.out, a.command)
    elif a.cmd == "sweep":
        run_sweep(a.storage, a.steps, a.workload, a.separate_coalescence)
    elif a.cmd == "trace-summary":
        trace_summary(a.results, a.out, a.command, a.storage, a.workload)
    else:
        traffic_summary(a.copy_fetch, a.copy_write, a.sweep_fetch, a.sweep_write, a.out, a.command, a.storage)


if __name__ == "__main__":
    main()
