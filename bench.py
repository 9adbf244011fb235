"""Jacobi3D benchmark on one MI355X.

Default workload: a 512^3 FP64 grid decomposed into 2x2x2 blocks of 256^3;
every step is one full iteration of the hot path: the faces of every block
are packed, moved through the pre-posted pairing and read as ghosts, and
the blocks are swept -- by default in one fused launch per iteration
(`--mode staged` runs the separate pack, exchange, unpack and sweep
kernels; both are also compared with host-staged exchange).  Prints one
JSON line with whole-job throughput in GLUP/s (1e9 interior lattice-site
updates per second), the sweep kernel's bandwidth against the HBM roofline
and the CPU oracle timed on a bounded sample of the same workload.

  python bench.py [--gpus 1] [--steps 1000] [--warmup 50] [--workload 512_2x2x2]
                  [--mode staged|fused] [--no-cpu] [--copy-probe]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, vendor peak
METRIC = "Jacobi3D GLUP/s + HBM GB/s (% peak); served solves/s, p50/p99 at 1e-10 resid"

WORKLOADS = {
    # name: (grid, block_dims or None, uneven cuts seed or None, default mode)
    "512_2x2x2": ((512, 512, 512), (256, 256, 256), None, "fused"),
    "64_single": ((64, 64, 64), None, None, "staged"),
    "768_8x8x8": ((768, 768, 768), (96, 96, 96), None, "fused"),
    "768_uneven": ((768, 768, 768), None, 12416, "fused"),
    # one GPU's share of the paper's weak-scaling base (1536^3 per node of
    # six GPUs, section 4.3): a single 512 x 768 x 1536 block
    "paper_share": ((512, 768, 1536), None, None, "fused"),
}

# Tile shapes picked by jc_autotune on an MI355X for the default mode
# (rows per tile, planes per work item); other workloads tune at start-up.
# The paper's Jacobi3D results (section 4.3; hardware in section 4.1), quoted
# as context beside the one-GPU exchange comparison: not the same transfer
# (there between processes and nodes), not a target.
PAPER_COMM_SPEEDUPS = {
    "hardware": "Summit: IBM AC922 nodes, 2x Power9 + 6x NVIDIA V100 each, NVLink 50 GB/s in a socket, "
                "EDR InfiniBand between nodes",
    "comm_speedup_gpu_aware_vs_host_staged": {"Charm++ GPU Messaging, weak scaling": "1.1-12.4x",
                                              "AMPI, weak scaling": "1.3-12.8x",
                                              "Charm4py, weak scaling": "1.9-19.7x"},
    "source": "paper section 4.3",
}

TUNED_TILES = {
    ("512_2x2x2", "fused"): (256, 8, 256),
    ("512_2x2x2", "staged"): (256, 8, 128),
    ("768_8x8x8", "fused"): (96, 16, 16),
    ("768_uneven", "fused"): (32, 16, 16),
}

# two-sweep launch shape (rows, planes per work-group) from jc_autotune on
# MI355X: 24-row tiles, one work-group per compute unit over the whole depth
TUNED_TEMPORAL = {
    "paper_share": (24, 1536),
}


def parse():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=400)
    ap.add_argument("--settle-ms", type=float, default=250.0,
                    help="sustained sweeps (in ms of wall time) after set-up and before the warm-up steps: the device "
                         "runs launches slower for tens of ms after tuning and graph capture left it idle")
    ap.add_argument("--workload", default="512_2x2x2",
                    choices=sorted(WORKLOADS) + ["refine", "serve", "768_grids", "batch", "small"])
    ap.add_argument("--batch-grids", type=int, default=64, help="batch: independent grids solved to 1e-10")
    ap.add_argument("--batch-edge", type=int, default=64, help="batch: cubic edge of each grid")
    ap.add_argument("--small-edges", type=int, nargs="*", default=[32, 24, 16],
                    help="small: cubic edges solved to 1e-10 with each launch form")
    ap.add_argument("--small-group-sizes", type=int, nargs="*", default=[256, 1024],
                    help="small: group sizes of members swept together")
    ap.add_argument("--small-group-edge", type=int, default=32, help="small: cubic edge of the group members")
    ap.add_argument("--ir-edge", type=int, default=1024, help="refine: grid edge of the per-sweep rates")
    ap.add_argument("--ir-sweeps", type=int, default=100, help="refine: sweeps timed per precision")
    ap.add_argument("--ir-tile", default="", help="refine: tile_x,tile_y,z_chunk of the refinement solvers "
                    "(default: the library's choice)")
    ap.add_argument("--ir-solve-edges", type=int, nargs="*", default=[64, 128],
                    help="refine: edges solved to 1e-10 end to end")
    ap.add_argument("--serve-requests", type=int, default=200)
    ap.add_argument("--serve-capacity-requests", type=int, default=0,
                    help="requests of the closed-loop capacity run (0: the same set as the timed run)")
    ap.add_argument("--serve-max-edge", type=int, default=384)
    ap.add_argument("--serve-min-edge", type=int, default=32)
    ap.add_argument("--serve-resident", action="store_true",
                    help="serve: binary64 requests of edge <= 32 in a lane of resident sweeps")
    ap.add_argument("--serve-no-graphs", action="store_true",
                    help="serve: launch every window eagerly instead of replaying a captured graph")
    ap.add_argument("--serve-max-iter", type=int, default=20000)
    ap.add_argument("--serve-budget-gb", type=float, default=64.0)
    ap.add_argument("--serve-lanes", default="64,160",
                    help="ascending edge bounds of the server's size lanes ('none': one group for all)")
    ap.add_argument("--serve-tile", default="", help="tile_x,tile_y,z_chunk of the server's groups "
                    "(default: the library's group tile)")
    ap.add_argument("--serve-rate", type=float, default=0.0,
                    help="Poisson arrival rate (requests/s); 0 = 0.7 x the measured closed-loop capacity")
    ap.add_argument("--mode", default=None, choices=["staged", "fused"])
    ap.add_argument("--temporal", action="store_true",
                    help="one-block workloads: two sweeps per launch (temporal blocking)")
    ap.add_argument("--sweeps-per-launch", type=int, default=2, choices=[2, 3],
                    help="with --temporal: sweeps per launch (two or three)")
    ap.add_argument("--temporal-tile", default="",
                    help="rows,z_chunk of the two-sweep launch (8, 16 or 24 rows; default: stored or autotuned)")
    ap.add_argument("--seed", type=int, default=12416)
    ap.add_argument("--tile-x", type=int, default=0, help="cells per tile row, 32 or 64 (0: library default)")
    ap.add_argument("--tile-y", type=int, default=0, help="rows per tile (0: library default)")
    ap.add_argument("--z-chunk", type=int, default=0, help="planes per tile (0: library default)")
    ap.add_argument("--pace", type=int, default=-1,
                    help="pace of the one-sweep launch in ticks of the 100 MHz clock (-1: tune it at start-up; "
                         "0: none)")
    ap.add_argument("--no-autotune", action="store_true",
                    help="keep the library's default tile shape instead of timing the candidates")
    ap.add_argument("--autotune", action="store_true",
                    help="re-tune even where a tuned shape is recorded for the workload")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-ab", action="store_true", help="skip the device / host-staged exchange comparison")
    ap.add_argument("--no-forms", action="store_true",
                    help="512_2x2x2: skip the reduced runs of the added forms (refinement, serving)")
    ap.add_argument("--forms-serve-requests", type=int, default=32)
    ap.add_argument("--forms-serve-max-edge", type=int, default=128)
    ap.add_argument("--no-temporal-context", action="store_true",
                    help="512_2x2x2: skip the one-block, two-sweeps-per-launch context figure")
    ap.add_argument("--ab-iters", type=int, default=100)
    ap.add_argument("--graphs", choices=["auto", "on", "off"], default="auto",
                    help="time a hipGraph replay of the whole window (fused mode; the sweep's time is then the "
                         "stream time per iteration) instead of eager launches with HIP events around each; "
                         "auto: on in fused mode")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--copy-probe", action="store_true",
                    help="only run a plain device copy of known size (counter calibration)")
    return ap.parse_args()


def tmode(args):
    """The temporal argument of Solver / Group / Server for --temporal and
    --sweeps-per-launch: False, True (two sweeps per launch) or 3."""
    if not args.temporal:
        return False
    return 3 if args.sweeps_per_launch == 3 else True


def copy_probe():
    """A plain device copy of known size: its HBM counters calibrate the
    sweep's, and its rate is the practical streaming ceiling."""
    import torch
    n = 1 << 28                                   # 2 GiB of float64
    a = torch.ones(n, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    reps = 10
    e0.record()
    for _ in range(reps):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    print(json.dumps({"copy_probe_bytes_read": n * 8, "copy_probe_bytes_written": n * 8,
                      "launches": 3 + reps, "ms_per_copy": round(ms, 4),
                      "copy_gbs": round(2 * n * 8 / (ms * 1e-3) / 1e9, 1)}))


def recorded_traffic(workload, mode, tile, pace=0):
    """HBM bytes per sweep launch from the committed rocprofv3 counters, if
    they were taken on the current kernel source and the same launch shape
    and pace (a pace within 5 % of the recorded one: it is tuned on each
    device) -- else None."""
    path = os.path.join(ROOT, "profiles", "k_sweep_%s_%s_fp64.counters.json" % (workload, mode))
    try:
        rec = json.load(open(path))
        sha = sweep_source_sha256()
    except (OSError, ValueError):
        return None
    if rec.get("sweep_source_sha256") != sha or rec.get("mode") != mode or list(rec.get("tile", [])) != list(tile):
        return None
    rp = rec.get("pace", 0)
    if (rp == 0) != (pace == 0) or abs(pace - rp) > 0.05 * max(rp, 1):
        return None
    return rec.get("traffic_bytes_per_launch")


def sweep_source_sha256(kernel="k_sweep"):
    """Fingerprint of a sweep kernel: its region of jc_kernels.hip (the
    one-sweep kernel with the helpers it defines; the two-sweep kernel
    also with those helpers) plus the shared table definitions and the
    division helpers it includes."""
    import hashlib
    csrc = os.path.join(ROOT, "paper_2102_12416_amd", "csrc")
    text = open(os.path.join(csrc, "jc_kernels.hip")).read()
    a = text.index("// ---- sweep kernel: begin")
    b = text.index("// ---- sweep kernel: end")
    h = hashlib.sha256(text[a:b].encode())
    if kernel == "k_sweep2":
        c = text.index("// ---- two-step sweep (temporal blocking): begin")
        d = text.index("// ---- two-step sweep: end")
        h.update(text[c:d].encode())
    h.update(open(os.path.join(csrc, "jc_types.h"), "rb").read())
    h.update(open(os.path.join(csrc, "jc_div6.h"), "rb").read())
    return h.hexdigest()


def recorded_traffic_temporal(workload, shape):
    """HBM bytes per two-sweep launch from the committed rocprofv3 counters,
    if taken on the current kernel source and the same shape (else None)."""
    path = os.path.join(ROOT, "profiles", "k_sweep2_%s_fp64.counters.json" % workload)
    try:
        rec = json.load(open(path))
        sha = sweep_source_sha256("k_sweep2")
    except (OSError, ValueError):
        return None
    if rec.get("sweep_source_sha256") != sha or list(rec.get("temporal_tile", [])) != list(shape):
        return None
    return rec.get("traffic_bytes_per_launch")


def exchange_ab(grid, bd, seed, iters, tiles):
    """The paper's comparison on one GPU: the same staged iteration with the
    faces moved by the pre-posted device pairing, by host staging, and by a
    device copy announced through a host metadata round trip.  Returns ms
    per iteration and the communication part (pack + exchange + unpack)."""
    import torch

    import synth
    from paper_2102_12416_amd import Solver, _lib as L
    u0 = synth.boundary_field(grid, seed=seed)
    out = {}
    for mode in ("device", "host", "metadata", "device_overlap"):
        overlap = mode == "device_overlap"
        with Solver(grid, block_dims=bd, mode="staged", use_graphs=False, exchange=mode.split("_")[0],
                    overlap=overlap) as s:
            s.set_tiles(*tiles)
            s.load(u0)
            s.iterate(20)
            # the iteration time with no per-kernel events, eager launches
            s.synchronize()
            t0 = time.perf_counter()
            s.iterate(iters)
            s.synchronize()
            wall = time.perf_counter() - t0
            # then the kernels, each bracketed by events
            s.set_timing(True)
            s.iterate(iters)
            s.synchronize()
            comm = sum(s.kernel_time(k)[0] for k in (L.JC_K_PACK, L.JC_K_EXCHANGE, L.JC_K_UNPACK))
            sweep = s.kernel_time(L.JC_K_SWEEP)[0]
            s.set_timing(False)
        out[mode] = dict(ms_per_iter=round(wall * 1e3 / iters, 4), comm_ms_per_iter=round(comm / iters, 4),
                         sweep_ms_per_iter=round(sweep / iters, 4))
    d = out["device"]
    for mode in ("host", "metadata"):
        out[mode]["comm_speedup_of_device"] = round(out[mode]["comm_ms_per_iter"] / d["comm_ms_per_iter"], 2)
        out[mode]["iter_speedup_of_device"] = round(out[mode]["ms_per_iter"] / d["ms_per_iter"], 2)
    o = out["device_overlap"]
    o["note"] = ("boundary tiles first, then pack / exchange / unpack of the new iterate on a second stream while "
                 "the interior tiles sweep; comm and sweep times overlap, the iteration is ms_per_iter")
    o["iter_speedup_over_device"] = round(d["ms_per_iter"] / o["ms_per_iter"], 3)
    return out


def temporal_one_block(grid, seed, iters=198):
    """Context for the bench line: the grid as one block with temporal
    blocking, two and three sweeps per launch (shapes from jc_autotune),
    each timed as one graph replay of `iters` iterations after a warm-up,
    apart from the headline measurement."""
    import torch

    from paper_2102_12416_amd import Solver, synth_field
    out = {"grid": list(grid), "blocks": 1, "iterations": iters,
           "note": "the same grid as one block (no inter-block exchange), several sweeps per launch: bitwise the "
                   "same iterate; not the headline, which exchanges halos between 8 blocks every iteration"}
    for depth, temporal in ((2, True), (3, 3)):
        with Solver(grid, mode="fused", temporal=temporal) as s:
            s.load(synth_field(grid, seed, 0))
            s.autotune(reps=3)
            s.iterate(iters)
            s.iterate(iters)                 # captures the window's graph
            s.synchronize()
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(s.stream)
            s.iterate(iters)
            e1.record(s.stream)
            e1.synchronize()
            ms = e0.elapsed_time(e1)
            t2 = s.temporal_info()
        cells = float(grid[0]) * grid[1] * grid[2]
        launch_ms = depth * ms / iters
        out["%s_sweeps" % ("two" if depth == 2 else "three")] = {
            "kernel": "k_sweep%d" % depth, "temporal_tile": [t2["rows"], t2["z_chunk"]],
            "glups": round(cells * iters / (ms * 1e-3) / 1e9, 1), "ms_per_launch": round(launch_ms, 5),
            "roofline_frac": round(16 * cells / (launch_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
            "bytes_per_unit": "16 B per cell per launch (%.2f B per update)" % (16.0 / depth)}
    return out


def cpu_baseline(grid, seed, seconds):
    """The oracle as it stands, on the undecomposed grid, for a bounded
    number of sweeps; returns GLUP/s and what was run."""
    import numpy as np

    import oracle
    import synth
    u = synth.boundary_field(grid, seed=seed)
    v = u.copy()
    lib = oracle.lib()
    dp = oracle._dptr
    nx, ny, nz = grid
    sweeps = 0
    t0 = time.perf_counter()
    while True:
        lib.oracle_sweep(dp(u), dp(v), None, nx, ny, nz)
        u, v = v, u
        sweeps += 1
        if time.perf_counter() - t0 >= seconds and sweeps >= 2:
            break
    dt = time.perf_counter() - t0
    lups = float(nx) * ny * nz * sweeps
    del u, v
    model = ""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return dict(value=lups / dt / 1e9, unit="GLUP/s", cores=oracle.num_threads(), cpu_model=model,
                kind="oracle",
                sample="%d sweeps of the undecomposed %dx%dx%d grid (C oracle, OpenMP) in %.1f s"
                       % (sweeps, nx, ny, nz, dt),
                host_cpus=len(os.sched_getaffinity(0)))


# tile shapes of the per-sweep refinement rates at 1024^3 in the default run
# (the inner sweep of the correction for the refined forms), from jc_autotune
# on MI355X; the pace is tuned at start-up
FORM_TILES = {"f64": (64, 32, 1024), "f32": (64, 32, 1024), "bf16": (64, 8, 128)}


def host_residual_norm(u, b):
    """|b + s(u) - 6u|_2 over the interior in binary64 on the host (numpy):
    the certificate of a served result, computed apart from the GPU path."""
    import numpy as np
    c = u[1:-1, 1:-1, 1:-1]
    s = u[1:-1, 1:-1, :-2] + u[1:-1, 1:-1, 2:]
    s = s + u[1:-1, :-2, 1:-1]
    s = s + u[1:-1, 2:, 1:-1]
    s = s + u[:-2, 1:-1, 1:-1]
    s = s + u[2:, 1:-1, 1:-1]
    r = (b[1:-1, 1:-1, 1:-1] + s) - 6.0 * c
    return float(np.sqrt(np.sum(r * r)))


def forms(args):
    """The added forms in reduced configurations, for the default run (each
    named in its own config): mixed precision at 1024^3 (per-sweep rates of
    the binary64 sweep with a source and of the binary32- and
    bfloat16-stored refinement, one outer step of 50 inner sweeps), time to
    a 1e-10 relative residual at 128^3 for binary64 and the refined forms
    (error against binary64 per result), and a served Poisson run with a
    host certificate of every result."""
    import numpy as np
    import torch

    import synth
    from paper_2102_12416_amd import Solver, _lib as L, synth_field
    from paper_2102_12416_amd.server import Request, Server, summarize
    res = {}
    # ---- mixed precision, per sweep, 1024^3 with a source
    n = 1024
    grid = (n, n, n)
    lups = float(n) ** 3
    g = synth_field(grid, args.seed, 0)
    b = synth_field(grid, args.seed, 1)
    rates = {}
    for dt in ("f64", "f32", "bf16"):
        ir = None if dt == "f64" else dt
        with Solver(grid, with_source=True, ir_dtype=ir, use_graphs=False) as s:
            s.load(g, b)
            s.set_tiles(*FORM_TILES[dt])
            pace = s.autotune_pace(reps=4)[0]
            s.set_timing(True)
            if ir is None:
                s.iterate(50)
                ms, k = s.kernel_time(L.JC_K_SWEEP)
                rates["f64_plain"] = dict(glups=round(lups * k / (ms * 1e-3) / 1e9, 1),
                                          gbs=round(24 * lups * k / (ms * 1e-3) / 1e9, 1),
                                          ms_per_sweep=round(ms / k, 4), tile=list(FORM_TILES[dt]), pace=pace,
                                          bytes_per_update=24)
            else:
                info = s.solve_ir(inner=50, rtol=0.0, max_inner=50)
                ms_in, k_in = s.kernel_time(L.JC_K_IR_INNER)
                ms_out, _ = s.kernel_time(L.JC_K_IR_OUTER)
                rates["%s_refined" % dt] = dict(
                    glups=round(lups * info["iters"] / ((ms_in + ms_out) * 1e-3) / 1e9, 1),
                    inner_gbs=round((12 if dt == "f32" else 6) * lups * k_in / (ms_in * 1e-3) / 1e9, 1),
                    ms_per_sweep_with_outer=round((ms_in + ms_out) / info["iters"], 4), tile=list(FORM_TILES[dt]),
                    pace=pace, bytes_per_update=12 if dt == "f32" else 6)
            s.set_timing(False)
    del g, b
    torch.cuda.empty_cache()
    for k in ("f32_refined", "bf16_refined"):
        rates[k]["speedup_vs_f64"] = round(rates[k]["glups"] / rates["f64_plain"]["glups"], 2)
    res["refinement_1024"] = dict(config="1024^3 interior, source U[-1,1), boundary U[0,1); refinement: one outer "
                                         "step of 50 inner sweeps (binary64 residual, update and norm included)",
                                  per_sweep=rates)
    print("[bench] forms: refinement per sweep %s" % json.dumps(rates), file=sys.stderr, flush=True)
    # ---- time to 1e-10 at 128^3: binary64 vs the refined forms (two and three sweeps per launch)
    m = 128
    gm = (m, m, m)
    gg = synth_field(gm, args.seed, 0)
    bb = synth_field(gm, args.seed, 1)
    row = {}
    for tag, ir, temporal in (("f64", None, False), ("f64_temporal", None, True), ("f32_refined_temporal", "f32", True),
                              ("bf16_refined_temporal", "bf16", True), ("f64_three_sweeps", None, 3),
                              ("f32_refined_three_sweeps", "f32", 3), ("bf16_refined_three_sweeps", "bf16", 3)):
        with Solver(gm, with_source=True, ir_dtype=ir, temporal=temporal) as s:
            s.load(gg, bb)
            s.autotune(reps=2)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            info = s.solve(rtol=1e-10, max_iter=2000000, check_every=50) if ir is None else \
                s.solve_ir(inner=50, rtol=1e-10, max_inner=2000000)
            sec = time.perf_counter() - t0
            u = s.store()
            if tag == "f64":
                u64, scale = u, float(u.abs().max())
            row[tag] = dict(seconds=round(sec, 3), sweeps_per_launch=3 if temporal == 3 else 2 if temporal else 1,
                            sweeps=info["iters"], rel_resid=info["rel_resid"],
                            converged=info["converged"],
                            max_rel_err_vs_f64=float((u - u64).abs().max()) / scale)
    for tag in row:
        row[tag]["speedup_vs_f64"] = round(row["f64"]["seconds"] / row[tag]["seconds"], 2)
    res["time_to_1e-10_128"] = row
    del gg, bb, u, u64
    print("[bench] forms: time to 1e-10 at 128^3 %s" % json.dumps(row), file=sys.stderr, flush=True)
    # ---- serving: Poisson arrivals, continuous batching, certificates
    nreq, hi = args.forms_serve_requests, args.forms_serve_max_edge
    budget = int(args.serve_budget_gb * (1 << 30))

    def reqs(rate):
        return [Request(id=r["id"], arrival=r["arrival"], n=r["n"], precision=r["precision"], seed=r["seed"])
                for r in synth.serving_requests(nreq, rate, seed=args.seed, lo=32, hi=hi)]

    def server(keep):
        return Server(budget_bytes=budget, window=50, rtol=1e-10, max_iter=args.serve_max_iter, lanes=(64, 160),
                      temporal=3, keep_fields=keep)
    t0 = time.perf_counter()
    cap = summarize(server(False).run(reqs(0.0), realtime=False), 1.0)
    cap_s = time.perf_counter() - t0
    capacity = cap["served"] / cap_s
    rate = 0.7 * capacity
    run = reqs(rate)
    srv = server(True)
    t0 = time.perf_counter()
    out = srv.run(run, realtime=True)
    span = time.perf_counter() - t0
    summ = summarize(out, span)
    worst, certified = 0.0, 0
    for rq, r in zip(run, out):
        if r.rejected:
            continue
        nn = (rq.n, rq.n, rq.n)
        u0 = synth.boundary_field(nn, seed=rq.seed)
        bs = synth.source_field(nn, seed=rq.seed)
        rel = host_residual_norm(r.field, bs) / host_residual_norm(u0, bs)
        worst = max(worst, abs(rel - r.rel_resid) / max(rel, 1e-300))
        certified += int((rel <= 1e-10 * (1 + 1e-9)) == r.converged)
        r.field = None
    res["serving"] = dict(
        config=dict(requests=nreq, edges="log-uniform [32, %d]" % hi, precision="Bernoulli(0.5) f64 / f32-refined",
                    rtol=1e-10, max_iter=args.serve_max_iter, window=50, lanes=[64, 160],
                    sweeps_per_launch=3, budget_gb=args.serve_budget_gb,
                    rate_per_s=round(rate, 3), rate_source="0.7 x closed-loop capacity of the same requests"),
        solves_per_s=round(summ["solves_per_s"], 3), p50_s=round(summ["p50_s"], 4), p99_s=round(summ["p99_s"], 4),
        mean_s=round(summ["mean_s"], 4), converged=summ["converged"], capped=summ["capped"],
        rejected=summ["rejected"], closed_loop_capacity_per_s=round(capacity, 3),
        certificate=dict(checked=summ["served"], stop_confirmed=certified,
                         max_rel_diff_host_vs_gpu_residual=worst,
                         how="numpy binary64 residual of every returned iterate over that of the initial one"))
    print("[bench] forms: serving %s" % json.dumps(res["serving"]), file=sys.stderr, flush=True)
    res["small_grids"] = small_group_rates(args, 256, 32, forms_=("three_sweeps", "resident"))
    print("[bench] forms: small grids %s" % json.dumps(res["small_grids"]), file=sys.stderr, flush=True)
    return res


def small_group_rates(args, count, m, forms_=("one_sweep", "three_sweeps", "resident"), window=300):
    """A group of `count` independent m^3 grids (binary64, with a source)
    swept together in each launch form: time per sweep of all members over
    a window of shared launches (HIP events, graph replay), aggregate
    GLUP/s, and whether a member's iterate equals the first form's."""
    import torch

    from paper_2102_12416_amd import Group, Solver, synth_field
    gm = (m, m, m)
    kws = {"one_sweep": dict(), "three_sweeps": dict(temporal=3), "resident": dict(resident=True)}
    stream = torch.cuda.Stream()
    solvers = [Solver(gm, mode="fused", with_source=True, use_graphs=False, stream=stream) for _ in range(count)]
    row, ref = {}, None
    for tag in forms_:
        for i, s in enumerate(solvers):
            s.load(synth_field(gm, args.seed + i, 0), synth_field(gm, args.seed + i, 1))
        with Group(solvers, use_graphs=True, stream=stream, **kws[tag]) as grp:
            grp.iterate(window)                   # warm-up and graph capture
            grp.stream.synchronize()
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(grp.stream)
            grp.iterate(window)
            e1.record(grp.stream)
            e1.synchronize()
            ms = e0.elapsed_time(e1) / window
        u = solvers[count // 2].store()
        if ref is None:
            ref = u
        row[tag] = dict(us_per_sweep=round(ms * 1e3, 2), glups=round(count * m ** 3 / (ms * 1e-3) / 1e9, 2),
                        bitwise_equal_first_form=bool(torch.equal(u, ref)))
    for s in solvers:
        s.close()
    del solvers
    torch.cuda.empty_cache()
    return dict(config="group of %d independent %d^3 grids, binary64 with a source, fused, %d-sweep windows"
                       % (count, m, window), forms=row)


def bench_refinement(args):
    """Mixed precision at 1024^3 with a source: per-sweep rate of the plain
    binary64 sweep and of the binary32 / bfloat16 inner sweeps (one outer
    step of 50 inner sweeps each), and time to 1e-10 at smaller grids."""
    import torch

    from paper_2102_12416_amd import Solver, _lib as L, synth_field
    n = args.ir_edge
    grid = (n, n, n)
    lups = float(n) ** 3
    out = {"metric": "Jacobi3D refinement: GLUP/s per sweep and time to 1e-10 relative residual",
           "unit": "GLUP/s", "n_gpus": 1, "higher_is_better": True, "data": "synthetic",
           "config": {"workload": "refine_%d" % n, "grid": list(grid), "inner_sweeps": 50,
                      "source": "U[-1,1) SplitMix64", "boundary": "U[0,1) SplitMix64"}}
    g = synth_field(grid, args.seed, 0)
    b = synth_field(grid, args.seed, 1)
    rates = {}
    # plain binary64 sweeps with the source: 24 bytes per update
    with Solver(grid, with_source=True, use_graphs=False) as s:
        s.load(g, b)
        s.autotune(reps=2)
        s.iterate(5)
        s.set_timing(True)
        s.iterate(args.ir_sweeps)
        ms, k = s.kernel_time(L.JC_K_SWEEP)
        rates["f64_plain"] = dict(glups=lups * k / (ms * 1e-3) / 1e9, gbs=24 * lups * k / (ms * 1e-3) / 1e9,
                                  ms_per_sweep=ms / k)
        s.set_timing(False)
    # the same binary64 sweeps, two per launch (temporal blocking): 24 bytes
    # per cell per launch (read u and b, write u), 12 per update
    with Solver(grid, with_source=True, use_graphs=False, temporal=True) as s:
        s.load(g, b)
        s.autotune(reps=2)
        s.iterate(4)
        s.set_timing(True)
        s.iterate(2 * (args.ir_sweeps // 2))
        ms, k = s.kernel_time(L.JC_K_SWEEP2)
        t2 = s.temporal_info()
        rates["f64_temporal"] = dict(glups=2 * lups * k / (ms * 1e-3) / 1e9, gbs=24 * lups * k / (ms * 1e-3) / 1e9,
                                     ms_per_sweep=ms / (2 * k), tile=[t2["rows"], t2["z_chunk"]])
        s.set_timing(False)
    # refinement, one inner sweep per launch (12 / 6 bytes per update with
    # r_lo), then two per launch (temporal blocking: 12 / 6 bytes per cell
    # per launch, 6 / 3 per update)
    for dt, inner_bytes, temporal in (("f32", 12, False), ("bf16", 6, False), ("f32", 12, True),
                                      ("bf16", 6, True)):
        tag = dt + ("_temporal" if temporal else "")
        with Solver(grid, with_source=True, ir_dtype=dt, use_graphs=False, temporal=temporal) as s:
            s.load(g, b)
            if args.ir_tile and not temporal:
                s.set_tiles(*[int(v) for v in args.ir_tile.split(",")])
            else:
                s.autotune(reps=2)      # tunes the inner sweep of the correction
            out["config"]["ir_tile_%s" % tag] = list(s.tile_info().values())[:3]
            if temporal:
                t2 = s.temporal_info()
                out["config"]["ir_temporal_tile_%s" % dt] = [t2["rows"], t2["z_chunk"]]
            s.set_timing(True)
            t0 = time.perf_counter()
            info = s.solve_ir(inner=50, rtol=0.0, max_inner=args.ir_sweeps)
            wall = time.perf_counter() - t0
            ms_in, k_in = s.kernel_time(L.JC_K_IR_INNER)
            ms_out, k_out = s.kernel_time(L.JC_K_IR_OUTER)
            s.set_timing(False)
            total_ms = ms_in + ms_out
            rates["%s_refined%s" % (dt, "_temporal" if temporal else "")] = dict(
                glups=lups * info["iters"] / (total_ms * 1e-3) / 1e9,
                # the first sweep of each step (no neighbour reads) is one of
                # the launches timed; per launch bytes of the later sweeps
                inner_gbs=inner_bytes * lups * k_in / (ms_in * 1e-3) / 1e9,
                inner_launches=k_in, ms_per_inner_sweep=ms_in / max(info["iters"], 1), outer_ms_total=ms_out,
                inner_sweeps=info["iters"], rel_resid=info["rel_resid"], wall_s=wall)
    del g, b
    torch.cuda.empty_cache()
    out["per_sweep"] = rates
    out["value"] = round(rates["f32_refined"]["glups"], 2)
    # time to 1e-10 at grids where it is feasible in a benchmark run
    ttt = {}
    for m in args.ir_solve_edges:
        gm = (m, m, m)
        gg = synth_field(gm, args.seed, 0)
        bb = synth_field(gm, args.seed, 1)
        row = {}
        with Solver(gm, with_source=True) as s:
            s.load(gg, bb)
            s.autotune(reps=2)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            info = s.solve(rtol=1e-10, max_iter=2000000, check_every=50)
            row["f64_plain"] = dict(seconds=time.perf_counter() - t0, sweeps=info["iters"],
                                    rel=info["rel_resid"], converged=info["converged"])
            u64 = s.store()          # the FP64 path is bitwise the oracle's Jacobi (parity tests)
            scale = float(u64.abs().max())
        with Solver(gm, with_source=True, temporal=True) as s:
            s.load(gg, bb)
            s.autotune(reps=2)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            info = s.solve(rtol=1e-10, max_iter=2000000, check_every=50)
            row["f64_temporal"] = dict(seconds=time.perf_counter() - t0, sweeps=info["iters"],
                                       rel=info["rel_resid"], converged=info["converged"],
                                       bitwise_equal_f64_plain=bool(torch.equal(s.store(), u64)))
        for dt, temporal in (("f32", False), ("bf16", False), ("f32", True), ("bf16", True)):
            with Solver(gm, with_source=True, ir_dtype=dt, temporal=temporal) as s:
                s.load(gg, bb)
                s.autotune(reps=2)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                info = s.solve_ir(inner=50, rtol=1e-10, max_inner=2000000)
                row["%s_refined%s" % (dt, "_temporal" if temporal else "")] = dict(seconds=time.perf_counter() - t0, sweeps=info["iters"],
                                              rel=info["rel_resid"], converged=info["converged"],
                                              max_rel_err_vs_f64=float((s.store() - u64).abs().max()) / scale)
        del u64
        ttt[str(m)] = row
        print("[bench] time to 1e-10 at %d^3: %s" % (m, json.dumps(row)), file=sys.stderr, flush=True)
    out["time_to_1e-10"] = ttt
    print(json.dumps(out), flush=True)


def bench_batch(args):
    """Independent FP64 solves to 1e-10 relative residual, one after another
    (each its own context, graph-captured windows) against all of them in one
    group (shared launches, continuous batching with no arrivals).  The two
    stop every solve at the same check, so the work is identical."""
    import torch

    from paper_2102_12416_amd import Solver
    from paper_2102_12416_amd.server import Request, Server, summarize
    n, count = args.batch_edge, args.batch_grids
    rtol, window, cap = 1e-10, 50, 200000
    reqs = [Request(id=i, arrival=0.0, n=n, precision="f64", seed=args.seed + 1000 + i) for i in range(count)]
    from paper_2102_12416_amd import synth_field
    # one after another: each solve with its own context and stream
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    seq_iters = []
    for r in reqs:
        with Solver((n, n, n), mode="fused", with_source=True, temporal=tmode(args)) as s:
            s.load(synth_field((n, n, n), r.seed, 0), synth_field((n, n, n), r.seed, 1))
            info = s.solve(rtol=rtol, max_iter=cap, check_every=window)
            seq_iters.append(info["iters"])
    torch.cuda.synchronize()
    seq_s = time.perf_counter() - t0
    print("[bench] one after another: %.3f s" % seq_s, file=sys.stderr, flush=True)
    srv = Server(budget_bytes=1 << 40, window=window, rtol=rtol, max_iter=cap, lanes=(), temporal=tmode(args))
    t0 = time.perf_counter()
    res = srv.run(reqs, realtime=False)
    bat_s = time.perf_counter() - t0
    same = [a == b.iters for a, b in zip(seq_iters, res)]
    out = {"metric": "time to 1e-10 relative residual for independent solves: batched vs one after another",
           "value": round(seq_s / bat_s, 3), "unit": "x (speedup of batching)", "n_gpus": 1, "higher_is_better": True,
           "data": "synthetic", "dtype": "f64",
           "config": {"workload": "batch", "grids": count, "grid": [n, n, n], "rtol": rtol, "check_every": window,
                      "temporal": bool(args.temporal), "sweeps_per_launch": args.sweeps_per_launch if args.temporal else 1,
                      "source": "U[-1,1) SplitMix64", "boundary": "U[0,1) SplitMix64"},
           "one_after_another_s": round(seq_s, 3), "batched_s": round(bat_s, 3),
           "sweeps_per_solve": [min(seq_iters), max(seq_iters)], "same_stop_as_alone": all(same),
           "batched_summary": summarize(res, bat_s)}
    print(json.dumps(out), flush=True)


def bench_small(args):
    """Small grids (binary64, with source) solved to 1e-10 with each launch
    form: one, two and three sweeps per launch (graph-captured windows,
    shapes tuned by jc_autotune), and resident sweeps (one launch per
    window, the grid on chip).  Per form: time per sweep over a long
    window (HIP events on the context's stream) and wall time to 1e-10
    with a residual check every 50 sweeps; every form's final iterate is
    compared with the one-sweep form's."""
    import torch

    from paper_2102_12416_amd import Solver, _lib as L, synth_field
    forms_ = (("one_sweep", dict()), ("two_sweeps", dict(temporal=True)), ("three_sweeps", dict(temporal=3)),
              ("resident", dict(resident=True)))
    rows = {}
    for m in args.small_edges:
        gm = (m, m, m)
        g = synth_field(gm, args.seed, 0)
        b = synth_field(gm, args.seed, 1)
        row, ref = {}, None
        for tag, kw in forms_:
            with Solver(gm, mode="fused", with_source=True, **kw) as s:
                s.load(g, b)
                if not kw.get("resident"):
                    s.autotune(reps=2)
                window = 3000
                s.iterate(window)                 # warm-up (and graph capture)
                s.stream.synchronize()
                e0 = torch.cuda.Event(enable_timing=True)
                e1 = torch.cuda.Event(enable_timing=True)
                e0.record(s.stream)
                s.iterate(window)
                e1.record(s.stream)
                e1.synchronize()
                ms = e0.elapsed_time(e1) / window
                s.load(g, b)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                info = s.solve(rtol=1e-10, max_iter=2000000, check_every=50)
                sec = time.perf_counter() - t0
                u = s.store()
                if ref is None:
                    ref = u
                row[tag] = dict(us_per_sweep=round(ms * 1e3, 3), glups=round(m ** 3 / (ms * 1e-3) / 1e9, 3),
                                seconds_to_1e10=round(sec, 4), sweeps=info["iters"], converged=info["converged"],
                                bitwise_equal_one_sweep=bool(torch.equal(u, ref)))
        rows[str(m)] = row
        print("[bench] small %d^3: %s" % (m, json.dumps(row)), file=sys.stderr, flush=True)
    # many small solves at once: a group of 32^3 members, each form's
    # launches shared by all members (one work-group per member when resident)
    batch = {}
    ge = args.small_group_edge
    for count in args.small_group_sizes:
        batch[str(count)] = small_group_rates(args, count, ge)["forms"]
        print("[bench] small group of %d x %d^3: %s" % (count, ge, json.dumps(batch[str(count)])), file=sys.stderr,
              flush=True)
    first = rows[str(args.small_edges[0])]
    best_other = min(first[t]["seconds_to_1e10"] for t in ("one_sweep", "two_sweeps", "three_sweeps"))
    out = {"metric": "time to 1e-10 relative residual for a small grid: resident sweeps vs launches per sweep",
           "value": round(best_other / first["resident"]["seconds_to_1e10"], 3),
           "unit": "x (speedup of resident sweeps over the fastest launch form, first edge)", "n_gpus": 1,
           "higher_is_better": True, "data": "synthetic", "dtype": "f64",
           "config": {"workload": "small", "edges": list(args.small_edges), "rtol": 1e-10, "check_every": 50,
                      "mode": "fused, one block", "source": "U[-1,1) SplitMix64", "boundary": "U[0,1) SplitMix64"},
           "forms": rows, "group_edge": ge, "groups": batch}
    if batch:
        # the resident kernel is neither HBM- nor matrix-bound: price its
        # binary64 vector arithmetic (per update five neighbour additions,
        # the source addition, a multiply and two fused multiply-adds = 10
        # flops; the rarely taken IEEE division aside) against the part's
        # binary64 vector peak, at the largest group
        big = str(max(args.small_group_sizes))
        rate = batch[big]["resident"]["glups"] * 1e9 * 10 / 1e12
        out["roofline"] = {"bound": "alu", "kernel": "k_resident (group of %s x %d^3)" % (big, ge),
                           "achieved": round(rate, 3), "peak": 78.6, "unit": "TFLOP/s", "frac": round(rate / 78.6, 4),
                           "flops_per_update": 10, "traffic": None,
                           "note": "latency-bound plane steps (LDS round trip, barrier, dependent binary64 chains); "
                                   "HBM traffic is one read and write of each block per launch"}
    print(json.dumps(out), flush=True)


def bench_grids(args):
    """Many independent grids in one launch per iteration: 512 grids of
    96^3 (the 768^3 volume as separate solves, seeds seed + i), swept by a
    group.  Throughput over all grids; the kernel time per launch is the
    stream time per iteration (one launch each)."""
    import torch

    from paper_2102_12416_amd import Group, Solver, synth_field
    n, count = 96, 512
    stream = torch.cuda.Stream()
    solvers = []
    for i in range(count):
        s = Solver((n, n, n), mode="fused", use_graphs=False, stream=stream)
        g = synth_field((n, n, n), args.seed + i, 0)
        s.load(g)
        solvers.append(s)
    # a whole 96-cell row per tile (1.309 ms per iteration against 1.369 for
    # 32 x 32 x 16 tiles on MI355X)
    tile = (args.tile_x or 96, args.tile_y or 16, args.z_chunk or 16)
    out = {"metric": METRIC, "unit": "GLUP/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
           "config": {"workload": "768_grids", "grids": count, "grid": [n, n, n], "tile": list(tile),
                      "mode": "group of independent single-block solves",
                      "temporal": bool(args.temporal), "sweeps_per_launch": args.sweeps_per_launch if args.temporal else 1,
                      "launch": "hipGraph replay of the timed window"}}
    if args.temporal and args.steps % 2:
        print("bench.py: --temporal needs an even --steps", file=sys.stderr)
        sys.exit(2)
    with Group(solvers, use_graphs=True, tile=tile, temporal=tmode(args)) as grp:
        grp.iterate(args.warmup)
        # capture the timed window's graph outside the timed region (both
        # start parities when the window is odd)
        grp.iterate(args.steps)
        if args.steps % 2:
            grp.iterate(args.steps)
        grp.stream.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(grp.stream)
        grp.iterate(args.steps)
        e1.record(grp.stream)
        e1.synchronize()
        ms = e0.elapsed_time(e1)
        norms = grp.residuals()
    lups = float(count) * n ** 3
    per = ms / args.steps
    out["ms_per_step"] = round(per, 5)
    out["value"] = round(lups / (per * 1e-3) / 1e9, 3)
    if args.temporal:
        # one two-sweep launch per two iterations: 16 B per cell per launch
        launch_ms = 2 * per
        out["roofline"] = {"bound": "hbm", "kernel": "k_sweep2(group)",
                           "achieved": round(16 * lups / (launch_ms * 1e-3) / 1e9, 1), "peak": HBM_PEAK_GBS,
                           "unit": "GB/s", "frac": round(16 * lups / (launch_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                           "traffic": None, "bytes_per_launch": 16 * lups, "avg_launch_ms": round(launch_ms, 5),
                           "bytes_per_unit": "16 B per cell per two-sweep launch (8 B per update)"}
    else:
        out["roofline"] = {"bound": "hbm", "kernel": "k_sweep(group)",
                           "achieved": round(16 * lups / (per * 1e-3) / 1e9, 1), "peak": HBM_PEAK_GBS,
                           "unit": "GB/s", "frac": round(16 * lups / (per * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                           "traffic": None, "bytes_per_launch": 16 * lups, "avg_launch_ms": round(per, 5)}
    out["residual_norm_range"] = [min(norms), max(norms)]
    for s in solvers:
        s.close()
    print(json.dumps(out), flush=True)


def bench_serve(args):
    """Continuous-batching server: closed-loop capacity, then Poisson
    arrivals at 0.7x capacity (or a given rate); p50/p99 latency and solves/s."""
    import numpy as np

    import synth
    from paper_2102_12416_amd.server import Request, Server, summarize

    def reqs(count, rate, seed):
        return [Request(id=r["id"], arrival=r["arrival"], n=r["n"], precision=r["precision"], seed=r["seed"])
                for r in synth.serving_requests(count, rate, seed=seed, lo=args.serve_min_edge, hi=args.serve_max_edge)]

    budget = int(args.serve_budget_gb * (1 << 30))
    lanes = () if args.serve_lanes in ("", "none") else tuple(int(v) for v in args.serve_lanes.split(","))

    def server():
        return Server(budget_bytes=budget, window=50, rtol=1e-10, max_iter=args.serve_max_iter,
                      progress_every=15.0, lanes=lanes, temporal=tmode(args), resident=args.serve_resident,
                      use_graphs=not args.serve_no_graphs,
                      tile=[int(v) for v in args.serve_tile.split(",")] if args.serve_tile else None)

    cap = None
    rate = args.serve_rate
    if rate <= 0:
        # capacity: the same request mix, all queued at once (closed loop)
        ncap = args.serve_capacity_requests or args.serve_requests
        cap_reqs = reqs(ncap, 0.0, args.seed)
        srv = server()
        t0 = time.perf_counter()
        res = srv.run(cap_reqs, realtime=False)
        cap_time = time.perf_counter() - t0
        cap = summarize(res, cap_time)
        print("[bench] closed-loop capacity: %s" % json.dumps(cap), file=sys.stderr, flush=True)
        rate = 0.7 * cap["solves_per_s"]
    run_reqs = reqs(args.serve_requests, rate, args.seed)
    srv = server()
    t0 = time.perf_counter()
    res = srv.run(run_reqs, realtime=True)
    span = time.perf_counter() - t0
    summ = summarize(res, span)
    small = [r.latency for r in res if not r.rejected and r.n <= 64]
    summ["p50_s_edge_le_64"] = float(np.percentile(small, 50)) if small else None
    out = {"metric": "served solves/s, p50/p99 latency at 1e-10 relative residual or the sweep cap",
           "value": round(summ["solves_per_s"], 3), "unit": "solves/s", "n_gpus": 1, "higher_is_better": True,
           "data": "synthetic", "dtype": "f64 / f32-refined",
           "config": {"workload": "serve", "requests": args.serve_requests, "rate_per_s": round(rate, 3),
                      "edges": "log-uniform [%d, %d]" % (args.serve_min_edge, args.serve_max_edge),
                      "precision": "Bernoulli(0.5) f64/f32", "resident_lane": bool(args.serve_resident),
                      "graphs": not args.serve_no_graphs,
                      "rtol": 1e-10, "max_iter": args.serve_max_iter, "window": 50,
                      "budget_gb": args.serve_budget_gb, "lanes": list(lanes), "tile": args.serve_tile or "64,8,32 (group default)",
                      "rate_source": "given" if args.serve_rate > 0 else "0.7 x closed-loop capacity"},
           "p50_s": round(summ["p50_s"], 4), "p99_s": round(summ["p99_s"], 4), "summary": summ,
           "capacity": cap, "server_stats": srv.stats}
    print(json.dumps(out), flush=True)


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)
    if args.copy_probe:
        copy_probe()
        return
    if args.workload == "refine":
        bench_refinement(args)
        return
    if args.workload == "serve":
        bench_serve(args)
        return
    if args.workload == "768_grids":
        bench_grids(args)
        return
    if args.workload == "batch":
        bench_batch(args)
        return
    if args.workload == "small":
        bench_small(args)
        return

    import numpy as np
    import torch

    import synth
    from paper_2102_12416_amd import Solver, _lib as L

    grid, bd, uneven_seed, default_mode = WORKLOADS[args.workload]
    mode = args.mode or default_mode
    kw = {}
    if bd is not None:
        kw["block_dims"] = bd
    if uneven_seed is not None:
        kw["cuts"] = [synth.uneven_cuts(grid[a], 32, 160, seed=uneven_seed, axis=a) for a in range(3)]
    graphs = args.graphs == "on" or (args.graphs == "auto" and mode == "fused")
    temporal = bool(args.temporal)
    depth = (3 if args.sweeps_per_launch == 3 else 2) if temporal else 1
    if temporal and (bd is not None or uneven_seed is not None or args.steps % depth):
        print("bench.py: --temporal needs a one-block workload and --steps a multiple of the sweeps per launch",
              file=sys.stderr)
        sys.exit(2)
    if graphs and mode != "fused":
        print("bench.py: --graphs needs the fused mode (one launch per iteration)", file=sys.stderr)
        sys.exit(2)
    print("[bench] workload %s mode %s: building inputs" % (args.workload, mode), file=sys.stderr, flush=True)
    u0 = synth.boundary_field(grid, seed=args.seed)
    s = Solver(grid, mode=mode, use_graphs=graphs, tile_x=args.tile_x, tile_y=args.tile_y, z_chunk=args.z_chunk,
               temporal=tmode(args), **kw)
    s.load(u0)
    del u0
    nb = s.num_blocks
    given = bool(args.tile_x or args.tile_y or args.z_chunk)
    tile_source = "given" if given else "library default"
    if temporal:
        # the timed launches are all two-sweep launches: tune their shape
        if args.temporal_tile:
            s.set_temporal_tiles(*[int(v) for v in args.temporal_tile.split(",")])
            tile_source = "given"
        elif args.workload in TUNED_TEMPORAL and depth == 2 and not args.autotune:
            s.set_temporal_tiles(*TUNED_TEMPORAL[args.workload])
            tile_source = "tuned (jc_autotune on MI355X)"
        else:
            s.autotune(reps=3)
            tile_source = "jc_autotune at start-up"
    elif not given:
        if (args.workload, mode) in TUNED_TILES and not args.autotune:
            s.set_tiles(*TUNED_TILES[(args.workload, mode)])
            tile_source = "tuned (jc_autotune on MI355X)"
        elif not args.no_autotune:
            tuned = s.autotune(reps=3)
            tile_source = "jc_autotune at start-up"
            print("[bench] autotuned tile_x=%d tile_y=%d z_chunk=%d (%.1f us per sweep)" % tuned, file=sys.stderr,
                  flush=True)
    pace = None
    if True:
        # the pace of the timed launch (the one-sweep launch, or the multi-
        # sweep launch of a temporal context), for the shape just set: tuned
        # at start-up (it depends on the device as much as on the shape)
        if args.pace >= 0:
            s.set_pace(args.pace)
            pace = {"ticks": s.pace, "source": "given"}
        elif tile_source == "jc_autotune at start-up":
            pace = {"ticks": s.pace, "source": "jc_autotune at start-up"}
        else:
            p_ticks, us_paced, us_free = s.autotune_pace(reps=10)
            pace = {"ticks": p_ticks, "source": "jc_autotune_pace at start-up", "us_per_sweep_paced": us_paced,
                    "us_per_sweep_unpaced": us_free}
        print("[bench] pace %s" % pace, file=sys.stderr, flush=True)
    tiles = s.tile_info()
    if graphs:
        # capture the timed window's and the warm-up's graphs outside the
        # timed region (both start parities when a window is odd)
        for n in (args.steps, args.warmup):
            if n > 0:
                s.iterate(n)
                if n % 2:
                    s.iterate(n)
    # set-up (tuning, capture) leaves the device idle or lightly loaded, and
    # the next launches then run slower until it has swept for tens of ms (the
    # first 20-iteration window after 5 warm-up steps measured 2 % slow): the
    # settle phase sweeps for a fixed wall time, then the warm-up steps run
    # last, right before the timed window
    settle_iters, t_settle = 0, time.perf_counter()
    while args.settle_ms > 0 and (time.perf_counter() - t_settle) * 1e3 < args.settle_ms:
        s.iterate(args.steps)
        settle_iters += args.steps
        s.synchronize()
    s.iterate(args.warmup)
    s.synchronize()

    if not graphs:
        s.set_timing(True)
    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    ev0.record(s.stream)
    t0 = time.perf_counter()
    s.iterate(args.steps)
    ev1.record(s.stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    gpu_ms = ev0.elapsed_time(ev1)
    kinds = {"sweep": L.JC_K_SWEEP, "pack": L.JC_K_PACK, "exchange": L.JC_K_EXCHANGE,
             "unpack": L.JC_K_UNPACK, "fused": L.JC_K_FUSED, "sweep2": L.JC_K_SWEEP2, "sweep3": L.JC_K_SWEEP3}
    if graphs and temporal:
        # one multi-sweep launch per `depth` iterations
        ktime = {"sweep%d" % depth: (gpu_ms, args.steps // depth)}
    elif graphs:
        # one fused launch per iteration: the stream time per iteration bounds
        # the sweep's launch time from above
        ktime = {"fused": (gpu_ms, args.steps)}
    else:
        ktime = {k: s.kernel_time(v) for k, v in kinds.items()}
        s.set_timing(False)
    print("[bench] %d warm-up iterations, then %d timed%s: %.3f s wall, %.3f ms on the stream"
          % (args.warmup, args.steps, " as one graph replay" if graphs else "", wall, gpu_ms), file=sys.stderr,
          flush=True)

    t2_shape = [s.temporal_info()["rows"], s.temporal_info()["z_chunk"]] if temporal else None
    nx, ny, nz = grid
    lups = float(nx) * ny * nz
    ms_per_step = max(gpu_ms, wall * 1e3) / args.steps
    glups = lups * args.steps / (ms_per_step * args.steps * 1e-3) / 1e9
    dom = ("sweep%d" % depth) if temporal else "fused" if mode == "fused" else "sweep"
    dom_ms, dom_n = ktime[dom]
    avg_ms = dom_ms / max(dom_n, 1)
    # read u, write u' per cell update; the two-sweep launch reads iterate k
    # and writes iterate k + 2 once per cell (8 B per update)
    sweep_bytes = 16.0 / depth * lups
    launch_bytes = 16.0 * lups
    halo_values = sum(s.pair_info(q)["count"] for q in range(s.num_pairs))
    # the fused sweep also moves the halo: each exchanged face value is
    # written once (epilogue) and read once (the neighbour's ghost); the
    # staged sweep leaves that to pack / exchange / unpack (48 B per value)
    kernel_bytes = launch_bytes + (16.0 * halo_values if mode == "fused" else 0.0)
    achieved = kernel_bytes / (avg_ms * 1e-3) / 1e9
    step_bytes = sweep_bytes + (16.0 if mode == "fused" else 48.0) * halo_values
    out = {
        "metric": METRIC,
        "value": round(glups, 3),
        "unit": "GLUP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": args.workload, "grid": list(grid), "blocks": nb, "mode": mode,
                   "iterations": args.steps, "tile": [tiles["tile_x"], tiles["tile_y"], tiles["z_chunk"]],
                   "temporal": temporal,
                   "sweeps_per_launch": depth,
                   "temporal_tile": t2_shape,
                   "pace": pace,
                   "settle": {"iterations": settle_iters, "ms": args.settle_ms,
                              "note": "untimed sweeps after set-up, before the warm-up steps"},
                   "tile_source": tile_source,
                   "launch": "hipGraph replay of the timed window" if graphs else "eager, HIP events per launch",
                   "boundary": "U[0,1) SplitMix64 seed %d, interior 0, no source" % args.seed},
        "hbm_gbs_step": round(step_bytes / (ms_per_step * 1e-3) / 1e9, 1),
        "pct_hbm_peak_step": round(100 * step_bytes / (ms_per_step * 1e-3) / 1e9 / HBM_PEAK_GBS, 2),
        "roofline": {"bound": "hbm",
                     "kernel": ("k_sweep%d" % depth) if temporal else "k_sweep" if mode == "staged" else "k_sweep(fused)",
                     "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": (recorded_traffic_temporal(args.workload, t2_shape) if depth == 2 else None)
                     if temporal else recorded_traffic(
                         args.workload, mode, [tiles["tile_x"], tiles["tile_y"], tiles["z_chunk"]],
                         pace["ticks"] if pace else 0),
                     "bytes_per_launch": kernel_bytes, "avg_launch_ms": round(avg_ms, 5),
                     "bytes_per_unit": (("16 B per cell per %d-sweep launch (%.2f B per update)" % (depth, 16.0 / depth))
                                        if temporal else
                                        "16 B per update" + (" + 16 B per exchanged face value (%d values)"
                                                             % halo_values if mode == "fused" else ""))},
        "kernel_ms_per_step": {k: round(v[0] / max(v[1], 1), 5) for k, v in ktime.items() if v[1]},
        "device": {"name": torch.cuda.get_device_name(0),
                   "arch": getattr(torch.cuda.get_device_properties(0), "gcnArchName", ""),
                   "compute_units": torch.cuda.get_device_properties(0).multi_processor_count},
    }
    tr = out["roofline"]["traffic"]
    # counter-measured DRAM bytes (recorded for this kernel source) over the live launch time
    out["roofline"]["traffic_gbs"] = None if tr is None else round(tr / (avg_ms * 1e-3) / 1e9, 1)
    s.close()
    del s
    torch.cuda.empty_cache()
    if args.workload == "512_2x2x2" and not args.no_temporal_context:
        print("[bench] context: the same grid as one block, two sweeps per launch", file=sys.stderr, flush=True)
        out["temporal_one_block"] = temporal_one_block(grid, args.seed)
    if not args.no_ab and bd is not None:
        print("[bench] exchange A/B: device pairing vs host staging vs host metadata", file=sys.stderr, flush=True)
        st_tiles = TUNED_TILES.get((args.workload, "staged"), (tiles["tile_x"], tiles["tile_y"], tiles["z_chunk"]))
        out["exchange_ab"] = exchange_ab(grid, bd, args.seed, args.ab_iters, st_tiles)
        out["exchange_ab"]["paper_context"] = PAPER_COMM_SPEEDUPS
    if args.workload == "512_2x2x2" and not args.no_forms:
        print("[bench] forms: refinement at 1024^3, time to 1e-10 at 128^3, serving", file=sys.stderr, flush=True)
        out["forms"] = forms(args)
    if not args.no_cpu:
        print("[bench] CPU oracle baseline (%.0f s budget)" % args.cpu_seconds, file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(grid, args.seed, args.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
