"""Benchmark: D8 flow routing of a 43,360 x 43,360 (1.88e9-cell) DEM on one GPU.

One step = the whole hot path over the grid: local flow routing
(fr_receivers, D8) + global flow routing (fr_accumulate: float32 rain with
float-float accumulation, exact uint64 unit-rain counts, float64 sink mass
balance).  Inputs are generated on the host, copied to HBM once, and are
resident before the timed region starts.

Prints one JSON line (see the repository's design notes for the fields).
"""
from __future__ import annotations

import argparse
import ctypes
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# Algorithmic bytes per cell of each timed phase (each array its kernels
# must touch, counted once per kernel):
PHASE_BYTES = {
    "receivers": 4 + 1,        # z read, code written
    "d8_up": 1 + 1 + 4,        # phase A: code (root sweep), code + rain (local sweep); exits are sparse
    "d8_down": 1 + 4 + 4 + 8,  # code, rain read; q (f32), counts (u64) written
    # Tile forest (flow in every direction): its phase A reads code + rain,
    # its phase C code + rain and writes q + counts; the exit forest between
    # them is not counted (exits are a few per cent of the cells).
    "d8_tiles": (1 + 4) + (1 + 4 + 4 + 8),
}
PHASE_KERNEL = {"receivers": "k_receivers", "d8_up": "k_d8_a (root + local sweep)", "d8_down": "k_d8_c",
                "d8_tiles": "k_d8t (tile forest, phases A and C) + exit forest work queue"}
ACC_BYTES = 1 + 4 + 4 + 8     # whole accumulate call: code, rain in; q, counts out
ROUTE_BYTES = 4 + 1 + ACC_BYTES  # whole route: receivers (z in, code out) + accumulate
# HBM bytes per launch from rocprofv3 FETCH_SIZE / WRITE_SIZE runs calibrated
# against a device copy, keyed by workload and phase, with the summary they
# come from.  Only counters taken on the kernels as they are now are listed;
# a phase without one reports traffic null.
MEASURED_TRAFFIC = {
    ("d8", 43360, 43360): {
        "receivers": (1.0632e10, "profiles/d8_43360_hbm_traffic.md"),
        "d8_up": (1.3366e10, "profiles/d8_43360_hbm_traffic.md"),
        "d8_down": (3.3176e10, "profiles/d8_43360_hbm_traffic.md"),
    },
    # The tile phase of the filled route: both tile kernels and the exit
    # forest's work queue (link with the children's counts, leaves, queue,
    # totals).
    ("d8_filled", 43360, 43360): {"d8_tiles": (9.3017e10, "profiles/d8_43360_filled_tile_forest.md")},
    ("mfd", 16384, 16384): {"row_sweep": (5.3063e9, "profiles/mfd_16384_row_sweep.md")},
    ("adjoint", 4096, 4096): {"sweep": (6.987e8, "profiles/sweep_and_batch_hbm_traffic.md")},
    ("batched", 512): {"batch": (2.472e10, "profiles/sweep_and_batch_hbm_traffic.md")},
}
# Algorithmic bytes per cell of the secondary workloads' dominant kernel
# (arrays visible at the C ABI, each touched once): MFD float32 sweep z 4 +
# mask 1 + q 4; adjoint z 4 + mask 1 + qbar 4 + rbar 4; batched D8 tiles z 4 +
# counts 8, MFD tiles z 4 + q 4 (codes stay in the batch workspace).
SWEEP_BYTES = {"mfd": 4 + 1 + 4, "adjoint": 4 + 1 + 4 + 4}
# Depression filling, algorithmic bytes per cell: elevation read, filled
# surface written.
FILL_BYTES = 4 + 4
METRIC = "cells routed/sec (D8 & MFD) at 1 MI355X; % HBM peak; batched vs per-tile"


def traffic(key, phase):
    """(bytes per launch, profile summary) of a counted phase, or (None, None)."""
    t = MEASURED_TRAFFIC.get(key, {}).get(phase)
    return (t[0], t[1]) if t else (None, None)


def roofline(achieved_gbs, kernel, key, phase, **extra):
    tb, src = traffic(key, phase)
    r = {"bound": "hbm", "achieved": achieved_gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
         "frac": achieved_gbs / HBM_PEAK_GBS, "traffic": tb, "kernel": kernel}
    if src:
        r["traffic_unit"] = "HBM bytes per launch (FETCH_SIZE + WRITE_SIZE, copy-calibrated)"
        r["traffic_source"] = src
    r.update(extra)
    return r


def copy_probe(dev):
    """One 1 GiB device copy: the reference for HBM byte counters."""
    import torch
    src = torch.empty(1 << 28, dtype=torch.float32, device=dev)
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    del src, dst


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def cpu_baseline(size: int, seed: int):
    """The oracle, single-threaded, on a size x size sample of the same workload."""
    import numpy as np
    import oracle
    import synth
    z = synth.dem(seed, size, size)
    rain = synth.rain(seed, size, size)
    t0 = time.perf_counter()
    code = oracle.receivers(z)
    t1 = time.perf_counter()
    order = oracle.order(z)
    t2 = time.perf_counter()
    q, c = oracle.accumulate_single(code, rain, order)
    t3 = time.perf_counter()
    s, t = oracle.mass_single(code, q, rain)
    t4 = time.perf_counter()
    n = size * size
    return {
        "value": n / (t4 - t0), "unit": "cells/s", "cores": 1, "kind": "oracle",
        "sample": (f"D8 {size}x{size} DEM seed {seed} (same generator): receivers {t1 - t0:.2f}s, "
                   f"high-to-low sort {t2 - t1:.2f}s, push q+counts {t3 - t2:.2f}s, mass {t4 - t3:.2f}s; "
                   f"host nproc={os.cpu_count()}"),
    }


def cpu_baseline_mfd(size: int, seed: int, adjoint: bool):
    """The oracle, single-threaded, on a size x size MFD sample of the same
    generator: high-to-low order, then the push (or the transpose sweep for
    the adjoint) with fractions computed from z as it goes."""
    import numpy as np
    import oracle
    import synth
    z = synth.dem(seed, size, size)
    t0 = t1 = time.perf_counter()
    order = oracle.order(z)
    t2 = time.perf_counter()
    if adjoint:
        qbar = np.zeros(size * size)
        cells = synth.distinct_cells(6, synth.STREAM_PICK, 64, size * size)
        qbar[cells] = synth.normal(6, synth.STREAM_NORMAL, 64)
        oracle.adjoint_mfd(z, qbar.reshape(size, size), 1.1, order)
    else:
        oracle.accumulate_mfd(z, None, 1.1, order)
    t3 = time.perf_counter()
    n = size * size
    what = "transpose sweep" if adjoint else "push"
    return {
        "value": n / (t3 - t0), "unit": "cells/s", "cores": 1, "kind": "oracle",
        "sample": (f"MFD {size}x{size} DEM seed {seed} (same generator): high-to-low sort {t2 - t1:.2f}s, "
                   f"{what} with fractions {t3 - t2:.2f}s; host nproc={os.cpu_count()}"),
    }


def run_secondary(args, workload):
    """MFD (16384^2, seed 3) or adjoint (MFD 4096^2, seed 5) timing lines."""
    import torch
    import synth
    import paper_2606_12800_amd as fr
    lib = fr.load_library()
    dev = torch.device("cuda:0")
    n = args.size if args.size_given else (16384 if workload == "mfd" else 4096)
    seed = 3 if workload == "mfd" else 5
    log(f"generating {n}x{n} DEM (seed {seed}) ...")
    z = torch.from_numpy(synth.dem(seed, n, n)).to(dev)
    code = torch.empty((n, n), dtype=torch.uint8, device=dev)
    status = torch.zeros(1, dtype=torch.int32, device=dev)
    stream = torch.cuda.current_stream(dev)
    sp = ctypes.c_void_p(stream.cuda_stream)
    P = lambda t: ctypes.c_void_p(t.data_ptr())
    out = {}
    fr.timing_enable(True)
    for name, dt, tdt in [("f32", fr.F32, torch.float32), ("f64", fr.F64, torch.float64)]:
        q = torch.empty((n, n), dtype=tdt, device=dev)
        wsb = fr.workspace_bytes(fr.FN_ACCUMULATE if workload == "mfd" else fr.FN_ADJOINT, n, n, fr.MFD, dt)
        ws = torch.empty(wsb, dtype=torch.uint8, device=dev)
        gbar = None
        if workload == "adjoint":
            gbar = torch.zeros((n, n), dtype=tdt, device=dev)
            cells = synth.distinct_cells(6, synth.STREAM_PICK, 64, n * n)
            w = synth.normal(6, synth.STREAM_NORMAL, 64)
            gbar.view(-1)[torch.from_numpy(cells).to(dev)] = torch.from_numpy(w).to(dev, tdt)
        times = []
        phases = {}
        for i in range(args.warmup + args.steps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            if lib.fr_receivers(P(z), n, n, fr.MFD, P(code), P(status), sp) != 0:
                raise RuntimeError("fr_receivers failed")
            if workload == "mfd":
                rc = lib.fr_accumulate(P(z), P(code), n, n, fr.MFD, 1.1, None, fr.F32, dt, P(q), None, None,
                                       P(status), P(ws), wsb, sp)
            else:
                rc = lib.fr_accumulate_adjoint(P(z), P(code), n, n, fr.MFD, 1.1, P(gbar), dt, P(q), P(status),
                                               P(ws), wsb, sp)
            if rc != 0:
                raise fr.FlowRouteError(rc, workload)
            torch.cuda.synchronize()
            if i >= args.warmup:
                times.append(time.perf_counter() - t0)
                for k, v in fr.timing_last().items():
                    phases.setdefault(k, []).append(v)
        if int(status.item()) != 0:
            raise fr.FlowRouteError(int(status.item()), "device status")
        t = sum(times) / len(times)
        out[name] = {"ms_per_step": 1e3 * t, "cells_per_s": n * n / t,
                     "phase_ms": {k: sum(v) / len(v) for k, v in phases.items()}}
        del q, ws
        torch.cuda.empty_cache()
        log(f"  {name}: {1e3 * t:.2f} ms per step")
    line = {
        "metric": METRIC,
        "value": out["f32"]["cells_per_s"], "unit": "cells/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": out["f32"]["ms_per_step"], "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": (f"MFD {n}x{n} fractal DEM (seed {seed}), unit rain, p=1.1" if workload == "mfd"
                                else f"MFD adjoint {n}x{n} (seed {seed}), 64 gauges (seed 6)"),
                   "cells": n * n},
        "detail": out,
    }
    # The sweeps are bound by the latency of their row steps, not by HBM;
    # the roofline below states how far from the HBM bound that leaves them.
    # The dominant sweep is the row sweep (k_ms) where no cell sends
    # against the row order, else the windowed wavefront sweep.
    ph = out["f32"]["phase_ms"]
    phase = "row_sweep" if ph.get("row_sweep", 0.0) >= ph.get("sweep", 0.0) else "sweep"
    ms = ph.get(phase, out["f32"]["ms_per_step"])
    kernel = "k_ms (row sweep, producer + consumer)" if phase == "row_sweep" else "k_ws_pass (all passes)"
    achieved = SWEEP_BYTES[workload] * n * n / (ms * 1e-3) / 1e9
    line["roofline"] = roofline(achieved, kernel, (workload, n, n), phase,
                                bytes_per_cell=SWEEP_BYTES[workload], ms_per_launch=ms, row_step_us=1e3 * ms / n)
    if args.copy_probe:
        copy_probe(torch.device("cuda:0"))
    if not args.no_cpu_baseline:
        # MFD: an 8192^2 sample (~15 s on one core); adjoint: the whole 4096^2 workload.
        size = args.cpu_size if "--cpu-size" in sys.argv else (8192 if workload == "mfd" else n)
        log(f"cpu baseline: oracle on {size}^2 ...")
        del z, code
        torch.cuda.empty_cache()
        line["cpu_baseline"] = cpu_baseline_mfd(size, seed, workload == "adjoint")
    return line


def run_fill(args):
    """Depression filling (epsilon variant, 8 neighbours) of an untilted
    fractal DEM (seed 2; default 43360^2; about a quarter of the cells lie
    in depressions), timed from elevations in HBM to the filled surface,
    with the oracle's priority flood on a sample as CPU baseline."""
    import torch
    import synth
    import paper_2606_12800_amd as fr
    lib = fr.load_library()
    dev = torch.device("cuda:0")
    nr = args.rows or args.size
    nc = args.cols or args.size
    log(f"generating {nr}x{nc} untilted DEM (seed {args.seed}) ...")
    z = torch.from_numpy(synth.dem(args.seed, nr, nc, tilt=0.0)).to(dev)
    f = torch.empty_like(z)
    status = torch.zeros(1, dtype=torch.int32, device=dev)
    wsb = fr.workspace_bytes(fr.FN_FILL, nr, nc, fr.D8, fr.F32)
    ws = torch.empty(wsb, dtype=torch.uint8, device=dev)
    sp = ctypes.c_void_p(torch.cuda.current_stream(dev).cuda_stream)
    P = lambda t: ctypes.c_void_p(t.data_ptr())
    launches = ctypes.c_int32(0)
    fr.timing_enable(True)
    times, dev_ms = [], []
    for i in range(args.warmup + args.steps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        rc = lib.fr_fill_depressions(P(z), nr, nc, fr.D8, 1, P(f), ctypes.byref(launches), P(status), P(ws), wsb,
                                     sp)
        if rc != 0:
            raise fr.FlowRouteError(rc, "fr_fill_depressions")
        torch.cuda.synchronize()
        if i >= args.warmup:
            times.append(time.perf_counter() - t0)
            dev_ms.append(fr.timing_last().get("fill", 0.0))
    fr._raise_status(status, "fill")
    raised = float((f > z).float().mean().item())
    t_fill = sum(times) / len(times)
    ms = sum(dev_ms) / len(dev_ms)
    ncell = nr * nc
    achieved = FILL_BYTES * ncell / (ms * 1e-3) / 1e9
    log(f"  fill: {1e3 * t_fill:.2f} ms per step ({launches.value} launches, {100 * raised:.2f}% cells raised)")
    line = {
        "metric": METRIC,
        "value": ncell / t_fill, "unit": "cells/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": 1e3 * t_fill, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "u32", "data": "synthetic",
        "config": {"workload": f"depression filling (epsilon, 8 neighbours) of the {nr}x{nc} untilted fractal "
                               f"DEM (seed {args.seed})", "cells": ncell},
        "roofline": roofline(achieved, "k_fill_tile (all launches)", ("fill", nr, nc), "fill",
                             bytes_per_cell=FILL_BYTES, ms_per_launch=ms),
        "detail": {"launches": launches.value, "fraction_raised": raised, "device_ms": ms},
    }
    if not args.no_cpu_baseline:
        size = args.cpu_size if "--cpu-size" in sys.argv else 4096
        del z, f, ws
        torch.cuda.empty_cache()
        import oracle
        zh = synth.dem(args.seed, size, size, tilt=0.0)
        log(f"cpu baseline: oracle priority flood on {size}^2 ...")
        t0 = time.perf_counter()
        oracle.fill_depressions(zh, 8, True)
        dt = time.perf_counter() - t0
        line["cpu_baseline"] = {"value": size * size / dt, "unit": "cells/s", "cores": 1, "kind": "oracle",
                                "sample": f"priority flood (binary heap) of a {size}x{size} DEM, same generator "
                                          f"and seed: {dt:.2f}s; host nproc={os.cpu_count()}"}
    print(json.dumps(line), flush=True)


def run_batched(args):
    """512 independent tiles, sides uniform in [64, 2048] (seed 4), tile i's DEM
    from seed 1000 + i; even tiles D8 with uint64 counts, odd tiles MFD with
    float32 water, unit rain.  Times the batched float32 route (one persistent
    launch, autotuned schedule, replayed from a HIP graph) against per-tile
    launches (fr_receivers + fr_accumulate per tile) in float32 and float64."""
    import torch
    import synth
    import paper_2606_12800_amd as fr
    dev = torch.device("cuda:0")
    ntiles = args.tiles
    shapes = synth.batch_shapes(4, ntiles)
    ncell = sum(a * b for a, b in shapes)
    log(f"generating {ntiles} tiles ({ncell / 1e6:.1f} Mcells) ...")
    tiles = []
    for i, (nr, nc) in enumerate(shapes):
        z = torch.from_numpy(synth.dem(1000 + i, nr, nc)).to(dev)
        t = {"z": z, "rule": "d8" if i % 2 == 0 else "mfd"}
        if i % 2 == 0:
            t["counts"] = torch.empty((nr, nc), dtype=torch.int64, device=dev)
        else:
            t["q"] = torch.empty((nr, nc), dtype=torch.float32, device=dev)
        tiles.append(t)
    b = fr.Batch(tiles)
    log(f"  workspace {b.ws_bytes / 2**30:.2f} GiB; autotuning ...")
    plan = b.autotune(reps=1)
    log(f"  plan: workers {plan.workers} order {plan.order}")
    b.run(plan=plan)
    # One batched route captured in a HIP graph (the call allocates nothing,
    # clears its counters with kernels and never synchronises with the host);
    # the timed steps are replays of that graph.
    cap = torch.cuda.Stream()
    cap.wait_stream(torch.cuda.current_stream())
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.stream(cap):
        b.run(check=False, plan=plan)
        torch.cuda.synchronize()
        with torch.cuda.graph(graph, stream=cap):
            b.run(check=False, plan=plan)
    torch.cuda.current_stream().wait_stream(cap)
    for _ in range(args.warmup):
        graph.replay()
    torch.cuda.synchronize()
    fr._raise_status(b.status, "batched route (graph)")
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    ev0.record()
    for _ in range(args.steps):
        graph.replay()
    ev1.record()
    torch.cuda.synchronize()
    t_batch = (time.perf_counter() - t0) / args.steps
    gpu_ms = ev0.elapsed_time(ev1) / args.steps
    fr._raise_status(b.status, "batched route")
    log(f"  batched float32 (graph replay): {1e3 * t_batch:.2f} ms per batch, {gpu_ms:.2f} ms on the GPU")
    # Algorithmic bytes: D8 tiles z + counts, MFD tiles z + q.
    alg = sum(a * b_ * (4 + 8 if i % 2 == 0 else 4 + 4) for i, (a, b_) in enumerate(shapes))
    del b, graph
    torch.cuda.empty_cache()
    per_tile = {}
    if not args.no_per_tile:
        for name, dt in (("f32", fr.F32), ("f64", fr.F64)):
            per_tile[name] = per_tile_route(shapes, tiles, dt)

    line = {
        "metric": METRIC,
        "value": ncell / t_batch, "unit": "cells/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": 1e3 * t_batch, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"batched: {ntiles} tiles, sides U[64,2048] (seed 4), even D8 uint64 counts, "
                               f"odd MFD float32, unit rain", "cells": ncell},
        "roofline": roofline(alg / (gpu_ms * 1e-3) / 1e9, "k_batch", ("batched", ntiles), "batch", bytes=alg,
                             ms_per_launch=gpu_ms),
        "detail": {"plan": {"workers": plan.workers, "order": plan.order}, "timing": "HIP graph replay"},
    }
    for name, t_tile in per_tile.items():
        line["detail"][f"per_tile_{name}_ms"] = 1e3 * t_tile
        line["detail"][f"per_tile_{name}_cells_per_s"] = ncell / t_tile
        line["detail"][f"batched_over_per_tile_{name}"] = t_tile / t_batch
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline_tiles(shapes)
    return line


def per_tile_route(shapes, tiles, q_dtype):
    """Seconds for routing the batch's tiles one by one (one fr_receivers +
    fr_accumulate per tile, on the same stream, a workspace allocated once),
    with q_dtype water for every tile (D8 tiles also get their counts)."""
    import torch
    import paper_2606_12800_amd as fr
    dev = torch.device("cuda:0")
    big = max(a * b_ for a, b_ in shapes)
    q = torch.empty(big, dtype=torch.float64 if q_dtype == fr.F64 else torch.float32, device=dev)
    cnt = torch.empty(big, dtype=torch.uint64, device=dev)
    code = torch.empty(big, dtype=torch.uint8, device=dev)
    ws = fr.Workspace()
    status = torch.zeros(1, dtype=torch.int32, device=dev)
    lib = fr.load_library()
    stream = fr._stream(dev)
    P = lambda t: ctypes.c_void_p(t.data_ptr())
    wsb_max = max(fr.workspace_bytes(fr.FN_ACCUMULATE, a, b_, fr.MFD if i % 2 else fr.D8, q_dtype)
                  for i, (a, b_) in enumerate(shapes))
    wbuf = ws.get(wsb_max, dev)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i, (nr, nc) in enumerate(shapes):
        rule = fr.D8 if i % 2 == 0 else fr.MFD
        z = tiles[i]["z"]
        if lib.fr_receivers(P(z), nr, nc, rule, P(code), P(status), stream) != 0:
            raise RuntimeError("fr_receivers")
        rc = lib.fr_accumulate(P(z), P(code), nr, nc, rule, 1.1, None, fr.F32, q_dtype, P(q),
                               P(cnt) if rule == fr.D8 else None, None, P(status), P(wbuf), wsb_max, stream)
        if rc != 0:
            raise fr.FlowRouteError(rc, "per-tile fr_accumulate")
    torch.cuda.synchronize()
    t_tile = time.perf_counter() - t0
    fr._raise_status(status, "per-tile route")
    log(f"  per-tile {'float64' if q_dtype == fr.F64 else 'float32'}: {1e3 * t_tile:.2f} ms for the batch")
    return t_tile


def cpu_baseline_tiles(shapes, budget_s: float = 15.0):
    """The oracle, single-threaded, on the batch's tiles in order (same
    seeds and rules) until about budget_s of CPU work."""
    import oracle
    import synth
    cells, spent, k = 0, 0.0, 0
    for i, (nr, nc) in enumerate(shapes):
        z = synth.dem(1000 + i, nr, nc)
        t0 = time.perf_counter()
        order = oracle.order(z)
        if i % 2 == 0:
            code = oracle.receivers(z)
            oracle.accumulate_single(code, None, order, q=False, counts=True)
        else:
            oracle.accumulate_mfd(z, None, 1.1, order)
        spent += time.perf_counter() - t0
        cells += nr * nc
        k += 1
        if spent >= budget_s:
            break
    return {"value": cells / spent, "unit": "cells/s", "cores": 1, "kind": "oracle",
            "sample": (f"the first {k} of the batch's tiles ({cells / 1e6:.1f} Mcells; even D8 counts, odd "
                       f"MFD float64): high-to-low sort + push, {spent:.1f}s; host nproc={os.cpu_count()}")}


def run_blockiter(args):
    """The paper's parallel scheme on the GPU: D8 unit-rain counts on the
    43360^2 DEM (seed 2) by block iterations (I+X and (I-X)(I+X), blocks of
    --block cells, each solved exactly), timed beside the direct path on the
    same codes."""
    import numpy as np
    import torch
    import synth
    import paper_2606_12800_amd as fr
    lib = fr.load_library()
    dev = torch.device("cuda:0")
    nr = args.rows or args.size
    nc = args.cols or args.size
    log(f"generating {nr}x{nc} DEM (seed {args.seed}) ...")
    z = torch.from_numpy(synth.dem(args.seed, nr, nc)).to(dev)
    code = torch.empty((nr, nc), dtype=torch.uint8, device=dev)
    cnt = torch.empty((nr, nc), dtype=torch.uint64, device=dev)
    cnt2 = torch.empty((nr, nc), dtype=torch.uint64, device=dev)
    status = torch.zeros(1, dtype=torch.int32, device=dev)
    P = lambda t: ctypes.c_void_p(t.data_ptr())
    sp = ctypes.c_void_p(torch.cuda.current_stream(dev).cuda_stream)
    if lib.fr_receivers(P(z), nr, nc, fr.D8, P(code), P(status), sp) != 0:
        raise RuntimeError("fr_receivers")
    del z
    wsb = max(fr.workspace_bytes(fr.FN_ACCUMULATE, nr, nc, fr.D8, fr.NONE),
              fr.workspace_bytes(fr.FN_BLOCK_ITER, nr, nc, fr.D8, fr.NONE),
              fr.workspace_bytes(fr.FN_BLOCK_ITER_PRE, nr, nc, fr.D8, fr.NONE))
    ws = torch.empty(wsb, dtype=torch.uint8, device=dev)
    iters = ctypes.c_int32(0)
    iters_pre = ctypes.c_int32(0)

    def forest():
        return lib.fr_accumulate(None, P(code), nr, nc, fr.D8, 1.1, None, fr.F32, fr.NONE, None, P(cnt2), None,
                                 P(status), P(ws), wsb, sp)

    br, bc = args.block

    def blocks():
        return lib.fr_accumulate_block_iterations(None, P(code), nr, nc, fr.D8, 0.0, br, bc, fr.SCHEME_IX, None,
                                                  fr.F32, fr.NONE, None, P(cnt), 100000, ctypes.byref(iters),
                                                  P(status), P(ws), wsb, sp)

    def blocks_pre():
        return lib.fr_accumulate_block_iterations(None, P(code), nr, nc, fr.D8, 0.0, br, bc, fr.SCHEME_IMX_IX,
                                                  None, fr.F32, fr.NONE, None, P(cnt2), 100000,
                                                  ctypes.byref(iters_pre), P(status), P(ws), wsb, sp)

    times = {}
    same_pre = None
    for name, fn in (("forest", forest), ("block_iterations", blocks), ("block_iterations_imx_ix", blocks_pre)):
        if name == "block_iterations_imx_ix":
            same = bool(torch.equal(cnt, cnt2))
        for _ in range(args.warmup):
            if fn() != 0:
                raise RuntimeError(name)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            if fn() != 0:
                raise RuntimeError(name)
        torch.cuda.synchronize()
        times[name] = (time.perf_counter() - t0) / args.steps
        log(f"  {name}: {1e3 * times[name]:.2f} ms")
    fr._raise_status(status, "block iterations")
    same_pre = bool(torch.equal(cnt, cnt2))
    ncell = nr * nc
    t_it = times["block_iterations"]
    per_iter_ms = 1e3 * t_it / max(iters.value + 1, 1)
    # Per iteration: codes read, counts written, previous counts read.
    achieved = (1 + 8 + 8) * ncell / (per_iter_ms * 1e-3) / 1e9
    line = {
        "metric": "cells routed/sec (D8 & MFD) at 1 MI355X; % HBM peak; batched vs per-tile",
        "value": ncell / t_it, "unit": "cells/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": 1e3 * t_it, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "u64", "data": "synthetic",
        "config": {"workload": f"D8 {nr}x{nc} fractal DEM (seed {args.seed}), unit-rain counts by the paper's "
                               f"block iterations (I+X), blocks of {br}x{bc} cells solved exactly",
                   "cells": ncell},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                     "kernel": "one block solve (k_d8_a, forest, k_d8_c)",
                     "bytes_per_cell": 17, "ms_per_launch": per_iter_ms},
        "detail": {"iterations_until_exact": iters.value, "launches": iters.value + 1,
                   "forest_path_ms": 1e3 * times["forest"], "same_counts_as_forest_path": same,
                   "block_iterations_over_forest": t_it / times["forest"],
                   "imx_ix_iterations_until_exact": iters_pre.value,
                   "imx_ix_ms": 1e3 * times["block_iterations_imx_ix"],
                   "imx_ix_same_counts": same_pre},
    }
    print(json.dumps(line), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", default="d8", choices=["d8", "mfd", "adjoint", "batched", "blockiter", "fill"],
                    help="d8: the headline 1.88e9-cell route (default); the others: one line for that workload")
    ap.add_argument("--tiles", type=int, default=512, help="batched workload: number of tiles")
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--size", type=int, default=43360, help="grid side (default: 1.88e9-cell DEM)")
    ap.add_argument("--rows", type=int, default=0, help="D8: grid rows (with --cols; default: --size)")
    ap.add_argument("--cols", type=int, default=0, help="D8: grid columns (e.g. the paper's 57345 x 32769)")
    ap.add_argument("--seed", type=int, default=2)
    ap.add_argument("--cpu-size", type=int, default=8192)
    ap.add_argument("--block", type=int, nargs=2, default=[4096, 4096],
                    help="blockiter: block rows and columns (multiples of 16 and 256)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-per-tile", action="store_true", help="batched: skip the per-tile comparisons")
    ap.add_argument("--filled", action="store_true",
                    help="d8: route the untilted DEM after depression filling (the paper's workflow)")
    ap.add_argument("--headline-only", action="store_true",
                    help="d8: time only the headline route (not the MFD and batched workloads in detail)")
    ap.add_argument("--copy-probe", action="store_true",
                    help="after timing, run one 1 GiB device copy (reference for HBM byte counters)")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py: the library routes on one GPU; multi-GPU runs are not supported "
              f"(asked for --gpus {args.gpus}, WORLD_SIZE {world})", flush=True)
        sys.exit(2)
    args.size_given = "--size" in sys.argv
    if args.workload == "batched":
        print(json.dumps(run_batched(args)), flush=True)
        return
    if args.workload == "blockiter":
        run_blockiter(args)
        return
    if args.workload == "fill":
        run_fill(args)
        return
    if args.workload != "d8":
        print(json.dumps(run_secondary(args, args.workload)), flush=True)
        return
    out = run_d8(args)
    if not args.headline_only and not args.rows and not args.cols and not args.size_given and not args.filled:
        # The other configurations of the metric, timed in the same run:
        # MFD 16384^2 (float32 and float64), the 512-tile batch (HIP graph
        # replay against per-tile float32 and float64 launches) and the
        # paper's workflow -- the untilted 43360^2 DEM depression-filled
        # (not timed), then routed D8.  Each keeps its own roofline; none has
        # a CPU baseline here (bench.py --workload mfd / batched time the
        # oracle beside them).
        import torch
        torch.cuda.empty_cache()
        sub = argparse.Namespace(**vars(args))
        sub.no_cpu_baseline = True
        sub.steps, sub.warmup = 3, 1
        sub.size_given = False
        filled = argparse.Namespace(**vars(sub))
        filled.filled = True
        filled.headline_only = True
        for name, fn in (("mfd_16384", lambda: run_secondary(sub, "mfd")), ("batched_512", lambda: run_batched(sub)),
                         ("d8_filled_43360", lambda: run_d8(filled))):
            log(f"{name} ...")
            line = fn()
            out["detail"][name] = {k: line[k] for k in ("value", "unit", "ms_per_step", "dtype", "config",
                                                        "roofline", "detail") if k in line}
            torch.cuda.empty_cache()
    print(json.dumps(out), flush=True)


def run_d8(args):
    """The headline route: D8 receivers + accumulation (float32 rain with
    float-float sums, uint64 counts, float64 mass balance) of the 43360^2
    DEM (seed 2), inputs resident in HBM."""
    import numpy as np
    import torch
    import synth
    import paper_2606_12800_amd as fr

    lib = fr.load_library()
    dev = torch.device("cuda:0")
    nr = args.rows or args.size
    nc = args.cols or args.size
    ncell = nr * nc

    log(f"generating {nr}x{nc} DEM (seed {args.seed}) ...")
    t0 = time.perf_counter()
    z_h = synth.dem(args.seed, nr, nc, tilt=0.0 if args.filled else synth.TILT)
    rain_h = synth.rain(args.seed, nr, nc)
    log(f"  generated in {time.perf_counter() - t0:.1f}s; copying to HBM")
    z = torch.from_numpy(z_h).to(dev)
    del z_h
    if args.filled:
        # The paper's workflow (Section 4): the untilted DEM filled first
        # (not timed), then routed.
        z = fr.fill_depressions(z, "d8", eps=True)
        fr._default_ws.buf = None
        torch.cuda.synchronize()
    rain = torch.from_numpy(rain_h).to(dev)
    del rain_h
    code = torch.empty((nr, nc), dtype=torch.uint8, device=dev)
    q = torch.empty((nr, nc), dtype=torch.float32, device=dev)
    cnt = torch.empty((nr, nc), dtype=torch.uint64, device=dev)
    mass = torch.empty(2, dtype=torch.float64, device=dev)
    status = torch.zeros(1, dtype=torch.int32, device=dev)
    wsb = fr.workspace_bytes(fr.FN_ACCUMULATE, nr, nc, fr.D8, fr.F32)
    ws = torch.empty(wsb, dtype=torch.uint8, device=dev)
    stream = torch.cuda.current_stream(dev)
    sp = ctypes.c_void_p(stream.cuda_stream)
    P = lambda t: ctypes.c_void_p(t.data_ptr())
    log(f"  resident: {torch.cuda.memory_allocated(dev) / 1e9:.1f} GB allocated")

    ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
    recv_ms, acc_ms = [], []
    phase_ms = {}
    fr.timing_enable(True)

    def step(record: bool):
        ev[0].record(stream)
        rc = lib.fr_receivers(P(z), nr, nc, fr.D8, P(code), P(status), sp)
        ev[1].record(stream)
        if rc != 0:
            raise fr.FlowRouteError(rc, "fr_receivers")
        ph = fr.timing_last() if record else {}
        rc = lib.fr_accumulate(None, P(code), nr, nc, fr.D8, 1.1, P(rain), fr.F32, fr.F32, P(q), P(cnt),
                               P(mass), P(status), P(ws), wsb, sp)
        ev[2].record(stream)
        if rc != 0:
            raise fr.FlowRouteError(rc, "fr_accumulate")
        if record:
            ph.update(fr.timing_last())
            for k, v in ph.items():
                phase_ms.setdefault(k, []).append(v)
            ev[2].synchronize()
            recv_ms.append(ev[0].elapsed_time(ev[1]))
            acc_ms.append(ev[1].elapsed_time(ev[2]))

    for i in range(args.warmup):
        step(False)
        log(f"  warmup {i} done")
    torch.cuda.synchronize()
    st = int(status.item())
    if st != 0:
        raise fr.FlowRouteError(st, "device status")

    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        step(True)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    log(f"  timed {args.steps} steps in {wall:.3f}s")
    fr.timing_enable(False)

    if args.copy_probe:
        copy_probe(dev)

    m = mass.cpu().numpy()
    total_cells_counts = int(cnt.view(torch.int64)[code == 0xFF].sum().item())
    ms_step = 1e3 * wall / args.steps
    value = ncell * args.steps / wall
    recv_avg = sum(recv_ms) / len(recv_ms)
    acc_avg = sum(acc_ms) / len(acc_ms)
    acc_gbs = ACC_BYTES * ncell / (acc_avg * 1e-3) / 1e9
    route_gbs = ROUTE_BYTES * ncell / ((recv_avg + acc_avg) * 1e-3) / 1e9
    phase_avg = {k: sum(v) / len(v) for k, v in phase_ms.items()}
    # Dominant phase: the one with the largest device time.
    single = {k: v for k, v in phase_avg.items() if k in PHASE_BYTES}
    dom = max(single, key=single.get)
    achieved = PHASE_BYTES[dom] * ncell / (single[dom] * 1e-3) / 1e9
    phase_gbs = {k: PHASE_BYTES[k] * ncell / (single[k] * 1e-3) / 1e9 for k in single}
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "cells/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": (f"D8 {nr}x{nc} fractal DEM (seed {args.seed}"
                                + (", untilted, depression-filled" if args.filled else "") + "), f32 rain + u64 counts"),
                   "cells": ncell},
        "roofline": roofline(achieved, PHASE_KERNEL[dom], ("d8_filled" if args.filled else "d8", nr, nc), dom,
                             bytes_per_cell=PHASE_BYTES[dom],
                             ms_per_launch=single[dom]),
        "detail": {"receivers_ms": recv_avg, "accumulate_ms": acc_avg,
                   "accumulate_alg_GBs": acc_gbs,
                   # The whole route (receivers + accumulate, 22 algorithmic
                   # bytes per cell) against the HBM peak.
                   "route_roofline": {"bytes_per_cell": ROUTE_BYTES, "achieved": route_gbs, "unit": "GB/s",
                                      "frac": route_gbs / HBM_PEAK_GBS, "ms": recv_avg + acc_avg},
                   "phase_ms": phase_avg, "phase_alg_GBs": phase_gbs,
                   "phase_frac": {k: v / HBM_PEAK_GBS for k, v in phase_gbs.items()},
                   "mass_sinks": float(m[0]), "mass_rain": float(m[1]),
                   "mass_rel_err": abs(float(m[0]) - float(m[1])) / float(m[1]),
                   "sink_counts_total": total_cells_counts,
                   "cells_leaving_row_sweep": int((code > 2).sum().item()) / ncell},
    }
    del z, rain, code, q, cnt, ws
    torch.cuda.empty_cache()
    if not args.no_cpu_baseline:
        log(f"cpu baseline: oracle on {args.cpu_size}^2 ...")
        out["cpu_baseline"] = cpu_baseline(args.cpu_size, args.seed)
    return out


if __name__ == "__main__":
    main()
