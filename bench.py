#!/usr/bin/env python3
"""Benchmark of the MI355X 2D FFT: forward + inverse round trip of a
4096 x 4096 complex64 grid (128 MiB), inputs resident in HBM.

One step = forward 2D FFT (row pass + column pass) then inverse 2D FFT (row
pass + column pass), out of place: x -> y -> z. Prints ONE JSON line:
GFLOP/s under the 5 N log2 N convention (two transforms per step), the
effective HBM bandwidth, the roofline of the dominant kernel (algorithmic
bytes per launch over its mean duration, timed with HIP events bound to the
kernel's launch on the stream it runs on), the FP64 oracle timed on the host cores as CPU baseline,
and the backward (adjoint) and batched forms against the plain path.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W]
"""

from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "2D FFT GFLOP/s (5NlogN) + HBM GB/s at 4096²; batched & backward vs plain"
HBM_PEAK_GBS = 8000.0
BYTES_PER_POINT_PER_PASS = 16  # each pass reads and writes every complex64 point once


TRAFFIC_PROFILE = os.path.join(ROOT, "profiles", "hbm_traffic_fft2d_4096x4096_roundtrip.txt")
PASS_NAMES = ["fwd_row", "fwd_col", "inv_row", "inv_col"]


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_source_hash():
    """SHA-256 over the sources of the plain path's kernels and plan logic
    (csrc/, batched sources excluded): counters taken from an older build do not
    describe the current one."""
    import hashlib
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2506_15437_amd", "csrc")
    files = sorted(f for f in os.listdir(csrc)
                   if f.endswith((".hip", ".hpp", ".h", ".cpp")) and not f.startswith("fft_batched"))
    for f in files:
        with open(os.path.join(csrc, f), "rb") as fh:
            h.update(f.encode() + b"\0" + fh.read())
    return h.hexdigest()[:16]


def _counter_rows(run_dir):
    import csv
    path = os.path.join(run_dir, "run_counter_collection.csv")
    with open(path, newline="") as fh:
        return list(csv.DictReader(fh))


def summarize_traffic(fetch_dir, write_dir, copy_fetch_dir, copy_write_dir):
    """HBM bytes per launch of each pass from rocprofv3 FETCH_SIZE / WRITE_SIZE
    runs (KiB per dispatch), each scaled by the factor that makes the same
    counter read the known size of a plain device copy (bench.py --copy-only)."""
    copy_bytes = 4096 * 4096 * 8  # bytes read, and bytes written, by one copy of the grid
    factors = {}
    for name, d in (("FETCH_SIZE", copy_fetch_dir), ("WRITE_SIZE", copy_write_dir)):
        vals = [float(r["Counter_Value"]) for r in _counter_rows(d)
                if "copyBuffer" in r["Kernel_Name"] and r["Counter_Name"] == name]
        kib = float(np.median(vals))
        factors[name] = (copy_bytes / 1024.0) / kib
    per_pass = {}
    for name, d in (("FETCH_SIZE", fetch_dir), ("WRITE_SIZE", write_dir)):
        rows = [r for r in _counter_rows(d) if "fft2d::dev::" in r["Kernel_Name"] and r["Counter_Name"] == name]
        rows.sort(key=lambda r: int(r["Dispatch_Id"]))
        for i, r in enumerate(rows):
            p = PASS_NAMES[i % 4]
            per_pass.setdefault(p, {}).setdefault(name, []).append(float(r["Counter_Value"]))
            per_pass[p]["kernel"] = r["Kernel_Name"]
    lines = ["source_hash = %s" % kernel_source_hash(),
             "fetch_factor = %.4f" % factors["FETCH_SIZE"],
             "write_factor = %.4f" % factors["WRITE_SIZE"],
             "algorithmic_bytes_per_pass = %d" % (BYTES_PER_POINT_PER_PASS * 4096 * 4096)]
    for p in PASS_NAMES:
        e = per_pass[p]
        fk = float(np.mean(e["FETCH_SIZE"]))
        wk = float(np.mean(e["WRITE_SIZE"]))
        rd = fk * 1024 * factors["FETCH_SIZE"]
        wr = wk * 1024 * factors["WRITE_SIZE"]
        lines.append("pass %s bytes %d read %d write %d fetch_kib %.1f write_kib %.1f dispatches %d kernel %s"
                     % (p, rd + wr, rd, wr, fk, wk, len(e["FETCH_SIZE"]), e["kernel"]))
    return "\n".join(lines)


def summarize_counters(*run_dirs):
    """Mean per launch of every counter of rocprofv3 --pmc runs (one folder per
    run), for each pass of the round trip, and the count per wave where the
    counter counts instructions (wave count SQ_WAVES from the same runs)."""
    per_pass = {}
    for d in run_dirs:
        rows = [r for r in _counter_rows(d) if "fft2d::dev::" in r["Kernel_Name"]]
        for name in sorted({r["Counter_Name"] for r in rows}):
            sel = sorted((r for r in rows if r["Counter_Name"] == name), key=lambda r: int(r["Dispatch_Id"]))
            for i, r in enumerate(sel):
                e = per_pass.setdefault(PASS_NAMES[i % 4], {"kernel": r["Kernel_Name"]})
                e.setdefault(name, []).append(float(r["Counter_Value"]))
    lines = []
    for p in PASS_NAMES:
        e = per_pass[p]
        waves = float(np.mean(e["SQ_WAVES"])) if "SQ_WAVES" in e else None
        lines.append("pass %s kernel %s" % (p, e["kernel"]))
        for name in sorted(k for k in e if k != "kernel"):
            v = float(np.mean(e[name]))
            extra = ("  per wave %.1f" % (v / waves)) if waves and name.startswith("SQ_INSTS_") else ""
            lines.append("  %-24s %16.1f  (%d launches)%s" % (name, v, len(e[name]), extra))
    return "\n".join(lines)


def summarize_stats(stats_dir):
    """The fft2d rows of a rocprofv3 --kernel-trace --stats run (kernel_stats.csv)."""
    import csv
    with open(os.path.join(stats_dir, "run_kernel_stats.csv"), newline="") as fh:
        rows = list(csv.DictReader(fh))
    out = ["calls  avg_us   min_us   max_us   total_%  kernel"]
    for r in rows:
        out.append("%5s %8.2f %8.2f %8.2f %8.2f  %s" % (r["Calls"], float(r["AverageNs"]) / 1e3,
                                                      float(r["MinNs"]) / 1e3, float(r["MaxNs"]) / 1e3,
                                                      float(r["Percentage"]), r["Name"]))
    return "\n".join(out)


def measured_traffic(pass_name):
    """HBM bytes per launch of `pass_name` from the committed counter summary,
    or None when it is missing or was taken from other kernel sources."""
    try:
        with open(TRAFFIC_PROFILE) as fh:
            text = fh.read()
    except OSError:
        return None
    vals = {}
    for line in text.splitlines():
        f = line.split()
        if len(f) >= 3 and f[1] == "=":
            vals[f[0]] = f[2]
        elif len(f) >= 4 and f[0] == "pass" and f[2] == "bytes":
            vals["pass " + f[1]] = f[3]
    if vals.get("source_hash") != kernel_source_hash() or ("pass " + pass_name) not in vals:
        return None
    return int(vals["pass " + pass_name])


def flops_2d(rows, cols, batch=1):
    p = rows * cols
    return 5.0 * p * math.log2(p) * batch if p > 1 else 0.0


def time_plain(F, torch, rows, cols, steps, warmup, seed):
    """Forward + inverse round trip. The step time comes from `steps` steps of
    two fft2d_exec calls with nothing else on the stream; the per-pass
    durations from a second run of `steps` steps launched pass by pass with
    fft2d_exec_pass_timed, whose start and stop events are bound to the pass's
    kernel (hipExtLaunchKernel): each pair spans that kernel alone, and no
    marker packet sits between the launches."""
    import synth
    x_h = synth.complex_grid(seed, (rows, cols))
    x = torch.from_numpy(x_h).to("cuda")
    y = torch.empty_like(x)
    z = torch.empty_like(x)
    plan = F.get_plan(1, rows, cols, x.device)
    stream = torch.cuda.current_stream()
    sh = int(stream.cuda_stream)
    xp, yp, zp = x.data_ptr(), y.data_ptr(), z.data_ptr()

    def step_plain():
        F.fft2d_exec(plan.handle, xp, yp, F.FORWARD, sh)
        F.fft2d_exec(plan.handle, yp, zp, F.INVERSE, sh)

    passes = ((xp, yp, F.FORWARD, 0), (xp, yp, F.FORWARD, 1), (yp, zp, F.INVERSE, 0), (yp, zp, F.INVERSE, 1))

    def step_timed(evs):
        for (src, dst, direction, index), (a, b) in zip(passes, evs):
            F.fft2d_exec_pass_timed(plan.handle, src, dst, direction, index, a.cuda_event, b.cuda_event, sh)

    for _ in range(warmup):
        step_plain()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        step_plain()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    # per-pass durations: the same steps, each pass kernel with its own pair of HIP events on the stream it
    # runs on (each event is recorded once first, which creates it and gives torch a handle to pass on)
    events = [[(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(4)]
              for _ in range(steps)]
    for evs in events:
        for a, b in evs:
            a.record(stream)
            b.record(stream)
    torch.cuda.synchronize()
    for i in range(steps):
        step_timed(events[i])
    torch.cuda.synchronize()
    per = np.array([[a.elapsed_time(b) for a, b in events[i]] for i in range(steps)])
    # correctness of what was timed: round trip error, computed on the GPU
    rt = float(torch.linalg.vector_norm(z - x) / torch.linalg.vector_norm(x))
    y_h = y.cpu().numpy()
    return dict(wall=wall, per_pass_ms=per, x=x_h, y=y_h, roundtrip_rel_l2=rt, plan=plan.describe())


CONFIGS = [  # (name, batch, rows, cols, seed)
    ("64x64 forward", 1, 64, 64, 0),
    ("8192 x 64x64 forward", 8192, 64, 64, 6),
    ("1024x1024 forward", 1, 1024, 1024, 0),
    ("4096x4096 forward", 1, 4096, 4096, 1),
    ("8192x8192 forward", 1, 8192, 8192, 2),
    ("16384x2048 forward", 1, 16384, 2048, 3),
    ("1D: 4096 rows of 16384 points forward", 4096, 1, 16384, 0),
]


def time_configs(F, torch, iters):
    """Forward transform of each configuration, warm (back to back), cold (a
    1 GiB scratch tensor is zeroed before each iteration, outside the timed
    events, so the 256 MB MALL holds none of the input, but holds dirty lines
    of the scratch that are written back while the transform runs) and
    cold_clean (the scratch is read instead: no input in the MALL and nothing
    to write back): median, mean, min."""
    import synth
    stream = torch.cuda.current_stream()
    sh = int(stream.cuda_stream)
    scratch = torch.empty(1 << 28, dtype=torch.float32, device="cuda")
    res = {}
    for name, batch, rows, cols, seed in CONFIGS:
        shape = (batch, rows, cols) if batch > 1 else (rows, cols)
        x = torch.from_numpy(synth.complex_grid(seed, shape)).to("cuda")
        y = torch.empty_like(x)
        plan = F.get_plan(batch, rows, cols, x.device)
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(iters)]
        out = {}
        # HBM passes: a length-1 dimension needs none; a whole-grid plan reads and writes once
        npass = 1 if " grid[" in plan.describe() else int(rows > 1) + int(cols > 1)
        for mode in ("warm", "cold", "cold_clean"):
            for _ in range(3):
                F.fft2d_exec(plan.handle, x.data_ptr(), y.data_ptr(), F.FORWARD, sh)
            for a, b in ev:
                if mode == "cold":
                    scratch.zero_()
                elif mode == "cold_clean":
                    scratch.sum()  # reads the 1 GiB; the result is not needed
                a.record(stream)
                F.fft2d_exec(plan.handle, x.data_ptr(), y.data_ptr(), F.FORWARD, sh)
                b.record(stream)
            torch.cuda.synchronize()
            t = np.array([a.elapsed_time(b) for a, b in ev])
            med = float(np.median(t))
            pts = batch * rows * cols
            out[mode] = {"median_ms": round(med, 5), "mean_ms": round(float(t.mean()), 5),
                         "min_ms": round(float(t.min()), 5),
                         "gflops": round(flops_2d(rows, cols, batch) / med / 1e6, 1),
                         "hbm_gbps": round(npass * BYTES_PER_POINT_PER_PASS * pts / med / 1e6, 1)}
        out["plan"] = plan.describe()
        res[name] = out
        del x, y
    del scratch
    torch.cuda.empty_cache()
    return res


def device_copy_gbps(torch, rows, cols, iters=20):
    """Read+write bandwidth of a plain device copy of one rows x cols complex64
    grid (torch's copy kernel), warm (source and destination stay in the 256 MB
    MALL) and cold (1 GiB scrubbed before each copy)."""
    x = torch.zeros((rows, cols), dtype=torch.complex64, device="cuda")
    y = torch.empty_like(x)
    scratch = torch.empty(1 << 28, dtype=torch.float32, device="cuda")
    stream = torch.cuda.current_stream()
    out = {}
    for mode in ("warm", "cold"):
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(iters)]
        for _ in range(3):
            y.copy_(x)
        for a, b in ev:
            if mode == "cold":
                scratch.zero_()
            a.record(stream)
            y.copy_(x)
            b.record(stream)
        torch.cuda.synchronize()
        med = float(np.median([a.elapsed_time(b) for a, b in ev]))
        out[mode + "_gbps"] = round(2 * x.numel() * 8 / med / 1e6, 1)
    del x, y, scratch
    torch.cuda.empty_cache()
    return out


def vendor_fft_context(F, torch, iters=20):
    """Context only: torch.fft.fft2 (the ROCm vendor FFT that torch calls) and
    fft2d_exec on the same inputs, forward, warm medians of `iters` transforms
    with HIP events around each, and the relative difference of the two
    results. Nothing of the library's path goes through torch.fft."""
    import synth
    stream = torch.cuda.current_stream()
    sh = int(stream.cuda_stream)
    res = {}
    for batch, rows, cols in ((1, 4096, 4096), (1, 8192, 8192), (1, 16384, 2048), (8, 2048, 2048)):
        shape = (batch, rows, cols) if batch > 1 else (rows, cols)
        x = torch.from_numpy(synth.complex_grid(1, shape)).to("cuda")
        y = torch.empty_like(x)
        plan = F.get_plan(batch, rows, cols, x.device)
        vendor_out = torch.fft.fft2(x)
        med = {}
        for name, fn in (("vendor", lambda: torch.fft.fft2(x)),
                         ("library", lambda: F.fft2d_exec(plan.handle, x.data_ptr(), y.data_ptr(), F.FORWARD, sh))):
            for _ in range(3):
                fn()
            ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(iters)]
            for a, b in ev:
                a.record(stream)
                fn()
                b.record(stream)
            torch.cuda.synchronize()
            med[name] = float(np.median([a.elapsed_time(b) for a, b in ev]))
        diff = float(torch.linalg.vector_norm(y - vendor_out) / torch.linalg.vector_norm(vendor_out))
        name = ("%d x %dx%d forward" % (batch, rows, cols)) if batch > 1 else ("%dx%d forward" % (rows, cols))
        res[name] = {"torch_fft2_ms": round(med["vendor"], 5), "fft2d_exec_ms": round(med["library"], 5),
                     "speedup": round(med["vendor"] / med["library"], 2), "rel_l2_difference": diff}
        del x, y, vendor_out
    torch.cuda.empty_cache()
    return res


def energy(F, torch, rows, cols, seconds):
    """Energy of forward rows x cols transforms from the GPU's energy counter
    (amdsmi, whole board), over a loop of about `seconds`. None when the
    counter cannot be read."""
    try:
        import amdsmi
        amdsmi.amdsmi_init()
        h = amdsmi.amdsmi_get_processor_handles()[0]
    except Exception as e:  # no counter on this machine: report nothing
        log("bench: energy counter unavailable (%s)" % e)
        return None

    def joules():
        c = amdsmi.amdsmi_get_energy_count(h)
        return c["energy_accumulator"] * c["counter_resolution"] * 1e-6

    try:
        import synth
        x = torch.from_numpy(synth.complex_grid(0, (rows, cols))).to("cuda")
        y = torch.empty_like(x)
        plan = F.get_plan(1, rows, cols, x.device)
        sh = int(torch.cuda.current_stream().cuda_stream)

        def run(n):
            for _ in range(n):
                F.fft2d_exec(plan.handle, x.data_ptr(), y.data_ptr(), F.FORWARD, sh)

        run(20)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        run(200)
        torch.cuda.synchronize()
        per = (time.perf_counter() - t0) / 200
        n = max(200, int(seconds / per))
        e0, t0 = joules(), time.perf_counter()
        run(n)
        torch.cuda.synchronize()
        e1, t1 = joules(), time.perf_counter()
        busy_w = (e1 - e0) / (t1 - t0)
        return {"workload": "%dx%d forward, %d back-to-back transforms" % (rows, cols, n),
                "seconds": round(t1 - t0, 3), "ms_per_transform": round((t1 - t0) / n * 1e3, 5),
                "avg_power_w": round(busy_w, 1),
                "energy_per_transform_j": (e1 - e0) / n,
                "source": "amdsmi energy counter (whole GPU)"}
    except Exception as e:
        log("bench: energy measurement failed (%s)" % e)
        return None
    finally:
        try:
            amdsmi.amdsmi_shut_down()
        except Exception:
            pass


def time_backward(F, torch, batch, rows, cols, steps, warmup, seed):
    """fft2d_backward (adjoint kernels) against fft2d_exec on the same plan and data."""
    import synth
    x = torch.from_numpy(synth.complex_grid(seed, (batch, rows, cols))).to("cuda")
    out = torch.empty_like(x)
    plan = F.get_plan(batch, rows, cols, x.device)
    stream = torch.cuda.current_stream()
    sh = int(stream.cuda_stream)

    def run(fn):
        for _ in range(warmup):
            fn()
        torch.cuda.synchronize()
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record(stream)
        for _ in range(steps):
            fn()
        b.record(stream)
        torch.cuda.synchronize()
        return a.elapsed_time(b) / steps

    fwd = run(lambda: F.fft2d_exec(plan.handle, x.data_ptr(), out.data_ptr(), F.FORWARD, sh))
    bwd = run(lambda: F.fft2d_backward(plan.handle, x.data_ptr(), out.data_ptr(), F.FORWARD, sh))
    fl = flops_2d(rows, cols, batch)
    return {"workload": "batch %d of %dx%d complex64" % (batch, rows, cols), "plain_ms": fwd, "backward_ms": bwd,
            "backward_over_plain": bwd / fwd, "plain_gflops": fl / fwd / 1e6, "backward_gflops": fl / bwd / 1e6}


def time_batched(F, torch, steps, warmup, seed):
    """512 transforms of 2^a x 2^b (a, b in [6, 11] from `seed`): one graph replay of the
    persistent kernel against 512 fft2d_exec calls (two kernel launches each) on one stream."""
    import synth
    shapes = synth.pow2_shapes(seed, 512)
    xs = [torch.from_numpy(x).to("cuda") for x in synth.batched_grids(seed, shapes)]
    ys = [torch.empty_like(x) for x in xs]
    zs = [torch.empty_like(x) for x in xs]
    plan = F.BatchedPlan(shapes)
    stream = torch.cuda.current_stream()
    sh = int(stream.cuda_stream)
    iptr = [x.data_ptr() for x in xs]
    iarr = F.pointer_array(iptr)  # built once: a replay converts nothing
    oarr = F.pointer_array([y.data_ptr() for y in ys])
    plans = [F.get_plan(1, r, c, xs[0].device) for r, c in shapes]
    zptr = [z.data_ptr() for z in zs]

    def batched():
        plan.exec_ptrs(iarr, oarr, F.FORWARD, sh)

    def plain():
        for p, a, b in zip(plans, iptr, zptr):
            F.fft2d_exec(p.handle, a, b, F.FORWARD, sh)

    def run(fn):
        for _ in range(warmup):
            fn()
        torch.cuda.synchronize()
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record(stream)
        for _ in range(steps):
            fn()
        b.record(stream)
        torch.cuda.synchronize()
        return a.elapsed_time(b) / steps

    t_b = run(batched)
    t_p = run(plain)
    num = sum(float(torch.linalg.vector_norm(y - z)) ** 2 for y, z in zip(ys, zs)) ** 0.5
    den = sum(float(torch.linalg.vector_norm(z)) ** 2 for z in zs) ** 0.5
    points = sum(r * c for r, c in shapes)
    fl = sum(flops_2d(r, c) for r, c in shapes)
    res = {"workload": "512 forward 2D FFTs of 2^a x 2^b, a, b in [6, 11] from seed %d, %d points" % (seed, points),
           "batched_ms": t_b, "plain_512_launches_ms": t_p, "speedup": t_p / t_b,
           "batched_gflops": fl / t_b / 1e6, "plain_gflops": fl / t_p / 1e6,
           "batched_hbm_gbps": 32.0 * points / t_b / 1e6,
           "batched_vs_plain_rel_l2": num / den, "plan": plan.describe()}
    plan.close()
    return res


def cpu_baseline(rows, cols, x, budget_s, max_reps, threads=0):
    """The FP64 oracle (plain recursive radix-2, OpenMP) on the same input;
    threads = 0 uses every host core."""
    import oracle
    used = threads if threads > 0 else oracle.max_threads()
    reps = 0
    t0 = time.perf_counter()
    ref = None
    while reps < max_reps:
        ref = oracle.fft2_forward(x, threads)
        oracle.ifft2(ref, threads)
        reps += 1
        if time.perf_counter() - t0 >= budget_s:
            break
    dt = time.perf_counter() - t0
    gflops = 2 * flops_2d(rows, cols) * reps / dt / 1e9
    return ref, {"value": gflops, "unit": "GFLOP/s", "cores": used, "kind": "oracle",
                 "sample": "%d forward+inverse round trips of the %dx%d grid, FP64 recursive radix-2 with OpenMP "
                           "over rows then columns, %.1f s" % (reps, rows, cols, dt)}


ORACLE_CASES = [  # (name, shape, seed): the configurations the FP64 oracle also runs, with their bench inputs
    ("64x64 forward", (64, 64), 0),
    ("8192 x 64x64 forward", (8192, 64, 64), 6),
    ("1024x1024 forward", (1024, 1024), 0),
    ("8192x8192 forward", (8192, 8192), 2),
    ("16384x2048 forward", (16384, 2048), 3),
    ("1D: 4096 rows of 16384 points forward", (4096, 1, 16384), 0),
    ("8 x 2048x2048 forward", (8, 2048, 2048), 5),
]
BATCHED_SEED = 4
BATCHED_COUNT = 512


def gpu_forward_outputs(F, torch):
    """The library's forward transform of every ORACLE_CASES input and of the
    512-shape batched set (one batched launch), copied to the host."""
    import synth
    out = {}
    for name, shape, seed in ORACLE_CASES:
        x = torch.from_numpy(synth.complex_grid(seed, shape)).to("cuda")
        out[name] = F.fft2(x).cpu().numpy()
        del x
    xs = [torch.from_numpy(g).to("cuda")
          for g in synth.batched_grids(BATCHED_SEED, synth.pow2_shapes(BATCHED_SEED, BATCHED_COUNT))]
    out["batched"] = [y.cpu().numpy() for y in F.fft2_batched(xs)]
    del xs
    torch.cuda.empty_cache()
    return out


def rel_l2(got, ref):
    return float(np.linalg.norm((got.astype(np.complex128) - ref).ravel()) / np.linalg.norm(ref.ravel()))


def cpu_configs(gpu_out, threads=0):
    """The FP64 oracle's forward transform of each configuration once (all host
    cores), for GPU/CPU context beside the 4096^2 baseline, and the relative L2
    error of the library's result for the same input against it."""
    import oracle
    import synth
    out = {}
    for name, shape, seed in ORACLE_CASES:
        x = synth.complex_grid(seed, shape)
        t0 = time.perf_counter()
        ref = oracle.fft2_forward(x, threads)
        dt = time.perf_counter() - t0
        batch = int(np.prod(shape[:-2])) if len(shape) > 2 else 1
        out[name] = {"seconds": round(dt, 4), "gflops": round(flops_2d(shape[-2], shape[-1], batch) / dt / 1e9, 2),
                     "gpu_rel_l2": rel_l2(gpu_out[name], ref)}
        del x, ref
    shapes = synth.pow2_shapes(BATCHED_SEED, BATCHED_COUNT)
    xs = synth.batched_grids(BATCHED_SEED, shapes)
    t0 = time.perf_counter()
    refs = [oracle.fft2_forward(x, threads) for x in xs]
    dt = time.perf_counter() - t0
    errs = [rel_l2(g, r) for g, r in zip(gpu_out["batched"], refs)]
    out["%d shapes 2^a x 2^b forward" % BATCHED_COUNT] = {"seconds": round(dt, 4),
                                           "gflops": round(sum(flops_2d(r, c) for r, c in shapes) / dt / 1e9, 2),
                                           "gpu_rel_l2_max": max(errs)}
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--seed", type=int, default=1)
    ap.add_argument("--cpu-budget", type=float, default=12.0, help="seconds of oracle work for the CPU baseline")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU baseline (profiling runs)")
    ap.add_argument("--no-extras", action="store_true", help="skip the backward and batched comparisons")
    ap.add_argument("--copy-only", action="store_true",
                    help="only run plain device copies of the 4096x4096 grid (calibrates rocprofv3 byte counters)")
    ap.add_argument("--summarize-traffic", nargs=4, metavar=("FETCH", "WRITE", "COPY_FETCH", "COPY_WRITE"),
                    help="print HBM bytes per pass from four rocprofv3 --pmc output folders, then exit")
    ap.add_argument("--summarize-counters", nargs="+", metavar="DIR",
                    help="print the mean of every counter per pass from rocprofv3 --pmc output folders, then exit")
    ap.add_argument("--summarize-stats", metavar="DIR",
                    help="print the kernel rows of a rocprofv3 --kernel-trace --stats output folder, then exit")
    args = ap.parse_args()
    if args.summarize_traffic:
        print(summarize_traffic(*args.summarize_traffic))
        return
    if args.summarize_counters:
        print(summarize_counters(*args.summarize_counters))
        return
    if args.summarize_stats:
        print(summarize_stats(args.summarize_stats))
        return

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py runs on one GPU only: this library has no multi-GPU path (a 2D FFT would need an "
              "all-to-all transpose across GPUs, which is not built); use --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch
    if not torch.cuda.is_available():
        print("no GPU visible", file=sys.stderr)
        sys.exit(1)
    import paper_2506_15437_amd as F

    rows = cols = 4096
    if args.copy_only:
        x = torch.empty((rows, cols), dtype=torch.complex64, device="cuda")
        y = torch.empty_like(x)
        x.zero_()
        for _ in range(args.warmup + args.steps):
            y.copy_(x)
        torch.cuda.synchronize()
        print(json.dumps({"copy_only": True, "bytes_per_copy": 2 * x.numel() * 8, "copies": args.warmup + args.steps}))
        return
    log("bench: %dx%d forward+inverse, steps=%d warmup=%d" % (rows, cols, args.steps, args.warmup))
    r = time_plain(F, torch, rows, cols, args.steps, args.warmup, args.seed)
    ms_per_step = r["wall"] / args.steps * 1e3
    step_flops = 2 * flops_2d(rows, cols)
    value = step_flops / (ms_per_step * 1e-3) / 1e9
    pass_names = PASS_NAMES
    mean_pass = r["per_pass_ms"].mean(axis=0)
    pass_bytes = BYTES_PER_POINT_PER_PASS * rows * cols
    dom = int(np.argmax(mean_pass))
    achieved = pass_bytes / (mean_pass[dom] * 1e-3) / 1e9
    step_bytes = 4 * pass_bytes
    log("bench: per-pass mean ms", dict(zip(pass_names, [round(float(v), 4) for v in mean_pass])))

    result = {
        "metric": METRIC,
        "value": round(value, 2),
        "unit": "GFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "fft2d forward+inverse round trip, 4096x4096 complex64 (128 MiB), out of place, "
                               "re/im uniform[-1,1) seed %d" % args.seed,
                   "rows": rows, "cols": cols, "batch": 1},
        "hbm_gbps_effective": round(step_bytes / (ms_per_step * 1e-3) / 1e9, 1),
        "roofline": {"bound": "hbm", "kernel": pass_names[dom] + " pass", "achieved": round(achieved, 1),
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": measured_traffic(pass_names[dom])},
        "per_pass_ms": {n: round(float(v), 5) for n, v in zip(pass_names, mean_pass)},
        "per_pass_gbps": {n: round(pass_bytes / (float(v) * 1e-3) / 1e9, 1) for n, v in zip(pass_names, mean_pass)},
        "roundtrip_rel_l2": r["roundtrip_rel_l2"],
        "plan": r["plan"],
    }

    if not args.no_extras:
        log("bench: backward vs plain, 8 x 2048 x 2048")
        result["backward_vs_plain"] = time_backward(F, torch, 8, 2048, 2048, 20, 3, 5)
        log("bench: forward transforms of every configuration, warm and cold")
        result["configs"] = time_configs(F, torch, 20)
        # One 4096^2 forward transform against the HBM roofline: two passes that
        # each read and write every point once (32 algorithmic bytes per point).
        one = result["configs"]["4096x4096 forward"]
        alg = 2 * BYTES_PER_POINT_PER_PASS * 4096 * 4096
        result["forward_4096_roofline"] = {
            "algorithmic_bytes": alg, "peak_gbps": HBM_PEAK_GBS,
            "cold_ms": one["cold"]["median_ms"], "warm_ms": one["warm"]["median_ms"],
            "frac_cold": round(alg / (one["cold"]["median_ms"] * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
            "cold_clean_ms": one["cold_clean"]["median_ms"],
            "frac_cold_clean": round(alg / (one["cold_clean"]["median_ms"] * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
            "frac_warm": round(alg / (one["warm"]["median_ms"] * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}
        log("bench: device copy bandwidth, 4096 x 4096 complex64")
        result["device_copy"] = device_copy_gbps(torch, rows, cols)
        log("bench: energy per transform (1024 x 1024 and 4096 x 4096)")
        result["energy"] = [energy(F, torch, 1024, 1024, 1.5), energy(F, torch, 4096, 4096, 1.5)]
        log("bench: batched 512 shapes vs 512 plain launches")
        result["batched_vs_plain"] = time_batched(F, torch, 10, 3, 4)
        log("bench: torch.fft.fft2 (vendor FFT) on the same inputs, context")
        result["vendor_fft_context"] = vendor_fft_context(F, torch)

    if not args.no_cpu:
        log("bench: CPU baseline (FP64 oracle)")
        ref, cpu = cpu_baseline(rows, cols, r["x"], args.cpu_budget, 200)
        result["cpu_baseline"] = cpu
        log("bench: CPU baseline on one core")
        _, cpu1 = cpu_baseline(rows, cols, r["x"], 4.0, 50, threads=1)
        result["cpu_baseline_1core"] = cpu1
        if not args.no_extras:
            log("bench: FP64 oracle on the other configurations (context, and the library's error on each)")
            result["cpu_oracle_configs"] = cpu_configs(gpu_forward_outputs(F, torch))
        num = np.linalg.norm((r["y"].astype(np.complex128) - ref).ravel())
        result["fwd_rel_l2_vs_oracle"] = float(num / np.linalg.norm(ref.ravel()))

    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
