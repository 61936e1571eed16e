#!/usr/bin/env python3
"""Benchmark of the MI355X 2D FFT: forward + inverse round trip of a
4096 x 4096 complex64 grid (128 MiB), inputs resident in HBM.

One step = forward 2D FFT (row pass + column pass) then inverse 2D FFT (row
pass + column pass), out of place: x -> y -> z. Prints ONE JSON line:
GFLOP/s under the 5 N log2 N convention (two transforms per step), the
effective HBM bandwidth, the roofline of the dominant kernel (algorithmic
bytes per launch over its mean duration, timed with HIP events bound to the
kernel's launch on the stream it runs on), the FP64 oracle timed on the host
cores as CPU baseline, every configuration's forward transform with its
passes against their data-movement floors (the same kernels with arithmetic,
then also the LDS exchanges, switched off), and the backward (adjoint) and
batched forms against the plain path.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W]
       python bench.py --only NAME [--steps K] [--warmup W]   (one configuration, for rocprofv3)
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


def kernel_role(name):
    """(kind, direction) of a library pass kernel from its demangled name:
    kind "row" (pass_kernel in row mode, rowc_kernel, rowx_kernel or
    row_wave_kernel) or "col" (pass_kernel in column mode), direction -1 or +1
    (the template argument after the configuration); None for any other
    kernel. A measurement variant (MODE template argument 1 or 2) has kind
    "row-probe" / "col-probe"."""
    import re
    m = re.search(r"fft2d::dev::(pass_kernel|rowc_kernel|rowx_kernel|row_wave_kernel)<fft2d::dev::Cfg<([^>]*)>,"
                  r"\s*(-?\d+)([^>]*)>", name)
    if not m:
        return None
    kernel, cfg, sign, rest = m.group(1), [v.strip() for v in m.group(2).split(",")], int(m.group(3)), m.group(4)
    kind = "col" if (kernel == "pass_kernel" and cfg[4] == "true") else "row"
    tail = [v.strip() for v in rest.split(",") if v.strip()]
    mode_at = 1 if kernel == "row_wave_kernel" else 3  # position of MODE after the sign
    if len(tail) > mode_at and tail[mode_at] in ("1", "2"):
        kind += "-probe"
    return kind, (-1 if sign < 0 else 1)


# expected (kind, direction) of each pass of the profiled sequences
ROUND_TRIP_ROLES = {"fwd_row": ("row", -1), "fwd_col": ("col", -1), "inv_row": ("row", 1), "inv_col": ("col", 1)}
FORWARD_ROLES = {"fwd_row": ("row", -1), "fwd_col": ("col", -1)}
# fft2d_backward with the forward direction runs the opposite-sign kernels
BACKWARD_ROLES = {"bwd_row": ("row", 1), "bwd_col": ("col", 1)}


def _assign_passes(rows, roles):
    """Dispatches of the library's pass kernels in dispatch order, each given
    the pass name whose role it has (the sequence cycles through `roles`);
    raises ValueError when a dispatch's kernel is not the expected one (an
    extra or missing dispatch would otherwise shift every later counter onto
    the wrong pass)."""
    names = list(roles)
    sel = [r for r in rows if kernel_role(r["Kernel_Name"]) is not None
           and not kernel_role(r["Kernel_Name"])[0].endswith("-probe")]
    sel.sort(key=lambda r: int(r["Dispatch_Id"]))
    out = []
    for i, r in enumerate(sel):
        want = names[i % len(names)]
        got = kernel_role(r["Kernel_Name"])
        if got != roles[want]:
            raise ValueError("dispatch %s (%s) is %s, expected %s for pass %s"
                             % (r["Dispatch_Id"], r["Kernel_Name"], got, roles[want], want))
        out.append((want, r))
    return out


def summarize_traffic(fetch_dir, write_dir, copy_fetch_dir, copy_write_dir, points=4096 * 4096,
                      roles=ROUND_TRIP_ROLES, copy_bytes=4096 * 4096 * 8):
    """HBM bytes per launch of each pass from rocprofv3 FETCH_SIZE / WRITE_SIZE
    runs (KiB per dispatch), each scaled by the factor that makes the same
    counter read the known size of a plain device copy (bench.py --copy-only:
    `copy_bytes` read and written per copy)."""
    factors = {}
    for name, d in (("FETCH_SIZE", copy_fetch_dir), ("WRITE_SIZE", copy_write_dir)):
        vals = [float(r["Counter_Value"]) for r in _counter_rows(d)
                if "copyBuffer" in r["Kernel_Name"] and r["Counter_Name"] == name]
        kib = float(np.median(vals))
        factors[name] = (copy_bytes / 1024.0) / kib
    per_pass = {}
    for name, d in (("FETCH_SIZE", fetch_dir), ("WRITE_SIZE", write_dir)):
        rows = [r for r in _counter_rows(d) if r["Counter_Name"] == name]
        for p, r in _assign_passes(rows, roles):
            per_pass.setdefault(p, {}).setdefault(name, []).append(float(r["Counter_Value"]))
            per_pass[p]["kernel"] = r["Kernel_Name"]
    lines = ["source_hash = %s" % kernel_source_hash(),
             "fetch_factor = %.4f" % factors["FETCH_SIZE"],
             "write_factor = %.4f" % factors["WRITE_SIZE"],
             "algorithmic_bytes_per_pass = %d" % (BYTES_PER_POINT_PER_PASS * points)]
    for p in roles:
        e = per_pass[p]
        fk = float(np.mean(e["FETCH_SIZE"]))
        wk = float(np.mean(e["WRITE_SIZE"]))
        rd = fk * 1024 * factors["FETCH_SIZE"]
        wr = wk * 1024 * factors["WRITE_SIZE"]
        lines.append("pass %s bytes %d read %d write %d fetch_kib %.1f write_kib %.1f dispatches %d kernel %s"
                     % (p, rd + wr, rd, wr, fk, wk, len(e["FETCH_SIZE"]), e["kernel"]))
    return "\n".join(lines)


def summarize_counters(*run_dirs, roles=ROUND_TRIP_ROLES):
    """Mean per launch of every counter of rocprofv3 --pmc runs (one folder per
    run), for each pass of the profiled sequence, and the count per wave where
    the counter counts instructions (wave count SQ_WAVES from the same runs)."""
    per_pass = {}
    for d in run_dirs:
        rows = _counter_rows(d)
        for name in sorted({r["Counter_Name"] for r in rows}):
            sel = [r for r in rows if r["Counter_Name"] == name]
            for p, r in _assign_passes(sel, roles):
                e = per_pass.setdefault(p, {"kernel": r["Kernel_Name"]})
                e.setdefault(name, []).append(float(r["Counter_Value"]))
    lines = []
    for p in roles:
        e = per_pass[p]
        waves = float(np.mean(e["SQ_WAVES"])) if "SQ_WAVES" in e else None
        lines.append("pass %s kernel %s" % (p, e["kernel"]))
        for name in sorted(k for k in e if k != "kernel"):
            v = float(np.mean(e[name]))
            extra = ("  per wave %.1f" % (v / waves)) if waves and name.startswith("SQ_INSTS_") else ""
            lines.append("  %-24s %16.1f  (%d launches)%s" % (name, v, len(e[name]), extra))
    return "\n".join(lines)


STATS_PROFILE = os.path.join(ROOT, "profiles", "kernel_stats_fft2d_4096x4096_roundtrip.txt")


def summarize_stats(stats_dir, timed=0):
    """The rows of a rocprofv3 --kernel-trace --stats run (kernel_stats.csv),
    after the hash of the plain path's sources they were taken from; with
    timed = K, also each library pass kernel's mean duration over its last K
    dispatches (from the kernel trace): the launches of the bench's timed
    region, which come last in a run."""
    import csv
    with open(os.path.join(stats_dir, "run_kernel_stats.csv"), newline="") as fh:
        rows = list(csv.DictReader(fh))
    last = {}
    if timed:
        with open(os.path.join(stats_dir, "run_kernel_trace.csv"), newline="") as fh:
            trace = list(csv.DictReader(fh))
        by_name = {}
        for r in trace:
            if kernel_role(r["Kernel_Name"]) is not None or "::batched_kernel(" in r["Kernel_Name"]:
                by_name.setdefault(r["Kernel_Name"], []).append(r)
        for name, rs in by_name.items():
            rs.sort(key=lambda r: int(r["Dispatch_Id"]))
            d = [(int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3 for r in rs[-timed:]]
            last[name] = float(np.mean(d))
    out = ["source_hash = %s" % kernel_source_hash(),
           "calls  avg_us   min_us   max_us   total_%%  last%d_us  kernel" % timed]
    for r in rows:
        lt = ("%9.2f" % last[r["Name"]]) if r["Name"] in last else "        -"
        out.append("%5s %8.2f %8.2f %8.2f %8.2f %s  %s" % (r["Calls"], float(r["AverageNs"]) / 1e3,
                                                          float(r["MinNs"]) / 1e3, float(r["MaxNs"]) / 1e3,
                                                          float(r["Percentage"]), lt, r["Name"]))
    return "\n".join(out)


def rocprof_roofline(pass_name, pass_bytes):
    """The dominant pass's mean duration over the timed region's launches in
    the committed rocprofv3 kernel trace of the round trip (the same bench
    command under rocprofv3), as a roofline fraction, beside its mean over all
    launches of that run; None when the summary is missing or was taken from
    other kernel sources."""
    try:
        with open(STATS_PROFILE) as fh:
            lines = fh.read().splitlines()
    except OSError:
        return None
    hashes = [l.split()[2] for l in lines if l.startswith("source_hash = ")]
    if not hashes or hashes[0] != kernel_source_hash():
        return None
    want = ROUND_TRIP_ROLES[pass_name]
    for l in lines:
        f = l.split(None, 6)
        if len(f) == 7 and f[0].isdigit() and kernel_role(f[6]) == want and f[5] != "-":
            timed_us, all_us = float(f[5]), float(f[1])
            return {"timed_avg_us": timed_us, "all_launches_avg_us": all_us, "calls": int(f[0]),
                    "achieved": round(pass_bytes / (timed_us * 1e-6) / 1e9, 1),
                    "frac": round(pass_bytes / (timed_us * 1e-6) / 1e9 / HBM_PEAK_GBS, 4)}
    return None


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
    ("8 x 2048x2048 forward", 8, 2048, 2048, 5),
]
# --only names: configuration (batch, rows, cols, seed)
ONLY = {"64x64": (1, 64, 64, 0), "8192x64x64": (8192, 64, 64, 6), "1024x1024": (1, 1024, 1024, 0),
        "4096x4096": (1, 4096, 4096, 1), "8192x8192": (1, 8192, 8192, 2), "16384x2048": (1, 16384, 2048, 3),
        "4096x1x16384": (4096, 1, 16384, 0), "8x2048x2048": (8, 2048, 2048, 5)}
SCRATCH_FLOATS = 1 << 28  # 1 GiB read before each cold transform


def _frac(nbytes, ms):
    return round(nbytes / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4) if ms and ms > 0 else None


def time_passes(F, torch, plan, batch, rows, cols, x, y, iters, scratch):
    """Per pass of a two-pass plan, the mean kernel duration (HIP events bound
    to each launch) of the pass itself ("fft"), of the same kernel with its
    arithmetic switched off ("no_arith": loads, LDS exchanges, stores) and with
    its arithmetic and exchanges switched off ("copy": a copy with the pass's
    access pattern), each transform preceded by a 1 GiB read (no input in the
    MALL, nothing dirty there), passes back to back as in fft2d_exec. The
    fraction of the copy is copy / fft: 1.0 means the pass runs at the speed
    of its own data movement."""
    stream = torch.cuda.current_stream()
    sh = int(stream.cuda_stream)
    passes = [p for p, n in ((0, cols), (1, rows)) if n > 1]
    nbytes = BYTES_PER_POINT_PER_PASS * batch * rows * cols
    xp, yp = x.data_ptr(), y.data_ptr()
    out = {}
    for variant, mode in (("fft", 0), ("no_arith", F.ABLATE_ARITHMETIC), ("copy", F.ABLATE_EXCHANGE)):
        ev = [[(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in passes]
              for _ in range(iters + 2)]
        for row in ev:
            for a, b in row:
                a.record(stream)
                b.record(stream)
        torch.cuda.synchronize()
        try:
            for row in ev:
                scratch.sum()
                for pidx, (a, b) in zip(passes, row):
                    if mode == 0:
                        F.fft2d_exec_pass_timed(plan.handle, xp, yp, F.FORWARD, pidx, a.cuda_event, b.cuda_event, sh)
                    else:
                        F.fft2d_exec_pass_ablated(plan.handle, xp, yp, pidx, mode, a.cuda_event, b.cuda_event, sh)
        except F.Fft2dError:  # no measurement variant compiled for this plan's kernels
            torch.cuda.synchronize()
            continue
        torch.cuda.synchronize()
        for i, pidx in enumerate(passes):
            t = float(np.mean([row[i][0].elapsed_time(row[i][1]) for row in ev[2:]]))
            out.setdefault("row" if pidx == 0 else "col", {})[variant + "_ms"] = round(t, 5)
    for name, e in out.items():
        e["frac"] = _frac(nbytes, e.get("fft_ms"))
        if "copy_ms" in e:
            e["copy_frac"] = _frac(nbytes, e["copy_ms"])
            e["fft_over_copy"] = round(e["fft_ms"] / e["copy_ms"], 3)
        if "no_arith_ms" in e:
            e["fft_over_no_arith"] = round(e["fft_ms"] / e["no_arith_ms"], 3)
    return out


def time_configs(F, torch, iters):
    """Forward transform of each configuration, warm (back to back), cold (a
    1 GiB scratch tensor is zeroed before each iteration, outside the timed
    events, so the 256 MB MALL holds none of the input, but holds dirty lines
    of the scratch that are written back while the transform runs) and
    cold_clean (the scratch is read instead: no input in the MALL and nothing
    to write back): median, mean, min; and for two-pass plans each pass,
    cold_clean, against its data-movement floors (time_passes)."""
    import synth
    stream = torch.cuda.current_stream()
    sh = int(stream.cuda_stream)
    scratch = torch.empty(SCRATCH_FLOATS, dtype=torch.float32, device="cuda")
    res = {}
    for name, batch, rows, cols, seed in CONFIGS:
        shape = (batch, rows, cols) if batch > 1 else (rows, cols)
        x = torch.from_numpy(synth.complex_grid(seed, shape)).to("cuda")
        y = torch.empty_like(x)
        plan = F.get_plan(batch, rows, cols, x.device)
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(iters)]
        out = {}
        # HBM passes: a length-1 dimension needs none; a whole-grid plan reads and writes once
        whole = " grid[" in plan.describe()
        npass = 1 if whole else int(rows > 1) + int(cols > 1)
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
                         "hbm_gbps": round(npass * BYTES_PER_POINT_PER_PASS * pts / med / 1e6, 1),
                         "frac": _frac(npass * BYTES_PER_POINT_PER_PASS * pts, med)}
        if not whole:
            out["passes_cold_clean"] = time_passes(F, torch, plan, batch, rows, cols, x, y, iters, scratch)
        out["plan"] = plan.describe()
        res[name] = out
        del x, y
    del scratch
    torch.cuda.empty_cache()
    return res


def only_config(F, torch, name, steps, warmup):
    """One configuration's forward transform alone, for rocprofv3 (its kernel
    statistics then hold that configuration's passes only), under the same
    protocol as the per-pass figures of the default run (time_passes): every
    transform preceded by a 1 GiB read. `warmup` + `steps` transforms by
    fft2d_exec, then `steps` pass by pass with events bound to each launch;
    prints one JSON line with the per-pass mean durations."""
    import synth
    batch, rows, cols, seed = ONLY[name]
    shape = (batch, rows, cols) if batch > 1 else (rows, cols)
    x = torch.from_numpy(synth.complex_grid(seed, shape)).to("cuda")
    y = torch.empty_like(x)
    scratch = torch.empty(SCRATCH_FLOATS, dtype=torch.float32, device="cuda")
    plan = F.get_plan(batch, rows, cols, x.device)
    stream = torch.cuda.current_stream()
    sh = int(stream.cuda_stream)
    for _ in range(warmup):
        scratch.sum()
        F.fft2d_exec(plan.handle, x.data_ptr(), y.data_ptr(), F.FORWARD, sh)
    torch.cuda.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    for a, b in ev:
        scratch.sum()
        a.record(stream)
        F.fft2d_exec(plan.handle, x.data_ptr(), y.data_ptr(), F.FORWARD, sh)
        b.record(stream)
    torch.cuda.synchronize()
    per_transform = float(np.mean([a.elapsed_time(b) for a, b in ev]))
    whole = " grid[" in plan.describe()
    passes = [] if whole else [p for p, n in ((0, cols), (1, rows)) if n > 1]
    pev = [[(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in passes]
           for _ in range(steps)]
    for row in pev:
        for a, b in row:
            a.record(stream)
            b.record(stream)
    torch.cuda.synchronize()
    for row in pev:
        scratch.sum()
        for pidx, (a, b) in zip(passes, row):
            F.fft2d_exec_pass_timed(plan.handle, x.data_ptr(), y.data_ptr(), F.FORWARD, pidx, a.cuda_event,
                                    b.cuda_event, sh)
    torch.cuda.synchronize()
    nbytes = BYTES_PER_POINT_PER_PASS * batch * rows * cols
    per = {}
    for i, pidx in enumerate(passes):
        t = float(np.mean([row[i][0].elapsed_time(row[i][1]) for row in pev]))
        per["row" if pidx == 0 else "col"] = {"ms": round(t, 5), "frac": _frac(nbytes, t)}
    npass = 1 if whole else len(passes)
    print(json.dumps({"only": name, "steps": steps, "warmup": warmup, "protocol": "1 GiB read before each transform",
                      "ms_per_transform": round(per_transform, 5),
                      "frac": _frac(npass * nbytes, per_transform), "passes": per, "plan": plan.describe()}),
          flush=True)


def device_copy_gbps(torch, iters=20):
    """Read+write bandwidth of a plain device copy (torch's copy_ of a
    contiguous tensor, which runs the HIP runtime's copy kernel), 512 MiB to
    512 MiB (1 GiB of traffic): warm (back to back), and cold_clean (a
    different 1 GiB buffer read before each copy, so neither source nor
    destination sits in the MALL and nothing dirty is left there)."""
    n = 1 << 26  # complex64 points: 512 MiB
    x = torch.zeros(n, dtype=torch.complex64, device="cuda")
    y = torch.empty_like(x)
    scratch = torch.empty(SCRATCH_FLOATS, dtype=torch.float32, device="cuda")
    stream = torch.cuda.current_stream()
    out = {"bytes_per_copy": 2 * n * 8}
    for mode in ("warm", "cold_clean"):
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(iters)]
        for _ in range(3):
            y.copy_(x)
        for a, b in ev:
            if mode == "cold_clean":
                scratch.sum()
            a.record(stream)
            y.copy_(x)
            b.record(stream)
        torch.cuda.synchronize()
        med = float(np.median([a.elapsed_time(b) for a, b in ev]))
        out[mode + "_ms"] = round(med, 5)
        out[mode + "_gbps"] = round(2 * n * 8 / med / 1e6, 1)
        out[mode + "_frac"] = _frac(2 * n * 8, med)
    del x, y, scratch
    torch.cuda.empty_cache()
    return out


def probe_rates(F, torch, iters=10):
    """The probes behind the pass kernels' design: copies of an 8192 x 8192
    grid in column tiles of the 8192^2 split column pass's rows (M1 = 4) with
    128-, 256- and 512-byte row segments (fft2d_probe_tile_copy; every tile
    256 KiB; only the 128-byte form fits a 2048-point column FFT in one
    workgroup), plain and nontemporal loads, each copy after a 1 GiB read
    (mean, GB/s of read + write); and the LDS read and write bandwidth of one
    1024-thread workgroup per CU with 4-, 8- and 16-byte accesses
    (fft2d_probe_lds; bytes per clock per CU at the 2.4 GHz peak clock)."""
    stream = torch.cuda.current_stream()
    sh = int(stream.cuda_stream)
    n = 8192
    x = torch.zeros((n, n), dtype=torch.complex64, device="cuda")
    y = torch.empty_like(x)
    scratch = torch.empty(SCRATCH_FLOATS, dtype=torch.float32, device="cuda")
    out = {}

    def timed(fn, cold):
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(iters + 1)]
        for a, b in ev:  # torch computes elapsed times only of events it has recorded once
            a.record(stream)
            b.record(stream)
        torch.cuda.synchronize()
        for a, b in ev:
            if cold:
                scratch.sum()
            fn(a.cuda_event, b.cuda_event)
        torch.cuda.synchronize()
        return float(np.mean([a.elapsed_time(b) for a, b in ev[1:]]))

    for cw in (16, 32, 64):
        for nt in (False, True):
            ms = timed(lambda a, b: F.fft2d_probe_tile_copy(x.data_ptr(), y.data_ptr(), n, n, cw, 4, nt, a, b, sh),
                       True)
            nbytes = 2 * n * n * 8
            out["tile_copy_%dB%s" % (cw * 8, "_nt" if nt else "")] = {
                "ms": round(ms, 5), "gbps": round(nbytes / (ms * 1e-3) / 1e9, 1), "frac": _frac(nbytes, ms)}
    del x, y, scratch
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    sink = torch.empty(cus * 1024, dtype=torch.float32, device="cuda")
    for width in (4, 8, 16):
        for write in (False, True):
            moved = {}

            def run(a, b):
                moved["bytes"] = F.fft2d_probe_lds(width, write, sink.data_ptr(), sink.numel(), a, b, sh)
            ms = timed(run, False)
            out["lds_%s_b%d" % ("write" if write else "read", width * 8)] = {
                "ms": round(ms, 5), "bytes_per_clk_per_cu": round(moved["bytes"] / (ms * 1e-3) / 2.4e9 / cus, 1)}
    del sink
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
    """fft2d_backward (adjoint kernels) against fft2d_exec on the same plan and
    data, and one whole differentiation step of sum |W * FFT2(x)|^2."""
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
    # One differentiation step of the loss sum |W * FFT2(x)|^2 (W real [rows][cols], uniform [0, 1) from seed
    # seed + 100, broadcast over the batch): the library's forward and adjoint kernels plus torch's elementwise
    # ops and reduction, as a training step would run them.
    w = torch.from_numpy(synth.real_weights(seed + 100, (rows, cols))).to("cuda")
    xg = x.clone().requires_grad_(True)

    def train_step():
        xg.grad = None
        y = F.fft2_diff(xg, F.FORWARD)
        loss = (w * w * (y.real * y.real + y.imag * y.imag)).sum()
        loss.backward()

    step = run(train_step)
    return {"workload": "batch %d of %dx%d complex64" % (batch, rows, cols), "plain_ms": fwd, "backward_ms": bwd,
            "backward_over_plain": bwd / fwd, "plain_gflops": fl / fwd / 1e6, "backward_gflops": fl / bwd / 1e6,
            "loss_step_ms": step, "loss_step": "fft2_diff forward, loss = sum |W * FFT2(x)|^2 (torch), backward",
            "fft_share_of_loss_step": (fwd + bwd) / step}


def _batched_plan(F, shapes, tune, cache):
    """A batched plan made with FFT2D_TUNE=`tune` and the tuning cache at `cache`."""
    saved = {k: os.environ.get(k) for k in ("FFT2D_TUNE", "FFT2D_TUNE_CACHE")}
    os.environ["FFT2D_TUNE"] = tune
    os.environ["FFT2D_TUNE_CACHE"] = cache
    try:
        return F.BatchedPlan(shapes)
    finally:
        for k, v in saved.items():
            if v is None:
                os.environ.pop(k, None)
            else:
                os.environ[k] = v


BATCHED_SEED = 4  # the 512-shape workload of the default run
ONLY_EXTRA = ("backward-8x2048x2048", "batched-512")


def only_batched(F, torch, steps, warmup):
    """The 512-shape batched workload alone, for rocprofv3: the tuned plan (its
    tuning trials launch the batched kernel too), `warmup` graph replays, then
    `steps` replays each bracketed by events; the timed replays are the
    kernel's last `steps` dispatches. Prints one JSON line."""
    import tempfile

    import synth
    shapes = synth.pow2_shapes(BATCHED_SEED, 512)
    xs = [torch.from_numpy(x).to("cuda") for x in synth.batched_grids(BATCHED_SEED, shapes)]
    ys = [torch.empty_like(x) for x in xs]
    with tempfile.TemporaryDirectory() as tmp:
        plan = _batched_plan(F, shapes, "full", os.path.join(tmp, "tune.txt"))
    stream = torch.cuda.current_stream()
    sh = int(stream.cuda_stream)
    iarr = F.pointer_array([x.data_ptr() for x in xs])
    oarr = F.pointer_array([y.data_ptr() for y in ys])
    for _ in range(warmup):
        plan.exec_ptrs(iarr, oarr, F.FORWARD, sh)
    torch.cuda.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    for a, b in ev:
        a.record(stream)
        plan.exec_ptrs(iarr, oarr, F.FORWARD, sh)
        b.record(stream)
    torch.cuda.synchronize()
    ms = float(np.mean([a.elapsed_time(b) for a, b in ev]))
    points = sum(r * c for r, c in shapes)
    print(json.dumps({"only": "batched-512", "steps": steps, "warmup": warmup, "protocol": "graph replays back to back",
                      "ms_per_replay": round(ms, 5), "points": points,
                      "gbps_at_32_bytes_per_point": round(32.0 * points / (ms * 1e-3) / 1e9, 1),
                      "frac": _frac(32.0 * points, ms), "plan": plan.describe()}), flush=True)
    plan.close()


def only_backward(F, torch, steps, warmup):
    """fft2d_backward (forward-direction adjoint) of a batch of 8 grids of
    2048 x 2048 alone, for rocprofv3, under the protocol of only_config: every
    call preceded by a 1 GiB read; prints one JSON line."""
    import synth
    x = torch.from_numpy(synth.complex_grid(5, (8, 2048, 2048))).to("cuda")
    y = torch.empty_like(x)
    scratch = torch.empty(SCRATCH_FLOATS, dtype=torch.float32, device="cuda")
    plan = F.get_plan(8, 2048, 2048, x.device)
    stream = torch.cuda.current_stream()
    sh = int(stream.cuda_stream)
    for _ in range(warmup):
        scratch.sum()
        F.fft2d_backward(plan.handle, x.data_ptr(), y.data_ptr(), F.FORWARD, sh)
    torch.cuda.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    for a, b in ev:
        scratch.sum()
        a.record(stream)
        F.fft2d_backward(plan.handle, x.data_ptr(), y.data_ptr(), F.FORWARD, sh)
        b.record(stream)
    torch.cuda.synchronize()
    ms = float(np.mean([a.elapsed_time(b) for a, b in ev]))
    nbytes = 2 * BYTES_PER_POINT_PER_PASS * 8 * 2048 * 2048
    print(json.dumps({"only": "backward-8x2048x2048", "steps": steps, "warmup": warmup,
                      "protocol": "1 GiB read before each call", "ms_per_call": round(ms, 5),
                      "frac": _frac(nbytes, ms), "plan": plan.describe()}), flush=True)


def summarize_batched_traffic(fetch_dir, write_dir, copy_fetch_dir, copy_write_dir, timed,
                              copy_bytes=4096 * 4096 * 8):
    """HBM bytes per launch of the batched kernel from rocprofv3 FETCH_SIZE /
    WRITE_SIZE runs of `bench.py --only batched-512`, over its last `timed`
    dispatches (the timed graph replays), scaled as in summarize_traffic."""
    import synth
    factors = {}
    for name, d in (("FETCH_SIZE", copy_fetch_dir), ("WRITE_SIZE", copy_write_dir)):
        vals = [float(r["Counter_Value"]) for r in _counter_rows(d)
                if "copyBuffer" in r["Kernel_Name"] and r["Counter_Name"] == name]
        factors[name] = (copy_bytes / 1024.0) / float(np.median(vals))
    kib = {}
    kernel = None
    for name, d in (("FETCH_SIZE", fetch_dir), ("WRITE_SIZE", write_dir)):
        rows = [r for r in _counter_rows(d) if r["Counter_Name"] == name and "batched_kernel" in r["Kernel_Name"]]
        if len(rows) < timed:
            raise ValueError("%d batched_kernel dispatches in %s, fewer than %d" % (len(rows), d, timed))
        rows.sort(key=lambda r: int(r["Dispatch_Id"]))
        kib[name] = float(np.mean([float(r["Counter_Value"]) for r in rows[-timed:]]))
        kernel = rows[-1]["Kernel_Name"]
    points = sum(r * c for r, c in synth.pow2_shapes(BATCHED_SEED, 512))
    rd = kib["FETCH_SIZE"] * 1024 * factors["FETCH_SIZE"]
    wr = kib["WRITE_SIZE"] * 1024 * factors["WRITE_SIZE"]
    return "\n".join([
        "source_hash = %s" % kernel_source_hash(),
        "fetch_factor = %.4f" % factors["FETCH_SIZE"],
        "write_factor = %.4f" % factors["WRITE_SIZE"],
        "points = %d" % points,
        "algorithmic_bytes_at_32_per_point = %d" % (32 * points),
        "launch bytes %d read %d write %d fetch_kib %.1f write_kib %.1f dispatches %d kernel %s"
        % (rd + wr, rd, wr, kib["FETCH_SIZE"], kib["WRITE_SIZE"], timed, kernel)])


def summarize_batched_counters(run_dir, timed):
    """Mean of every counter of a rocprofv3 --pmc run of `bench.py --only
    batched-512` over the batched kernel's last `timed` dispatches."""
    rows = [r for r in _counter_rows(run_dir) if "batched_kernel" in r["Kernel_Name"]]
    by = {}
    for r in rows:
        by.setdefault(r["Counter_Name"], []).append(r)
    lines = ["source_hash = %s" % kernel_source_hash()]
    for name in sorted(by):
        rs = sorted(by[name], key=lambda r: int(r["Dispatch_Id"]))[-timed:]
        lines.append("%s %.6g (mean of %d dispatches)" % (name, float(np.mean([float(r["Counter_Value"]) for r in rs])),
                                                          len(rs)))
    return "\n".join(lines)


def time_batched(F, torch, steps, warmup, seed):
    """512 transforms of 2^a x 2^b (a, b in [6, 11] from `seed`): one graph
    replay of the persistent kernel, with the autotuner's choice (grid size,
    item order, group size and the radix/tile variant of every length, tuned
    afresh into a scratch cache file) and with the untuned defaults, against
    512 fft2d_exec calls (two kernel launches each) on one stream."""
    import tempfile

    import synth
    shapes = synth.pow2_shapes(seed, 512)
    xs = [torch.from_numpy(x).to("cuda") for x in synth.batched_grids(seed, shapes)]
    ys = [torch.empty_like(x) for x in xs]
    zs = [torch.empty_like(x) for x in xs]
    with tempfile.TemporaryDirectory() as tmp:
        cache = os.path.join(tmp, "tune.txt")
        t0 = time.perf_counter()
        plan = _batched_plan(F, shapes, "full", cache)
        tune_s = time.perf_counter() - t0
        default = _batched_plan(F, shapes, "off", cache)
    stream = torch.cuda.current_stream()
    sh = int(stream.cuda_stream)
    iptr = [x.data_ptr() for x in xs]
    iarr = F.pointer_array(iptr)  # built once: a replay converts nothing
    oarr = F.pointer_array([y.data_ptr() for y in ys])
    plans = [F.get_plan(1, r, c, xs[0].device) for r, c in shapes]
    zptr = [z.data_ptr() for z in zs]

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

    def plain():
        for p, a, b in zip(plans, iptr, zptr):
            F.fft2d_exec(p.handle, a, b, F.FORWARD, sh)

    t_d = run(lambda: default.exec_ptrs(iarr, oarr, F.FORWARD, sh))
    t_b = run(lambda: plan.exec_ptrs(iarr, oarr, F.FORWARD, sh))
    t_p = run(plain)
    num = sum(float(torch.linalg.vector_norm(y - z)) ** 2 for y, z in zip(ys, zs)) ** 0.5
    den = sum(float(torch.linalg.vector_norm(z)) ** 2 for z in zs) ** 0.5
    points = sum(r * c for r, c in shapes)
    fl = sum(flops_2d(r, c) for r, c in shapes)
    res = {"workload": "512 forward 2D FFTs of 2^a x 2^b, a, b in [6, 11] from seed %d, %d points" % (seed, points),
           "batched_ms": t_b, "batched_untuned_ms": t_d, "tuned_over_untuned": t_b / t_d, "tuning_s": tune_s,
           "plain_512_launches_ms": t_p, "speedup": t_p / t_b,
           "batched_gflops": fl / t_b / 1e6, "plain_gflops": fl / t_p / 1e6,
           "batched_hbm_gbps": 32.0 * points / t_b / 1e6,
           "batched_vs_plain_rel_l2": num / den, "plan": plan.describe(), "plan_untuned": default.describe()}
    plan.close()
    default.close()
    return res


def cpu_model():
    """The host CPU's model name (/proc/cpuinfo), or None."""
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


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
    return ref, {"value": gflops, "unit": "GFLOP/s", "cores": used, "kind": "oracle", "cpu_model": cpu_model(),
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


BACKWARD_CASE = ("8 x 2048x2048 backward (adjoint)", (8, 2048, 2048), 5)


def gpu_forward_outputs(F, torch):
    """The library's forward transform of every ORACLE_CASES input, its
    adjoint (fft2d_backward of the forward transform) of the BACKWARD_CASE
    input, and the forward transforms of the 512-shape batched set (one
    batched launch), copied to the host."""
    import synth
    out = {}
    for name, shape, seed in ORACLE_CASES:
        x = torch.from_numpy(synth.complex_grid(seed, shape)).to("cuda")
        out[name] = F.fft2(x).cpu().numpy()
        del x
    name, shape, seed = BACKWARD_CASE
    x = torch.from_numpy(synth.complex_grid(seed, shape)).to("cuda")
    out[name] = F.get_plan(shape[0], shape[1], shape[2], x.device).backward(x, F.FORWARD).cpu().numpy()
    del x
    xs = [torch.from_numpy(g).to("cuda")
          for g in synth.batched_grids(BATCHED_SEED, synth.pow2_shapes(BATCHED_SEED, BATCHED_COUNT))]
    out["batched"] = [y.cpu().numpy() for y in F.fft2_batched(xs)]
    del xs
    torch.cuda.empty_cache()
    return out


def errors(got, ref):
    """(relative L2, largest element error over the reference's RMS magnitude), in FP64."""
    d = np.abs(got.astype(np.complex128) - ref).ravel()
    den = float(np.linalg.norm(ref.ravel()))
    rms = den / math.sqrt(ref.size)
    return float(np.linalg.norm(d)) / den, float(d.max()) / rms


def rel_l2(got, ref):
    return errors(got, ref)[0]


def cpu_configs(gpu_out, threads=0):
    """The FP64 oracle's transform of each configuration once (all host
    cores), for GPU/CPU context beside the 4096^2 baseline, and the error of
    the library's result for the same input against it: relative L2 and the
    largest element error over the reference's RMS magnitude (the GPU tests'
    two bounds, 1e-5 each). The backward case checks fft2d_backward against
    the oracle's adjoint."""
    import oracle
    import synth
    out = {}
    for name, shape, seed in ORACLE_CASES + [BACKWARD_CASE]:
        x = synth.complex_grid(seed, shape)
        t0 = time.perf_counter()
        ref = oracle.adjoint(x, oracle.FORWARD, threads) if name == BACKWARD_CASE[0] else oracle.fft2_forward(x, threads)
        dt = time.perf_counter() - t0
        batch = int(np.prod(shape[:-2])) if len(shape) > 2 else 1
        rel, mx = errors(gpu_out[name], ref)
        out[name] = {"seconds": round(dt, 4), "gflops": round(flops_2d(shape[-2], shape[-1], batch) / dt / 1e9, 2),
                     "gpu_rel_l2": rel, "gpu_max_elem": mx}
        del x, ref
    shapes = synth.pow2_shapes(BATCHED_SEED, BATCHED_COUNT)
    xs = synth.batched_grids(BATCHED_SEED, shapes)
    t0 = time.perf_counter()
    refs = [oracle.fft2_forward(x, threads) for x in xs]
    dt = time.perf_counter() - t0
    errs = [errors(g, r) for g, r in zip(gpu_out["batched"], refs)]
    out["%d shapes 2^a x 2^b forward" % BATCHED_COUNT] = {"seconds": round(dt, 4),
                                           "gflops": round(sum(flops_2d(r, c) for r, c in shapes) / dt / 1e9, 2),
                                           "gpu_rel_l2_max": max(e[0] for e in errs),
                                           "gpu_max_elem_max": max(e[1] for e in errs)}
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
    ap.add_argument("--only", choices=sorted(ONLY) + list(ONLY_EXTRA),
                    help="run only this configuration's forward transform (warmup + steps back to back, then "
                         "steps pass by pass with bound events) and print its per-pass times; "
                         "backward-8x2048x2048: fft2d_backward calls; batched-512: replays of the batched plan")
    ap.add_argument("--vendor-context", action="store_true",
                    help="also time torch.fft.fft2 (ROCm's FFT library) on the large configurations, for context")
    ap.add_argument("--summarize-traffic", nargs=4, metavar=("FETCH", "WRITE", "COPY_FETCH", "COPY_WRITE"),
                    help="print HBM bytes per pass from four rocprofv3 --pmc output folders, then exit")
    ap.add_argument("--summarize-batched-traffic", nargs=4, metavar=("FETCH", "WRITE", "COPY_FETCH", "COPY_WRITE"),
                    help="print HBM bytes per launch of the batched kernel (its last --timed dispatches) from four "
                         "rocprofv3 --pmc output folders of --only batched-512 and --copy-only, then exit")
    ap.add_argument("--summarize-batched-counters", metavar="DIR",
                    help="print the mean of every counter over the batched kernel's last --timed dispatches from a "
                         "rocprofv3 --pmc output folder of --only batched-512, then exit")
    ap.add_argument("--summarize-counters", nargs="+", metavar="DIR",
                    help="print the mean of every counter per pass from rocprofv3 --pmc output folders, then exit")
    ap.add_argument("--summarize-stats", metavar="DIR",
                    help="print the kernel rows of a rocprofv3 --kernel-trace --stats output folder, then exit")
    ap.add_argument("--timed", type=int, default=0,
                    help="for --summarize-stats: also average each pass kernel's last TIMED dispatches")
    ap.add_argument("--profiled", default="roundtrip", choices=["roundtrip", "backward-8x2048x2048"] + sorted(ONLY),
                    help="for --summarize-*: the workload profiled: the 4096x4096 round trip (default), "
                         "fft2d_backward at 8x2048x2048, or the forward transform of an --only configuration")
    args = ap.parse_args()
    roles = {"roundtrip": ROUND_TRIP_ROLES, "backward-8x2048x2048": BACKWARD_ROLES}.get(args.profiled, FORWARD_ROLES)
    if args.summarize_traffic:
        b, r_, c_, _ = ONLY[{"roundtrip": "4096x4096", "backward-8x2048x2048": "8x2048x2048"}.get(args.profiled,
                                                                                                   args.profiled)]
        print(summarize_traffic(*args.summarize_traffic, points=b * r_ * c_, roles=roles))
        return
    if args.summarize_batched_counters:
        print(summarize_batched_counters(args.summarize_batched_counters, args.timed or 1))
        return
    if args.summarize_batched_traffic:
        print(summarize_batched_traffic(*args.summarize_batched_traffic, timed=args.timed or 1))
        return
    if args.summarize_counters:
        print(summarize_counters(*args.summarize_counters, roles=roles))
        return
    if args.summarize_stats:
        print(summarize_stats(args.summarize_stats, args.timed))
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
    if args.only == "batched-512":
        only_batched(F, torch, args.steps, args.warmup)
        return
    if args.only == "backward-8x2048x2048":
        only_backward(F, torch, args.steps, args.warmup)
        return
    if args.only:
        only_config(F, torch, args.only, args.steps, args.warmup)
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
        "roofline_rocprof": rocprof_roofline(pass_names[dom], pass_bytes),
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
        passes = one.get("passes_cold_clean", {})
        if "row" in passes and "copy_ms" in passes["row"]:
            # the dominant kernel (the forward row pass) against a copy with its own access pattern
            result["roofline"]["frac_of_same_pattern_copy"] = round(passes["row"]["copy_ms"] / passes["row"]["fft_ms"], 4)
        log("bench: device copy bandwidth, 512 MiB to 512 MiB")
        result["device_copy"] = device_copy_gbps(torch)
        log("bench: column-tile copy and LDS bandwidth probes")
        result["probes"] = probe_rates(F, torch)
        log("bench: energy per transform (1024 x 1024 and 4096 x 4096)")
        result["energy"] = [energy(F, torch, 1024, 1024, 1.5), energy(F, torch, 4096, 4096, 1.5)]
        log("bench: batched 512 shapes vs 512 plain launches")
        result["batched_vs_plain"] = time_batched(F, torch, 10, 3, BATCHED_SEED)
        if args.vendor_context:
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
        rel, mx = errors(r["y"], ref)
        result["fwd_rel_l2_vs_oracle"] = rel
        result["fwd_max_elem_vs_oracle"] = mx

    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
