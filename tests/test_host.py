"""Host-side logic that needs no GPU: argument checks of the Python binding,
the pointer-array marshalling, and bench.py's rocprofv3 summaries and its
one-GPU rule."""

from __future__ import annotations

import csv
import os
import subprocess
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def F():
    import paper_2506_15437_amd as F
    return F


def test_binding_rejects_bad_tensors_without_a_gpu(F):
    import torch
    with pytest.raises(TypeError):
        F.fft2(np.zeros((4, 4), np.complex64))
    with pytest.raises(TypeError):
        F.fft2(torch.zeros(4, 4, dtype=torch.complex64))  # host tensor
    with pytest.raises(TypeError):
        F.fft2(torch.zeros(4, 4, dtype=torch.float32))


def test_pointer_array(F):
    a = F.pointer_array([0x1000, 0x2008, 2**40])
    assert a.dtype == np.uint64 and a.tolist() == [0x1000, 0x2008, 2**40]
    assert F.pointer_array(a) is a  # an array of the right type passes through unconverted


# demangled names of the round trip's four pass kernels, as rocprofv3 reports them
_RC = "void fft2d::dev::rowc_kernel<fft2d::dev::Cfg<4096, 32, 4, 2, false, 16, 16, 16>, %d, 4, 0, true, 0>(fft2d::PassArgs)"
_PK = ("void fft2d::dev::pass_kernel<fft2d::dev::Cfg<1024, 32, 16, 2, true, 16, 16, 4>, %d, false, 1, 0, 0>"
       "(fft2d::PassArgs)")
ROUND_TRIP_NAMES = [_RC % -1, _PK % -1, _RC % 1, _PK % 1]


def _write_counters(path, rows):
    os.makedirs(path, exist_ok=True)
    with open(os.path.join(path, "run_counter_collection.csv"), "w", newline="") as fh:
        w = csv.writer(fh)
        w.writerow(["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"])
        for r in rows:
            w.writerow(r)


def test_traffic_summary_scales_by_the_copy(tmp_path, monkeypatch):
    """FETCH_SIZE reading half of a copy's bytes gives a factor of 2; the
    per-pass figure is the scaled sum, dispatches assigned in step order."""
    import bench
    grid = 4096 * 4096 * 8  # bytes of one grid
    kib = grid / 1024
    names = ROUND_TRIP_NAMES
    fetch, write = [], []
    for step in range(2):
        for i, n in enumerate(names):
            d = 10 + step * 4 + i
            fetch.append([d, n, "FETCH_SIZE", kib / 2 * (1.05 if i == 0 else 1.0)])
            write.append([d, n, "WRITE_SIZE", kib])
    _write_counters(tmp_path / "f", fetch + [[1, "some_other_kernel", "FETCH_SIZE", 1.0]])
    _write_counters(tmp_path / "w", write)
    _write_counters(tmp_path / "cf", [[1, "__amd_rocclr_copyBuffer", "FETCH_SIZE", kib / 2]])
    _write_counters(tmp_path / "cw", [[1, "__amd_rocclr_copyBuffer", "WRITE_SIZE", kib]])
    text = bench.summarize_traffic(str(tmp_path / "f"), str(tmp_path / "w"), str(tmp_path / "cf"),
                                   str(tmp_path / "cw"))
    lines = {l.split()[1]: l.split() for l in text.splitlines() if l.startswith("pass ")}
    assert "fetch_factor = 2.0000" in text and "write_factor = 1.0000" in text
    assert int(lines["fwd_row"][3]) == round(grid * 1.05) + grid
    assert int(lines["fwd_col"][3]) == 2 * grid
    assert "pass_kernel" in " ".join(lines["inv_col"]) and ", 1, false" in " ".join(lines["inv_col"])
    # the bench reads the figure back only while the source hash matches
    prof = tmp_path / "profile.txt"
    prof.write_text("# header\n" + text + "\n")
    monkeypatch.setattr(bench, "TRAFFIC_PROFILE", str(prof))
    assert bench.measured_traffic("fwd_col") == 2 * grid
    prof.write_text(text.replace(bench.kernel_source_hash(), "0" * 16))
    assert bench.measured_traffic("fwd_col") is None


def test_bench_refuses_more_than_one_gpu():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2 and "one GPU" in r.stderr


def test_cpu_configs_reports_the_error_of_each_result(monkeypatch):
    """bench.py's per-configuration error report: outputs equal to the oracle's
    (rounded to complex64) give errors at FP32 rounding level; a planted
    mistake (a conjugated result) is reported as an error of order one."""
    import bench
    import oracle
    import synth
    monkeypatch.setattr(bench, "ORACLE_CASES", [("a", (16, 32), 0), ("b", (3, 8, 4), 1), ("c", (2, 1, 64), 2)])
    monkeypatch.setattr(bench, "BATCHED_COUNT", 3)
    monkeypatch.setattr(synth, "pow2_shapes", lambda seed, count: [(8, 16), (4, 4), (32, 2)][:count])
    gpu = {name: oracle.fft2_forward(synth.complex_grid(seed, shape)).astype(np.complex64)
           for name, shape, seed in bench.ORACLE_CASES}
    gpu["b"] = np.conj(gpu["b"])
    monkeypatch.setattr(bench, "BACKWARD_CASE", ("d", (2, 8, 16), 3))
    gpu["d"] = oracle.adjoint(synth.complex_grid(3, (2, 8, 16)), oracle.FORWARD).astype(np.complex64)
    gpu["batched"] = [oracle.fft2_forward(x).astype(np.complex64)
                      for x in synth.batched_grids(bench.BATCHED_SEED, synth.pow2_shapes(bench.BATCHED_SEED, 3))]
    out = bench.cpu_configs(gpu)
    assert out["a"]["gpu_rel_l2"] < 1e-7 and out["c"]["gpu_rel_l2"] < 1e-7 and out["d"]["gpu_rel_l2"] < 1e-7
    assert out["a"]["gpu_max_elem"] < 1e-6 and out["d"]["gpu_max_elem"] < 1e-6
    assert out["b"]["gpu_rel_l2"] > 0.5 and out["b"]["gpu_max_elem"] > 0.5
    assert out["3 shapes 2^a x 2^b forward"]["gpu_rel_l2_max"] < 1e-7
    assert out["3 shapes 2^a x 2^b forward"]["gpu_max_elem_max"] < 1e-6


def test_counter_summary_means_per_pass(tmp_path):
    """--summarize-counters: dispatches assigned to passes in step order, the
    mean per launch of each counter, instruction counts per wave."""
    import bench
    names = ROUND_TRIP_NAMES
    a, b = [], []
    for step in range(2):
        for i, n in enumerate(names):
            d = 10 + step * 4 + i
            a.append([d, n, "SQ_WAVES", 100.0])
            a.append([d, n, "SQ_INSTS_VALU", 1000.0 * (i + 1) + 100.0 * step])
            b.append([d, n, "SQ_WAIT_ANY", 7.0])
    _write_counters(tmp_path / "a", a + [[1, "some_other_kernel", "SQ_WAVES", 1.0]])
    _write_counters(tmp_path / "b", b)
    text = bench.summarize_counters(str(tmp_path / "a"), str(tmp_path / "b"))
    blocks = {}
    for line in text.splitlines():
        f = line.split()
        if f[0] == "pass":
            cur = blocks.setdefault(f[1], {})
        else:
            cur[f[0]] = f
    assert float(blocks["fwd_row"]["SQ_INSTS_VALU"][1]) == 1050.0
    assert blocks["fwd_row"]["SQ_INSTS_VALU"][-1] == "10.5"  # per wave
    assert float(blocks["inv_col"]["SQ_INSTS_VALU"][1]) == 4050.0
    assert float(blocks["fwd_col"]["SQ_WAIT_ANY"][1]) == 7.0 and "per" not in blocks["fwd_col"]["SQ_WAIT_ANY"]


def test_element_bound_catches_a_wrong_tile_that_the_norm_misses():
    """The GPU tests' element-wise bound fails a result whose global relative
    L2 passes: a 16-column x 1024-row tile of a 4096^2-sized output off by 3e-4
    relative (planted on the CPU), and a single point off by 1 % of the RMS."""
    from tests.gpu_util import ELEM_TOL, TOL, errors
    rng = np.random.default_rng(0)
    ref = (rng.standard_normal((1024, 1024)) + 1j * rng.standard_normal((1024, 1024))) * 64.0
    good = ref * (1 + 2e-7)
    rel, mx = errors(good, ref)
    assert rel <= TOL and mx <= ELEM_TOL
    tile = ref.copy()
    tile[:256, 16:20] *= 1 + 3e-4  # 1/1024 of the points
    rel, mx = errors(tile, ref)
    assert rel <= TOL < mx
    spike = ref.copy()
    spike[5, 7] += 0.0095 * np.sqrt(np.mean(np.abs(ref) ** 2))
    rel, mx = errors(spike, ref)
    assert rel <= TOL < mx
    assert errors(np.zeros(4), np.zeros(4)) == (0.0, 0.0)


def test_batched_schedule_invariants(tmp_path):
    """The batched path's scheduler (csrc/fft_schedule.hpp, plain C++) on
    random shape sets, for every queue count, item order and group size: each
    tile appears once, a transform's items share one queue with all its row
    items before its column items, and groups tile the item table
    (tests/c/schedule_check.cpp)."""
    exe = str(tmp_path / "schedule_check")
    src = os.path.join(ROOT, "tests", "c", "schedule_check.cpp")
    subprocess.run(["g++", "-std=c++17", "-O2", "-Wall", "-Wextra", "-Werror", src, "-o", exe], check=True,
                   timeout=120)
    r = subprocess.run([exe, "120"], capture_output=True, text=True, timeout=300)
    assert r.returncode == 0 and r.stdout.startswith("ok "), r.stdout + r.stderr


def test_counter_summaries_reject_a_shifted_trace(tmp_path):
    """A profiled run with one dispatch missing (or one extra) would shift
    every later counter onto the wrong pass: the summaries check each
    dispatch's kernel (row or column pass, sign) and raise instead."""
    import bench
    rows = []
    for step in range(2):
        for i, n in enumerate(ROUND_TRIP_NAMES):
            rows.append([10 + step * 4 + i, n, "SQ_WAVES", 100.0])
    _write_counters(tmp_path / "ok", rows)
    assert "pass inv_col" in bench.summarize_counters(str(tmp_path / "ok"))
    _write_counters(tmp_path / "shifted", rows[1:])
    with pytest.raises(ValueError):
        bench.summarize_counters(str(tmp_path / "shifted"))
    # measurement variants and other kernels are not passes of the sequence
    probe = ROUND_TRIP_NAMES[0].replace("true, 0>", "true, 2>")
    assert bench.kernel_role(probe) == ("row-probe", -1)
    _write_counters(tmp_path / "extra", rows + [[99, probe, "SQ_WAVES", 1.0], [98, "copyBuffer", "SQ_WAVES", 1.0]])
    assert bench.summarize_counters(str(tmp_path / "extra")) == bench.summarize_counters(str(tmp_path / "ok"))
    # the other row-pass kernels: last stage across rows, one row per wave
    rx = "void fft2d::dev::rowx_kernel<fft2d::dev::Cfg<4096, 32, 4, 2, false, 16, 32, 8>, %d, 4, 0, true, %d>(fft2d::PassArgs)"
    rw = "void fft2d::dev::row_wave_kernel<fft2d::dev::Cfg<1024, 16, 1, 1, false, 16, 16, 4>, %d, true, %d>(fft2d::PassArgs)"
    assert bench.kernel_role(rx % (-1, 0)) == ("row", -1) and bench.kernel_role(rx % (1, 0)) == ("row", 1)
    assert bench.kernel_role(rx % (-1, 1)) == ("row-probe", -1)
    assert bench.kernel_role(rw % (1, 0)) == ("row", 1) and bench.kernel_role(rw % (-1, 2)) == ("row-probe", -1)
    fwd = [[i, n, "SQ_WAVES", 1.0] for i, n in enumerate(ROUND_TRIP_NAMES[:2] * 3)]
    _write_counters(tmp_path / "fwd", fwd)
    assert "pass fwd_col" in bench.summarize_counters(str(tmp_path / "fwd"), roles=bench.FORWARD_ROLES)
    with pytest.raises(ValueError):
        bench.summarize_counters(str(tmp_path / "fwd"))  # a forward-only trace is not a round trip


def test_tune_cache_parsing(tmp_path):
    """The batched tuner's cache (csrc/fft_tune_cache.hpp): a missing, empty,
    binary or malformed cache file yields no choice, so the plan tunes again
    (or keeps its defaults with FFT2D_TUNE=off) rather than using bad values;
    a valid line is found among junk and the last one for a key wins
    (tests/c/tune_cache_check.cpp)."""
    exe = str(tmp_path / "tune_cache_check")
    src = os.path.join(ROOT, "tests", "c", "tune_cache_check.cpp")
    subprocess.run(["g++", "-std=c++17", "-O2", "-Wall", "-Wextra", "-Werror", src, "-o", exe], check=True,
                   timeout=120)
    r = subprocess.run([exe, str(tmp_path)], capture_output=True, text=True, timeout=60)
    assert r.returncode == 0 and r.stdout.strip() == "ok", r.stdout + r.stderr


def test_batched_traffic_summary_uses_the_timed_dispatches(tmp_path):
    """The batched kernel's bytes per launch are the scaled mean over its last
    `timed` dispatches (tuning trials come first in a run and are left out);
    other kernels are ignored, and too few dispatches are an error."""
    import bench
    grid = 4096 * 4096 * 8
    kib = grid / 1024
    name = "fft2d::(anonymous namespace)::batched_kernel(fft2d::(anonymous namespace)::BatchArgs)"
    fetch = [[d, name, "FETCH_SIZE", 999.0] for d in range(1, 4)]  # tuning trials
    fetch += [[d, name, "FETCH_SIZE", 3000.0 + d] for d in (10, 11)]
    fetch += [[5, "some_other_kernel", "FETCH_SIZE", 1.0e9]]
    write = [[d, name, "WRITE_SIZE", 500.0] for d in range(1, 4)] + [[d, name, "WRITE_SIZE", 4000.0] for d in (10, 11)]
    _write_counters(tmp_path / "f", fetch)
    _write_counters(tmp_path / "w", write)
    _write_counters(tmp_path / "cf", [[1, "__amd_rocclr_copyBuffer", "FETCH_SIZE", kib / 2]])
    _write_counters(tmp_path / "cw", [[1, "__amd_rocclr_copyBuffer", "WRITE_SIZE", kib]])
    args = [str(tmp_path / d) for d in ("f", "w", "cf", "cw")]
    text = bench.summarize_batched_traffic(*args, timed=2)
    launch = [l.split() for l in text.splitlines() if l.startswith("launch ")][0]
    assert int(launch[4]) == round(3010.5 * 1024 * 2) and int(launch[6]) == round(4000.0 * 1024)
    assert int(launch[2]) == int(launch[4]) + int(launch[6])
    assert "fetch_factor = 2.0000" in text and "dispatches 2" in text
    with pytest.raises(ValueError):
        bench.summarize_batched_traffic(*args, timed=6)
