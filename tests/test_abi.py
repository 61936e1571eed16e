"""CPU-only checks of the C ABI: the library loads, exports every declared
symbol, and rejects bad arguments before touching the GPU."""

from __future__ import annotations

import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "fft2d.h")


def _declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(fft2d_[a-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def L():
    from paper_2506_15437_amd import _lib
    return _lib


def test_header_declares_the_entry_points():
    names = _declared_functions()
    for required in ("fft2d_plan", "fft2d_exec", "fft2d_exec_batched", "fft2d_backward"):
        assert required in names


def test_library_exports_every_declared_symbol(L):
    names = _declared_functions()
    assert sorted(L.EXPORTS) == names
    raw = ctypes.CDLL(L.LIB_PATH)
    for n in names:
        assert hasattr(raw, n), n


def test_status_strings_and_version(L):
    assert L.status_string(0) == "success"
    for code in range(1, 12):
        s = L.status_string(code)
        assert s and s != "unknown status"
    assert L.status_string(99) == "unknown status"
    assert L.version() >= 100


@pytest.mark.parametrize("shape", [(1, 0, 8), (1, 8, 0), (1, 3, 8), (1, 8, 12), (1, 32768, 2), (1, 2, 32768),
                                   (0, 8, 8), (-1, 8, 8), (1, -4, 8)])
def test_plan_rejects_bad_sizes(L, shape):
    with pytest.raises(L.Fft2dError) as e:
        L.fft2d_plan(*shape)
    assert e.value.status == 2


def test_plan_rejects_null_out(L):
    st = L.lib.fft2d_plan(None, 1, 8, 8)
    assert st == 1


def test_batched_plan_validation(L):
    with pytest.raises(L.Fft2dError) as e:
        L.fft2d_plan_batched([64, 48], [64, 64])
    assert e.value.status == 2
    with pytest.raises(L.Fft2dError) as e:
        L.fft2d_plan_batched([], [])
    assert e.value.status == 2
    assert L.lib.fft2d_plan_batched(None, 1, None, None) == 1


def test_exec_rejects_null_and_dead_plans(L):
    assert L.lib.fft2d_exec(None, 8, 8, -1, None) == 1
    assert L.lib.fft2d_backward(None, 8, 8, -1, None) == 1
    # A handle that was never created is not live: rejected without being dereferenced.
    bogus = ctypes.c_void_p(0x1000)
    assert L.lib.fft2d_exec(bogus, 8, 8, -1, None) == 8
    assert "not live" in L.last_error()
    assert L.lib.fft2d_exec_batched(bogus, None, None, -1, None) == 8
    assert L.lib.fft2d_exec_pass(None, 8, 8, -1, 0, None) == 1
    assert L.lib.fft2d_exec_pass(bogus, 8, 8, -1, 0, None) == 8
    # the timed pass checks its events first, then the plan like fft2d_exec_pass
    assert L.lib.fft2d_exec_pass_timed(bogus, 8, 8, -1, 0, None, 16, None) == 1
    assert L.lib.fft2d_exec_pass_timed(bogus, 8, 8, -1, 0, 16, None, None) == 1
    assert "event" in L.last_error()
    assert L.lib.fft2d_exec_pass_timed(None, 8, 8, -1, 0, 16, 16, None) == 1
    assert L.lib.fft2d_exec_pass_timed(bogus, 8, 8, -1, 0, 16, 16, None) == 8
    # the ablated pass checks its ablation and events first, then the plan like fft2d_exec_pass
    assert L.lib.fft2d_exec_pass_ablated(bogus, 8, 8, 0, 3, None, None, None) == 3
    assert L.lib.fft2d_exec_pass_ablated(bogus, 8, 8, 0, 1, 16, None, None) == 1
    assert L.lib.fft2d_exec_pass_ablated(None, 8, 8, 0, 2, None, None, None) == 1
    assert L.lib.fft2d_exec_pass_ablated(bogus, 8, 8, 0, 1, None, None, None) == 8
    assert L.lib.fft2d_destroy(bogus) == 8
    assert L.lib.fft2d_destroy(None) == 0
    buf = ctypes.create_string_buffer(16)
    assert L.lib.fft2d_plan_describe(bogus, buf, 16) == 8
    n = ctypes.c_int64(-1)
    assert L.lib.fft2d_plan_twiddles(None, 0, None, 0, ctypes.byref(n)) == 1
    assert L.lib.fft2d_plan_twiddles(bogus, 0, None, 0, None) == 1
    assert L.lib.fft2d_plan_twiddles(bogus, 0, None, 0, ctypes.byref(n)) == 8


def test_last_error_is_thread_local(L):
    import threading
    with pytest.raises(L.Fft2dError):
        L.fft2d_plan(1, 3, 3)
    main_msg = L.last_error()
    seen = []

    def other():
        seen.append(L.last_error())

    th = threading.Thread(target=other)
    th.start()
    th.join()
    assert main_msg and seen == [""]


def test_product_package_does_not_import_the_oracle():
    import subprocess
    import sys
    code = ("import sys; import paper_2506_15437_amd; "
            "bad = [m for m in sys.modules if m == 'oracle' or m.startswith('oracle.')]; "
            "print(bad); sys.exit(1 if bad else 0)")
    r = subprocess.run([sys.executable, "-c", code], cwd=ROOT, capture_output=True, text=True)
    assert r.returncode == 0, r.stdout + r.stderr
    for dirpath, _, files in os.walk(os.path.join(ROOT, "paper_2506_15437_amd")):
        for f in files:
            if f.endswith((".py", ".cpp", ".hip", ".h")):
                src = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in src and "from oracle" not in src, f
                assert "fft_oracle" not in src, f


def test_noalloc_rejects_bad_arguments_before_touching_the_gpu(L):
    """fft2d_exec_noalloc validates sizes, direction and pointers on the host
    (no device call is made for a rejected call)."""
    f = L.lib.fft2d_exec_noalloc
    assert f(1, 3, 8, 16, 32, -1, None) == 2
    assert f(0, 8, 8, 16, 32, -1, None) == 2
    assert f(1, 8, 32768, 16, 32, -1, None) == 2
    assert f(1 << 30, 256, 256, 16, 32, -1, None) == 2  # beyond 2^35 points
    assert f(1, 8, 8, None, 32, -1, None) == 1
    assert f(1, 8, 8, 16, 32, 0, None) == 3
    assert f(1, 8, 8, 12, 1024, -1, None) == 4
    assert f(1, 64, 64, 16, 24, -1, None) == 9
    assert "overlap" in L.last_error()


def test_dft16_probe_rejects_bad_arguments_before_touching_the_gpu(L):
    f = L.lib.fft2d_probe_dft16
    assert f(2, 16, 8192, 64, 8, None, None, None) == 3
    assert f(0, None, 8192, 64, 8, None, None, None) == 1
    assert f(0, 16, 8192, 64, 8, 16, None, None) == 1
    for count, reps in ((0, 8), (63, 8), (96, 8), (64, 0), (64, 12), (64, 8192), (1 << 27, 8)):
        assert f(1, 16, 1 << 40, count, reps, None, None, None) == 2, (count, reps)
    assert f(1, 12, 1 << 40, 64, 8, None, None, None) == 4
    assert f(1, 16, 24, 64, 8, None, None, None) == 9


def test_pattern_probes_reject_bad_arguments_before_touching_the_gpu(L):
    """fft2d_probe_tile_copy validates pointers, tile width, shape, alignment
    and overlap, and fft2d_probe_lds its width and pointers, on the host."""
    f = L.lib.fft2d_probe_tile_copy
    big = 1 << 40
    assert f(None, big, 2048, 64, 16, 1, 0, None, None, None) == 1
    assert f(16, big, 2048, 64, 16, 1, 0, 16, None, None) == 1
    for rows, cols, tc, res in ((2048, 64, 8, 1), (1000, 64, 16, 1), (2048, 64, 16, 0), (2048, 60, 16, 1),
                                (4096, 64, 16, 3), (1 << 15, 1 << 14, 16, 1)):
        assert f(16, big, rows, cols, tc, res, 0, None, None, None) == 2, (rows, cols, tc, res)
    assert f(12, big, 2048, 64, 16, 1, 0, None, None, None) == 4
    assert f(16, 24, 2048, 64, 16, 1, 0, None, None, None) == 9
    import ctypes
    g = L.lib.fft2d_probe_lds
    n = ctypes.c_int64(0)
    assert g(8, 0, None, 1 << 20, ctypes.byref(n), None, None, None) == 1
    assert g(8, 0, 16, 1 << 20, None, None, None, None) == 1
    assert g(12, 0, 16, 1 << 20, ctypes.byref(n), None, None, None) == 2
    assert g(8, 1, 16, 1 << 20, ctypes.byref(n), 16, None, None) == 1
