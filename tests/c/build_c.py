"""Builds the plain-C client of the C ABI (``tests/c/abi_roundtrip``) with gcc
against ``include/fft2d.h``, the in-tree ``libfft2d.so`` and the HIP runtime."""

from __future__ import annotations

import os
import shutil
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
BIN = os.path.join(HERE, "abi_roundtrip")


def build() -> str:
    rocm = os.environ.get("ROCM_PATH", "/opt/rocm")
    cc = shutil.which("gcc") or "gcc"
    pkg = os.path.join(ROOT, "paper_2506_15437_amd")
    cmd = [cc, "-std=c11", "-O2", "-Wall", "-Wextra", "-D__HIP_PLATFORM_AMD__",
           "-I" + os.path.join(ROOT, "include"), "-I" + os.path.join(rocm, "include"),
           os.path.join(HERE, "abi_roundtrip.c"), "-o", BIN,
           "-L" + pkg, "-lfft2d", "-Wl,-rpath," + pkg, "-Wl,-rpath,$ORIGIN/../../paper_2506_15437_amd",
           "-L" + os.path.join(rocm, "lib"), "-lamdhip64", "-Wl,-rpath," + os.path.join(rocm, "lib")]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("C client build failed: %s\n%s%s" % (" ".join(cmd), r.stdout, r.stderr))
    return BIN


if __name__ == "__main__":
    print(build())
