"""Host code of the library under AddressSanitizer and UndefinedBehaviorSanitizer.

Every library source is compiled with the sanitizers on its host side only
(`-Xarch_host`; the device code is built as usual and never launched here),
linked with the C driver `host_sanitize/abi_errors.c`, and run: the driver
calls every C-ABI entry point on its documented error paths (null plans and
buffers, degrees, methods and curve kinds out of range, knot vectors that are
not open or not simple, malformed curves, a valid patch that no device can
take) and checks each status and message. A sanitizer report (invalid access,
leak, undefined behaviour) fails the run as well.

Runs where there is no GPU: with one, the valid descriptor would build a plan.
"""
import os
import shutil
import subprocess
from concurrent.futures import ThreadPoolExecutor

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2101_08053_amd", "csrc")
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")
HIPCC = os.path.join(ROCM, "bin", "hipcc")
CLANG = os.path.join(ROCM, "llvm", "bin", "clang")

pytestmark = [
    pytest.mark.skipif(not (os.path.exists(HIPCC) and os.path.exists(CLANG)), reason="ROCm toolchain not found"),
    pytest.mark.skipif(os.path.exists("/dev/kfd"), reason="host-only checks; a GPU is present"),
]

HOST_SAN = ["-Xarch_host", "-fsanitize=address",
            "-Xarch_host", "-fsanitize=undefined",
            "-Xarch_host", "-fno-omit-frame-pointer", "-Xarch_host", "-g"]


def _run(cmd):
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, f"{' '.join(cmd)}\n{r.stderr[-3000:]}"


def test_abi_error_paths_under_sanitizers(tmp_path):
    srcs = sorted(f for f in os.listdir(CSRC) if f.endswith(".hip"))
    objs = [str(tmp_path / (f[:-4] + ".o")) for f in srcs]

    def compile_one(i):
        _run([HIPCC, "-O1", "-std=c++17", "-fPIC", *HOST_SAN, "--offload-arch=gfx950",
              "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
              "-I", os.path.join(ROOT, "include"), "-Wno-unused-command-line-argument",
              "-c", os.path.join(CSRC, srcs[i]), "-o", objs[i]])

    with ThreadPoolExecutor(max_workers=min(8, os.cpu_count() or 1)) as ex:
        list(ex.map(compile_one, range(len(srcs))))
    drv = str(tmp_path / "abi_errors.o")
    exe = str(tmp_path / "abi_errors")
    san = "-fsanitize=address,undefined"
    _run([CLANG, "-O1", "-g", san, "-fno-omit-frame-pointer", "-I", os.path.join(ROOT, "include"),
          "-c", os.path.join(ROOT, "tests", "host_sanitize", "abi_errors.c"), "-o", drv])
    _run([CLANG + "++", san, drv, *objs, "-L" + os.path.join(ROCM, "lib"), "-lamdhip64",
          "-Wl,-rpath," + os.path.join(ROCM, "lib"), "-o", exe])

    env = dict(os.environ,
               ASAN_OPTIONS="detect_leaks=1:halt_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=120)
    report = r.stdout[-4000:] + r.stderr[-4000:]
    assert r.returncode == 0, report
    assert "all checks passed" in r.stdout, report
    for marker in ("AddressSanitizer", "LeakSanitizer", "runtime error:"):
        assert marker not in r.stderr, report
    assert r.stdout.count("\nok ") + r.stdout.startswith("ok ") >= 50, report
    shutil.rmtree(tmp_path, ignore_errors=True)
