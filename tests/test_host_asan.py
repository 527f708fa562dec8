"""Host AddressSanitizer and UndefinedBehaviorSanitizer runs (CPU only):
the oracle on small and degenerate lattices, and the C-ABI's argument
validation (every path that returns before any device work).  The HIP
library's host code is built with the sanitizers on its host side only."""
import os
import shutil
import subprocess

import pytest

from conftest import ROOT

ASAN_DIR = os.path.join(ROOT, "tests", "asan")
CSRC = os.path.join(ROOT, "paper_1702_01690_amd", "csrc")
SAN_ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")


def _run(exe):
    r = subprocess.run([exe], capture_output=True, text=True, env=SAN_ENV, timeout=300)
    print(r.stdout, r.stderr)
    assert r.returncode == 0, r.stderr[-4000:]
    assert "ERROR: AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr


def test_oracle_under_host_sanitizers(tmp_path):
    exe = str(tmp_path / "oracle_asan")
    subprocess.run(["gcc", "-std=c11", "-O1", "-g", "-fsanitize=address,undefined", "-fno-omit-frame-pointer",
                    "-fno-sanitize-recover=all", "-I", os.path.join(ROOT, "oracle"),
                    os.path.join(ROOT, "oracle", "olb_oracle.c"), os.path.join(ASAN_DIR, "oracle_driver.c"),
                    "-o", exe, "-lm"], check=True)
    _run(exe)


@pytest.mark.skipif(shutil.which("hipcc") is None, reason="needs hipcc")
def test_abi_validation_under_host_sanitizers(tmp_path):
    # device code is compiled as usual; the sanitizers apply to host code only
    flags = ["hipcc", "--offload-arch=gfx950", "-std=c++17", "-O1", "-g",
             "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
             "-fno-omit-frame-pointer", "-I", os.path.join(ROOT, "include"), "-w"]
    srcs = [os.path.join(CSRC, s) for s in ("olb_kernels.hip", "olb_runtime.hip", "olb_closure.hip")]
    srcs.append(os.path.join(ASAN_DIR, "abi_driver.cpp"))
    objs = [str(tmp_path / (os.path.basename(s) + ".o")) for s in srcs]
    procs = [subprocess.Popen(flags + ["-c", s, "-o", o]) for s, o in zip(srcs, objs)]
    assert all(p.wait() == 0 for p in procs)
    exe = str(tmp_path / "abi_asan")
    subprocess.run(flags + objs + ["-o", exe], check=True)
    _run(exe)
