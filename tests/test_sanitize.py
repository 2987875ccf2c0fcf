"""Sanitizer builds on the CPU: the oracle, and the host-side paths of the
library that run without a GPU, compiled with AddressSanitizer and
UndefinedBehaviorSanitizer (host code only; no GPU code is built with a
sanitizer) and driven through their C interfaces.  Any report aborts the
driver and fails the test."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN_ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")


def _run(exe):
    r = subprocess.run([exe], capture_output=True, text=True, env=SAN_ENV, timeout=300)
    out = r.stdout + r.stderr
    assert r.returncode == 0, out[-4000:]
    assert "ERROR: AddressSanitizer" not in out and "runtime error" not in out, out[-4000:]
    return out


def test_oracle_under_sanitizers(tmp_path):
    if not shutil.which("g++"):
        pytest.skip("no g++")
    exe = str(tmp_path / "oracle_san")
    subprocess.run(["g++", "-std=c++17", "-O1", "-g", "-pthread", "-ffp-contract=off",
                    "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
                    "-fno-omit-frame-pointer", "-o", exe,
                    os.path.join(ROOT, "tests", "sanitize_oracle.cpp")], check=True)
    assert "oracle sanitize: ok" in _run(exe)


def test_library_host_paths_under_sanitizers(tmp_path):
    if not shutil.which("hipcc"):
        pytest.skip("no hipcc")
    exe = str(tmp_path / "host_san")
    csrc = os.path.join(ROOT, "paper_1803_01237_amd", "csrc")
    srcs = sorted(os.path.join(csrc, f) for f in os.listdir(csrc) if f.endswith(".hip"))
    # the sanitizers go to the host compilation only
    cmd = ["hipcc", "--offload-arch=gfx950", "-std=c++17", "-O1", "-g",
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
           "-Xarch_host", "-fsanitize=address,undefined", "-Xarch_host", "-fno-sanitize-recover=all",
           "-Xarch_host", "-fno-omit-frame-pointer",
           "-I" + os.path.join(ROOT, "include"), "-o", exe,
           os.path.join(ROOT, "tests", "sanitize_host.cpp"), *srcs]
    subprocess.run(cmd, check=True, capture_output=True)
    assert "host sanitize: ok" in _run(exe)
