"""Host code under the sanitizers (CPU only).

* The oracle (oracle/oracle.c) with AddressSanitizer and
  UndefinedBehaviorSanitizer, leak detection on: every entry point on small
  graphs (tests/host/oracle_sanitize_check.c).
* The top-k driver's host logic (topk.cpp with the sequential and the
  parallel push-relabel of pflow.hpp, union-find over host threads) with
  AddressSanitizer and UndefinedBehaviorSanitizer, and again with
  ThreadSanitizer, running the battery of tests/host/host_logic_check.cpp.
  The sanitizers instrument the host side of the hipcc build only; nothing
  here runs on a GPU.

Each program prints "ok" and exits 0 when its checks hold; a sanitizer
report ends it with a non-zero status."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
HOST_ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1",
                TSAN_OPTIONS="halt_on_error=1")


def _hipcc():
    h = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    if os.path.exists(h):
        return h
    return shutil.which("hipcc")


def _run(exe, timeout):
    r = subprocess.run([exe], capture_output=True, text=True, timeout=timeout, env=HOST_ENV)
    assert r.returncode == 0 and r.stdout.startswith("ok"), (r.stdout + r.stderr)[-4000:]


def test_oracle_asan_ubsan(tmp_path):
    cc = shutil.which("gcc")
    if cc is None:
        pytest.skip("gcc not available")
    exe = str(tmp_path / "oracle_sanitize_check")
    src = os.path.join(HERE, "host", "oracle_sanitize_check.c")
    flags = ["-O1", "-g", "-std=gnu11", "-fno-omit-frame-pointer", "-fno-sanitize-recover=all"]
    san = ["-fsanitize=address,undefined"]
    r = subprocess.run([cc] + flags + san + [src, "-o", exe, "-lm"], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-2000:]
    _run(exe, 300)


def _host_logic(tmp_path, tag, host_flags):
    hipcc = _hipcc()
    if hipcc is None:
        pytest.skip("hipcc not available")
    exe = str(tmp_path / ("host_logic_" + tag))
    src = os.path.join(HERE, "host", "host_logic_check.cpp")
    cmd = [hipcc, "-O1", "-g", "-std=c++17", "-I" + os.path.join(ROOT, "include"),
           "-I" + os.path.join(ROOT, "paper_2504_10937_amd", "csrc"), "-pthread"] + host_flags + [src, "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-2000:]
    _run(exe, 600)


def test_host_logic_asan_ubsan(tmp_path):
    # each sanitizer flag applies to the host compilation only
    _host_logic(tmp_path, "asan", ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
                                   "-Xarch_host", "-fno-omit-frame-pointer",
                                   "-Xarch_host", "-fno-sanitize-recover=all"])


def test_host_logic_tsan(tmp_path):
    _host_logic(tmp_path, "tsan", ["-Xarch_host", "-fsanitize=thread", "-Xarch_host", "-fno-omit-frame-pointer"])
