"""Host code under AddressSanitizer, UndefinedBehaviorSanitizer and ThreadSanitizer (CPU only).

The FP64 oracle (``oracle/bp_oracle.c``, multithreaded over z-planes and voxel lists) is built
with ASan + UBSan and with TSan around a driver that runs its entries on several threads; the
library's host-only matrix composition (``bp_geometry.cpp``) is built with ASan + UBSan around a
driver of its own.  Each build must run clean: exit status 0 and no sanitizer report.  (The
serving scheduler is Python: its cross-thread cancellation is tested in ``test_serve``.)
"""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HERE = os.path.join(ROOT, "tests", "sanitize")
ORACLE = os.path.join(ROOT, "oracle", "bp_oracle.c")
GEOMETRY = os.path.join(ROOT, "paper_1401_7494_amd", "csrc", "bp_geometry.cpp")

pytestmark = pytest.mark.skipif(shutil.which("gcc") is None or shutil.which("g++") is None,
                                reason="needs gcc and g++")

REPORTS = ("AddressSanitizer", "ThreadSanitizer", "runtime error", "LeakSanitizer")


def _build_and_run(cmd, exe, env_extra):
    subprocess.run(cmd + ["-o", exe], check=True, capture_output=True, text=True)
    env = dict(os.environ, **env_extra)
    env.pop("LD_PRELOAD", None)  # a sanitizer runtime must come first in the process
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    out = r.stdout + r.stderr
    assert r.returncode == 0, out
    assert not any(s in out for s in REPORTS), out
    return out


@pytest.mark.parametrize("san", ["address,undefined", "thread"])
def test_oracle_under_sanitizers(tmp_path, san):
    exe = str(tmp_path / f"oracle_{san.split(',')[0]}")
    cmd = ["gcc", "-O1", "-g", "-std=c99", f"-fsanitize={san}", "-fno-omit-frame-pointer", "-pthread",
           "-fno-sanitize-recover=undefined" if "undefined" in san else "-fno-common",
           ORACLE, os.path.join(HERE, "oracle_driver.c"), "-lm"]
    env = {"ASAN_OPTIONS": "detect_leaks=1:abort_on_error=0", "TSAN_OPTIONS": "halt_on_error=1",
           "UBSAN_OPTIONS": "halt_on_error=1:print_stacktrace=1"}
    assert "oracle driver ok" in _build_and_run(cmd, exe, env)


def test_host_geometry_under_asan(tmp_path):
    exe = str(tmp_path / "geometry_asan")
    cmd = ["g++", "-O1", "-g", "-std=c++17", "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
           "-fno-omit-frame-pointer", "-I", os.path.join(ROOT, "include"), GEOMETRY,
           os.path.join(HERE, "geometry_driver.cpp")]
    env = {"ASAN_OPTIONS": "detect_leaks=1", "UBSAN_OPTIONS": "halt_on_error=1:print_stacktrace=1"}
    assert "geometry driver ok" in _build_and_run(cmd, exe, env)
