"""Host logic of the library compiled for the CPU side only: the work list of
the polarizability contraction (tests/host/worklist_check.hip), and the
validation, plan and decomposition code under the address and
undefined-behaviour sanitizers (tests/host/host_logic_check.hip)."""
import os
import shutil
import subprocess
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def hipcc():
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if c and os.path.exists(c):
            return c
    return None


@pytest.mark.skipif(hipcc() is None, reason="hipcc not found")
def test_polarizability_worklist_covers_every_tile_once():
    src = os.path.join(ROOT, "tests", "host", "worklist_check.hip")
    with tempfile.TemporaryDirectory() as d:
        exe = os.path.join(d, "worklist_check")
        r = subprocess.run([hipcc(), "-O1", "-std=c++17", "--offload-arch=gfx950", "-Xclang", "-target-feature",
                            "-Xclang", "-packed-fp32-ops", "-I", os.path.join(ROOT, "include"), src, "-o", exe],
                           capture_output=True, text=True, timeout=600)
        assert r.returncode == 0, r.stderr[-2000:]
        r = subprocess.run([exe], capture_output=True, text=True, timeout=120)
        assert r.returncode == 0 and r.stdout.strip().endswith("ok"), r.stdout[-2000:]


@pytest.mark.skipif(hipcc() is None, reason="hipcc not found")
def test_host_logic_under_address_and_ub_sanitizers():
    """Argument validation, the workspace plan of many shapes, the skeleton
    decomposition, the fit ranges and the work lists (tests/host/
    host_logic_check.hip) run with the host side built under the address and
    undefined-behaviour sanitizers; a finding aborts the check."""
    src = os.path.join(ROOT, "tests", "host", "host_logic_check.hip")
    with tempfile.TemporaryDirectory() as d:
        exe = os.path.join(d, "host_logic_check")
        r = subprocess.run([hipcc(), "-O1", "-g", "-std=c++17", "--offload-arch=gfx950",
                            "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
                            "-fno-omit-frame-pointer", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
                            "-I", os.path.join(ROOT, "include"), src, "-o", exe],
                           capture_output=True, text=True, timeout=600)
        assert r.returncode == 0, r.stderr[-2000:]
        env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
                   UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
        r = subprocess.run([exe], capture_output=True, text=True, timeout=300, env=env)
        assert r.returncode == 0 and r.stdout.strip().endswith("ok"), (r.stdout[-2000:], r.stderr[-2000:])
