"""The library's host code under AddressSanitizer and
UndefinedBehaviorSanitizer (CPU only).

The library sources are compiled with the sanitizers on host code only
(`-Xarch_host`; device code is built as usual) and linked with
`tests/cpu/host_checks.cpp`, a driver that makes host-only C-ABI calls:
circuit creation with adjacent and distant pairs, the compiled circuit,
light cones, cut bounds, validation errors and the all-outputs count.  Any
sanitizer report or failed check fails the test."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2510_26408_amd", "csrc")
SOURCES = ["api.cpp", "serve.cpp", "pool.cpp", "graph.cpp", "noalloc.hip", "tables.hip", "plan.hip", "frontier.hip",
           "dfs.hip", "reduce.hip", "contract.hip", "join.hip", "keys.hip"]

pytestmark = pytest.mark.slow


def _hipcc():
    for cand in (shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    return None


def test_host_code_under_address_and_ub_sanitizers(tmp_path):
    cc = _hipcc()
    if cc is None:
        pytest.skip("hipcc not available")
    exe = str(tmp_path / "host_checks")
    san = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
           "-Xarch_host", "-fno-sanitize-recover=undefined", "-Xarch_host", "-fno-omit-frame-pointer"]
    cmd = ([cc, "-O1", "-g", "-std=c++17", "--offload-arch=gfx950", "-I", os.path.join(ROOT, "include"), "-I", CSRC,
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", "-Wno-unused-command-line-argument"]
           + san + ["-x", "hip"] + [os.path.join(CSRC, s) for s in SOURCES]
           + ["-x", "none", os.path.join(ROOT, "tests", "cpu", "host_checks.cpp"), "-o", exe])
    subprocess.run(cmd, check=True, capture_output=True)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=0:halt_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    out = r.stdout + r.stderr
    assert r.returncode == 0, out[-4000:]
    assert "0 failures" in r.stdout
    assert "ERROR: AddressSanitizer" not in out and "runtime error" not in out, out[-4000:]
