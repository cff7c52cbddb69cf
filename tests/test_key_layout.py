"""The split contraction's grouping buffers across calls of different batch
sizes on one circuit (host bookkeeping, CPU only).

`tests/cpu/key_layout_check.cpp` replays on host memory what the insert and
jobs kernels do to the hash table and slot hulls, through the index functions
of `csrc/key_layout.h` that the kernels use, and checks that every slot a
call claims starts empty and every key's hull equals its members' hull.

The per-call layout (the two halves `cap` rows apart, cleared only when a
buffer is reallocated) is replayed too: a smaller call after a larger one
then reads its upper hull bounds from rows that held the larger call's lower
bounds (0x7f7f7f7f), which made the contraction jobs' intervals, their state
sizes and the join's strides far larger than the states they index.
"""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "tests", "cpu", "key_layout_check.cpp")
INC = os.path.join(ROOT, "paper_2510_26408_amd", "csrc")
SPAN_C2 = 9 * 15   # (depth + 1) x (m - 1) of the 16-mode, depth-8 workload


@pytest.fixture(scope="module")
def checker(tmp_path_factory):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not available")
    exe = str(tmp_path_factory.mktemp("klc") / "key_layout_check")
    subprocess.check_call([gxx, "-O1", "-std=c++17", "-I", INC, "-o", exe, SRC])
    return exe


def run(exe, layout, sizes, span=SPAN_C2):
    r = subprocess.run([exe, layout, str(span)] + [str(b) for b in sizes], capture_output=True, text=True)
    return r.returncode, r.stdout


@pytest.mark.parametrize("sizes", [
    [32768, 4096],               # the batch sizes of the large-batch test
    [4096, 904],                 # a 5000-pattern batch in passes of 4096
    [4096, 1000, 4096],
    [64, 4096, 904, 32768, 100, 5000],
])
def test_stride_layout_keeps_claimed_rows_empty(checker, sizes):
    rc, out = run(checker, "stride", sizes)
    assert rc == 0, out
    assert out.count(" ok") == len(sizes)


@pytest.mark.parametrize("sizes", [[32768, 4096], [4096, 904]])
def test_per_call_layout_reads_stale_upper_bounds(checker, sizes):
    # a smaller call after a larger one: the model must see the stale rows
    rc, out = run(checker, "per-call", sizes)
    assert rc == 1, out
    assert "stale hull row" in out and str(0x7F7F7F7F) in out


def test_growing_sizes_are_cleared_in_both_layouts(checker):
    # growth reallocates and clears in both layouts: the failure needs a
    # smaller call after a larger one
    for layout in ("stride", "per-call"):
        rc, out = run(checker, layout, [64, 4096, 32768])
        assert rc == 0, out
