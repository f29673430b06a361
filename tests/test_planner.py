"""CPU programs built with g++ and the host AddressSanitizer/UBSan.

The host-side recursion planner (csrc/planner.hpp) on the CPU: a C++
program built with g++ and the host AddressSanitizer/UBSan checks how one
level's bucket bounds become base-case bins and next-level subproblems --
bins pairwise disjoint (they are sorted at the same time), inside their task
and caller segment, every bucket of 2..cap elements in exactly one bin, no
bin touching a recursed bucket -- on hand-built cases (among them two tasks
with an earlier level's binned bucket between them) and random recursions."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.mark.skipif(shutil.which("g++") is None, reason="g++ not available")
def test_planner_bins(tmp_path):
    exe = str(tmp_path / "planner_check")
    subprocess.check_call(["g++", "-std=c++17", "-O1", "-g", "-fsanitize=address,undefined",
                           "-fno-sanitize-recover=all", "-o", exe, os.path.join(HERE, "planner_check.cpp")])
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "planner ok" in r.stdout


@pytest.mark.skipif(shutil.which("g++") is None, reason="g++ not available")
def test_permutation_word(tmp_path):
    """The permutation's packed (w, r, readers) word (csrc/wrword.hpp): field
    arithmetic at every extreme and a simulated claim/read/write
    interleaving in which a writer of a block that was full at the start
    always sees its reader counted."""
    exe = str(tmp_path / "wrword_check")
    subprocess.check_call(["g++", "-std=c++17", "-O1", "-g", "-fsanitize=address,undefined",
                           "-fno-sanitize-recover=all", "-o", exe, os.path.join(HERE, "wrword_check.cpp")])
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "wrword ok" in r.stdout
