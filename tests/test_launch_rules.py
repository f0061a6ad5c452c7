"""Host-side launch rules of the library, checked without a GPU: the header
that holds them has no HIP dependency, so a small C++ program built with the
host compiler evaluates them here."""
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2208_10006_amd", "csrc")

PROGRAM = r"""
#include <cstdio>
#include "launch_rules.hpp"
int main() {
  const int tuned[] = {64, 128, 256, 512, 1024};
  const int stack[] = {2 * 44, 4 * 16, 4 * 32, 4 * 64, 100000};
  for (int t : tuned)
    for (int s : stack) std::printf("%d %d %d\n", t, s, sbr::replay_block_for(t, (std::size_t)s));
  return 0;
}
"""


@pytest.fixture(scope="module")
def rules(tmp_path_factory):
    d = tmp_path_factory.mktemp("rules")
    src, exe = d / "rules.cpp", d / "rules"
    src.write_text(PROGRAM)
    subprocess.check_call(["g++", "-std=c++17", "-O1", "-I", CSRC, str(src), "-o", str(exe)])
    out = subprocess.check_output([str(exe)], text=True)
    return [tuple(int(x) for x in line.split()) for line in out.splitlines()]


def test_replay_block_fits_lds(rules):
    """The capture replay keeps one traversal stack per thread in LDS: the
    block size is the tuned one, cut in whole waves until the stacks fit the
    64 KiB a workgroup may allocate (one wave at least)."""
    for tuned, stack, rb in rules:
        assert rb % 64 == 0 and 64 <= rb <= tuned, (tuned, stack, rb)
        if rb > 64:
            assert rb * stack <= 65536, (tuned, stack, rb)
        if rb < tuned:  # cut only as far as needed
            assert (rb + 64) * stack > 65536, (tuned, stack, rb)
    got = {(t, s): rb for t, s, rb in rules}
    assert got[(1024, 4 * 64)] == 256      # 64-entry stacks: 256 threads at most
    assert got[(1024, 2 * 44)] == 704      # 44 two-byte entries
    assert got[(256, 4 * 32)] == 256       # fits as tuned
    assert got[(64, 100000)] == 64         # never below one wave
