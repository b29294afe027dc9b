"""CPU check of the workspace arena's bookkeeping (csrc/arena.hpp).

Blocking calls and serving requests take their workspace ranges from the one
arena under the context lock; the property that keeps them from corrupting
each other's scratch is that ranges in use never overlap and stay inside the
workspace.  A small C++ driver (compiled here with g++, host code only)
replays random interleavings of allocations (tickets and blocking leases)
and releases and checks that property after every step, plus the
first-fit and alignment rules."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HDR = os.path.join(ROOT, "paper_1906_04572_amd", "csrc")

DRIVER = r"""
#include <cstdio>
#include <cstdlib>
#include <random>
#include "arena.hpp"
using corutv::Arena;

static int check(const Arena& a, size_t cap) {
  const auto& r = a.ranges();
  for (size_t i = 0; i < r.size(); ++i) {
    if (r[i].first % 256 != 0) return 1;
    if (r[i].second > cap || r[i].first > r[i].second) return 2;
    if (i && r[i].first < r[i - 1].second) return 3;  // overlap
  }
  return 0;
}

int main() {
  // first fit and alignment
  Arena a(4096);
  size_t o1, o2, o3, o4;
  if (!a.alloc(1000, &o1) || o1 != 0) return 10;
  if (!a.alloc(1000, &o2) || o2 != 1024) return 11;
  if (!a.alloc(2000, &o3) || o3 != 2048) return 12;
  if (a.alloc(1, &o4)) return 13;          // full (4048 used, next at 4096)
  if (!a.release(o2) || a.release(o2)) return 14;
  if (!a.alloc(1024, &o4) || o4 != 1024) return 15;  // the hole is reused
  if (a.alloc(1025, &o4)) return 16;
  // random interleavings: tickets (several live) and a blocking lease
  std::mt19937_64 g(12345);
  for (int trial = 0; trial < 200; ++trial) {
    const size_t cap = 256 * (1 + g() % 4000);
    Arena b(cap);
    std::vector<size_t> live;
    for (int step = 0; step < 2000; ++step) {
      const int op = g() % 3;
      if (op < 2) {
        size_t off, bytes = 1 + g() % (cap / 3 + 1);
        if (b.alloc(bytes, &off)) live.push_back(off);
      } else if (!live.empty()) {
        const size_t i = g() % live.size();
        if (!b.release(live[i])) return 20;
        live.erase(live.begin() + i);
      }
      const int rc = check(b, cap);
      if (rc) {
        std::printf("trial %d step %d: rule %d broken\n", trial, step, rc);
        return 30 + rc;
      }
      if (b.ranges().size() != live.size()) return 40;
    }
  }
  std::printf("arena ok\n");
  return 0;
}
"""


def test_arena_ranges_never_overlap(tmp_path):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not available")
    src = tmp_path / "arena_check.cpp"
    src.write_text(DRIVER)
    exe = tmp_path / "arena_check"
    subprocess.run([gxx, "-std=c++17", "-O1", "-I", HDR, str(src), "-o", str(exe)], check=True,
                   capture_output=True, timeout=120)
    out = subprocess.run([str(exe)], capture_output=True, text=True, timeout=120)
    assert out.returncode == 0, (out.returncode, out.stdout)
    assert "arena ok" in out.stdout
