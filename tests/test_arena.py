"""Host-side check of the server's device-arena allocator (plain C++, compiled with g++).

Random alloc / release sequences must never hand out overlapping ranges,
must keep the free list coalesced, and must return to one free range."""
import os
import subprocess
import textwrap

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

DRIVER = textwrap.dedent(r"""
    #include <cstdio>
    #include <cstdlib>
    #include <map>
    #include <vector>
    #include "arena.hpp"
    int main() {
      const int64_t size = 64ll << 20;
      otkm::Arena a(size);
      std::map<int64_t, int64_t> live;  // offset -> rounded size
      unsigned seed = 12345;
      auto rnd = [&]() { seed = seed * 1103515245u + 12345u; return (seed >> 8); };
      for (int step = 0; step < 200000; ++step) {
        if (live.empty() || rnd() % 3 != 0) {
          const int n = 1 + rnd() % 1500;
          const int64_t bytes = 4ll * n * n;          // a cost matrix
          const int64_t off = a.alloc(bytes);
          if (off < 0) continue;
          const int64_t r = otkm::Arena::round(bytes);
          if (off % otkm::Arena::kAlign || off + r > size) { printf("bad range\n"); return 1; }
          auto nx = live.lower_bound(off);
          if (nx != live.end() && nx->first < off + r) { printf("overlap next\n"); return 1; }
          if (nx != live.begin()) { auto pv = std::prev(nx); if (pv->first + pv->second > off) { printf("overlap prev\n"); return 1; } }
          live[off] = r;
        } else {
          auto it = live.begin();
          std::advance(it, rnd() % live.size());
          a.release(it->first, it->second);
          live.erase(it);
        }
        int64_t prev_end = -1;
        for (auto &f : a.free_ranges()) {
          if (f.first <= prev_end) { printf("free list not coalesced\n"); return 1; }
          prev_end = f.first + f.second;
        }
      }
      for (auto &l : live) a.release(l.first, l.second);
      if (a.free_ranges().size() != 1 || a.used() != 0) { printf("not fully coalesced\n"); return 1; }
      printf("ok\n");
      return 0;
    }
""")


def test_arena_never_overlaps(tmp_path):
    src = tmp_path / "arena_check.cpp"
    src.write_text(DRIVER)
    exe = tmp_path / "arena_check"
    subprocess.run(["g++", "-O2", "-std=c++17", "-I", os.path.join(ROOT, "paper_2005_01182_amd", "csrc"), str(src),
                    "-o", str(exe)], check=True)
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0 and r.stdout.strip() == "ok", r.stdout + r.stderr
