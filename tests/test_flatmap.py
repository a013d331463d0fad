"""The host library's open-addressing table (FlatMap in csrc/mesh.hpp, used
for the octree's nodes and the leaf-id lookups of the plan build and the
remesh decisions) against std::map under random inserts, overwrites,
erasures (backward-shift deletion, including runs that wrap around the end of
the table) and lookups, with keys packed as the octree packs them and keys
chosen to collide.  Compiled with g++ on the host."""
import os
import subprocess
import tempfile

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "..", "paper_1810_01319_amd", "csrc")

PROG = r"""
#include <cstdio>
#include <map>
#include <random>
#include "mesh.hpp"
using amr::FlatMap;
static uint64_t pk(int l, int i, int j, int k) {
  return (uint64_t(l) << 60) | (uint64_t(k) << 40) | (uint64_t(j) << 20) | uint64_t(i);
}
int main() {
  std::mt19937_64 rng(12345);
  long checks = 0;
  for (int round = 0; round < 40; round++) {
    FlatMap<int32_t> f;
    std::map<uint64_t, int32_t> ref;
    const int span = 4 + round % 13;  // small key spaces force long probe runs
    const int ops = 20000;
    for (int o = 0; o < ops; o++) {
      const int l = int(rng() % 3), i = int(rng() % span), j = int(rng() % span), k = int(rng() % span);
      const uint64_t key = pk(l, i, j, k);
      const int r = int(rng() % 10);
      if (r < 5) {
        const int32_t v = int32_t(rng() % 1000000);
        f[key] = v;
        ref[key] = v;
      } else if (r < 8) {
        f.erase(key);
        ref.erase(key);
      } else {
        const int32_t* p = f.find(key);
        auto it = ref.find(key);
        if ((p == nullptr) != (it == ref.end()) || (p && *p != it->second)) {
          std::printf("lookup mismatch round %d op %d\n", round, o);
          return 1;
        }
      }
      checks++;
    }
    if (f.size() != ref.size()) {
      std::printf("size %zu vs %zu\n", f.size(), ref.size());
      return 1;
    }
    size_t seen = 0;
    bool bad = false;
    f.for_each([&](uint64_t key, int32_t v) {
      seen++;
      auto it = ref.find(key);
      if (it == ref.end() || it->second != v) bad = true;
    });
    if (bad || seen != ref.size()) {
      std::printf("iteration mismatch round %d\n", round);
      return 1;
    }
    for (const auto& kv : ref) {
      const int32_t* p = f.find(kv.first);
      if (!p || *p != kv.second) {
        std::printf("final lookup mismatch round %d\n", round);
        return 1;
      }
    }
    f.clear();
    if (f.size() != 0 || f.find(ref.begin()->first)) return 1;
  }
  std::printf("ok %ld\n", checks);
  return 0;
}
"""


def test_flatmap_matches_std_map():
    with tempfile.TemporaryDirectory() as d:
        src = os.path.join(d, "t.cpp")
        exe = os.path.join(d, "t")
        with open(src, "w") as f:
            f.write(PROG)
        r = subprocess.run(["g++", "-O1", "-std=c++17", "-I" + CSRC, "-I/opt/rocm/include", "-D__HIP_PLATFORM_AMD__",
                            src, "-o", exe], capture_output=True, text=True)
        assert r.returncode == 0, r.stderr[-2000:]
        out = subprocess.run([exe], capture_output=True, text=True, timeout=120)
        assert out.returncode == 0 and out.stdout.startswith("ok"), out.stdout + out.stderr
