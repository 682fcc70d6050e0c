"""The FP64 GEMM's workgroup -> tile schedule (csrc/tile_map.h), built for the host with g++ and
checked by brute force: every schedule must hand each live output tile of every batch item to
exactly one workgroup, and no dead one.  Host-only, no GPU.

  remap 0  row-major, one workgroup per tile of the rectangle;
  remap 1  XCD chunks over the rectangle;
  remap 2  XCD chunks over the lower trapezoid (tile column <= tile row, tiles_m >= tiles_n),
           the shape of the Cholesky updates C -= L L^T with or without the extra right-hand-side
           rows below the factor.
"""
import pathlib
import shutil
import subprocess

import pytest

CSRC = pathlib.Path(__file__).resolve().parents[1] / "paper_2605_21149_amd" / "csrc"

HARNESS = r"""
#include <cstdio>
#include <vector>
#include "tile_map.h"
using cf::tile_map;
static long check(int remap, int tm, int tn, int nz) {
  const int64_t nx = remap == 2 ? (int64_t)tn * (tn + 1) / 2 + (int64_t)(tm - tn) * tn : (int64_t)tm * tn;
  std::vector<int> seen((size_t)nz * tm * tn, 0);
  long bad = 0;
  for (int64_t bz = 0; bz < nz; ++bz)
    for (int64_t bx = 0; bx < nx; ++bx) {
      int64_t z; int a, b;
      if (!tile_map(remap, tm, tn, nx, nz, bx, bz, z, a, b)) { ++bad; continue; }
      if (z < 0 || z >= nz || a < 0 || a >= tm || b < 0 || b >= tn) { ++bad; continue; }
      ++seen[((size_t)z * tm + a) * tn + b];
    }
  for (size_t k = 0; k < seen.size(); ++k) {
    const int a = (int)((k / tn) % tm), b = (int)(k % tn);
    const int want = remap == 2 ? (b <= a) : 1;
    if (seen[k] != want) ++bad;
  }
  return bad;
}
int main() {
  long bad = 0, cases = 0;
  for (int remap = 0; remap <= 2; ++remap)
    for (int tn = 1; tn <= 30; ++tn)
      for (int tm = (remap == 2 ? tn : 1); tm <= tn + 20; ++tm)
        for (int nz : {1, 3, 8}) { bad += check(remap, tm, tn, nz); ++cases; }
  // factorisation shapes: n = 5952 in 64-wide tiles (93 tile rows), the trailing blocks after
  // 512-column panels, with and without one extra tile row of right-hand sides; batch 8
  for (int tn : {93, 85, 77, 13, 5, 1})
    for (int tm : {tn, tn + 1, tn + 7}) { bad += check(2, tm, tn, 8); ++cases; }
  std::printf("cases %ld bad %ld\n", cases, bad);
  return bad != 0;
}
"""


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs a host C++ compiler")
def test_every_live_tile_gets_exactly_one_workgroup(tmp_path):
    src = tmp_path / "tm.cpp"
    src.write_text(HARNESS)
    exe = tmp_path / "tm"
    subprocess.run(["g++", "-O2", "-std=c++17", "-D__host__=", "-D__device__=", f"-I{CSRC}", str(src),
                    "-o", str(exe)], check=True)
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stdout + r.stderr
    assert r.stdout.split()[-1] == "0"
