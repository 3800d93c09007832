"""Role map of the fused step launch (step_map.h, compiled for the host):
every role block is dealt to exactly one hardware block, padding blocks get
no role, and with the XCD-aware map each XCD's fluid blocks form one
contiguous run with its walker blocks spread among them."""
import os
import shutil
import subprocess
import tempfile

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "..", "paper_2308_05007_amd", "csrc")

PROGRAM = r"""
#include <cstdio>
#include <vector>
#include "step_map.h"
using namespace rwmi;
static int check(const int nb[3], bool xcd) {
  const int g = step_grid(nb, xcd);
  std::vector<int> seen[3];
  for (int r = 0; r < 3; ++r) seen[r].assign(nb[r], 0);
  std::vector<int> fluid_xcd(nb[2], -1);
  std::vector<int> last_fluid(8, -1);
  for (int i = 0; i < g; ++i) {
    int idx = -1;
    const int r = step_role(i, nb, xcd, idx);
    if (r == kRoleNone) continue;
    if (r < 0 || r > 2 || idx < 0 || idx >= nb[r]) { printf("bad role %d idx %d at %d\n", r, idx, i); return 1; }
    seen[r][idx]++;
    if (xcd && r == kRoleFluid) {
      const int x = i & 7;
      // fluid indices of one XCD are consecutive, in hardware-block order
      if (last_fluid[x] >= 0 && idx != last_fluid[x] + 1) { printf("fluid run broken on xcd %d\n", x); return 1; }
      last_fluid[x] = idx;
    }
  }
  for (int r = 0; r < 3; ++r)
    for (int k = 0; k < nb[r]; ++k)
      if (seen[r][k] != 1) { printf("role %d block %d dealt %d times (nb %d %d %d xcd %d)\n", r, k, seen[r][k], nb[0], nb[1], nb[2], (int)xcd); return 1; }
  if (!xcd && g != nb[0] + nb[1] + nb[2]) { printf("grid %d\n", g); return 1; }
  if (xcd && (g % 8 != 0 || g < nb[0] + nb[1] + nb[2] || g >= nb[0] + nb[1] + nb[2] + 8 * 3 + 8)) { printf("xcd grid %d\n", g); return 1; }
  return 0;
}
int main() {
  const int vals[] = {0, 1, 2, 3, 7, 8, 9, 15, 16, 17, 63, 64, 65, 100, 1000, 3907, 8064};
  long cases = 0;
  for (int a : vals) for (int b : vals) for (int c : vals)
    for (int x = 0; x < 2; ++x) {
      const int nb[3] = {a, b, c};
      if (check(nb, x != 0)) return 1;
      ++cases;
    }
  printf("ok %ld\n", cases);
  return 0;
}
"""


@pytest.mark.skipif(shutil.which("g++") is None, reason="g++ not available")
def test_role_map_is_a_bijection():
    with tempfile.TemporaryDirectory() as d:
        src = os.path.join(d, "t.cpp")
        exe = os.path.join(d, "t")
        with open(src, "w") as fh:
            fh.write(PROGRAM)
        subprocess.run(["g++", "-std=c++17", "-O1", "-I", CSRC, src, "-o", exe], check=True, capture_output=True)
        r = subprocess.run([exe], capture_output=True, text=True, timeout=120)
        assert r.returncode == 0, r.stdout + r.stderr
        assert r.stdout.startswith("ok")
