"""Device layouts of the element state and of the face inboxes (host logic).

A small host program built from the library's own layout header checks, for
every order and a ragged element count, that
* qidx maps (element, row, quantity) one-to-one into [0, q_size), row r of
  element el in tile r >> 4, slot v = (r >> 2) & 3 and lane el + 16 (r & 3)
  (rows run over the lane groups first inside a tile);
* inidx maps (element, face, node, quantity) one-to-one into [0, in_size);
* the quantities 0..7 of a node are eight consecutive values starting on a
  16-byte boundary (two vector stores), and quantity 8 sits in its block's
  trailing row at the same lane;
* node m of a face sits in tile m >> 4, register v and lane group g with
  m = 16 t + 4 v + g, the slot order the matrix-core kernels assume.
No GPU is needed; the program runs on the host.
"""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2107_06640_amd", "csrc")
HIPCC = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"

PROGRAM = r"""
#include "layout.hpp"
#include <cstdio>
#include <vector>
using namespace seis;
static int nb(int N) { return (N + 1) * (N + 2) * (N + 3) / 6; }
static int nf(int N) { return (N + 1) * (N + 2) / 2; }
int main() {
  const int64_t E = 37;  // two full groups of 16 and a ragged one
  int bad = 0;
  for (int N = 2; N <= 6; ++N) {
    const int B = nb(N), Bf = nf(N), RT = row_tiles(B), FT = row_tiles(Bf);
    std::vector<int> seen(q_size(E, RT), 0);
    for (int64_t e = 0; e < E; ++e)
      for (int r = 0; r < B; ++r)
        for (int p = 0; p < 9; ++p) {
          const int64_t i = qidx(e, r, p, RT);
          if (i < 0 || i >= (int64_t)seen.size() || seen[i]++) ++bad;
          // row r in tile r >> 4, slot v = (r >> 2) & 3, lane group g = r & 3
          const int64_t want = ((((e >> 4) * RT + (r >> 4)) * 4 + ((r >> 2) & 3)) * 9 + p) * 64 + (e & 15) + 16 * (r & 3);
          if (i != want) ++bad;
          if (tile_perm(tile_perm(r)) != r || (tile_perm(r) >> 4) != (r >> 4)) ++bad;
        }
    std::vector<int> in(in_size(E, FT), 0);
    for (int64_t e = 0; e < E; ++e)
      for (int f = 0; f < 4; ++f)
        for (int m = 0; m < Bf; ++m) {
          const int64_t b = in_block(e, f, m, FT);
          const int l = in_lane(e, m);
          const int t = m >> 4, v = int((b & 3)), g = (l >> 4);
          if (16 * t + 4 * v + g != m || (l & 15) != int(e & 15)) ++bad;
          if (inidx(e, f, m, 0, FT) % 4 != 0) ++bad;
          for (int p = 0; p < 9; ++p) {
            const int64_t i = inidx(e, f, m, p, FT);
            if (i < 0 || i >= (int64_t)in.size() || in[i]++) ++bad;
            if (p < 8 && i != inidx(e, f, m, 0, FT) + p) ++bad;
          }
          if (inidx(e, f, m, 8, FT) != 576 * b + 512 + l) ++bad;
        }
  }
  std::printf("violations %d\n", bad);
  return bad != 0;
}
"""


@pytest.mark.skipif(not os.path.exists(HIPCC), reason="hipcc not available")
def test_state_and_inbox_layouts(tmp_path):
    src = tmp_path / "layout_check.cpp"
    exe = tmp_path / "layout_check"
    src.write_text(PROGRAM)
    build = subprocess.run([HIPCC, "-O1", "-std=c++17", f"-I{CSRC}", "-x", "hip", "--offload-arch=gfx950", str(src),
                            "-o", str(exe)], capture_output=True, text=True, timeout=300)
    assert build.returncode == 0, build.stderr[-2000:]
    run = subprocess.run([str(exe)], capture_output=True, text=True, timeout=120)
    assert run.returncode == 0, run.stdout + run.stderr
    assert "violations 0" in run.stdout
