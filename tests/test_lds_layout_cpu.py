"""LDS layout of the width-32 tile kernel (paper_2302_01838_amd/csrc/vmap_internal.h), evaluated on
the host: for every wave count a launch accepts, the end-of-tile gradient copies fit in the
workgroup's staging space, the regions do not overlap, and the workgroup fits in the 160 KiB of
LDS of a CU (two four-wave BF16 workgroups per CU)."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HIPCC = "/opt/rocm/bin/hipcc"

DRIVER = r"""
#include <cstdio>
#include "vmap_internal.h"
using namespace vmapi;
int main() {
  for (int bf = 0; bf <= 1; ++bf)
    for (int nw = 1; nw <= 8; ++nw) {
      const LdsLayout L = lds_layout(32, bf != 0, nw);
      const int red = red_copies(nw) * round_up(n_params_of(32), 4) * 4;
      std::printf("%d %d %d %d %d %d %d %d %d\n", bf, nw, L.total, L.scratch_off,
                  nw * L.scratch_wave, red, L.loss_off, L.B_off, red_copies(nw));
    }
  return 0;
}
"""


def test_tile_kernel_lds_layout(tmp_path):
    if not os.path.exists(HIPCC) or shutil.which("g++") is None:
        pytest.skip("hipcc not available")
    src = tmp_path / "drv.cpp"
    src.write_text(DRIVER)
    exe = tmp_path / "drv"
    subprocess.run([HIPCC, "-std=c++17", "-I", os.path.join(ROOT, "include"),
                    "-I", os.path.join(ROOT, "paper_2302_01838_amd", "csrc"), str(src), "-o", str(exe)],
                   check=True, capture_output=True)
    rows = [list(map(int, ln.split())) for ln in
            subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.splitlines()]
    assert len(rows) == 16
    for bf, nw, total, scratch_off, staging, red, loss_off, b_off, nc in rows:
        assert nc == (4 if nw >= 8 else 2 if nw >= 2 else 1)
        # the copies of the tile's gradient and the per-wave staging share the scratch region
        assert total - scratch_off >= max(staging, red)
        # the loss of each copy and the non-finite flag (at +16 bytes) sit before the scratch
        assert loss_off + 16 + 4 <= scratch_off
        assert b_off < loss_off
        assert total <= 160 * 1024
        if bf and nw == 4:  # two workgroups per CU, with the in-kernel tile table of 50 objects
            assert 2 * (total + 3 * 52 * 4) <= 160 * 1024
