"""The tile kernels' BF16 packing helpers (paper_2302_01838_amd/csrc/vmap_bf16.h), compiled for
the host with clang and compared with torch's own float32 -> bfloat16 cast: rounding to BF16
(nearest even), ReLU on packed BF16 pairs, and the ReLU derivative applied to packed deltas."""
import os
import shutil
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CLANG = "/opt/rocm/llvm/bin/clang++"

DRIVER = r"""
#include <cstdio>
#include <cstdint>
#include <cstring>
#include "vmap_bf16.h"
using namespace vmapi;
static uint16_t bits(__bf16 x) { uint16_t u; std::memcpy(&u, &x, 2); return u; }
int main() {
  float buf[16];
  while (std::fread(buf, sizeof(float), 16, stdin) == 16) {
    f32x16 acc;
    for (int i = 0; i < 16; ++i) acc[i] = buf[i];
    const bf16x8 r = round8(acc, 0), h = relu_round8(acc, 8), m = relu_mask(r, h);
    for (int i = 0; i < 8; ++i) std::printf("%u %u %u\n", bits(r[i]), bits(h[i]), bits(m[i]));
  }
  return 0;
}
"""


def _bf16_bits(x):
    """The 16-bit patterns of torch's rounding of float32 values to BF16 (nearest even)."""
    import torch
    t = torch.from_numpy(np.ascontiguousarray(x, np.float32)).to(torch.bfloat16)
    return t.view(torch.int16).numpy().view(np.uint16)


@pytest.mark.skipif(not os.path.exists(CLANG), reason="clang++ of ROCm not available")
def test_bf16_helpers_against_torch(tmp_path):
    src = tmp_path / "drv.cpp"
    src.write_text(DRIVER)
    exe = tmp_path / "drv"
    subprocess.run([CLANG, "-std=c++17", "-O2", "-I", os.path.join(ROOT, "paper_2302_01838_amd", "csrc"),
                    str(src), "-o", str(exe)], check=True)
    rng = np.random.default_rng(3)
    n = 4000
    a = rng.standard_normal((n, 16)).astype(np.float32) * np.float32(3.0)
    a[::7, 8:] = 0.0                     # exact zeros
    a[1::7, 8:] = -0.0                   # negative zeros
    a[2::7, 8:] = np.float32(1e-39)      # FP32 subnormals
    a[3::7, :] = np.float32(1e-3) * a[3::7, :]
    out = subprocess.run([str(exe)], input=a.tobytes(), capture_output=True, check=True).stdout
    got = np.array([[int(v) for v in ln.split()] for ln in out.decode().splitlines()], dtype=np.uint32)
    got = got.reshape(n, 8, 3)
    r_ref = _bf16_bits(a[:, :8])
    assert np.array_equal(got[:, :, 0], r_ref)
    hpos = a[:, 8:] > 0
    h_ref = np.where(hpos, _bf16_bits(np.where(hpos, a[:, 8:], 0)), 0).astype(np.uint16)
    assert np.array_equal(got[:, :, 1], h_ref)
    m_ref = np.where(h_ref != 0, r_ref, 0)
    assert np.array_equal(got[:, :, 2], m_ref)
