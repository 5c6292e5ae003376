"""Host-side logic of bench.py, on the CPU: the refusal of more than one GPU, and the traffic
figure read from the committed counter summary, which applies only to the kernel source it was
measured on and only to the launch shape and step form it lists."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    proc = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                          capture_output=True, text=True, timeout=120)
    assert proc.returncode == 2
    assert "one GPU" in proc.stderr


def _summary_fields():
    fields = {}
    for line in open(bench.TRAFFIC_FILE).read().splitlines():
        if line.startswith("- ") and ":" in line:
            key, val = line[2:].split(":", 1)
            fields[key.strip()] = val.strip().strip("`")
    return fields


def test_traffic_figure_follows_the_kernel_source():
    fields = _summary_fields()
    if fields.get("kernel source sha256") != bench.tile_kernel_fingerprint():
        pytest.skip("the tile-kernel sources changed since the counters were taken")
    want = int(fields["traffic bytes per launch (bf16, rays_per_tile 36, waves 4, table)"].replace(",", ""))
    assert bench.measured_traffic("bf16", 36, 4) == want
    assert bench.measured_traffic("fp32", 36, 2) == int(
        fields["traffic bytes per launch (fp32, rays_per_tile 36, waves 2, table)"].replace(",", ""))
    # another launch shape or step form has no figure
    assert bench.measured_traffic("bf16", 24, 4) is None
    assert bench.measured_traffic("bf16", 36, 8) is None
    assert bench.measured_traffic("bf16", 36, 4, split_step=True) is None


def test_fingerprint_changes_with_the_tile_kernel_source(tmp_path, monkeypatch):
    """A copy of the sources with one character changed inside the tile kernel's region gives
    another fingerprint, so a stale counter summary is not reported."""
    csrc = os.path.join(ROOT, "paper_2302_01838_amd", "csrc")
    fake_root = tmp_path / "repo"
    fake_csrc = fake_root / "paper_2302_01838_amd" / "csrc"
    fake_csrc.mkdir(parents=True)
    for name in ("vmap_kernels.hip", "vmap_internal.h", "vmap_math.h", "vmap_bf16.h"):
        text = open(os.path.join(csrc, name)).read()
        if name == "vmap_kernels.hip":
            a = text.index("// Activations of one 32-sample pass")
            b = text.index("{", a)  # the first brace inside the region
            text = text[:b] + "{ " + text[b + 1:]
        (fake_csrc / name).write_text(text)
    before = bench.tile_kernel_fingerprint()
    monkeypatch.setattr(bench, "ROOT", str(fake_root))
    assert bench.tile_kernel_fingerprint() != before
