"""Device-side bounds of the work list (paper_2302_01838_amd/csrc/vmap_internal.h), evaluated on the
host: the kernels take a batch's tile count and every ray index from ray offsets in device memory,
which the host never reads. The helpers they use (batch_segment_ok, tiles_of, clamp_tiles,
clamp_tile_range, tile_ray_range, partial_bad, make_batch_dev) are compiled here for the CPU and
driven with valid and corrupted offset arrays: whatever the offsets hold, every tile lies inside the
workspace and every ray index inside the batch; a valid CSR batch is accepted and its tiles cover
its rays exactly once; a corrupted one is rejected."""
import os
import shutil
import struct
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HIPCC = "/opt/rocm/bin/hipcc"

# A line-oriented driver: each input line names a helper and its integer arguments.
DRIVER = r"""
#include <cstdio>
#include <cstring>
#include <string>
#include <iostream>
#include <sstream>
#include "vmap_internal.h"
using namespace vmapi;
int main() {
  std::string line;
  while (std::getline(std::cin, line)) {
    std::istringstream in(line);
    std::string op;
    in >> op;
    if (op == "seg") {
      long long j, n, o0, o1, nr;
      in >> j >> n >> o0 >> o1 >> nr;
      std::printf("%d\n", (int)batch_segment_ok((int)j, (int)n, (int)o0, (int)o1, (int)nr));
    } else if (op == "tiles") {
      long long nr, rpt;
      in >> nr >> rpt;
      std::printf("%d\n", tiles_of((int)nr, (int)rpt));
    } else if (op == "clamp") {
      long long t, m;
      in >> t >> m;
      std::printf("%d\n", clamp_tiles((int)t, (int)m));
    } else if (op == "range") {
      long long t0, t1, n;
      in >> t0 >> t1 >> n;
      const TileRange r = clamp_tile_range((int)t0, (int)t1, (int)n);
      std::printf("%d %d\n", r.t0, r.t1);
    } else if (op == "rays") {
      long long o0, o1, t, rpt, nr;
      in >> o0 >> o1 >> t >> rpt >> nr;
      const RayRange r = tile_ray_range((int)o0, (int)o1, (int)t, (int)rpt, (int)nr);
      std::printf("%d %d\n", r.lo, r.hi);
    } else if (op == "bad") {
      unsigned bits;
      in >> bits;
      float g;
      std::memcpy(&g, &bits, 4);
      std::printf("%d\n", (int)partial_bad(g));
    } else if (op == "bd") {
      // a descriptor written over memory full of 0xAB: every byte must come from the fields
      BatchDev b;
      std::memset(&b, 0xAB, sizeof b);
      b = make_batch_dev(3, 20, 77, (const int32_t*)16, (const int32_t*)32, (const float*)48,
                         (const float*)64, (const float*)80, (const float*)96, (const float*)112,
                         (const float*)128, (float*)144, (const float*)160);
      const unsigned char* p = reinterpret_cast<const unsigned char*>(&b);
      for (size_t i = 0; i < sizeof b; ++i) std::printf("%d ", p[i]);
      std::printf("\n");
    }
    std::fflush(stdout);
  }
  return 0;
}
"""


@pytest.fixture(scope="module")
def drv(tmp_path_factory):
    if not os.path.exists(HIPCC) or shutil.which("g++") is None:
        pytest.skip("hipcc not available")
    d = tmp_path_factory.mktemp("bounds")
    src = d / "drv.cpp"
    src.write_text(DRIVER)
    exe = d / "drv"
    subprocess.run([HIPCC, "-std=c++17", "-I", os.path.join(ROOT, "include"),
                    "-I", os.path.join(ROOT, "paper_2302_01838_amd", "csrc"), str(src), "-o", str(exe)],
                   check=True, capture_output=True)

    def run(lines):
        out = subprocess.run([str(exe)], input="\n".join(lines) + "\n", check=True,
                             capture_output=True, text=True).stdout.splitlines()
        assert len(out) == len(lines)
        return [list(map(int, ln.split())) for ln in out]
    return run


def work_list(run, offs, n_rays, rpt, max_tiles):
    """The tile kernel's work list from the header helpers, as its table scan builds it: per
    object ok and tile count, exclusive scan, -1 when any object fails; then every tile's rays."""
    n = len(offs) - 1
    ok = [r[0] for r in run([f"seg {j} {n} {offs[j]} {offs[j + 1]} {n_rays}" for j in range(n)])]
    cnt = [r[0] if k else 0 for r, k in
           zip(run([f"tiles {offs[j + 1] - offs[j]} {rpt}" for j in range(n)]), ok)]
    first = np.concatenate([[0], np.cumsum(cnt)]).astype(np.int64)
    n_tiles = -1 if not all(ok) else int(first[-1])
    n_clamped = run([f"clamp {n_tiles} {max_tiles}"])[0][0]
    tiles = []
    if n_clamped:
        owners = [int(np.searchsorted(first, t, side="right") - 1) for t in range(n_clamped)]
        rr = run([f"rays {offs[j]} {offs[j + 1]} {t - first[j]} {rpt} {n_rays}"
                  for t, j in zip(range(n_clamped), owners)])
        tiles = [(j, lo, hi) for j, (lo, hi) in zip(owners, rr)]
    return all(ok), n_clamped, tiles


def test_valid_batches_cover_their_rays_once(drv):
    rng = np.random.default_rng(0)
    for case in range(40):
        n = int(rng.integers(1, 30))
        counts = rng.integers(0, 200, n)
        counts[rng.random(n) < 0.2] = 0  # objects without rays
        offs = np.concatenate([[0], np.cumsum(counts)]).astype(int).tolist()
        R = offs[-1]
        rpt = int(rng.integers(1, 64))
        max_tiles = (R + rpt - 1) // rpt + n  # the host's capacity check
        ok, n_tiles, tiles = work_list(drv, offs, R, rpt, max_tiles)
        assert ok
        assert n_tiles <= max_tiles
        seen = np.zeros(R, np.int64)
        for j, lo, hi in tiles:
            assert offs[j] <= lo < hi <= offs[j + 1]
            seen[lo:hi] += 1
        assert np.all(seen == 1)


@pytest.mark.parametrize("kind", ["decreasing", "beyond", "negative", "first", "last", "overlap",
                                  "huge"])
def test_corrupted_offsets_are_rejected_and_stay_in_bounds(drv, kind):
    rng = np.random.default_rng(1)
    for case in range(10):
        n = int(rng.integers(2, 20))
        offs = np.concatenate([[0], np.cumsum(rng.integers(1, 100, n))]).astype(np.int64)
        R = int(offs[-1])
        j = int(rng.integers(1, n))
        if kind == "decreasing":
            offs[j] = offs[j - 1] - 1 if offs[j - 1] > 0 else -1
        elif kind == "beyond":
            offs[j] = R + 1000
        elif kind == "negative":
            offs[j] = -5
        elif kind == "first":
            offs[0] = 3
        elif kind == "last":
            offs[-1] = R - 1
        elif kind == "overlap":  # 0, R, 0, R, ...: each even segment alone is in range
            offs[:] = [(i % 2) * R for i in range(n + 1)]
            offs[-1] = R
        elif kind == "huge":
            offs[j] = 2 ** 31 - 1
        offs = offs.tolist()
        rpt = 7
        max_tiles = (R + rpt - 1) // rpt + n
        ok, n_tiles, tiles = work_list(drv, offs, R, rpt, max_tiles)
        assert not ok
        assert n_tiles == 0  # the kernels run no tile of a rejected batch


def test_clamps_keep_indices_in_bounds(drv):
    rng = np.random.default_rng(2)
    big = [-(2 ** 31), -(2 ** 20), -1, 0, 1, 5, 2 ** 20, 2 ** 31 - 1]
    lines, args = [], []
    for _ in range(400):
        o0, o1, t = (int(rng.choice(big)) if rng.random() < 0.5 else int(rng.integers(-50, 500))
                     for _ in range(3))
        rpt = int(rng.integers(1, 2 ** 16))
        nr = int(rng.integers(0, 1000))
        lines.append(f"rays {o0} {o1} {t} {rpt} {nr}")
        args.append(nr)
    for (lo, hi), nr in zip(drv(lines), args):
        assert 0 <= lo <= hi <= nr
    lines, args = [], []
    for _ in range(400):
        t0, t1 = (int(rng.choice(big)) if rng.random() < 0.5 else int(rng.integers(-10, 100))
                  for _ in range(2))
        n = int(rng.integers(0, 100))
        lines.append(f"range {t0} {t1} {n}")
        args.append(n)
    for (a, b), n in zip(drv(lines), args):
        assert 0 <= a <= b <= n
    for t, m, want in [(-1, 10, 0), (0, 10, 0), (5, 10, 5), (10, 10, 10), (11, 10, 10),
                       (2 ** 31 - 1, 10, 10)]:
        assert drv([f"clamp {t} {m}"])[0][0] == want


def test_partial_limit(drv):
    def bits(x):
        return struct.unpack("<I", struct.pack("<f", x))[0]
    cases = [(0.0, 0), (-0.0, 0), (1.0, 0), (-3.5e18, 0), (float(np.nextafter(np.float32(2.0 ** 64),
                                                                               np.float32(0)) ), 0),
             (2.0 ** 64, 1), (-(2.0 ** 64), 1), (3e38, 1), (float("inf"), 1), (float("-inf"), 1)]
    lines = [f"bad {bits(x)}" for x, _ in cases] + ["bad 2143289344", "bad 4290772992"]  # NaNs
    want = [w for _, w in cases] + [1, 1]
    assert [r[0] for r in drv(lines)] == want
    # the bound: 2^27 tiles of magnitude below 2^64, each addition rounding up by at most 2^-24
    assert 2.0 ** 27 * 2.0 ** 64 * np.exp(2.0 ** 27 * 2.0 ** -24) < 2.0 ** 128


def test_batch_descriptor_sets_every_byte(drv):
    b = bytes(drv(["bd"])[0])
    assert len(b) == 96
    n_objects, S, n_rays, pad = struct.unpack_from("<4i", b, 0)
    assert (n_objects, S, n_rays, pad) == (3, 20, 77, 0)
    assert list(struct.unpack_from("<10Q", b, 16)) == [16, 32, 48, 64, 80, 96, 112, 128, 144, 160]
