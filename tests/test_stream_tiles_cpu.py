"""Tile-to-request mapping and descriptor checks of the request kernels
(csrc/xs_stream_tiles.h), compiled for the host and run on the CPU.

The persistent request kernel loops over tiles up to a count passed as a
kernel argument and, for each tile, picks a descriptor with request_of and
uses it only if descriptor_ok accepts it.  These tests feed the two
functions valid batches, descriptors left over from another batch, and
arbitrary bytes, and check that (a) a valid batch maps every tile to the
request that owns it, (b) request_of always returns an index in [0, count)
whatever memory holds, and (c) a descriptor not written for the batch is
never accepted, so its pointers are never used."""
import os
import struct
import subprocess
import tempfile

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2402_09222_amd", "csrc")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

HARNESS = r"""
#include "xs_stream_tiles.h"
#include <cstdio>
#include <vector>
// stdin: count, tiles, tag, max_n, then count descriptors (64 bytes each).
// stdout: for each tile g < tiles, "r ok".
int main() {
  int count; long long tiles; unsigned long long tag; long long max_n;
  if (std::fread(&count, 4, 1, stdin) != 1) return 2;
  if (std::fread(&tiles, 8, 1, stdin) != 1) return 2;
  if (std::fread(&tag, 8, 1, stdin) != 1) return 2;
  if (std::fread(&max_n, 8, 1, stdin) != 1) return 2;
  std::vector<xs::ReqDev> reqs(count);
  if (std::fread(reqs.data(), sizeof(xs::ReqDev), count, stdin) != (size_t)count)
    return 2;
  for (long long g = 0; g < tiles; ++g) {
    const int r = xs::request_of(reqs.data(), count, g);
    const bool ok = xs::descriptor_ok(reqs[r], g, tag, max_n);
    std::printf("%d %d\n", r, ok ? 1 : 0);
  }
  return 0;
}
"""


@pytest.fixture(scope="module")
def harness():
    if not os.path.exists(HIPCC):
        pytest.skip("hipcc not available")
    d = tempfile.mkdtemp(prefix="xs_tiles_")
    src = os.path.join(d, "tiles.cpp")
    exe = os.path.join(d, "tiles")
    with open(src, "w") as f:
        f.write(HARNESS)
    # host-only compile of the host/device header: runs without a GPU
    subprocess.run([HIPCC, "--cuda-host-only", "-x", "hip", "-O1",
                    "-std=c++17", "-I", CSRC, "-I",
                    os.path.join(ROOT, "include"), src, "-o", exe],
                   check=True, capture_output=True)
    return exe


def pack(count, tiles, tag, max_n, descs):
    b = struct.pack("<iqQq", count, tiles, tag, max_n)
    for d in descs:
        b += struct.pack("<QQQqqqQq", d["E"], d["mat"], d["out"], d["n"],
                         d["tile_begin"], d["begin"], d["tag"], 0)
    return b


def run(exe, count, tiles, tag, max_n, descs=None, raw=None):
    data = pack(count, tiles, tag, max_n, descs or [])
    if raw is not None:
        data = struct.pack("<iqQq", count, tiles, tag, max_n) + raw
    r = subprocess.run([exe], input=data, capture_output=True, timeout=60)
    assert r.returncode == 0, r.stderr
    rows = [tuple(map(int, ln.split())) for ln in r.stdout.decode().split("\n")
            if ln]
    assert len(rows) == tiles
    return rows


def batch(sizes, tag):
    descs, t, b = [], 0, 0
    for i, n in enumerate(sizes):
        descs.append(dict(E=0x1000 + i, mat=0x2000 + i, out=0x3000 + i, n=n,
                          tile_begin=t, begin=b, tag=tag))
        t += (n + 1023) // 1024
        b += n
    return descs, t


def owner(sizes, g):
    t = 0
    for i, n in enumerate(sizes):
        k = (n + 1023) // 1024
        if t <= g < t + k:
            return i
        t += k
    raise AssertionError(g)


@pytest.mark.parametrize("seed", range(6))
def test_valid_batch_maps_every_tile_to_its_owner(harness, seed):
    rng = np.random.default_rng(seed)
    sizes = [int(x) for x in np.floor(np.exp(rng.uniform(0, np.log(2e5), 40)))]
    sizes[3] = 0
    sizes[7] = 0
    sizes[-1] = 0  # empty requests anywhere, also last
    sizes[10] = 1024
    sizes[11] = 1025
    tag = 0x9E3779B97F4A7C15 * (seed + 1) % 2**64
    descs, tiles = batch(sizes, tag)
    rows = run(harness, len(sizes), tiles, tag, max(sizes), descs)
    for g, (r, ok) in enumerate(rows):
        assert r == owner(sizes, g) and ok == 1, (g, r, ok)


def test_descriptors_of_another_batch_are_refused(harness):
    sizes = [3000, 0, 1, 70000, 1024]
    descs, tiles = batch(sizes, tag=111)
    rows = run(harness, len(sizes), tiles, 222, max(sizes), descs)
    assert all(ok == 0 for _, ok in rows)
    assert all(0 <= r < len(sizes) for r, _ in rows)


def test_sizes_beyond_the_hosts_bound_are_refused(harness):
    sizes = [5000, 2000]
    descs, tiles = batch(sizes, tag=5)
    rows = run(harness, 2, tiles, 5, 4999, descs)  # host said max 4999
    assert [ok for _, ok in rows[:5]] == [0] * 5  # request 0 (n = 5000)
    assert [ok for _, ok in rows[5:]] == [1, 1]   # request 1


def test_tiles_past_a_request_are_refused(harness):
    # tile counts from the host larger than the descriptors cover
    sizes = [1024, 1]
    descs, tiles = batch(sizes, tag=9)
    rows = run(harness, 2, tiles + 5, 9, 1024, descs)
    assert [ok for _, ok in rows] == [1, 1, 0, 0, 0, 0, 0]
    assert all(r == 1 for r, _ in rows[1:])


@pytest.mark.parametrize("seed", range(4))
def test_arbitrary_memory_gives_valid_indices_and_no_accept(harness, seed):
    rng = np.random.default_rng(100 + seed)
    count = int(rng.integers(1, 300))
    raw = rng.integers(0, 256, size=64 * count, dtype=np.uint8).tobytes()
    tag = int(rng.integers(1, 2**63))
    rows = run(harness, count, 2000, tag, 10**6, raw=raw)
    assert all(0 <= r < count for r, _ in rows)
    # a random 64-bit word equals the tag with probability 2^-64
    assert all(ok == 0 for _, ok in rows)
