"""The halo-lane layout of the D2Q9 step kernel (lbm_kernels.hip: kHaloLane,
halo_dir, halo_rho): the two maps are inverse to each other, and the kernel's
four-level butterfly of lane-pair sums (DPP quad_perm [1,0,3,2], quad_perm
[2,3,0,1], row_half_mirror, row_mirror on rows of 16 lanes), emulated here in
binary32, gives every lane of the row the density rho9 computes, bit for bit,
on random populations.  A halo density equal to the inner nodes' one is what
makes the results independent of the tiling.  CPU only: the source is read,
not run."""
import os
import re

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "paper_1601_00918_amd", "csrc", "lbm_kernels.hip")


def _tables():
    s = open(SRC).read()
    lane = [int(v) for v in re.search(r"kHaloLane\[9\]\s*=\s*\{([^}]*)\}", s).group(1).split(",")]
    body = re.search(r"int halo_dir\(int lane\)\s*\{(.*?)\}", s, re.S).group(1)
    pairs = {int(a): int(b) for a, b in re.findall(r"lane == (\d+) \? (\d+)", body)}
    return lane, pairs


def _rho9(f):
    a13, a24 = f[1] + f[3], f[2] + f[4]
    a57, a68 = f[5] + f[7], f[6] + f[8]
    return ((f[0] + a13) + a24) + (a57 + a68)


def _butterfly(v):
    def level(v, partner):
        return np.stack([v[partner(i)] + v[i] for i in range(16)])
    q1, q2 = [1, 0, 3, 2], [2, 3, 0, 1]
    v = level(v, lambda i: (i & ~3) | q1[i & 3])
    v = level(v, lambda i: (i & ~3) | q2[i & 3])
    v = level(v, lambda i: (i & ~7) | (7 - (i & 7)))
    return level(v, lambda i: 15 - i)


def test_lane_maps_are_inverse():
    lane, pairs = _tables()
    assert sorted(lane) == sorted(pairs)            # nine distinct lanes
    assert all(pairs[lane[j]] == j for j in range(9))
    assert max(lane) < 16


def test_butterfly_reproduces_rho9_bit_for_bit():
    lane, _ = _tables()
    rng = np.random.default_rng(11)
    n = 20000
    f = (rng.random((9, n)) * 10.0 ** rng.integers(-7, 1, (9, n))).astype(np.float32)
    v = np.zeros((16, n), dtype=np.float32)
    for j in range(9):
        v[lane[j]] = f[j]
    out = _butterfly(v)
    want = _rho9(f)
    assert out.dtype == np.float32 and want.dtype == np.float32
    assert np.array_equal(out.view(np.uint32), np.broadcast_to(want, out.shape).view(np.uint32))
