"""The storage-rounding emulation that the 16-bit floors come from
(tests/storage_floor.py), checked on its own, on D3Q19 and D2Q9: source
indices by brute force on a tiny tube and channel, every re-encoded
population within half a unit in the last place of its deviation, and each
node's stored mass equal to its density up to the rounding of the stochastic
rest remainder.  CPU only."""
import numpy as np
import pytest

import synth
from oracle import lbm3d as o3
from tests import storage_floor as sf


def _tiny_tube():
    cfg = synth.config_tube(lam=12.0, r0=3.0, a=1.0, nx=12, ny=10, nz=10, theta=90.0)
    return cfg, synth.mask3_of(cfg)


def test_source_index3_by_brute_force():
    cfg, mask = _tiny_tube()
    idx, w = sf.source_index3(mask, False)
    cx, cy, cz, _, _ = o3.lattice()
    nz, ny, nx = mask.shape
    assert np.isclose(w.sum(), 1.0) and np.isclose(w.max(), 1 / 3)
    for i in range(len(cx)):
        for z in range(nz):
            for y in range(ny):
                for x in range(nx):
                    xs, ys, zs = (x - cx[i]) % nx, y - cy[i], z - cz[i]
                    inside = 0 <= ys < ny and 0 <= zs < nz and mask[zs, ys, xs] == 1
                    want = (zs * ny + ys) * nx + xs if inside else (z * ny + y) * nx + x
                    assert idx[i, z, y, x] == want


# ulp: the format's spacing relative to a value's leading power of two (10 and
# 7 fraction bits), so a value d rounds to within ulp |d| / 2 in the normal range
@pytest.mark.parametrize("fmt,ulp", [("f16", 2.0 ** -10), ("bf16", 2.0 ** -7)])
def test_reencode3_rounds_each_deviation_and_keeps_node_mass(fmt, ulp):
    cfg, mask = _tiny_tube()
    idx, w = sf.source_index3(mask, False)
    rng = np.random.default_rng(3)
    fluid = mask == 1
    n = mask.size
    # densities of the source nodes (species 0 ~ 1, species 1 ~ 0.03) and
    # populations near w_i rho(source) with deviations of a few per cent
    rho = np.stack([1.0 + 0.05 * rng.random(mask.shape), 0.03 * (1 + 0.5 * rng.random(mask.shape))])
    rho *= fluid
    f = np.zeros((2, len(w)) + mask.shape)
    for s in range(2):
        src = rho[s].ravel()[idx]
        f[s] = w[:, None, None, None] * src * (1 + 0.03 * rng.standard_normal(src.shape))
    f *= fluid
    out = sf.reencode3(f, rho, mask, idx, w, fmt, np.random.default_rng(7))
    i0 = int(np.argmax(w))
    moving = [i for i in range(len(w)) if i != i0]
    for s in range(2):
        R = rho[s].astype(np.float32).astype(np.float16).astype(np.float64).ravel()
        ref = R[idx]
        dev = f[s] / w[:, None, None, None] - ref
        err = np.abs(out[s] - f[s]) / w[:, None, None, None]
        # round to nearest: half a unit of the deviation (plus its FP32 step);
        # binary16 below 2^-14 is subnormal, with a fixed spacing of 2^-24
        sub = 2.0 ** -25 if fmt == "f16" else 0.0
        bound = (0.5 * ulp + 2.0 ** -23) * np.abs(dev) + sub + 1e-15
        assert np.all(err[moving][:, fluid] <= bound[moving][:, fluid])
        # each node's stored mass: the populations it emitted (moving ones at
        # their destinations, the rest in place) sum to its FP32 density up to
        # the rest remainder's stochastic rounding (below one unit of it)
        emitted = np.zeros(n)
        np.add.at(emitted, idx[moving].ravel(), out[s][moving].ravel())
        emitted += out[s][i0].ravel()
        r32 = rho[s].astype(np.float32).astype(np.float64).ravel()
        rest_dev = np.abs(out[s][i0].ravel() / w[i0] - R)
        assert np.all(np.abs(emitted - r32)[fluid.ravel()] <=
                      (w[i0] * (ulp * rest_dev + 2.0 ** -24) + 1e-15)[fluid.ravel()])


def _tiny_channel():
    cfg = synth.config_channel(lam=16, theta=90.0)
    return cfg, synth.mask_of(cfg)


def test_source_index_by_brute_force():
    cfg, mask = _tiny_channel()
    idx = sf.source_index(mask, False)
    ny, nx = mask.shape
    for i in range(9):
        for y in range(ny):
            for x in range(nx):
                xs, ys = (x - sf.CX[i]) % nx, y - sf.CY[i]
                inside = 0 <= ys < ny and mask[ys, xs] == 1
                assert idx[i, y, x] == (ys * nx + xs if inside else y * nx + x)


@pytest.mark.parametrize("fmt,ulp", [("f16", 2.0 ** -10), ("bf16", 2.0 ** -7), ("f32", 2.0 ** -23)])
def test_reencode_rounds_each_deviation_and_keeps_node_mass(fmt, ulp):
    cfg, mask = _tiny_channel()
    idx = sf.source_index(mask, False)
    rng = np.random.default_rng(4)
    fluid = mask == 1
    rho = np.stack([1.0 + 0.05 * rng.random(mask.shape), 0.03 * (1 + 0.5 * rng.random(mask.shape))])
    rho *= fluid
    W = sf.W[:, None, None]
    f = np.zeros((2, 9) + mask.shape)
    for s in range(2):
        f[s] = W * rho[s].ravel()[idx] * (1 + 0.03 * rng.standard_normal(idx.shape))
    f *= fluid
    out = sf.reencode(f, rho, mask, idx, fmt, np.random.default_rng(9))
    if fmt == "f32":   # every population rounded to binary32
        assert np.all(np.abs(out - f) <= 0.5 * ulp * np.abs(f))
        return
    sub = 2.0 ** -25 if fmt == "f16" else 0.0
    for s in range(2):
        R = rho[s].astype(np.float32).astype(np.float16).astype(np.float64).ravel()
        dev = f[s] / W - R[idx]
        err = np.abs(out[s] - f[s]) / W
        bound = (0.5 * ulp + 2.0 ** -23) * np.abs(dev) + sub + 1e-15
        assert np.all(err[1:][:, fluid] <= bound[1:][:, fluid])
        emitted = np.zeros(mask.size)
        np.add.at(emitted, idx[1:].ravel(), out[s][1:].ravel())
        emitted += out[s][0].ravel()
        r32 = rho[s].astype(np.float32).astype(np.float64).ravel()
        rest_dev = np.abs(out[s][0].ravel() / sf.W[0] - R)
        assert np.all(np.abs(emitted - r32)[fluid.ravel()] <=
                      (sf.W[0] * (ulp * rest_dev + 2.0 ** -24) + 1e-15)[fluid.ravel()])
