"""Storage-rounding floor of the 16-bit population formats (not a test).

Runs the FP64 oracle and, beside it, the same run whose state is re-encoded
after every step the way the 16-bit formats store it: per node and species a
binary16 reference density R (the node's density), deviations
d_i = f_i / w_i - R rounded to nearest even for i >= 1 and the rest d_0
carrying the mass remainder with stochastic rounding.  The difference between
the two runs is the error the storage alone puts on the result; the GPU
tolerances are a multiple of it.  Arithmetic stays FP64: only the rounding of
the stored state is emulated.

    python tests/storage_floor.py            # prints the floors after 1000 steps
    python tests/storage_floor.py --write    # also stores them in
                                             # tests/golden/storage_floor.json
    python tests/storage_floor.py --tube     # floors of the D3Q19 tube workload
                                             # after 20 steps, stored in
                                             # tests/golden/storage_floor_tube.json
    python tests/storage_floor.py --batch    # floors of the sampled instances
                                             # of the 256-channel batch after 100
                                             # steps, stored in
                                             # tests/golden/storage_floor_batch.json

Format "f32" rounds every population to binary32 instead: the floor of the
FP32 storage itself (arithmetic still FP64).
"""
import os
import sys

import numpy as np

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))

import synth  # noqa: E402
from tests.gpu_util import field_rel_err, oracle_lattice  # noqa: E402

W = np.array([4 / 9] + [1 / 9] * 4 + [1 / 36] * 4)
CX = [0, 1, 0, -1, 0, 1, -1, -1, 1]
CY = [0, 0, 1, 0, -1, 1, 1, -1, -1]


def source_index(mask, periodic_y):
    """Flat index of the node each pulled population f_i(x) came from (the
    node itself after bounce-back)."""
    ny, nx = mask.shape
    idx = np.zeros((9, ny, nx), dtype=np.int64)
    own = np.arange(ny)[:, None] * nx + np.arange(nx)[None, :]
    for i in range(9):
        ys = np.arange(ny)[:, None] - CY[i] + 0 * np.arange(nx)[None, :]
        xs = (np.arange(nx)[None, :] - CX[i]) % nx + 0 * ys
        if periodic_y:
            ys = ys % ny
        ok = (ys >= 0) & (ys < ny)
        ysc = np.clip(ys, 0, ny - 1)
        fluid = ok & (mask[ysc, xs] == 1)
        idx[i] = np.where(fluid, ysc * nx + xs, own)
    return idx


def _rne(v, fmt):
    v = np.asarray(v, dtype=np.float32)
    if fmt == "f16":
        return v.astype(np.float16).astype(np.float64)
    u = v.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) >> 16 << 16
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def _sr(v, fmt, rng):
    v = np.asarray(v, dtype=np.float64)
    if fmt == "bf16":
        u = v.astype(np.float32).view(np.uint32).astype(np.uint64)
        u = (u + rng.integers(0, 1 << 16, size=v.shape, dtype=np.uint64)) >> 16 << 16
        return u.astype(np.uint32).view(np.float32).astype(np.float64)
    h = v.astype(np.float16)
    hv = h.astype(np.float64)
    lo = np.where(hv > v, np.nextafter(h, np.float16(-np.inf)), h).astype(np.float64)
    hi = np.where(hv > v, h, np.nextafter(h, np.float16(np.inf))).astype(np.float64)
    p = np.where(hi > lo, (v - lo) / (hi - lo), 0.0)
    return np.where(rng.random(v.shape) < p, hi, lo)


def reencode(f, rho, mask, idx, fmt, rng):
    """f: pulled populations [2, 9, ny, nx] after a step whose sources had
    densities rho [2, ny, nx] (before the step); returns the decoded state.
    fmt "f32": every population rounded to binary32 (the FP32 storage)."""
    if fmt == "f32":
        return f.astype(np.float32).astype(np.float64)
    ny, nx = mask.shape
    out = np.empty_like(f)
    fluid = (mask == 1)
    for s in range(2):
        r32 = rho[s].astype(np.float32).astype(np.float64).ravel()
        R = r32.astype(np.float16).astype(np.float64)
        ref = R[idx]
        d = _rne(f[s] / W[:, None, None] - ref, fmt) * fluid[None]
        dsum = np.zeros(ny * nx)
        np.add.at(dsum, idx[1:].ravel(), (W[1:, None, None] * d[1:]).ravel())
        rest = (r32 - R - dsum) / (4 / 9)
        d[0] = (_sr(rest, fmt, rng) * fluid.ravel()).reshape(ny, nx)
        out[s] = W[:, None, None] * (ref + d)
    out[:, :, ~fluid] = 0.0
    return out


def floor(cfg, fmt, steps=1000, seed=5):
    """Max relative field errors (rho, u, p) and mass drift after `steps`."""
    ref, mask, _ = oracle_lattice(cfg)
    ref.step(steps)
    emu, _, _ = oracle_lattice(cfg)
    idx = source_index(mask, cfg["kind"] == "box")
    rng = np.random.default_rng(seed)
    m0 = emu.moments()["mon"]
    for _ in range(steps):
        rho = emu.f.sum(axis=1)
        emu.step(1)
        emu.f[...] = reencode(emu.f, rho, mask, idx, fmt, rng)
    R, M = ref.moments(), emu.moments()
    return (max(field_rel_err(R["rho"], M["rho"], mask)),
            max(field_rel_err(R["u"], M["u"], mask)),
            max(field_rel_err(R["p"][None], M["p"][None], mask)),
            max(abs(M["mon"][k] / m0[k] - 1) for k in (0, 1)))


def oracle_lattice3(cfg):
    """FP64 D3Q19 oracle lattice of a tube or box configuration."""
    from oracle import lbm3d as o3
    mask = synth.mask3_of(cfg)
    p = o3.Params3(cfg["nx"], cfg["ny"], cfg["nz"], tau=cfg["tau"], G=cfg["G"],
                   rho_s=cfg["rho_s"], g=cfg["g"], periodic_yz=(cfg["kind"] == "box3d"))
    return o3.Lattice3(p, mask, synth.rho03_of(cfg, mask)), mask


def source_index3(mask, periodic_yz):
    """D3Q19 counterpart of source_index, in the oracle's direction order;
    also returns the weights w_i."""
    from oracle import lbm3d as o3
    cx, cy, cz, _, _ = o3.lattice()
    nz, ny, nx = mask.shape
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    own = (z * ny + y) * nx + x
    idx = np.zeros((len(cx), nz, ny, nx), dtype=np.int64)
    for i in range(len(cx)):
        xs, ys, zs = (x - cx[i]) % nx, y - cy[i], z - cz[i]
        if periodic_yz:
            ys, zs = ys % ny, zs % nz
        ok = (ys >= 0) & (ys < ny) & (zs >= 0) & (zs < nz)
        ysc, zsc = np.clip(ys, 0, ny - 1), np.clip(zs, 0, nz - 1)
        fluid = ok & (mask[zsc, ysc, xs] == 1)
        idx[i] = np.where(fluid, (zsc * ny + ysc) * nx + xs, own)
    c2 = np.asarray(cx) ** 2 + np.asarray(cy) ** 2 + np.asarray(cz) ** 2
    w = np.where(c2 == 0, 1 / 3, np.where(c2 == 1, 1 / 18, 1 / 36))
    return idx, w


def reencode3(f, rho, mask, idx, w, fmt, rng):
    """reencode on D3Q19: f [2, 19, nz, ny, nx] in the oracle's direction
    order, w the weights (the rest direction has w = 1/3)."""
    out = np.empty_like(f)
    fluid = (mask == 1)
    i0 = int(np.argmax(w))
    W = w[:, None, None, None]
    moving = [i for i in range(len(w)) if i != i0]
    for s in range(2):
        r32 = rho[s].astype(np.float32).astype(np.float64).ravel()
        R = r32.astype(np.float16).astype(np.float64)
        ref = R[idx]
        d = _rne(f[s] / W - ref, fmt) * fluid[None]
        dsum = np.zeros(r32.size)
        np.add.at(dsum, idx[moving].ravel(), (W[moving] * d[moving]).ravel())
        rest = (r32 - R - dsum) / w[i0]
        d[i0] = (_sr(rest, fmt, rng) * fluid.ravel()).reshape(mask.shape)
        out[s] = W * (ref + d)
    out[:, :, ~fluid] = 0.0
    return out


def floor3(cfg, fmt, steps, seed=5):
    """floor() for a D3Q19 configuration: max relative errors of rho, u, p."""
    ref, mask = oracle_lattice3(cfg)
    ref.step(steps)
    R = ref.moments()
    del ref
    emu, _ = oracle_lattice3(cfg)
    idx, w = source_index3(mask, cfg["kind"] == "box3d")
    rng = np.random.default_rng(seed)
    for _ in range(steps):
        rho = emu.f.sum(axis=1)
        emu.step(1)
        emu.f[...] = reencode3(emu.f, rho, mask, idx, w, fmt, rng)
    M = emu.moments()
    m = mask.astype(bool)

    def rel(a, b):
        return max(float(np.abs(a[k][m] - b[k][m]).max() / np.abs(a[k][m]).max())
                   for k in range(a.shape[0]))
    return rel(R["rho"], M["rho"]), rel(R["u"], M["u"]), rel(R["p"][None], M["p"][None])


def tube_config():
    """The D3Q19 tube workload bench.py times."""
    return synth.config_tube(lam=256, r0=40.0, a=16.0, nx=512, ny=128, nz=128, theta=60.0,
                             tau=(1.0, 1.0), g=1e-6, slug_len=384, slug_x0=64)


def write_tube_floors(steps=20):
    import json
    cfg = tube_config()
    table = {"steps": steps, "seed": 5, "fields": ["rho", "u", "p"],
             "workload": "D3Q19 tube 512 x 128 x 128, r(x) = 40 + 16 cos(2 pi x / 256), slug 384, "
                         "theta 60 deg, g = 1e-6"}
    for fmt in ("f16", "bf16"):
        e = floor3(cfg, fmt, steps)
        table[fmt] = [float("%.3e" % v) for v in e]
        print("tube %-5s rho %.1e  u %.1e  p %.1e" % ((fmt,) + e), flush=True)
    out = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                       "storage_floor_tube.json")
    with open(out, "w") as fh:
        json.dump(table, fh, indent=1)
        fh.write("\n")


def batch_sample(cfgs):
    """The sampled instances of the 256-channel batch: the first of each
    wavelength."""
    return [next(k for k, c in enumerate(cfgs) if c["lam"] == lam) for lam in (64, 128, 256, 512)]


def write_batch_floors(steps=100):
    import json
    cfgs = synth.config_batch(n_inst=256, seed=1601)
    table = {"steps": steps, "seed": 5, "fields": ["rho", "u", "p", "mass_drift"],
             "batch": "synth.config_batch(n_inst=256, seed=1601)", "instances": {}}
    for k in batch_sample(cfgs):
        row = {"lam": int(cfgs[k]["lam"])}
        for fmt in ("f16", "bf16"):
            e = floor(cfgs[k], fmt, steps=steps)
            row[fmt] = [float("%.3e" % v) for v in e]
            print("instance %d (lambda %d) %-5s rho %.1e  u %.1e  p %.1e  mass drift %.1e"
                  % ((k, cfgs[k]["lam"], fmt) + e), flush=True)
        table["instances"][str(k)] = row
    out = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                       "storage_floor_batch.json")
    with open(out, "w") as fh:
        json.dump(table, fh, indent=1)
        fh.write("\n")


if __name__ == "__main__" and "--batch" in sys.argv:
    write_batch_floors()
elif __name__ == "__main__" and "--tube" in sys.argv:
    write_tube_floors()
elif __name__ == "__main__":
    import json
    cfgs = {"droplet": synth.config_droplet(n=128, r=20.0),
            "poiseuille": synth.config_poiseuille(),
            "channel": synth.config_channel(lam=64, theta=120.0, g=1e-5)}
    table = {"steps": 1000, "seed": 5, "fields": ["rho", "u", "p", "mass_drift"]}
    for fmt in ("f32", "f16", "bf16"):
        table[fmt] = {}
        for name, cfg in cfgs.items():
            e = floor(cfg, fmt)
            table[fmt][name] = [float("%.3e" % v) for v in e]
            print("%-5s %-10s rho %.1e  u %.1e  p %.1e  mass drift %.1e" % ((fmt, name) + e),
                  flush=True)
    if "--write" in sys.argv:
        out = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                           "storage_floor.json")
        with open(out, "w") as fh:
            json.dump(table, fh, indent=1)
            fh.write("\n")
