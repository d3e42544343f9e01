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
