"""Helpers shared by the GPU parity tests (inputs from synth, reference from
the oracle, device side through the C ABI binding)."""
import numpy as np

import synth
from oracle import lbm as orc


def oracle_lattice(cfg, rho0=None, mask=None):
    mask = synth.mask_of(cfg) if mask is None else mask
    rho0 = synth.rho0_of(cfg, mask) if rho0 is None else rho0
    p = orc.Params(cfg["nx"], cfg["ny"], tau=cfg["tau"], G=cfg["G"], rho_s=cfg["rho_s"],
                   g=cfg["g"], periodic_y=(cfg["kind"] == "box"),
                   reg_order=cfg.get("reg_order", 2))
    return orc.Lattice(p, mask, rho0), mask, rho0


def field_rel_err(ref, got, mask):
    """max |got - ref| / max |ref| over fluid nodes, per leading index."""
    m = mask.astype(bool)
    out = []
    for k in range(ref.shape[0]):
        a = ref[k][m]
        b = got[k][m]
        scale = np.abs(a).max()
        out.append(float(np.abs(a - b).max() / scale) if scale > 0 else float(np.abs(b).max()))
    return out


def fp32_storage_floor_u(make_lattice, steps, mask):
    """Velocity error (max over components of max|du| / max|u|) that binary32
    storage of the populations alone leaves after `steps`: the FP64 oracle
    against the same oracle run whose populations are rounded to binary32
    initially and after every step (arithmetic stays FP64).  make_lattice()
    returns a fresh oracle lattice (D2Q9 or D3Q19) at t = 0."""
    ref, emu = make_lattice(), make_lattice()
    ref.step(steps)
    emu.f[...] = emu.f.astype(np.float32).astype(np.float64)
    for _ in range(steps):
        emu.step(1)
        emu.f[...] = emu.f.astype(np.float32).astype(np.float64)
    return max(field_rel_err(ref.moments()["u"], emu.moments()["u"], mask))


def velocity_bound(floor):
    """Velocity tolerance of a 1000-step FP32 parity test: the 1e-5 moment
    bar, or four times the binary32 storage floor where that floor alone is
    larger (the GPU adds FP32 arithmetic rounding to the storage rounding)."""
    return max(1e-5, 4.0 * floor)


def assert_monitors_match(ref_mon, got_mon, rtol=1e-5):
    """GPU monitors (dict) against the oracle's mon[8] (mass o/w, momentum
    x/y, oil flux, oil cos/sin moments, bad nodes).  Sums of signed terms are
    compared on the scale of the total mass times the largest |term| / rho."""
    mass = ref_mon[0] + ref_mon[1]
    np.testing.assert_allclose(got_mon["mass"], ref_mon[:2], rtol=1e-6)
    mom_scale = max(abs(ref_mon[2]), abs(ref_mon[3]), abs(ref_mon[4]), 1e-300)
    for got, want in ((got_mon["momentum"][0], ref_mon[2]), (got_mon["momentum"][1], ref_mon[3]),
                      (got_mon["oil_flux"], ref_mon[4])):
        assert abs(got - want) <= rtol * mom_scale + 1e-12 * mass, (got, want)
    for got, want in ((got_mon["oil_cos"], ref_mon[5]), (got_mon["oil_sin"], ref_mon[6])):
        assert abs(got - want) <= rtol * abs(want) + 1e-6 * ref_mon[0], (got, want)
    assert got_mon["bad_nodes"] == 0 and ref_mon[7] == 0
