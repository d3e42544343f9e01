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


def fp32_storage_floor(make_lattice, steps, mask):
    """Field errors (max over components of max|d| / max|ref|, for rho, u
    and p) that binary32 storage of the populations alone leaves after
    `steps`: the FP64 oracle against the same oracle run whose populations
    are rounded to binary32 after every step (arithmetic stays FP64).  The
    floor is itself a chaotic sum of roundings (rounding the initial state
    too moves it by up to 4x on the two-layer Poiseuille), so each field
    takes the larger of the runs with and without a rounded initial state.
    make_lattice() returns a fresh oracle lattice (D2Q9 or D3Q19) at t = 0."""
    ref = make_lattice()
    ref.step(steps)
    R = ref.moments()
    worst = {"rho": 0.0, "u": 0.0, "p": 0.0}
    for round_initial in (False, True):
        emu = make_lattice()
        if round_initial:
            emu.f[...] = emu.f.astype(np.float32).astype(np.float64)
        for _ in range(steps):
            emu.step(1)
            emu.f[...] = emu.f.astype(np.float32).astype(np.float64)
        M = emu.moments()
        for k in worst:
            a, b = (R[k], M[k]) if k != "p" else (R[k][None], M[k][None])
            worst[k] = max(worst[k], max(field_rel_err(a, b, mask)))
    return worst


def fp32_storage_floor_u(make_lattice, steps, mask):
    """The velocity part of fp32_storage_floor."""
    return fp32_storage_floor(make_lattice, steps, mask)["u"]


def velocity_bound(floor):
    """Tolerance of a field after a long FP32 parity run: the 1e-5 moment bar,
    or four times the binary32 storage floor of that field where the floor
    alone is larger (the GPU adds FP32 arithmetic rounding to the storage
    rounding; measured 1.5-2.5 x the floor)."""
    return max(1e-5, 4.0 * floor)


def assert_monitors_match(ref_mon, got_mon, flow_rtol=1e-5, G=0.0):
    """GPU monitors (dict) against the oracle's mon[8] (mass o/w, momentum
    x/y, oil flux, oil cos/sin moments, bad nodes).  Masses to 1e-6 and the
    oil distribution moments to 1e-5; the flow sums (momentum, oil flux) to
    flow_rtol, the velocity tolerance of the same run, on the scale of the
    largest of them, plus the FP32 rounding of the node forces they contain
    (2^-24 |G| per unit of mass: at wall nodes the force G rho rho_s / 6 is
    large and cancels against j node by node, so a flow at rest still sums to
    a few units in the last place of those forces)."""
    np.testing.assert_allclose(got_mon["mass"], ref_mon[:2], rtol=1e-6)
    mass = ref_mon[0] + ref_mon[1]
    flow_scale = max(abs(ref_mon[2]), abs(ref_mon[3]), abs(ref_mon[4]), 1e-300)
    force_floor = 2.0 ** -24 * max(abs(G), 1.0) * mass
    for got, want in ((got_mon["momentum"][0], ref_mon[2]), (got_mon["momentum"][1], ref_mon[3]),
                      (got_mon["oil_flux"], ref_mon[4])):
        assert abs(got - want) <= flow_rtol * flow_scale + force_floor, (got, want)
    for got, want in ((got_mon["oil_cos"], ref_mon[5]), (got_mon["oil_sin"], ref_mon[6])):
        assert abs(got - want) <= 1e-5 * abs(want) + 1e-6 * ref_mon[0], (got, want)
    assert got_mon["bad_nodes"] == 0 and ref_mon[7] == 0
