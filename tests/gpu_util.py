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
