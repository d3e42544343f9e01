"""Independent vectorised numpy transcription of the two-component step on
the D3Q19 lattice, used only to cross-check the C oracle on tiny lattices.
The velocity set is generated here (all c in {-1,0,1}^3 with |c|^2 <= 2, in
this file's own order) and the weights from |c|^2; streaming is done with
array shifts instead of node loops.  Same equations as the oracle: Eqs. 1,
3-10, wall potentials, half-way bounce-back.  Test infrastructure."""
import itertools

import numpy as np

VEL = np.array([c for c in itertools.product((-1, 0, 1), repeat=3) if sum(v * v for v in c) <= 2])
WT = np.array([{0: 1 / 3, 1: 1 / 18, 2: 1 / 36}[int((c * c).sum())] for c in VEL])
OPP = np.array([int(np.nonzero((VEL == -c).all(axis=1))[0][0]) for c in VEL])


def _shift(a, c, periodic_yz, fill):
    """b[..., z, y, x] = a[..., z + cz, y + cy, x + cx] (x periodic; y, z
    periodic or filled with `fill` outside the box)."""
    cx, cy, cz = (int(v) for v in c)
    out = np.roll(a, -cx, axis=-1)
    if periodic_yz:
        return np.roll(np.roll(out, -cy, axis=-2), -cz, axis=-3)
    for ax, d in ((-2, cy), (-3, cz)):
        if d == 0:
            continue
        moved = np.roll(out, -d, axis=ax)
        idx = [slice(None)] * out.ndim
        idx[ax] = slice(-1, None) if d == 1 else slice(0, 1)
        moved[tuple(idx)] = fill
        out = moved
    return out


def run(f, mask, tau, G, rho_s, g, steps, periodic_yz):
    """f: [2, 19, nz, ny, nx] in this file's velocity order."""
    fl = mask.astype(bool)
    T0 = 1.0 / 3.0
    nb_fluid = [_shift(fl, c, periodic_yz, False) for c in VEL]
    src_fluid = [_shift(fl, -c, periodic_yz, False) for c in VEL]
    for _ in range(steps):
        rho = f.sum(axis=1)
        j = np.einsum('ia,sizyx->sazyx', VEL.astype(float), f)
        rt = np.where(fl, rho[0] + rho[1], 1.0)
        u = (j[0] + j[1]) / rt
        nu = T0 * (np.array(tau) - 0.5)
        taum = (rho[0] * nu[0] + rho[1] * nu[1]) / rt / T0 + 0.5
        om = 1.0 - 1.0 / taum
        fnew = np.zeros_like(f)
        for s in range(2):
            b = 1 - s
            S = np.zeros((3,) + mask.shape)
            for i, c in enumerate(VEL):
                if not c.any():
                    continue
                rb = np.where(nb_fluid[i], _shift(rho[b], c, periodic_yz, 0.0), rho_s[b])
                S += WT[i] * c[:, None, None, None] * rb
            rs = np.where(fl, rho[s], 1.0)
            vs = u + G * S + np.array(g)[:, None, None, None]
            vo = j[s] / rs

            def feq(v, i):
                cu = np.tensordot(VEL[i].astype(float), v, axes=1)
                usq = (v * v).sum(axis=0)
                return rho[s] * WT[i] * (1 + cu / T0 + cu * cu / (2 * T0 ** 2) - usq / (2 * T0)
                                         + cu ** 3 / (6 * T0 ** 3) - cu * usq / (2 * T0 ** 2))
            P = np.zeros((3, 3) + mask.shape)
            for i, c in enumerate(VEL):
                d = f[s, i] - feq(vo, i)
                P += np.outer(c, c)[:, :, None, None, None] * d
            for i, c in enumerate(VEL):
                H = np.outer(c, c) - T0 * np.eye(3)
                fneq = WT[i] / (2 * T0 ** 2) * np.einsum('ab,abzyx->zyx', H, P)
                fp = (feq(vs, i) + om * fneq) * fl
                fnew[s, i] += np.where(src_fluid[i], _shift(fp, -c, periodic_yz, 0.0), 0.0)
                fnew[s, OPP[i]] += np.where(~nb_fluid[i], fp, 0.0)
        f = fnew * fl
    return f
