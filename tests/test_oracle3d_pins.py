"""Pins of the D3Q19 oracle (oracle/lbm3d_oracle.c) against what mathematics
and an independent implementation fix: lattice isotropy, equilibrium and
regularization moments, a numpy transcription of the step on tiny lattices,
exact mass conservation in a closed tube, the Laplace law for 3-D droplets,
and the interpolated tube walls (link fractions in closed form, second-order
Hagen-Poiseuille, mass kept)."""
import itertools

import numpy as np
import pytest

import synth
from oracle import lbm3d as o3
from tests import np_bruteforce3d as bf

T0 = 1.0 / 3.0


def test_lattice_isotropy():
    cx, cy, cz, w, opp = o3.lattice()
    c = np.stack([cx, cy, cz], axis=1).astype(float)
    assert len(w) == 19 and w.sum() == pytest.approx(1.0, abs=1e-15)
    assert np.allclose(c[opp], -c)
    assert np.allclose(np.einsum('i,ia->a', w, c), 0)
    assert np.allclose(np.einsum('i,ia,ib->ab', w, c, c), T0 * np.eye(3), atol=1e-15)
    assert np.allclose(np.einsum('i,ia,ib,ic->abc', w, c, c, c), 0)
    d = np.eye(3)
    iso4 = T0 ** 2 * (np.einsum('ab,cd->abcd', d, d) + np.einsum('ac,bd->abcd', d, d) +
                      np.einsum('ad,bc->abcd', d, d))
    assert np.allclose(np.einsum('i,ia,ib,ic,id->abcd', w, c, c, c, c), iso4, atol=1e-15)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_equilibrium_moments(seed):
    """Eq. 7 on D3Q19: mass rho, momentum rho u and momentum flux
    rho T0 I + rho u u exactly (the cubic terms cancel in the first moment by
    fourth-order isotropy and vanish in the even moments)."""
    rng = np.random.default_rng(seed)
    rho = 0.3 + rng.random()
    u = 0.1 * rng.standard_normal(3)
    feq = o3.equilibrium(rho, *u)
    cx, cy, cz, w, _ = o3.lattice()
    c = np.stack([cx, cy, cz], axis=1).astype(float)
    assert feq.sum() == pytest.approx(rho, rel=1e-14)
    assert np.allclose(c.T @ feq, rho * u, rtol=0, atol=1e-15)
    assert np.allclose(np.einsum('ia,ib,i->ab', c, c, feq),
                       rho * T0 * np.eye(3) + rho * np.outer(u, u), rtol=0, atol=1e-15)


def test_regularized_part_reproduces_the_nonequilibrium_flux():
    rng = np.random.default_rng(4)
    f = 0.05 + 0.02 * rng.random(19)
    feq = o3.equilibrium(f.sum(), 0.02, -0.01, 0.03)
    fneq = o3.regularize(f, feq)
    cx, cy, cz, _, _ = o3.lattice()
    c = np.stack([cx, cy, cz], axis=1).astype(float)
    P = np.einsum('ia,ib,i->ab', c, c, f - feq)
    assert abs(fneq.sum()) < 1e-15 and np.allclose(c.T @ fneq, 0, atol=1e-15)
    assert np.allclose(np.einsum('ia,ib,i->ab', c, c, fneq), P, atol=1e-15)


def _to_bf(f):
    """oracle direction order -> the brute force's velocity order."""
    cx, cy, cz, _, _ = o3.lattice()
    c = np.stack([cx, cy, cz], axis=1)
    perm = [int(np.nonzero((c == v).all(axis=1))[0][0]) for v in bf.VEL]
    return f[:, perm]


@pytest.mark.parametrize("case", ["box", "tube"])
def test_step_matches_independent_numpy_transcription(case):
    rng = np.random.default_rng(7)
    if case == "box":
        nz, ny, nx = 3, 4, 5
        mask = np.ones((nz, ny, nx), dtype=np.uint8)
        periodic = True
    else:
        nz, ny, nx = 5, 6, 6
        mask = (rng.random((nz, ny, nx)) < 0.75).astype(np.uint8)
        periodic = False
    p = o3.Params3(nx, ny, nz, tau=(0.8, 1.3), G=-2.7, rho_s=(0.3, 0.6),
                   g=(1e-3, -2e-4, 5e-4), periodic_yz=periodic)
    w = o3.lattice()[3]
    base = 0.03 + 0.97 * rng.random((2, 1, nz, ny, nx))
    f = w[None, :, None, None, None] * base * (1 + 0.05 * rng.uniform(-1, 1, (2, 19, nz, ny, nx)))
    f *= mask[None, None]
    got = f.copy()
    for _ in range(3):
        got, bad = o3.step_once(p, mask, got)
        assert bad == 0
    ref = bf.run(_to_bf(f), mask, (0.8, 1.3), -2.7, (0.3, 0.6), (1e-3, -2e-4, 5e-4), 3,
                 periodic)
    assert np.abs(_to_bf(got) - ref).max() < 1e-14


def test_closed_tube_conserves_each_species_mass():
    cfg = synth.config_tube(lam=32, r0=6.0, a=2.0, theta=60.0, g=2e-4)
    mask = synth.mask3_of(cfg)
    p = o3.Params3(cfg["nx"], cfg["ny"], cfg["nz"], tau=cfg["tau"], G=cfg["G"],
                   rho_s=cfg["rho_s"], g=cfg["g"])
    L = o3.Lattice3(p, mask, synth.rho03_of(cfg, mask))
    m0 = L.moments()["mon"][:2]
    L.step(200)
    m1 = L.moments()["mon"][:2]
    assert np.allclose(m1, m0, rtol=1e-12, atol=0)


def test_laplace_law_for_3d_droplets():
    """Delta p = 2 sigma / R (Eq. 11 in 3-D): the jump between the droplet
    centre and the far field is linear in 1/R through the origin."""
    inv_r, dp = [], []
    for r in (5.0, 6.5, 8.0):
        cfg = synth.config_box3d(n=24, r=r)
        mask = synth.mask3_of(cfg)
        p = o3.Params3(24, 24, 24, tau=cfg["tau"], G=cfg["G"], periodic_yz=True)
        L = o3.Lattice3(p, mask, synth.rho03_of(cfg, mask))
        L.step(1200)
        m = L.moments()
        rho_o = m["rho"][0]
        R = (3.0 * (rho_o > 0.5).sum() / (4.0 * np.pi)) ** (1.0 / 3.0)  # from the volume
        pr = m["p"]
        dp.append(pr[10:14, 10:14, 10:14].mean() - pr[0:3, 0:3, 0:3].mean())
        inv_r.append(1.0 / R)
    slope, icpt = np.polyfit(inv_r, dp, 1)
    fit = np.polyval([slope, icpt], inv_r)
    resid = np.abs(fit - dp).max() / max(dp)
    print("1/R", inv_r, "dp", dp, "slope", slope, "intercept", icpt)
    assert slope > 0 and resid < 0.02
    assert abs(icpt) < 0.1 * min(dp)


def test_momentum_budget_with_body_force():
    """D3Q19: from rest on a periodic box with body acceleration g, the
    physical momentum (u_mix + (F^o + F^w) / (2 rho)) after t steps is
    M g (t + 1/2), since every collision adds the node's force and the
    pairwise interaction forces cancel (Eqs. 8-9)."""
    cfg = synth.config_box3d(n=16, r=5.0, tau=(0.8, 1.1))
    mask = synth.mask3_of(cfg)
    g = (1e-5, -4e-6, 2.5e-6)
    L = o3.Lattice3(o3.Params3(16, 16, 16, tau=cfg["tau"], G=cfg["G"], g=g, periodic_yz=True),
                    mask, synth.rho03_of(cfg, mask))
    for t in (0, 1, 10, 40):
        L.step(t - L.t)
        m = L.moments()
        rho = m["rho"].sum(axis=0)
        mass = m["rho"].sum()
        for k in range(3):
            want = mass * g[k] * (t + 0.5)
            assert abs((rho * m["u"][k]).sum() / want - 1) < 1e-10, (t, k)


def test_flat_interface_equal_bulk_pressures():
    """D3Q19 flat oil band with unequal inventories at rest: equal bulk
    pressures under the bulk equation of state T0 sum rho - G T0 rho^o rho^w,
    unequal ones (beyond 1e-4) under the opposite sign of the interaction
    term.  The bands are 32 rows wide so that their centres are bulk to
    rounding (24-row bands leave 2e-8 of interface tail at the centre)."""
    nx, ny, nz = 2, 2, 64
    mask = np.ones((nz, ny, nx), dtype=np.uint8)
    z = np.arange(nz)[:, None, None] * np.ones((1, ny, nx))
    oil = (z >= 16) & (z < 48)
    rho0 = np.stack([np.where(oil, 1.0, 0.03), np.where(oil, 0.02, 0.6)])
    G = synth.G_DEFAULT
    L = o3.Lattice3(o3.Params3(nx, ny, nz, tau=(1.0, 1.0), G=G, periodic_yz=True), mask, rho0)
    L.step(20000)
    m = L.moments()
    po, pw = m["p"][32, 0, 0], m["p"][0, 0, 0]
    ro, rw = m["rho"][:, 32, 0, 0], m["rho"][:, 0, 0, 0]
    assert not np.allclose(ro[::-1], rw, rtol=1e-4)
    assert abs(po / pw - 1) < 1e-9
    assert abs(po - (T0 * ro.sum() - G * T0 * ro[0] * ro[1])) < 1e-15

    def flipped(r):
        return T0 * r.sum() + G * T0 * r[0] * r[1]

    assert abs(flipped(ro) / flipped(rw) - 1) > 1e-4


# ---- interpolated (sub-lattice) tube walls -----------------------------------
def test_tube_wall_fraction_geometry():
    """Link fractions against the straight tube's closed form along the axes
    and a direct root of the sinusoidal wall along a face diagonal."""
    from scipy.optimize import brentq
    import math
    cx, cy, cz, _, _ = o3.lattice()
    R, side = 5.3, 13
    yc = zc = 0.5 * (side - 1)
    p = o3.Params3(4, side, side, wall=(yc, zc, R, 0.0, 1.0))
    mask = synth.tube_mask(4, side, side, 1.0, R, 0.0)
    checked = 0
    for z, y in itertools.product(range(side), range(side)):
        if not mask[z, y, 0]:
            continue
        for i in (3, 4, 5, 6):          # +-y, +-z
            if mask[z + cz[i], y + cy[i], 0]:
                continue
            if cy[i]:
                want = math.sqrt(R * R - (z - zc) ** 2) - cy[i] * (y - yc)
            else:
                want = math.sqrt(R * R - (y - yc) ** 2) - cz[i] * (z - zc)
            assert 0.0 < want <= 1.0
            assert o3.wall_fraction(p, 1, y, z, i) == pytest.approx(want, abs=1e-12)
            checked += 1
    assert checked > 20
    cfg = synth.config_tube(lam=32, r0=6.0, a=2.0)
    ny, nz = cfg["ny"], cfg["nz"]
    yc, zc = 0.5 * (ny - 1), 0.5 * (nz - 1)
    ps = o3.Params3(cfg["nx"], ny, nz, wall=(yc, zc, cfg["r0"], cfg["a"], cfg["lam"]))
    m = synth.mask3_of(cfg)
    checked = 0
    for x in (3, 11, 20):
        for z, y in itertools.product(range(nz), range(ny)):
            if not m[z, y, x]:
                continue
            for i in (7, 11, 16):       # (1,1,0), (1,0,1), (0,-1,-1)
                xn = (x + cx[i]) % cfg["nx"]
                if m[z + cz[i], y + cy[i], xn]:
                    continue

                def gap(t):
                    X, Y, Z = x + t * cx[i], y + t * cy[i], z + t * cz[i]
                    r = cfg["r0"] + cfg["a"] * math.cos(2 * math.pi * X / cfg["lam"])
                    return math.hypot(Y - yc, Z - zc) - r
                want = brentq(gap, 0.0, 1.0, xtol=1e-15)
                assert o3.wall_fraction(ps, x, y, z, i) == pytest.approx(want, abs=1e-12)
                checked += 1
    assert checked > 20


def test_interpolated_tube_walls_give_hagen_poiseuille():
    """A single fluid (G = 0, uniform densities) driven along a straight tube
    whose radius R falls between nodes: the steady profile is Hagen-Poiseuille,
    u = g (R^2 - rho^2) / (4 nu), vanishing at the analytic wall.  With
    interpolated walls the error falls by about four when R doubles (second
    order); the staircase of half-way bounce-back on the same nodes does not
    converge (its effective radius varies around the circle) and is over ten
    times further off at the finer radius."""
    tau = 0.8
    nu = (tau - 0.5) / 3.0
    errs = {}
    for R in (4.3, 8.6):
        g = 1e-5 * (4.3 / R) ** 2
        side = int(2 * R + 3)
        mask = synth.tube_mask(2, side, side, 1.0, R, 0.0)
        yc = zc = 0.5 * (side - 1)
        rho0 = np.stack([np.full(mask.shape, 0.5)] * 2) * mask
        zz, yy = np.meshgrid(np.arange(side), np.arange(side), indexing="ij")
        want = g * (R * R - (yy - yc) ** 2 - (zz - zc) ** 2) / (4.0 * nu)
        fl = mask[:, :, 0].astype(bool)
        for interp in (True, False):
            p = o3.Params3(2, side, side, tau=(tau, tau), G=0.0, g=(g, 0.0, 0.0),
                           wall=(yc, zc, R, 0.0, 1.0) if interp else None)
            L = o3.Lattice3(p, mask, rho0)
            L.step(int(3000 * (R / 4.3) ** 2))
            u = L.moments()["u"][0][:, :, 0]
            errs[R, interp] = np.abs(u[fl] - want[fl]).max() / want.max()
    print({k: "%.2e" % v for k, v in errs.items()})
    assert errs[4.3, True] < 0.025 and errs[8.6, True] < 0.005
    assert 3.3 < errs[4.3, True] / errs[8.6, True] < 5.5
    assert errs[8.6, False] > 10 * errs[8.6, True]


def test_interpolated_tube_walls_keep_each_species_mass():
    """Two-component slug with wall potentials in a sinusoidal tube: what the
    interpolated walls add returns through the rest population, so each
    species' mass stays constant to rounding."""
    cfg = synth.config_tube(lam=32, r0=6.0, a=2.0, theta=60.0, g=2e-4)
    mask = synth.mask3_of(cfg)
    yc, zc = 0.5 * (cfg["ny"] - 1), 0.5 * (cfg["nz"] - 1)
    p = o3.Params3(cfg["nx"], cfg["ny"], cfg["nz"], tau=cfg["tau"], G=cfg["G"],
                   rho_s=cfg["rho_s"], g=cfg["g"],
                   wall=(yc, zc, cfg["r0"], cfg["a"], cfg["lam"]))
    L = o3.Lattice3(p, mask, synth.rho03_of(cfg, mask))
    m0 = L.moments()["mon"][:2]
    L.step(200)
    m1 = L.moments()["mon"][:2]
    assert np.allclose(m1, m0, rtol=1e-12, atol=0)
