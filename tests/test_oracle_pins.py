"""Pins of the FP64 oracle against facts fixed by the paper and the mathematics
(not against the oracle itself).  CPU only."""
import itertools
import math

import numpy as np
import pytest

import synth
from oracle import lbm as orc

T0 = 1.0 / 3.0


def _D2Q9():
    cx, cy, w, opp = orc.lattice()
    return cx.astype(float), cy.astype(float), w, opp


# ------------------------------------------------------------ velocity set ---
def test_d2q9_moment_isotropy():
    """Sum w = 1, odd moments vanish, sum w c_a c_b = T0 delta_ab and the
    fourth moment is T0^2 (dd + dd + dd): the D2Q9 quadrature facts Eq. 7
    relies on (T0 = 1/3, Sec. 2)."""
    cx, cy, w, opp = _D2Q9()
    c = np.stack([cx, cy])
    assert abs(w.sum() - 1.0) < 1e-15
    for a in range(2):
        assert abs((w * c[a]).sum()) < 1e-15
        for b in range(2):
            assert abs((w * c[a] * c[b]).sum() - T0 * (a == b)) < 1e-15
            for g in range(2):
                assert abs((w * c[a] * c[b] * c[g]).sum()) < 1e-15
                for d in range(2):
                    want = T0 * T0 * ((a == b) * (g == d) + (a == g) * (b == d)
                                      + (a == d) * (b == g))
                    assert abs((w * c[a] * c[b] * c[g] * c[d]).sum() - want) < 1e-15
    assert np.all(cx[opp] == -cx) and np.all(cy[opp] == -cy)
    assert sorted(set(zip(cx, cy))) == sorted(itertools.product([-1, 0, 1], repeat=2))


# ------------------------------------------------------------ equilibrium ---
@pytest.mark.parametrize("seed", range(5))
def test_equilibrium_hermite_moments(seed):
    """Eq. 7 is the Hermite expansion to third order: its first three moments
    are rho, rho u, rho (T0 I + u u), and on D2Q9 the two representable third
    Hermite moments (H_xxy, H_xyy) are rho ux^2 uy and rho ux uy^2."""
    rng = np.random.default_rng(seed)
    rho = rng.uniform(0.02, 1.5)
    ux, uy = rng.uniform(-0.15, 0.15, size=2)
    cx, cy, w, _ = _D2Q9()
    f = orc.equilibrium(rho, ux, uy)
    assert abs(f.sum() - rho) < 1e-15 * 4
    assert abs((cx * f).sum() - rho * ux) < 1e-15 * 4
    assert abs((cy * f).sum() - rho * uy) < 1e-15 * 4
    assert abs((cx * cx * f).sum() - rho * (T0 + ux * ux)) < 1e-15 * 4
    assert abs((cx * cy * f).sum() - rho * ux * uy) < 1e-15 * 4
    assert abs((cy * cy * f).sum() - rho * (T0 + uy * uy)) < 1e-15 * 4
    assert abs(((cx * cx - T0) * cy * f).sum() - rho * ux * ux * uy) < 1e-15 * 4
    assert abs(((cy * cy - T0) * cx * f).sum() - rho * ux * uy * uy) < 1e-15 * 4


def test_equilibrium_worked_values():
    """Hand evaluation of Eq. 7 at rho = 1, u = (0.1, 0):
    bracket(c = +x) = 1 + .3 + .045 - .015 + .0045 - .0045 = 1.33,
    bracket(c = -x) = 0.73, bracket(c = +-y) = 0.985, bracket(rest) = 0.985,
    bracket(diagonals with c_x = +1) = 1.33, with c_x = -1: 0.73."""
    f = orc.equilibrium(1.0, 0.1, 0.0)
    want = [4 / 9 * 0.985, 1.33 / 9, 0.985 / 9, 0.73 / 9, 0.985 / 9,
            1.33 / 36, 0.73 / 36, 0.73 / 36, 1.33 / 36]
    np.testing.assert_allclose(f, want, rtol=1e-14)
    np.testing.assert_allclose(orc.equilibrium(0.7, 0.0, 0.0), 0.7 * _D2Q9()[2], rtol=1e-15)


# ------------------------------------------------------------ regularizer ---
@pytest.mark.parametrize("seed", range(5))
def test_regularizer_projection(seed):
    """Eq. 6: f' carries no mass and no momentum, its second moment is the
    non-equilibrium momentum flux, and projecting again changes nothing."""
    rng = np.random.default_rng(seed)
    cx, cy, w, _ = _D2Q9()
    rho = rng.uniform(0.1, 1.2)
    u = rng.uniform(-0.1, 0.1, size=2)
    feq = orc.equilibrium(rho, *u)
    f = feq * (1 + 0.05 * rng.uniform(-1, 1, size=9))
    fp, pi = orc.regularize(f, feq)
    d = f - feq
    assert abs(fp.sum()) < 1e-16
    assert abs((cx * fp).sum()) < 1e-16 and abs((cy * fp).sum()) < 1e-16
    np.testing.assert_allclose([(cx * cx * fp).sum(), (cx * cy * fp).sum(), (cy * cy * fp).sum()],
                               [(cx * cx * d).sum(), (cx * cy * d).sum(), (cy * cy * d).sum()],
                               atol=1e-16)
    np.testing.assert_allclose(pi, [(cx * cx * d).sum(), (cx * cy * d).sum(), (cy * cy * d).sum()],
                               atol=1e-16)
    fp2, _ = orc.regularize(feq + fp, feq)
    np.testing.assert_allclose(fp2, fp, atol=1e-17)


def test_regularizer_removes_higher_modes():
    """Modes with zero second moment (the third-order g_xxy-type and the
    fourth-order ghost) are filtered out entirely."""
    cx, cy, w, _ = _D2Q9()
    feq = orc.equilibrium(1.0, 0.02, -0.03)
    for mode in [(cx * cx - T0) * cy, (cy * cy - T0) * cx, (cx * cx - T0) * (cy * cy - T0)]:
        fp, _ = orc.regularize(feq + 1e-3 * w * mode, feq)
        assert np.abs(fp).max() < 1e-16  # perturbation is ~1e-4


# --------------------------------------------------------- mixed relaxation --
def test_tau_mix_limits():
    """Eqs. 4-5: a pure species relaxes with its own tau; equal taus give that
    tau for any mixture; the mixed viscosity is the density-weighted mean."""
    p = orc.Params(4, 4, tau=(0.6, 1.5))
    assert abs(orc.tau_mix(p, 1.0, 0.0) - 0.6) < 1e-15
    assert abs(orc.tau_mix(p, 0.0, 1.0) - 1.5) < 1e-15
    q = orc.Params(4, 4, tau=(0.8, 0.8))
    assert abs(orc.tau_mix(q, 0.3, 0.9) - 0.8) < 1e-15
    nu = T0 * (orc.tau_mix(p, 0.25, 0.75) - 0.5)
    assert abs(nu - (0.25 * T0 * 0.1 + 0.75 * T0 * 1.0)) < 1e-15


# ------------------------------------------------------- interaction force --
def test_force_uniform_and_linear():
    """Eq. 8: a uniform neighbour density exerts no force; a linear profile
    rho^b = a + b x gives sum_i w_i c_i rho^b(x + c_i) = T0 b exactly."""
    nx, ny = 16, 8
    mask = synth.box_mask(nx, ny)
    p = orc.Params(nx, ny, periodic_y=True)
    rho = np.zeros((2, ny, nx))
    rho[1] = 0.4
    assert orc.interaction_sum(p, mask, rho, 1, 5, 3) == (0.0, 0.0)
    rho[1] = 0.2 + 0.01 * np.arange(nx)[None, :]
    sx, sy = orc.interaction_sum(p, mask, rho, 1, 6, 4)
    assert abs(sx - T0 * 0.01) < 1e-16 and abs(sy) < 1e-17
    rho[1] = 0.2 + 0.03 * np.arange(ny)[:, None]
    sx, sy = orc.interaction_sum(p, mask, rho, 1, 6, 4)
    assert abs(sy - T0 * 0.03) < 1e-16 and abs(sx) < 1e-17


def test_force_flat_wall_potential():
    """A flat wall below a uniform fluid: the three solid neighbours carry the
    wall potential, so S_y = (rho^b - rho_s^b) (1/9 + 2/36) = (rho^b - rho_s^b)/6."""
    cfg = synth.config_poiseuille(nx=8, width=6, G=-3.0)
    mask = synth.mask_of(cfg)
    p = orc.Params(8, 8, rho_s=(0.37, 0.11))
    rho = np.zeros((2, 8, 8))
    rho[0][mask == 1] = 0.8
    rho[1][mask == 1] = 0.05
    sx, sy = orc.interaction_sum(p, mask, rho, 1, 3, 1)   # first fluid row, species w
    assert abs(sx) < 1e-17 and abs(sy - (0.05 - 0.11) / 6.0) < 1e-16
    sx, sy = orc.interaction_sum(p, mask, rho, 0, 3, 6)   # last fluid row, species o
    assert abs(sx) < 1e-17 and abs(sy + (0.8 - 0.37) / 6.0) < 1e-16


def test_force_pairwise_antisymmetry():
    """Newton's third law of Eq. 8: on a periodic wall-free lattice the forces
    of the two species on each other sum to zero over the domain."""
    nx, ny = 12, 10
    mask = synth.box_mask(nx, ny)
    p = orc.Params(nx, ny, periodic_y=True)
    rho = synth.random_field(nx, ny, mask, seed=3, amp=0.5)
    tot = np.zeros(2)
    for y in range(ny):
        for x in range(nx):
            so = orc.interaction_sum(p, mask, rho, 1, x, y)
            sw = orc.interaction_sum(p, mask, rho, 0, x, y)
            tot += rho[0, y, x] * np.array(so) + rho[1, y, x] * np.array(sw)
    assert np.abs(tot).max() < 1e-15


# ----------------------------------------------------------- whole steps ----
def test_bgk_special_case_tau_one():
    """With tau_mix = 1 the regularized collision (Eq. 3) reduces to
    f* = f^eq(rho^a, u*): the non-equilibrium part is multiplied by zero.
    Here G = 0 and g = 0, so u* = u_mix; checked through one full step on a
    periodic lattice, where streaming is a pure shift."""
    nx, ny = 6, 5
    mask = synth.box_mask(nx, ny)
    p = orc.Params(nx, ny, tau=(1.0, 1.0), G=0.0, periodic_y=True)
    f = synth.random_populations(nx, ny, mask, seed=7, amp=0.1)
    out, bad = orc.step_once(p, mask, f)
    assert bad == 0
    cx, cy, w, _ = _D2Q9()
    for y in range(ny):
        for x in range(nx):
            rho = f[:, :, y, x].sum(axis=1)
            j = np.array([(cx * f[:, :, y, x]).sum(), (cy * f[:, :, y, x]).sum()])
            u = j / rho.sum()
            for s in range(2):
                feq = orc.equilibrium(rho[s], *u)
                got = [out[s, i, (y + int(cy[i])) % ny, (x + int(cx[i])) % nx] for i in range(9)]
                np.testing.assert_allclose(got, feq, rtol=1e-14, atol=1e-17)


def test_mass_and_momentum_conservation():
    """Streaming with half-way bounce-back conserves each species' mass
    exactly; without walls and body force the pairwise interaction conserves
    total momentum (sum F = 0)."""
    cfg = synth.config_channel(lam=64, theta=120.0, g=1e-5, tau=(0.7, 1.3))
    L = orc.Lattice(orc.Params(cfg["nx"], cfg["ny"], tau=cfg["tau"], G=cfg["G"],
                               rho_s=cfg["rho_s"], g=cfg["g"]), synth.mask_of(cfg),
                    synth.rho0_of(cfg))
    m0 = L.moments()["mon"]
    L.step(300)
    m1 = L.moments()["mon"]
    np.testing.assert_allclose(m1[:2], m0[:2], rtol=1e-13)

    cfg = synth.config_droplet(n=32, r=7.0)
    mask = synth.mask_of(cfg)
    L = orc.Lattice(orc.Params(32, 32, tau=(0.8, 1.1), G=cfg["G"], periodic_y=True), mask,
                    synth.rho0_of(cfg, mask))
    L.step(300)
    m = L.moments()["mon"]
    assert abs(m[2]) < 1e-12 and abs(m[3]) < 1e-12


def test_momentum_budget_with_body_force():
    """Each collision adds the node's total force to its momentum (the shifted
    equilibrium of Eq. 9 carries rho^a u_mix + F^a), the interaction forces of
    Eq. 8 cancel in pairs on a periodic lattice, and the reported velocity is
    u_mix + (F^o + F^w) / (2 rho).  From rest, the physical momentum after t
    steps is therefore M g (t + 1/2) exactly: a dropped or doubled half-force
    term, or a force that enters the collision with the wrong weight, breaks
    it by at least 1 / (2 t + 1)."""
    cfg = synth.config_droplet(n=32, r=7.0)
    mask = synth.mask_of(cfg)
    g = (1e-5, -4e-6)
    L = orc.Lattice(orc.Params(32, 32, tau=(0.8, 1.1), G=cfg["G"], g=g, periodic_y=True),
                    mask, synth.rho0_of(cfg, mask))
    for t in (0, 1, 10, 100):
        L.step(t - L.t)
        m = L.moments()
        rho = m["rho"].sum(axis=0)
        mass = m["rho"].sum()
        for k in range(2):
            want = mass * g[k] * (t + 0.5)
            assert abs((rho * m["u"][k]).sum() / want - 1) < 1e-10, (t, k)
            assert abs(m["mon"][2 + k] / want - 1) < 1e-10, (t, k)


def test_uniform_flow_is_steady():
    """A uniform state moving at constant velocity is a fixed point of the
    step on a periodic lattice (equilibrium is reproduced by the collision and
    shifted onto itself by streaming)."""
    nx, ny = 8, 6
    mask = synth.box_mask(nx, ny)
    p = orc.Params(nx, ny, tau=(0.7, 1.4), G=0.0, periodic_y=True)
    f = np.zeros((2, 9, ny, nx))
    f[0] = orc.equilibrium(0.6, 0.05, -0.02)[:, None, None]
    f[1] = orc.equilibrium(0.4, 0.05, -0.02)[:, None, None]
    out, bad = orc.step_once(p, mask, f)
    np.testing.assert_allclose(out, f, rtol=1e-15, atol=1e-17)


@pytest.mark.parametrize("tau", [(0.6, 0.6), (0.6, 1.5)])
def test_shear_wave_decay_viscosity(tau):
    """A sinusoidal shear wave u_x = U sin(k y) decays as exp(-nu k^2 t), with
    the mixed viscosity nu = sum rho^a nu^a / rho (Eqs. 4-5) when the two
    species are uniformly mixed and do not interact (G = 0)."""
    nx, ny = 4, 64
    mask = synth.box_mask(nx, ny)
    ro, rw = 0.3, 0.7
    p = orc.Params(nx, ny, tau=tau, G=0.0, periodic_y=True)
    k = 2 * math.pi / ny
    U = 1e-3
    f = np.zeros((2, 9, ny, nx))
    for y in range(ny):
        for s, r in enumerate((ro, rw)):
            f[s, :, y, :] = orc.equilibrium(r, U * math.sin(k * y), 0.0)[:, None]
    L = orc.Lattice(p, mask, np.stack([np.full((ny, nx), ro), np.full((ny, nx), rw)]))
    L.f[...] = f
    nsteps = 600
    L.step(nsteps)
    ux = L.moments()["u"][0][:, 0]
    amp = 2.0 / ny * np.sum(ux * np.sin(k * np.arange(ny)))
    nu = (ro * T0 * (tau[0] - 0.5) + rw * T0 * (tau[1] - 0.5)) / (ro + rw)
    want = U * math.exp(-nu * k * k * nsteps)
    assert abs(amp / want - 1) < 5e-3


def test_numpy_brute_force_agrees():
    """An independent vectorised numpy transcription of the same step (written
    with array shifts instead of node loops) agrees with the C oracle on tiny
    lattices with walls, wall potentials, body force and random states."""
    from tests import np_bruteforce
    for cfg in (synth.config_channel(lam=8, h0=2, a=1, theta=60.0, g=1e-4, tau=(0.7, 1.2)),
                synth.config_droplet(n=6, r=2.0, tau=(0.9, 1.3))):
        cfg["nx"] = cfg["nx"] if cfg["kind"] != "box" else 6
        mask = synth.mask_of(cfg)
        f = synth.random_populations(cfg["nx"], cfg["ny"], mask, seed=11, amp=0.05)
        py = cfg["kind"] == "box"
        p = orc.Params(cfg["nx"], cfg["ny"], tau=cfg["tau"], G=cfg["G"], rho_s=cfg["rho_s"],
                       g=cfg["g"], periodic_y=py)
        a = f
        for _ in range(3):
            a, bad = orc.step_once(p, mask, a)
            assert bad == 0
        b = np_bruteforce.run(f, mask, cfg["tau"], cfg["G"], cfg["rho_s"], cfg["g"], 3, py)
        np.testing.assert_allclose(a, b, rtol=0, atol=1e-14)


# ---- third-order Hermite regularization (collision variant) -----------------
def _h3_tensor(c, T0=1.0 / 3.0):
    I = np.eye(2)
    return (np.einsum('a,b,c->abc', c, c, c) - T0 * (np.einsum('a,bc->abc', c, I) +
            np.einsum('b,ac->abc', c, I) + np.einsum('c,ab->abc', c, I)))


@pytest.mark.parametrize("seed", range(4))
def test_third_order_regularizer_projection(seed):
    """The third-order regularized part f' keeps the mass, momentum and second
    moment of the second-order one, reproduces the third-order Hermite moments
    of f - feq, is a projection (regularizing feq + f' returns f'), and on
    D2Q9 the xxx and yyy coefficients vanish (c^3 = c, so H_xxx = 0)."""
    rng = np.random.default_rng(100 + seed)
    f = 0.05 + 0.05 * rng.random(9)
    feq = orc.equilibrium(f.sum(), 0.05 * rng.standard_normal(), 0.05 * rng.standard_normal())
    f3, a3 = orc.regularize3(f, feq)
    f2, _ = orc.regularize(f, feq)
    cx, cy, w, _ = orc.lattice()
    C = np.stack([cx, cy], axis=1).astype(float)
    d = f3 - f2
    # rounding of values of order 1e-2
    assert abs(d.sum()) < 1e-16 and np.abs(C.T @ d).max() < 1e-16
    assert np.abs(np.einsum('ia,ib,i->ab', C, C, d)).max() < 1e-16
    H = np.array([_h3_tensor(c) for c in C])
    np.testing.assert_allclose(np.einsum('iabc,i->abc', H, f3),
                               np.einsum("iabc,i->abc", H, f - feq), rtol=0, atol=1e-15)
    assert a3[0, 0, 0] == 0.0 and a3[1, 1, 1] == 0.0
    g3, _ = orc.regularize3(feq + f3, feq)
    np.testing.assert_allclose(g3, f3, rtol=0, atol=1e-15)


def test_third_order_worked_values():
    """Closed form on D2Q9: only a_xxy and a_xyy survive; the additions are
    -+a_xyy / 2 on the x axis, -+a_xxy / 2 on the y axis and
    (s_y a_xxy + s_x a_xyy) / 4 on the diagonal (s_x, s_y) (w_i / (2 T0^3) times
    the Hermite value, checked here by hand for a distribution whose only
    non-equilibrium content is a unit xxy moment)."""
    feq = orc.equilibrium(1.0, 0.0, 0.0)
    # f - feq concentrated on the diagonals with s_y-odd, s_x-even weights:
    # sum H_xxy d = sum_diag (2 s_y / 3) d = 1 with d = (3/8) s_y on each diagonal
    d = np.zeros(9)
    for i, (sx, sy) in enumerate(zip(*orc.lattice()[:2])):
        if sx != 0 and sy != 0:
            d[i] = 0.375 * sy
    f3, a3 = orc.regularize3(feq + d, feq)
    f2, _ = orc.regularize(feq + d, feq)
    assert a3[0, 0, 1] == pytest.approx(1.0, abs=1e-15)
    assert a3[0, 1, 1] == pytest.approx(0.0, abs=1e-15)
    want = np.zeros(9)
    for i, (sx, sy) in enumerate(zip(*orc.lattice()[:2])):
        if sx == 0 and sy != 0:
            want[i] = -0.5 * sy
        elif sx != 0 and sy != 0:
            want[i] = 0.25 * sy
    np.testing.assert_allclose(f3 - f2, want, rtol=0, atol=1e-15)


def test_third_order_step_matches_numpy_and_reduces_at_tau_one():
    """The oracle step with reg_order = 3 agrees with the numpy transcription's
    tensor form, and at tau_mix = 1 (omega = 0: the regularized part drops out)
    it equals the second-order step bit for bit."""
    from tests import np_bruteforce
    cfg = synth.config_channel(lam=8, h0=2, a=1, theta=60.0, g=1e-4, tau=(0.7, 1.2))
    mask = synth.mask_of(cfg)
    f = synth.random_populations(cfg["nx"], cfg["ny"], mask, seed=12, amp=0.05)
    p3 = orc.Params(cfg["nx"], cfg["ny"], tau=cfg["tau"], G=cfg["G"], rho_s=cfg["rho_s"],
                    g=cfg["g"], reg_order=3)
    a = f
    for _ in range(3):
        a, bad = orc.step_once(p3, mask, a)
        assert bad == 0
    b = np_bruteforce.run(f, mask, cfg["tau"], cfg["G"], cfg["rho_s"], cfg["g"], 3, False,
                          reg3=True)
    np.testing.assert_allclose(a, b, rtol=0, atol=1e-14)
    a2, _ = orc.step_once(orc.Params(cfg["nx"], cfg["ny"], tau=cfg["tau"], G=cfg["G"],
                                     rho_s=cfg["rho_s"], g=cfg["g"]), mask, f)
    a3, _ = orc.step_once(p3, mask, f)
    assert np.abs(a3 - a2).max() > 1e-9          # the variant does change the step
    p2t = orc.Params(cfg["nx"], cfg["ny"], tau=(1.0, 1.0), G=cfg["G"], rho_s=cfg["rho_s"],
                     g=cfg["g"])
    p3t = orc.Params(cfg["nx"], cfg["ny"], tau=(1.0, 1.0), G=cfg["G"], rho_s=cfg["rho_s"],
                     g=cfg["g"], reg_order=3)
    assert np.array_equal(orc.step_once(p2t, mask, f)[0], orc.step_once(p3t, mask, f)[0])
