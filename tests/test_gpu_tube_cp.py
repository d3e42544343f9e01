"""Critical pressure in the D3Q19 sinusoidal tube (Sec. 3.4): the 3-D surface
tension from the Laplace law, the tube solve through lbm3d_critical_pressure
against the same driver on caller callbacks, and the LBM critical forcing
against the axisymmetric Young-Laplace estimate."""

import numpy as np
import pytest

import synth
from oracle import young_laplace as yl

pytestmark = pytest.mark.gpu

# Surface tension of the D3Q19 model at G = -2.7: slope / 2 of the Laplace fit
# of 3-D droplets (R = 9..14 in a periodic 48^3 box after 3000 steps), see
# test_laplace_law_gives_the_3d_surface_tension.
SIGMA_3D = 0.195
RHO_BAR = 1.03


def test_laplace_law_gives_the_3d_surface_tension(gpu_available):
    from paper_1601_00918_amd.binding3d import Simulation3D
    inv_r, dp = [], []
    for r in (8.0, 10.0, 12.0, 14.0):
        sim = Simulation3D(synth.config_box3d(n=48, r=r))
        sim.step(3000)
        m = sim.moments()
        R = (3.0 * (m["rho"][0] > 0.5).sum() / (4.0 * np.pi)) ** (1.0 / 3.0)
        p = m["p"]
        dp.append(p[22:26, 22:26, 22:26].mean() - p[0:4, 0:4, 0:4].mean())
        inv_r.append(1.0 / R)
    slope, icpt = np.polyfit(inv_r, dp, 1)
    resid = np.abs(np.polyval([slope, icpt], inv_r) - dp).max()
    print("slope %.5f intercept %.2e resid %.2e sigma %.5f" % (slope, icpt, resid, slope / 2))
    assert abs(slope / 2 - SIGMA_3D) <= 0.01
    assert abs(icpt) <= 0.15 * min(dp) and resid <= 0.02 * max(dp)


def _channel_view(cfg):
    """The tube's classification parameters as a planar problem (lambda, r0 as
    h0, a, nx), for the callback driver."""
    return dict(kind="channel", nx=cfg["nx"], ny=cfg["ny"], lam=cfg["lam"], h0=cfg["r0"],
                a=cfg["a"], tau=cfg["tau"], G=cfg["G"], rho_s=cfg["rho_s"], g=(0.0, 0.0),
                init=dict(kind="slug", x0=cfg["init"]["x0"], length=cfg["init"]["length"]))


class _TubeEngine:
    """The tube contexts driven from Python through the C ABI."""

    def __init__(self, cfgs, equil):
        from paper_1601_00918_amd.binding3d import Simulation3D
        self.sims = []
        for c in cfgs:
            s = Simulation3D(dict(c, g=(0.0, 0.0, 0.0)), snapshot=True)
            s.step(equil)
            s.snapshot_save()
            self.sims.append(s)

    def begin_probe(self, k, g):
        self.sims[k].snapshot_restore()
        self.sims[k].set_body_force(g)

    def advance(self, active, steps):
        for k, s in enumerate(self.sims):
            if active[k]:
                s.step(steps)

    def monitors(self):
        return [s.monitors() for s in self.sims]


def test_tube_solve_equals_callback_driver(gpu_available):
    from paper_1601_00918_amd import binding, binding3d as b3
    cfg = synth.config_tube(lam=32, r0=6.0, a=2.0, theta=120.0)
    g_lo, g_hi, equil, budget = 2e-5, 1e-3, 2000, 20000
    rules = dict(rel_tol=0.05, chunk_steps=500, min_steps=4000, still_chunks=3)
    native = b3.lbm3d_critical_pressure(
        [b3.cp3_problem(cfg, g_lo, g_hi, SIGMA_3D, RHO_BAR, equil, budget)],
        binding.cp_options(**rules))[0]
    prob = binding.cp_problem(_channel_view(cfg), g_lo, g_hi, SIGMA_3D, RHO_BAR, equil, budget)
    cb = binding.lbm_cp_drive(_TubeEngine([cfg], equil), [prob], binding.cp_options(**rules))[0]
    print("native", native, "callbacks", cb)
    for key in ("g_lo", "g_hi", "g_crit", "bo_crit", "probes", "flags"):
        assert native[key] == cb[key], key
    assert native["steps"] == cb["steps"] + equil


def test_tube_critical_forcing_vs_axisymmetric_young_laplace(gpu_available):
    """A slug of 1.5 wavelengths in a tube of three periods (lambda = 64, neck
    radius 6, widest 14), theta = 120 deg: the LBM critical forcing against
    the quasi-static axisymmetric Young-Laplace estimate with the model's own
    surface tension.  The model sits 4-15 % below the quasi-static value in
    the tubes tried, whatever the neck resolution, so the bound is 20 %."""
    from paper_1601_00918_amd import binding, binding3d as b3
    lam, r0, a, th = 64, 10.0, 4.0, 120.0
    cfg = synth.config_tube(lam=lam, r0=r0, a=a, theta=th)
    mask = synth.mask3_of(cfg)
    x = np.arange(cfg["nx"])
    slug = np.mod(x - cfg["init"]["x0"], cfg["nx"]) < cfg["init"]["length"]
    vol = float(mask[:, :, slug].sum())
    dps, _ = yl.critical_pressure(yl.Channel(r0, a, lam, axisymmetric=True), th, vol)
    g_yl = dps * SIGMA_3D / (RHO_BAR * cfg["nx"])
    prob = b3.cp3_problem(cfg, g_yl / 8, g_yl * 8, SIGMA_3D, RHO_BAR, 4000, 40000,
                          min_steps=5000)
    r = b3.lbm3d_critical_pressure(
        [prob], binding.cp_options(rel_tol=0.02, chunk_steps=500, still_chunks=3,
                                   verify_bracket=1))[0]
    ratio = r["g_crit"] / g_yl
    print("g_YL %.4e LBM %s ratio %.3f" % (g_yl, r, ratio))
    assert r["flags"] & ~binding._lib.CP_UNDECIDED == 0
    assert r["g_hi"] / r["g_lo"] - 1 <= 0.02 + 1e-12
    assert abs(ratio - 1) <= 0.2


def test_tube_critical_pressure_in_binary16_storage(gpu_available):
    """The tube solve with binary16 deviation storage against FP32 storage:
    same problem, same rules, bisection to 0.25 %; the critical forcings agree
    within the 1 % that 16-bit storage is held to."""
    from paper_1601_00918_amd import binding, binding3d as b3
    cfg = synth.config_tube(lam=32, r0=6.0, a=2.0, theta=120.0)
    rules = dict(rel_tol=0.0025, chunk_steps=500, min_steps=4000, still_chunks=3, verify_bracket=1)
    out = {}
    for storage in ("f32", "f16"):
        prob = b3.cp3_problem(cfg, 5e-5, 1e-3, SIGMA_3D, RHO_BAR, 2000, 40000)
        out[storage] = b3.lbm3d_critical_pressure(
            [prob], binding.cp_options(storage=storage, **rules))[0]
    print({k: (v["g_crit"], v["flags"]) for k, v in out.items()})
    assert all(v["flags"] & ~binding._lib.CP_UNDECIDED == 0 for v in out.values())
    assert abs(out["f16"]["g_crit"] / out["f32"]["g_crit"] - 1) <= 0.01


def test_full_size_tube_critical_pressure_binary16(gpu_available):
    """The full-size tube workload: 512 x 128 x 128, r(x) = 40 + 16 cos(2 pi x /
    256) (neck radius 24), a slug of 384 nodes, binary16 storage, probes of up
    to 100,000 steps, theta = 90 deg, bisection to 2 %: the critical forcing
    against the axisymmetric Young-Laplace value for the measured slug volume
    (the smaller tubes give 0.85-0.95 of it).  About three minutes; the
    driver logs every classified probe on stderr."""
    from paper_1601_00918_amd import binding, binding3d as b3
    cfg = synth.config_tube(lam=256, r0=40.0, a=16.0, nx=512, ny=128, nz=128, theta=90.0,
                            slug_len=384, slug_x0=64)
    sim = b3.Simulation3D(cfg, storage="f16")
    sim.step(40000)
    rho = sim.moments()["rho"]
    vol = float((rho[0] / np.maximum(rho[0] + rho[1], 1e-30) > 0.9).sum())
    del sim
    dps, _ = yl.critical_pressure(yl.Channel(40.0, 16.0, 256.0, axisymmetric=True), 90.0, vol)
    g_yl = dps * SIGMA_3D / (RHO_BAR * cfg["nx"])
    prob = b3.cp3_problem(cfg, 0.5 * g_yl, 1.5 * g_yl, SIGMA_3D, RHO_BAR, 40000, 100000,
                          min_steps=20000)
    r = b3.lbm3d_critical_pressure(
        [prob], binding.cp_options(storage="f16", rel_tol=0.02, chunk_steps=1000,
                                   still_chunks=3, verify_bracket=1, verbose=1))[0]
    print("volume %.0f g_YL %.4e result %s ratio %.3f" % (vol, g_yl, r, r["g_crit"] / g_yl),
          flush=True)
    assert r["flags"] & ~binding._lib.CP_UNDECIDED == 0
    assert abs(r["g_crit"] / g_yl - 1) <= 0.25
