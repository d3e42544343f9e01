"""Several slugs in series (the multi-slug workload the paper names as further
work): initial states of the D2Q9 and D3Q19 paths against the oracle, and the
critical forcing of two slugs against one."""
import numpy as np
import pytest

import synth
from oracle import lbm as orc

pytestmark = pytest.mark.gpu

SIGMA, RHO_BAR = 0.161, 1.03


def _channel(slugs, lam=64, theta=90.0):
    cfg = synth.config_channel(lam=lam, theta=theta)
    cfg["init"] = dict(kind="slug", slugs=[tuple(s) for s in slugs])
    return cfg


def test_two_slug_channel_matches_oracle(gpu_available):
    from paper_1601_00918_amd import Simulation
    cfg = _channel([(16, 40), (120, 56)], theta=60.0)
    mask = synth.mask_of(cfg)
    rho0 = synth.rho0_of(cfg, mask)
    oil = rho0[0] > 0.5
    assert oil[:, 16:56].all(where=mask[:, 16:56] > 0) and not oil[:, 60:116].any()
    p = orc.Params(cfg["nx"], cfg["ny"], tau=cfg["tau"], G=cfg["G"], rho_s=cfg["rho_s"],
                   g=(1e-5, 0.0))
    L = orc.Lattice(p, mask, rho0)
    sim = Simulation([dict(cfg, g=(1e-5, 0.0))])
    for n in (0, 1, 5):
        L.step(n - L.t)
        sim.step(n - sim.t)
        err = np.abs(sim.populations(0) - L.f).max()
        print("t=%d max|df| %.3e" % (n, err), flush=True)
        assert err < 2e-7 * max(n, 1)


def test_two_slug_tube_matches_oracle(gpu_available):
    from paper_1601_00918_amd.binding3d import Simulation3D
    from tests.test_gpu_d3q19 import _oracle, _to_oracle_order
    cfg = synth.config_tube(lam=32, r0=6.0, a=2.0, theta=120.0)
    cfg["init"] = dict(kind="slug", slugs=[(4, 20), (50, 24)])
    L, mask = _oracle(cfg)
    sim = Simulation3D(cfg)
    f = _to_oracle_order(sim.populations())
    np.testing.assert_allclose(f, L.f, rtol=1e-7, atol=0)
    L.step(3)
    sim.step(3)
    assert np.abs(_to_oracle_order(sim.populations()) - L.f).max() < 6e-7


def test_two_slugs_in_phase_double_the_critical_forcing(gpu_available):
    """lambda = 64, four periods, theta = 90 deg: slugs of 0.75 lambda one
    wavelength apart meet the same walls at the same phase, so their capillary
    resistances add and the critical forcing doubles (within the 1 %
    bisection and the equilibration's conditioning, bound 6 %).  Half a
    wavelength further apart, one slug's menisci sit where the other's pull
    the opposite way, and the pair holds much less than twice one slug."""
    from paper_1601_00918_amd import binding
    one = _channel([(16, 48)])
    two = _channel([(16, 48), (80, 48)])
    off = _channel([(16, 48), (112, 48)])
    probs = [binding.cp_problem(c, 2e-5, 2.4e-4, SIGMA, RHO_BAR, 10000, 300000)
             for c in (one, two, off)]
    res = binding.lbm_critical_pressure(
        probs, binding.cp_options(rel_tol=0.01, chunk_steps=500, verify_bracket=1))
    g1, g2, g3 = (r["g_crit"] for r in res)
    print("one slug %.4e, two in phase %.4e (x %.3f), two half a period apart %.4e (x %.3f)"
          % (g1, g2, g2 / g1, g3, g3 / g1), [r["flags"] for r in res], flush=True)
    assert all(r["flags"] & ~binding._lib.CP_UNDECIDED == 0 for r in res)
    assert abs(g2 / g1 - 2.0) <= 0.12
    assert g3 < 0.8 * g2


def test_two_slugs_in_phase_in_the_tube(gpu_available):
    """The same comparison on the D3Q19 tube (lambda = 32, neck 4, widest 8,
    four periods, theta = 90 deg, slugs of 0.75 lambda): two slugs one period
    apart hold about twice the critical forcing of one (measured 1.88, bound
    8 %), two slugs 1.5 periods apart less than 1.8 times (measured 1.20)."""
    from paper_1601_00918_amd import binding, binding3d as b3
    base = dict(lam=32, r0=6.0, a=2.0, nx=128, theta=90.0)
    cfgs = []
    for slugs in ([(8, 24)], [(8, 24), (40, 24)], [(8, 24), (56, 24)]):
        c = synth.config_tube(**base)
        c["init"] = dict(kind="slug", slugs=slugs)
        cfgs.append(c)
    probs = [b3.cp3_problem(c, 2e-5, 2e-3, 0.195, RHO_BAR, 4000, 100000, min_steps=10000)
             for c in cfgs]
    res = b3.lbm3d_critical_pressure(
        probs, binding.cp_options(rel_tol=0.01, chunk_steps=500, still_chunks=3,
                                  verify_bracket=1))
    g1, g2, g3 = (r["g_crit"] for r in res)
    print("tube: one slug %.4e, two in phase x %.3f, two 1.5 periods apart x %.3f"
          % (g1, g2 / g1, g3 / g1), [r["flags"] for r in res], flush=True)
    assert all(r["flags"] & ~binding._lib.CP_UNDECIDED == 0 for r in res)
    assert abs(g2 / g1 - 2.0) <= 0.16
    assert g3 < 1.8 * g1


@pytest.mark.parametrize("lattice", ["d2q9", "d3q19"])
def test_smooth_slug_start_matches_oracle(gpu_available, lattice):
    """Slugs started with tanh interfaces (lbm_init_fields.width): the initial
    populations equal the oracle's from the same synthetic field (FP64 tanh
    on both sides, then one binary32 rounding), and the first steps follow
    it within 2e-7 per step."""
    if lattice == "d2q9":
        from paper_1601_00918_amd import Simulation
        from tests.gpu_util import oracle_lattice
        cfg = synth.config_channel(lam=64, theta=90.0, tau=(1.5, 0.55), g=1e-5)
        cfg["init"]["width"] = 2.0
        L, mask, _ = oracle_lattice(cfg)
        sim = Simulation([cfg])

        def pops():
            return sim.populations(0)
    else:
        from oracle import lbm3d as o3
        from paper_1601_00918_amd.binding3d import C3, Simulation3D
        cfg = synth.config_tube(lam=48, r0=14.0, a=6.0, nx=144, theta=90.0, tau=(1.5, 0.55),
                                slug_len=46, slug_x0=4)
        cfg["init"]["width"] = 2.0
        mask = synth.mask3_of(cfg)
        L = o3.Lattice3(o3.Params3(cfg["nx"], cfg["ny"], cfg["nz"], tau=cfg["tau"], G=cfg["G"],
                                   rho_s=cfg["rho_s"], g=cfg["g"]), mask,
                        synth.rho03_of(cfg, mask))
        sim = Simulation3D(cfg)
        cx, cy, cz, _, _ = o3.lattice()
        oc = np.stack([cx, cy, cz], axis=1)
        perm = [int(np.nonzero((oc == c).all(axis=1))[0][0]) for c in C3]

        def pops():
            f = np.empty_like(L.f)
            f[:, perm] = sim.populations()
            return f
    np.testing.assert_allclose(pops(), L.f, rtol=2.5e-7, atol=0)
    for n in (1, 2, 5):
        L.step(n - L.t)
        sim.step(n - sim.t)
        err = np.abs(pops() - L.f).max()
        print(lattice, "t=%d max|df|=%.3e" % (n, err), flush=True)
        assert err < 2e-7 * n
