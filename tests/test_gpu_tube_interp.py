"""D3Q19 tube with interpolated walls (lbm3d_geom.wall_interp) against the
FP64 oracle's interpolated bounce-back on the same seeded inputs: populations
after a few steps, moments and monitors after 1000 steps, the 16-bit storage
formats, tiling independence, mass conservation and the Hagen-Poiseuille
profile of a straight tube whose wall falls between the nodes."""
import numpy as np
import pytest

import synth
from oracle import lbm3d as o3
from tests.gpu_util import assert_monitors_match, fp32_storage_floor_u, velocity_bound
from tests.test_gpu_d3q19 import _rel, _sim, _to_oracle_order

pytestmark = pytest.mark.gpu

TUBE = dict(lam=32, r0=6.0, a=2.0, theta=60.0, tau=(0.8, 1.3), g=1e-4, wall_interp=True)


def _oracle(cfg):
    mask = synth.mask3_of(cfg)
    wall = (0.5 * (cfg["ny"] - 1), 0.5 * (cfg["nz"] - 1), cfg["r0"], cfg["a"], cfg["lam"])
    p = o3.Params3(cfg["nx"], cfg["ny"], cfg["nz"], tau=cfg["tau"], G=cfg["G"],
                   rho_s=cfg["rho_s"], g=cfg["g"], wall=wall)
    return o3.Lattice3(p, mask, synth.rho03_of(cfg, mask)), mask


@pytest.mark.parametrize("storage,tol", [("f32", 1e-6), ("f16", 1e-3)])
def test_initial_state_matches_oracle(gpu_available, storage, tol):
    """The first pull, wall blends and mass return included, gives the rest
    equilibrium the oracle starts from."""
    cfg = synth.config_tube(**TUBE)
    L, mask = _oracle(cfg)
    sim = _sim(cfg, storage=storage)
    f = _to_oracle_order(sim.populations())
    err = np.abs(f - L.f).max() / np.abs(L.f).max()
    print(storage, "t=0 max|df|/max|f| = %.3e" % err, flush=True)
    assert err <= tol


def test_few_steps_populations(gpu_available):
    cfg = synth.config_tube(**TUBE)
    L, mask = _oracle(cfg)
    sim = _sim(cfg)
    assert np.array_equal(sim.fluid_mask(), mask)
    for n in (1, 2, 5):
        L.step(n - L.t)
        sim.step(n - sim.t)
        f = _to_oracle_order(sim.populations())
        err = np.abs(f - L.f).max()
        print("t=%d max|df|=%.3e" % (n, err), flush=True)
        assert err < 2e-7 * n


def test_moments_after_1000_steps(gpu_available):
    """One wavelength of the tube (the oracle's link fractions are recomputed
    every step, so it is kept short): rho and p to 1e-5, u to the velocity
    bound of its binary32 storage floor, monitors as in the half-way tests."""
    cfg = synth.config_tube(**dict(TUBE, lam=32), nx=32, slug_len=16, slug_x0=8)
    L, mask = _oracle(cfg)
    sim = _sim(cfg)
    sim.step(1000)
    L.step(1000)
    ref, got = L.moments(), sim.moments()
    erho = _rel(ref["rho"], got["rho"], mask)
    eu = _rel(ref["u"], got["u"], mask)
    ep = _rel(ref["p"][None], got["p"][None], mask)
    floor_u = fp32_storage_floor_u(lambda: _oracle(cfg)[0], 1000, mask)
    print("rho", erho, "u", eu, "(storage floor %.2e)" % floor_u, "p", ep, flush=True)
    assert max(erho) <= 1e-5
    assert max(ep) <= 1e-5
    assert max(eu) <= velocity_bound(floor_u)
    assert_monitors_match(ref["mon"], got["mon"], velocity_bound(floor_u), cfg["G"])


@pytest.mark.parametrize("storage,floor", [("f16", 2e-3), ("bf16", 1.5e-2)])
def test_16bit_storage_tracks_oracle(gpu_available, storage, floor):
    cfg = synth.config_tube(**TUBE)
    L, mask = _oracle(cfg)
    sim = _sim(cfg, storage=storage)
    sim.step(200)
    L.step(200)
    ref, got = L.moments(), sim.moments()
    erho = _rel(ref["rho"], got["rho"], mask)
    print(storage, "rho", erho, flush=True)
    assert max(erho) <= floor
    np.testing.assert_allclose(got["mon"]["mass"], ref["mon"][:2], rtol=1e-5)


def test_tiling_does_not_change_results(gpu_available):
    """Frame nodes blend their wall links like inner nodes, so every tiling
    gives bit-identical populations."""
    cfg = synth.config_tube(lam=32, r0=9.0, a=3.0, theta=120.0, g=1e-4, wall_interp=True)
    ref = None
    for bx, by, strip in [(32, 16, 16), (64, 8, 4), (32, 8, 7), (16, 12, 9), (32, 16, 100)]:
        sim = _sim(cfg)
        sim.set_tiling(bx, by, strip)
        sim.step(30)
        f = sim.populations()
        if ref is None:
            ref = f
        else:
            assert np.array_equal(f, ref), (bx, by, strip)


def test_each_species_mass_is_kept(gpu_available):
    """What the blends add returns through the rest population: each species'
    mass stays at its initial value to FP32 summation rounding over 3000
    forced steps."""
    cfg = synth.config_tube(**dict(TUBE, g=2e-4))
    sim = _sim(cfg)
    m0 = np.array(sim.monitors()["mass"])
    sim.step(3000)
    m1 = np.array(sim.monitors()["mass"])
    print("mass drift", (m1 - m0) / m0, flush=True)
    np.testing.assert_allclose(m1, m0, rtol=1e-6)


def test_hagen_poiseuille_between_the_nodes(gpu_available):
    """A single fluid driven along a straight tube of radius 8.6: the GPU
    profile is the oracle's, and both are within 0.5 % of Hagen-Poiseuille,
    u = g (R^2 - rho^2) / (4 nu), vanishing at the analytic wall."""
    R, tau, g = 8.6, 0.8, 2.5e-6
    nu = (tau - 0.5) / 3.0
    side = int(2 * R + 3)
    cfg = dict(name="tube", kind="tube", nx=4, ny=side, nz=side, lam=4.0, r0=R, a=0.0,
               tau=(tau, tau), G=0.0, rho_s=(0.0, 0.0), g=(g, 0.0, 0.0), wall_interp=True,
               init=dict(kind="uniform", rho_hi=0.5, rho_lo=0.5))
    sim = _sim(cfg)
    sim.step(12000)
    u = sim.moments()["u"][0][:, :, 0]
    mask = synth.mask3_of(cfg)[:, :, 0].astype(bool)
    yc = 0.5 * (side - 1)
    zz, yy = np.meshgrid(np.arange(side), np.arange(side), indexing="ij")
    want = g * (R * R - (yy - yc) ** 2 - (zz - yc) ** 2) / (4.0 * nu)
    err = np.abs(u[mask] - want[mask]).max() / want.max()
    print("Hagen-Poiseuille max error %.3e" % err, flush=True)
    assert err < 0.005
