"""D3Q19 HIP path (include/lbm3d.h) vs the FP64 D3Q19 oracle on the same seeded
inputs: initial state, populations after a few steps, moments after 1000
steps (tube and periodic droplet box), the droplet pressure jump, monitors,
tiling independence, the mask path, snapshots and the 16-bit storage formats."""
import numpy as np
import pytest

import synth
from oracle import lbm3d as o3
from tests.gpu_util import assert_monitors_match, fp32_storage_floor_u, velocity_bound

pytestmark = pytest.mark.gpu


def _oracle(cfg, mask=None):
    mask = synth.mask3_of(cfg) if mask is None else mask
    p = o3.Params3(cfg["nx"], cfg["ny"], cfg["nz"], tau=cfg["tau"], G=cfg["G"],
                   rho_s=cfg["rho_s"], g=cfg["g"], periodic_yz=(cfg["kind"] == "box3d"))
    return o3.Lattice3(p, mask, synth.rho03_of(cfg, mask)), mask


def _perm():
    """Library direction k -> oracle direction index."""
    from paper_1601_00918_amd.binding3d import C3
    cx, cy, cz, _, _ = o3.lattice()
    oc = np.stack([cx, cy, cz], axis=1)
    return [int(np.nonzero((oc == c).all(axis=1))[0][0]) for c in C3]


def _to_oracle_order(f):
    out = np.empty_like(f)
    out[:, _perm()] = f
    return out


def _sim(cfg, storage="f32", **kw):
    from paper_1601_00918_amd.binding3d import Simulation3D
    return Simulation3D(cfg, storage=storage, **kw)


def _rel(ref, got, mask):
    m = mask.astype(bool)
    out = []
    for k in range(ref.shape[0]):
        a, b = ref[k][m], got[k][m]
        s = np.abs(a).max()
        out.append(float(np.abs(a - b).max() / s) if s > 0 else float(np.abs(b).max()))
    return out


TUBE = dict(lam=32, r0=6.0, a=2.0, theta=60.0, tau=(0.8, 1.3), g=1e-4)


def _tube():
    return synth.config_tube(**TUBE)


def _box(n=20, r=5.0):
    return synth.config_box3d(n=n, r=r)


@pytest.mark.parametrize("which", ["tube", "box"])
def test_initial_state_matches_oracle(gpu_available, which):
    cfg = _tube() if which == "tube" else _box()
    L, mask = _oracle(cfg)
    sim = _sim(cfg)
    assert np.array_equal(sim.fluid_mask(), mask)
    f = _to_oracle_order(sim.populations())
    np.testing.assert_allclose(f, L.f, rtol=1e-7, atol=0)


@pytest.mark.parametrize("which", ["tube", "box"])
def test_few_steps_populations(gpu_available, which):
    cfg = _tube() if which == "tube" else _box()
    L, mask = _oracle(cfg)
    sim = _sim(cfg)
    for n in (1, 2, 5):
        L.step(n - L.t)
        sim.step(n - sim.t)
        f = _to_oracle_order(sim.populations())
        err = np.abs(f - L.f).max()
        print(which, "t=%d max|df|=%.3e" % (n, err), flush=True)
        assert err < 2e-7 * n


@pytest.mark.parametrize("which", ["tube", "box"])
def test_moments_after_1000_steps(gpu_available, which):
    cfg = _tube() if which == "tube" else _box(24, 6.0)
    L, mask = _oracle(cfg)
    sim = _sim(cfg)
    sim.step(1000)
    L.step(1000)
    ref = L.moments()
    got = sim.moments()
    erho = _rel(ref["rho"], got["rho"], mask)
    eu = _rel(ref["u"], got["u"], mask)
    ep = _rel(ref["p"][None], got["p"][None], mask)
    floor_u = fp32_storage_floor_u(lambda: _oracle(cfg)[0], 1000, mask)
    print(which, "rho", erho, "u", eu, "(storage floor %.2e)" % floor_u, "p", ep, flush=True)
    assert max(erho) <= 1e-5
    assert max(ep) <= 1e-5
    assert max(eu) <= velocity_bound(floor_u)
    assert_monitors_match(ref["mon"], got["mon"], velocity_bound(floor_u), cfg["G"])


def test_droplet_pressure_jump(gpu_available):
    """Centre-minus-far-field pressure of a 3-D droplet after 1000 steps:
    GPU against oracle to 1e-4 relative."""
    cfg = _box(24, 6.0)
    L, mask = _oracle(cfg)
    sim = _sim(cfg)
    sim.step(1000)
    L.step(1000)

    def dp(p):
        return p[10:14, 10:14, 10:14].mean() - p[0:3, 0:3, 0:3].mean()
    ref, got = dp(L.moments()["p"]), dp(sim.moments()["p"])
    print("dp ref %.9e got %.9e rel %.2e" % (ref, got, abs(got - ref) / abs(ref)), flush=True)
    assert abs(got - ref) <= 1e-4 * abs(ref)


def test_tiling_does_not_change_results(gpu_available):
    """Frame nodes are recomputed by neighbouring workgroups and strips meet
    at shared planes; every tiling must give bit-identical populations."""
    cfg = synth.config_tube(lam=32, r0=9.0, a=3.0, theta=120.0, g=1e-4)
    ref = None
    for bx, by, strip in [(32, 16, 16), (64, 8, 4), (32, 8, 7), (16, 12, 9), (32, 16, 100)]:
        sim = _sim(cfg)
        sim.set_tiling(bx, by, strip)
        assert sim.tiling()[:3] == (bx, by, strip)
        sim.step(30)
        f = sim.populations()
        if ref is None:
            ref = f
        else:
            assert np.array_equal(f, ref), (bx, by, strip)


def test_mask_path_equals_analytic_tube(gpu_available):
    cfg = _tube()
    mask = synth.mask3_of(cfg)
    sim_t = _sim(cfg)
    cfg_m = dict(cfg, kind="mask", mask=mask)
    sim_m = _sim(cfg_m)
    assert np.array_equal(sim_m.fluid_mask(), mask)
    sim_t.step(20)
    sim_m.step(20)
    assert np.array_equal(sim_t.populations(), sim_m.populations())


def test_snapshot_restores_state_and_time(gpu_available):
    cfg = _tube()
    sim = _sim(cfg, snapshot=True)
    sim.step(7)
    sim.snapshot_save()
    f7 = sim.populations()
    sim.step(5)
    sim.snapshot_restore()
    assert sim.t == 7
    assert np.array_equal(sim.populations(), f7)


def test_body_force_change_takes_effect(gpu_available):
    cfg = _tube()
    L, mask = _oracle(cfg)
    sim = _sim(cfg)
    sim.step(3)
    L.step(3)
    sim.set_body_force(3e-4, 1e-5, -2e-5)
    L.set_body_force(3e-4, 1e-5, -2e-5)
    sim.step(3)
    L.step(3)
    f = _to_oracle_order(sim.populations())
    assert np.abs(f - L.f).max() < 2e-6


@pytest.mark.parametrize("storage,floor", [("f16", 2e-3), ("bf16", 1.5e-2)])
def test_16bit_storage_tracks_oracle(gpu_available, storage, floor):
    """Deviation storage: densities within the 16-bit storage floor of the
    FP64 oracle after 200 steps, mass conserved to 1e-5."""
    cfg = _tube()
    L, mask = _oracle(cfg)
    sim = _sim(cfg, storage=storage)
    f0 = _to_oracle_order(sim.populations())
    assert np.abs(f0 - L.f).max() <= 1e-3 * np.abs(L.f).max()
    sim.step(200)
    L.step(200)
    ref, got = L.moments(), sim.moments()
    erho = _rel(ref["rho"], got["rho"], mask)
    print(storage, "rho", erho, flush=True)
    assert max(erho) <= floor
    np.testing.assert_allclose(got["mon"]["mass"], ref["mon"][:2], rtol=1e-5)


def test_rejects_bad_input_on_host(gpu_available):
    from paper_1601_00918_amd import _lib
    cfg = dict(_tube(), tau=(0.5, 1.0))
    with pytest.raises(_lib.LbmError) as e:
        _sim(cfg)
    assert "tau" in str(e.value)
    m = synth.mask3_of(_tube()).copy()
    m[3, :, :] = 0  # cuts every column's run in two
    with pytest.raises(_lib.LbmError) as e:
        _sim(dict(_tube(), kind="mask", mask=m))
    assert e.value.status == 6
