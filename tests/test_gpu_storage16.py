"""16-bit population storage (binary16 / bfloat16 deviations from a per-node
binary16 reference density, FP32 arithmetic) against the FP64 oracle, and the
exactness properties it shares with FP32 storage.  Through the C ABI.

Tolerances.  The oracle runs in FP64 with no storage rounding, so the bar is
the error that re-encoding the state every step the way the kernels store it
leaves on the FP64 run (the storage floor, measured by a CPU emulation of the
format on these workloads and sizes), times four to cover the FP32
arithmetic and the different stochastic-rounding sequence.  Floors after 1000 steps (max
relative field error; rho, u, p; python tests/storage_floor.py):
    binary16  droplet 1.7e-4 2.0e-3 1.2e-4   poiseuille 4.5e-4 4.5e-2 1.8e-4
              channel 1.2e-4 3.7e-3 9.4e-5
    bfloat16  droplet 4.5e-3 2.7e-2 2.0e-3   poiseuille 5.1e-3 3.7e-1 2.2e-3
              channel 1.5e-3 1.2e-1 7.9e-4
The Poiseuille velocity floor is the rounding of the large force-shifted
populations on the interface rows (about 4.5e-5 in binary16) against a
maximum velocity of 1e-3; bfloat16 has no useful velocity bound there and
its velocity is reported, not asserted."""
import numpy as np
import pytest

import synth
from tests.gpu_util import field_rel_err, oracle_lattice

pytestmark = pytest.mark.gpu

W = np.array([4 / 9] + [1 / 9] * 4 + [1 / 36] * 4)
FLOOR = {
    "f16": {"droplet": (1.7e-4, 2.0e-3, 1.2e-4), "poiseuille": (4.5e-4, 4.5e-2, 1.8e-4),
            "channel": (1.2e-4, 3.7e-3, 9.4e-5)},
    "bf16": {"droplet": (4.5e-3, 2.7e-2, 2.0e-3), "poiseuille": (5.1e-3, None, 2.2e-3),
             "channel": (1.5e-3, 1.2e-1, 7.9e-4)},
}


def _cfg(which, big=False):
    if which == "droplet":
        return synth.config_droplet(n=128 if big else 64, r=20.0 if big else 10.0)
    if which == "poiseuille":
        return synth.config_poiseuille() if big else synth.config_poiseuille(nx=64, width=32,
                                                                              wall_rows=8)
    return synth.config_channel(lam=64, theta=120.0, g=1e-5)


def _sim(cfgs, storage, **kw):
    from paper_1601_00918_amd import Simulation
    return Simulation(cfgs, storage=storage, **kw)


@pytest.mark.parametrize("storage", ["f16", "bf16"])
@pytest.mark.parametrize("which", ["droplet", "poiseuille", "channel"])
def test_initial_state_matches_oracle(gpu_available, which, storage):
    """The initial slot (x, i) holds rho0(reader) - R(x), rounded once: its
    error is at most half a unit in the last place of that difference."""
    cfg = _cfg(which)
    L, mask, rho0 = oracle_lattice(cfg)
    sim = _sim([cfg], storage)
    assert np.array_equal(sim.fluid_mask(0), mask)
    f = sim.populations(0)
    e = np.abs(f - L.f) / W[None, :, None, None]
    ulp = 2.0 ** -11 if storage == "f16" else 2.0 ** -8
    # |rho0(reader) - R(x)| <= max rho0, plus the FP32 decode
    bound = ulp * max(synth.RHO_HI, 1.0) + 1e-6
    print(which, storage, "max |df| / w = %.3e (bound %.3e)" % (e.max(), bound), flush=True)
    assert e.max() <= bound


@pytest.mark.parametrize("storage", ["f16", "bf16"])
@pytest.mark.parametrize("which", ["droplet", "poiseuille", "channel"])
def test_moments_after_1000_steps(gpu_available, which, storage):
    cfg = _cfg(which, big=True)
    L, mask, rho0 = oracle_lattice(cfg)
    sim = _sim([cfg], storage)
    m0 = sim.monitors()[0]["mass"]
    sim.step(1000)
    L.step(1000)
    ref = L.moments()
    got = sim.moments(0)
    erho = max(field_rel_err(ref["rho"], got["rho"], mask))
    eu = max(field_rel_err(ref["u"], got["u"], mask))
    ep = max(field_rel_err(ref["p"][None], got["p"][None], mask))
    m1 = sim.monitors()[0]["mass"]
    drift = [abs(m1[k] / m0[k] - 1) for k in range(2)]
    fr, fu, fp = FLOOR[storage][which]
    print(which, storage, "rho %.2e (floor %.1e)  u %.2e (floor %s)  p %.2e (floor %.1e)  "
          "mass drift %.1e %.1e" % (erho, fr, eu, fu, ep, fp, drift[0], drift[1]), flush=True)
    assert erho <= 4 * fr
    assert ep <= 4 * fp
    if fu is not None:
        assert eu <= 4 * fu
    # the encoder keeps each node's mass exact up to FP32 rounding and one
    # unbiased stochastic rounding of the rest deviation
    assert max(drift) <= (1e-5 if storage == "f16" else 5e-5)


@pytest.mark.parametrize("storage", ["f16", "bf16"])
def test_tiling_does_not_change_results(gpu_available, storage):
    cfg = synth.config_channel(lam=128, theta=60.0, g=1e-5)
    ref = None
    for bx, strip in [(256, 32), (64, 8), (128, 13), (256, 200)]:
        sim = _sim([cfg], storage)
        sim.set_tiling(bx, strip)
        sim.step(40)
        f = sim.populations(0)
        if ref is None:
            ref = f
        else:
            assert np.array_equal(f, ref), (bx, strip)


@pytest.mark.parametrize("storage", ["f16", "bf16"])
def test_batch_equals_single_instances(gpu_available, storage):
    cfgs = [synth.config_channel(lam=64, theta=40.0, g=2e-5, tau=(0.8, 1.3)),
            synth.config_droplet(n=96, r=15.0),
            synth.config_poiseuille(nx=200, width=30, wall_rows=7)]
    batch = _sim(cfgs, storage)
    batch.step(25)
    for k, cfg in enumerate(cfgs):
        one = _sim([cfg], storage)
        one.step(25)
        assert np.array_equal(batch.populations(k), one.populations(0)), k


def test_graph_replays_match_eager_steps(gpu_available):
    """Captured graphs take the step number of the rounding sequence from
    device memory; every replay must equal the eager steps bit for bit."""
    import torch
    cfg = synth.config_channel(lam=64, theta=120.0, g=1e-5)
    eager = _sim([cfg], "f16")
    graphed = _sim([cfg], "f16", stream=torch.cuda.Stream())
    for rep in range(3):
        eager.step(64)
        graphed.step(64)
        torch.cuda.synchronize()
        assert np.array_equal(eager.populations(0), graphed.populations(0)), rep
        eager.step(3)
        graphed.step(3)
        torch.cuda.synchronize()


def test_snapshot_restore_is_exact(gpu_available):
    cfgs = [synth.config_channel(lam=64, theta=60.0, g=1e-5), synth.config_droplet(n=64, r=10)]
    sim = _sim(cfgs, "f16", snapshot=True)
    sim.step(10)
    saved = [sim.populations(k) for k in range(2)]
    sim.snapshot_save()
    sim.step(7)
    sim.snapshot_restore(-1)
    for k in range(2):
        assert np.array_equal(sim.populations(k), saved[k])


# Storage floors after 1000 steps of the extended kernels' workloads (rho, u, p;
# tests/storage_floor.py's floor() on these configs): third-order
# regularization on the lambda = 64 channel, and the bypass channel with its
# solid island (two fluid runs per column in the island's columns).
EXT_FLOOR = {
    "f16": {"channel-reg3": (1.16e-4, 4.49e-3, 9.64e-5), "island64": (2.05e-4, 3.31e-3, 1.30e-4)},
    "bf16": {"channel-reg3": (1.77e-3, 6.25e-2, 8.03e-4), "island64": (1.39e-3, 5.27e-2, 8.64e-4)},
}


def _ext_cfg(which):
    if which == "channel-reg3":
        return dict(synth.config_channel(lam=64, theta=120.0, g=1e-5, tau=(0.7, 1.3)),
                    reg_order=3)
    return synth.config_bypass(lam=64, theta=120.0, g=1e-5, tau=(0.8, 1.2))


@pytest.mark.parametrize("storage", ["f16", "bf16"])
@pytest.mark.parametrize("which", ["channel-reg3", "island64"])
def test_extended_kernels_in_16bit_storage_track_the_oracle(gpu_available, which, storage):
    """The extended step instances (third-order regularization, two-run
    columns) in the 16-bit formats against the FP64 oracle after 1000 steps:
    every field within four times its storage floor, mass as in the plain
    kernels."""
    cfg = _ext_cfg(which)
    L, mask, rho0 = oracle_lattice(cfg)
    sim = _sim([cfg], storage)
    m0 = sim.monitors()[0]["mass"]
    sim.step(1000)
    L.step(1000)
    ref, got = L.moments(), sim.moments(0)
    erho = max(field_rel_err(ref["rho"], got["rho"], mask))
    eu = max(field_rel_err(ref["u"], got["u"], mask))
    ep = max(field_rel_err(ref["p"][None], got["p"][None], mask))
    m1 = sim.monitors()[0]["mass"]
    drift = [abs(m1[k] / m0[k] - 1) for k in range(2)]
    fr, fu, fp = EXT_FLOOR[storage][which]
    print(which, storage, "rho %.2e (floor %.1e)  u %.2e (floor %.1e)  p %.2e (floor %.1e)  "
          "mass drift %.1e %.1e" % (erho, fr, eu, fu, ep, fp, drift[0], drift[1]), flush=True)
    assert erho <= 4 * fr and eu <= 4 * fu and ep <= 4 * fp
    assert max(drift) <= (1e-5 if storage == "f16" else 5e-5)


@pytest.mark.parametrize("storage", ["f16", "bf16"])
@pytest.mark.parametrize("lattice", ["d2q9", "d3q19"])
def test_slug_list_with_tanh_interfaces_starts_at_the_oracle_state(gpu_available, lattice,
                                                                   storage):
    """Two slugs with tanh interfaces of width 2 in 16-bit storage: every
    initial population equals the oracle's rest equilibrium from the same
    synthetic field within one rounding of the stored deviation
    rho0(reader) - R(x) (half a unit in its last place, at most one unit of
    max rho0), times the weight."""
    ulp = 2.0 ** -11 if storage == "f16" else 2.0 ** -8
    slugs = [(6, 40), (100, 30)]
    if lattice == "d2q9":
        cfg = synth.config_channel(lam=64, theta=90.0)
        cfg["init"] = dict(kind="slug", slugs=slugs, width=2.0)
        L, mask, _ = oracle_lattice(cfg)
        f = _sim([cfg], storage).populations(0)
        w = W[None, :, None, None]
        ref = L.f
    else:
        from oracle import lbm3d as o3
        from paper_1601_00918_amd.binding3d import Simulation3D
        from tests.test_gpu_d3q19 import _to_oracle_order
        cfg = synth.config_tube(lam=48, r0=10.0, a=4.0, nx=144, theta=90.0)
        cfg["init"] = dict(kind="slug", slugs=slugs, width=2.0)
        mask = synth.mask3_of(cfg)
        L = o3.Lattice3(o3.Params3(cfg["nx"], cfg["ny"], cfg["nz"], tau=cfg["tau"], G=cfg["G"],
                                   rho_s=cfg["rho_s"], g=cfg["g"]), mask,
                        synth.rho03_of(cfg, mask))
        f = _to_oracle_order(Simulation3D(cfg, storage=storage).populations())
        w = o3.lattice()[3][None, :, None, None, None]
        ref = L.f
    e = (np.abs(f - ref) / w).max()
    bound = ulp * max(synth.RHO_HI, 1.0) + 1e-6
    print(lattice, storage, "max |df| / w = %.3e (bound %.3e)" % (e, bound), flush=True)
    assert e <= bound
