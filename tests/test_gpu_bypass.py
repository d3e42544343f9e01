"""Bypass channels (the paper's closing section names bypass channels as
further work): columns with two fluid runs, from the analytic channel with a
solid island in its wide part and from a mask.  Through the C ABI, against
the FP64 oracle on the same mask and inputs."""
import numpy as np
import pytest

import synth
from tests.gpu_util import (assert_monitors_match, field_rel_err, fp32_storage_floor,
                            oracle_lattice, velocity_bound)

pytestmark = pytest.mark.gpu


def _cases():
    return {"island64": synth.config_bypass(lam=64, theta=120.0, g=1e-5, tau=(0.8, 1.2)),
            "island128": synth.config_bypass(lam=128, theta=60.0, g=4e-6, island_h=5,
                                             island_len=40),
            # the C3 size (lambda = 256, 1024 x 98)
            "island256": synth.config_bypass(lam=256, theta=120.0, g=2e-6, tau=(0.8, 1.2))}


@pytest.mark.parametrize("which", ["island64", "island128", "island256"])
def test_fluid_mask_and_mask_geometry(gpu_available, which):
    """The library's voxelisation of the island equals the synthetic mask
    (two runs in the island columns), and the same mask passed as a mask
    geometry gives bit-identical populations."""
    from paper_1601_00918_amd import Simulation
    cfg = _cases()[which]
    mask = synth.mask_of(cfg)
    runs = (np.diff(np.concatenate([np.zeros((1, cfg["nx"]), np.uint8), mask,
                                    np.zeros((1, cfg["nx"]), np.uint8)]).astype(int),
                    axis=0) == 1).sum(axis=0)
    assert runs.max() == 2 and runs.min() == 1
    a = Simulation([cfg])
    assert np.array_equal(a.fluid_mask(0), mask)
    b = Simulation([dict(cfg, kind="mask", mask=mask)])
    a.step(50)
    b.step(50)
    assert np.array_equal(a.populations(0), b.populations(0))


@pytest.mark.parametrize("which", ["island64", "island128", "island256"])
def test_few_steps_and_1000_steps_match_oracle(gpu_available, which):
    from paper_1601_00918_amd import Simulation
    cfg = _cases()[which]
    L, mask, _ = oracle_lattice(cfg)
    sim = Simulation([cfg])
    for n in (1, 2, 5):
        L.step(n - L.t)
        sim.step(n - sim.t)
        err = np.abs(sim.populations(0) - L.f).max()
        print(which, "t=%d max|df|=%.3e" % (n, err), flush=True)
        assert err < 2e-7 * n
    sim.step(1000 - sim.t)
    L.step(1000 - L.t)
    ref, got = L.moments(), sim.moments(0)
    erho = field_rel_err(ref["rho"], got["rho"], mask)
    eu = field_rel_err(ref["u"], got["u"], mask)
    ep = field_rel_err(ref["p"][None], got["p"][None], mask)
    floor = fp32_storage_floor(lambda: oracle_lattice(cfg)[0], 1000, mask)
    print(which, "rho", erho, "u", eu, "p", ep, "floors", floor, flush=True)
    assert max(erho) <= velocity_bound(floor["rho"]) and max(ep) <= velocity_bound(floor["p"])
    assert max(eu) <= velocity_bound(floor["u"])
    assert_monitors_match(ref["mon"], got["mon"], velocity_bound(floor["u"]), cfg["G"])


def test_tiling_and_batching_do_not_change_results(gpu_available):
    """Halo columns and rows around the islands are recomputed by
    neighbouring workgroups: every tiling, and a batch with a plain channel,
    gives bit-identical populations (FP32 and binary16)."""
    from paper_1601_00918_amd import Simulation
    cfg = _cases()["island128"]
    for storage in ("f32", "f16"):
        ref = None
        for bx, strip in [(256, 8), (64, 5), (128, 32)]:
            sim = Simulation([cfg], storage=storage)
            sim.set_tiling(bx, strip)
            sim.step(40)
            f = sim.populations(0)
            if ref is None:
                ref = f
            else:
                assert np.array_equal(f, ref), (storage, bx, strip)
        both = Simulation([synth.config_channel(lam=64, theta=90.0, g=1e-5), cfg],
                          storage=storage)
        both.step(40)
        assert np.array_equal(both.populations(1), ref), storage
