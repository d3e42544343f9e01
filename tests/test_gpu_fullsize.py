"""The benchmark workload at full size, in the launch configuration bench.py
times (the 256-channel batch, default tiling, one launch per step):
properties that hold for every instance, and sampled instances element by
element against the oracle.  Plus degenerate inputs."""
import numpy as np
import pytest

import synth
from tests.gpu_util import field_rel_err, fp32_storage_floor_u, oracle_lattice, velocity_bound

pytestmark = pytest.mark.gpu


def test_full_batch_conserves_mass_and_matches_sampled_instances(gpu_available):
    from paper_1601_00918_amd import Simulation
    cfgs = synth.config_batch(n_inst=256, seed=1601)
    sim = Simulation(cfgs)
    m0 = sim.monitors()
    sim.step(100)
    m1 = sim.monitors()
    drift = max(abs(b["mass"][s] / a["mass"][s] - 1) for a, b in zip(m0, m1) for s in range(2))
    bad = sum(m["bad_nodes"] for m in m1)
    print("256 instances, 100 steps: max mass drift %.2e, bad nodes %d" % (drift, bad), flush=True)
    # bounce-back and the pull step conserve each species' mass exactly; only
    # FP32 rounding of the stored populations remains
    assert bad == 0 and drift <= 1e-6
    # sampled instances: the first of each wavelength, element by element
    sampled = [next(k for k, c in enumerate(cfgs) if c["lam"] == lam) for lam in (64, 128, 256, 512)]
    for k in sampled:
        L, mask, _ = oracle_lattice(cfgs[k])
        L.step(100)
        ref = L.moments()
        got = sim.moments(k)
        erho = max(field_rel_err(ref["rho"], got["rho"], mask))
        ep = max(field_rel_err(ref["p"][None], got["p"][None], mask))
        eu = max(field_rel_err(ref["u"], got["u"], mask))
        floor_u = fp32_storage_floor_u(lambda: oracle_lattice(cfgs[k])[0], 100, mask)
        print("instance %d (lambda %d): rho %.2e u %.2e (floor %.2e) p %.2e" % (
            k, cfgs[k]["lam"], erho, eu, floor_u, ep), flush=True)
        assert erho <= 1e-5 and ep <= 1e-5
        assert eu <= velocity_bound(floor_u)


def test_full_batch_third_order_matches_sampled_instances(gpu_available):
    """The 256-channel batch with the third-order regularization (what
    bench.py --reg-order 3 times): mass kept and the first instance of each
    wavelength element by element against the oracle's third-order step after
    100 steps (rho, p to 1e-5, u to the velocity bound of its binary32 storage
    floor)."""
    from paper_1601_00918_amd import Simulation
    cfgs = [dict(c, reg_order=3) for c in synth.config_batch(n_inst=256, seed=1601)]
    sim = Simulation(cfgs)
    m0 = sim.monitors()
    sim.step(100)
    m1 = sim.monitors()
    drift = max(abs(b["mass"][s] / a["mass"][s] - 1) for a, b in zip(m0, m1) for s in range(2))
    bad = sum(m["bad_nodes"] for m in m1)
    print("third order, 256 instances, 100 steps: max mass drift %.2e, bad nodes %d"
          % (drift, bad), flush=True)
    assert bad == 0 and drift <= 1e-6
    sampled = [next(k for k, c in enumerate(cfgs) if c["lam"] == lam) for lam in (64, 128, 256, 512)]
    for k in sampled:
        L, mask, _ = oracle_lattice(cfgs[k])
        L.step(100)
        ref, got = L.moments(), sim.moments(k)
        erho = max(field_rel_err(ref["rho"], got["rho"], mask))
        ep = max(field_rel_err(ref["p"][None], got["p"][None], mask))
        eu = max(field_rel_err(ref["u"], got["u"], mask))
        floor_u = fp32_storage_floor_u(lambda: oracle_lattice(cfgs[k])[0], 100, mask)
        print("instance %d (lambda %d): rho %.2e u %.2e (floor %.2e) p %.2e" % (
            k, cfgs[k]["lam"], erho, eu, floor_u, ep), flush=True)
        assert erho <= 1e-5 and ep <= 1e-5
        assert eu <= velocity_bound(floor_u)


@pytest.mark.parametrize("storage", ["f16", "bf16"])
def test_full_batch_in_16bit_storage_tracks_sampled_instances(gpu_available, storage):
    """The 256-channel batch in the 16-bit formats, in the launch configuration
    bench.py times with --storage: 100 steps without a bad node, each
    species' mass within the 16-bit drift bounds, and the first instance of
    each wavelength within four times its storage floor of the FP64 oracle
    (floors from tests/storage_floor.py --batch, which emulates the format's
    rounding on the oracle; the GPU's own random sequence and FP32 arithmetic
    differ, hence the factor)."""
    import json
    import os
    from paper_1601_00918_amd import Simulation
    from tests.storage_floor import batch_sample
    here = os.path.dirname(os.path.abspath(__file__))
    table = json.load(open(os.path.join(here, "golden", "storage_floor_batch.json")))
    steps = table["steps"]
    cfgs = synth.config_batch(n_inst=256, seed=1601)
    sim = Simulation(cfgs, storage=storage)
    m0 = sim.monitors()
    sim.step(steps)
    m1 = sim.monitors()
    drift = max(abs(b["mass"][s] / a["mass"][s] - 1) for a, b in zip(m0, m1) for s in range(2))
    bad = sum(m["bad_nodes"] for m in m1)
    print("%s, 256 instances, %d steps: max mass drift %.2e, bad nodes %d"
          % (storage, steps, drift, bad), flush=True)
    assert bad == 0 and drift <= (1e-5 if storage == "f16" else 5e-5)
    for k in batch_sample(cfgs):
        fr, fu, fp, _ = table["instances"][str(k)][storage]
        L, mask, _ = oracle_lattice(cfgs[k])
        L.step(steps)
        ref, got = L.moments(), sim.moments(k)
        erho = max(field_rel_err(ref["rho"], got["rho"], mask))
        eu = max(field_rel_err(ref["u"], got["u"], mask))
        ep = max(field_rel_err(ref["p"][None], got["p"][None], mask))
        print("instance %d (lambda %d): rho %.2e (floor %.1e) u %.2e (floor %.1e) "
              "p %.2e (floor %.1e)" % (k, cfgs[k]["lam"], erho, fr, eu, fu, ep, fp), flush=True)
        assert erho <= 4 * fr and eu <= 4 * fu and ep <= 4 * fp


@pytest.mark.parametrize("storage,G", [("f32", synth.G_DEFAULT), ("f16", 0.0)])
def test_uniform_mixture_at_rest_stays_at_rest(gpu_available, storage, G):
    """No density gradient: the interaction force vanishes exactly and the rest
    equilibrium is a fixed point of the step (up to one rounding per step).
    In FP32 every node does the same arithmetic, so the state stays uniform
    to the bit; binary16's stochastic rounding differs per node, which would
    seed the spinodal instability of the mixture at G = -2.7, so that case
    runs without interaction."""
    from paper_1601_00918_amd import Simulation
    cfg = synth.config_uniform(64, G=G)
    sim = Simulation([cfg], storage=storage)
    f0 = sim.populations(0)
    sim.step(200)
    f1 = sim.populations(0)
    mom = sim.moments(0)
    rel = np.abs(f1 - f0).max() / np.abs(f0).max()
    umax = np.abs(mom["u"]).max()
    print(storage, "max |df|/f %.2e  max |u| %.2e" % (rel, umax), flush=True)
    assert rel <= (1e-6 if storage == "f32" else 1e-3)
    assert umax <= 1e-6
