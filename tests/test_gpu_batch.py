"""Batched stepping with per-instance tiling and the autotuner, through the C
ABI: mixed workgroup widths run as separate launches of one step, graphs
capture all of them, and the tuner's steps are ordinary steps of the run."""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


def _cfgs():
    return [synth.config_channel(lam=64, theta=40.0, g=2e-5, tau=(0.8, 1.3)),
            synth.config_channel(lam=128, theta=140.0, g=5e-6),
            synth.config_droplet(n=96, r=15.0),
            synth.config_channel(lam=256, theta=90.0, g=1e-6),
            synth.config_poiseuille(nx=200, width=30, wall_rows=7)]


def _sim(cfgs, storage="f32", **kw):
    from paper_1601_00918_amd import Simulation
    return Simulation(cfgs, storage=storage, **kw)


@pytest.mark.parametrize("storage", ["f32", "f16"])
def test_mixed_instance_tilings_are_bitwise_equal(gpu_available, storage):
    cfgs = _cfgs()
    ref = _sim(cfgs, storage)
    ref.step(30)
    mixed = _sim(cfgs, storage)
    for k, (bx, strip) in enumerate([(64, 4), (128, 16), (256, 8), (64, 32), (128, 5)]):
        mixed.set_instance_tiling(k, bx, strip)
        assert mixed.instance_tiling(k) == (bx, strip)
    mixed.step(30)
    for k in range(len(cfgs)):
        assert np.array_equal(mixed.populations(k), ref.populations(k)), k


def test_mixed_tilings_in_graph_replays(gpu_available):
    import torch
    cfgs = _cfgs()
    eager = _sim(cfgs)
    graphed = _sim(cfgs, stream=torch.cuda.Stream())
    for sim in (eager, graphed):
        sim.set_instance_tiling(0, 64, 8)
        sim.set_instance_tiling(3, 128, 16)
    for rep in range(2):
        eager.step(64)
        graphed.step(64)
        torch.cuda.synchronize()
        for k in range(len(cfgs)):
            assert np.array_equal(eager.populations(k), graphed.populations(k)), (rep, k)


def test_autotune_steps_are_real_steps(gpu_available):
    """After tuning, the state equals that of plain steps of the same count,
    and the chosen tiling is not slower than the starting one."""
    cfgs = _cfgs()
    tuned = _sim(cfgs)
    rep = tuned.autotune(steps_per_trial=8)
    print("autotune", rep, [tuned.instance_tiling(k) for k in range(len(cfgs))], flush=True)
    assert rep["steps"] == 8 * rep["trials"] and tuned.t == rep["steps"]
    assert rep["buckets"] == 5          # widths 256, 512, 96, 1024, 200
    plain = _sim(cfgs)
    plain.step(rep["steps"])
    for k in range(len(cfgs)):
        assert np.array_equal(tuned.populations(k), plain.populations(k)), k
    assert rep["ms_after"] <= rep["ms_before"] * 1.05


def test_destroy_waits_for_queued_steps(gpu_available):
    """A context on its own stream replays captured graphs asynchronously;
    releasing it drains that stream, so the workspace can be freed at once."""
    import gc

    import torch
    from paper_1601_00918_amd import Simulation
    st = torch.cuda.Stream()
    sim = Simulation([synth.config_channel(lam=256, theta=90.0, g=1e-5)], stream=st)
    sim.step(640)
    del sim
    gc.collect()
    assert st.query()
