"""GPU critical-pressure driver against the oracle, snapshot/active-set and
graph-replay checks.  All through the C ABI."""
import time

import numpy as np
import pytest

import synth
from oracle import driver as odrv
from oracle import lbm as orc
from paper_1601_00918_amd import binding

pytestmark = pytest.mark.gpu

SIGMA = 0.161   # surface tension of the model at G = -2.7 (oracle Laplace fit)
RHO_BAR = 1.03


def _plain(cfg, g_lo, g_hi, max_steps):
    return dict(nx=cfg["nx"], lam=cfg["lam"], h0=cfg["h0"], a=cfg["a"], tau_w=cfg["tau"][1],
                g_lo=g_lo, g_hi=g_hi, max_steps=max_steps, sigma=SIGMA, rho_bar=RHO_BAR)


def test_critical_pressure_matches_oracle(gpu_available):
    """Same problem, same probe rules: the GPU solve and the oracle solve agree
    on the critical forcing to within the bisection tolerance."""
    cfg = synth.config_channel(lam=64, theta=90.0)
    rules = dict(rel_tol=0.01, chunk_steps=500, min_steps=5000, still_chunks=3)
    g_lo, g_hi, equil, budget = 1e-5, 1.6e-4, 4000, 30000
    t0 = time.time()
    prob = binding.cp_problem(cfg, g_lo, g_hi, SIGMA, RHO_BAR, equil, budget)
    gpu = binding.lbm_critical_pressure([prob], binding.cp_options(**rules))[0]
    t1 = time.time()
    mask = synth.mask_of(cfg)
    L = orc.Lattice(orc.Params(cfg["nx"], cfg["ny"], tau=cfg["tau"], G=cfg["G"],
                               rho_s=cfg["rho_s"]), mask, synth.rho0_of(cfg, mask))
    ref = odrv.solve(odrv.OracleEngine([L], equil), [_plain(cfg, g_lo, g_hi, budget)],
                     **rules)[0]
    t2 = time.time()
    print("gpu %s (%.1f s)  oracle %s (%.1f s)" % (gpu, t1 - t0, {k: v for k, v in ref.items()
                                                                  if k != "history"}, t2 - t1))
    assert gpu["g_lo"] < gpu["g_hi"] and gpu["flags"] & ~binding._lib.CP_UNDECIDED == 0
    assert abs(gpu["g_crit"] / ref["g_crit"] - 1) <= 0.011


def test_snapshot_restore_and_active_set(gpu_available):
    """Restoring a snapshot gives back the saved state bit for bit; inactive
    instances do not advance."""
    cfgs = [synth.config_channel(lam=64, theta=60.0, g=1e-5), synth.config_droplet(n=64, r=10)]
    sim = binding.Simulation(cfgs, snapshot=True)
    sim.step(10)
    saved = [sim.populations(k) for k in range(2)]
    sim.snapshot_save()
    sim.step(7)
    assert not np.array_equal(sim.populations(0), saved[0])
    sim.snapshot_restore(0)
    assert np.array_equal(sim.populations(0), saved[0])
    sim.set_active([False, True])
    before = sim.populations(0)
    sim.step(5)
    assert np.array_equal(sim.populations(0), before)
    assert not np.array_equal(sim.populations(1), saved[1])
    sim.snapshot_restore(-1)
    assert np.array_equal(sim.populations(1), saved[1])


def test_graph_replays_match_eager_steps(gpu_available):
    """On a non-null stream runs of 64 steps replay a captured graph; every
    replay, with eager work and synchronisation in between, must equal the
    eager (null-stream) result bit for bit."""
    import torch
    cfg = synth.config_channel(lam=64, theta=120.0, g=1e-5)
    eager = binding.Simulation([cfg])
    graphed = binding.Simulation([cfg], stream=torch.cuda.Stream())
    for rep in range(4):
        eager.step(64)
        graphed.step(64)
        torch.cuda.synchronize()
        assert np.array_equal(eager.populations(0), graphed.populations(0)), rep
        eager.step(3)    # eager work between replays (odd: flips the buffer parity)
        graphed.step(3)
        torch.cuda.synchronize()
