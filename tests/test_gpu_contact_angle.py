"""Contact angle of the wall potentials (Sec. 3.3): a slug at rest between
flat plates, the paper's detection (Eq. 12 fits, circle fit, Eq. 14) applied
to GPU fields, checked against the same detection on the FP64 oracle, and the
angle map over the wall potentials and the resolution H (the offset-0 column
of Table 1)."""
import numpy as np
import pytest

import synth
from oracle import analysis as an
from tests.gpu_util import oracle_lattice

pytestmark = pytest.mark.gpu


def _angles(cfg, rho):
    mask = synth.mask_of(cfg)
    frac = rho[0] / np.maximum(rho[0] + rho[1], 1e-30)
    x0, L = cfg["init"]["x0"], cfg["init"]["length"]
    front, _, _ = an.meniscus_contact_angle(frac, mask, x0 + L, oil_left=True)
    rear, _, _ = an.meniscus_contact_angle(frac, mask, x0, oil_left=False)
    return front, rear


def test_contact_angle_gpu_matches_oracle(gpu_available):
    from paper_1601_00918_amd import Simulation
    cfg = synth.config_plates(32, theta=60.0)
    sim = Simulation([cfg])
    sim.step(20000)
    L, mask, _ = oracle_lattice(cfg)
    L.step(20000)
    got = _angles(cfg, sim.moments(0)["rho"])
    ref = _angles(cfg, L.moments()["rho"])
    print("GPU front/rear", got, "oracle", ref)
    assert abs(got[0] - ref[0]) < 0.1 and abs(got[1] - ref[1]) < 0.1
    assert abs(got[0] - got[1]) < 1.0          # no forcing: both menisci alike


def test_contact_angle_map_and_resolution(gpu_available):
    """theta(rho_s) for the wall-potential map of the workloads, H = 16, 32,
    64, 40,000 steps: neutral walls give 90 deg, the map is monotonic and
    symmetric about 90 deg, and the angle depends little on H."""
    from paper_1601_00918_amd import Simulation
    thetas = (30.0, 60.0, 90.0, 120.0, 150.0)
    Hs = (16, 32, 64)
    cfgs = [synth.config_plates(H, theta=t) for H in Hs for t in thetas]
    sim = Simulation(cfgs)
    sim.step(40000)
    table = np.zeros((len(Hs), len(thetas)))
    for k, c in enumerate(cfgs):
        f, r = _angles(c, sim.moments(k)["rho"])
        table[k // len(thetas), k % len(thetas)] = 0.5 * (f + r)
    for H, row in zip(Hs, table):
        print("H=%d" % H, " ".join("%6.1f" % v for v in row), flush=True)
    assert np.all(np.abs(table[:, 2] - 90.0) < 1.0)
    assert np.all(np.diff(table, axis=1) > 0)
    assert np.all(np.abs(table + table[:, ::-1] - 180.0) < 2.0)
    assert np.all(table.max(axis=0) - table.min(axis=0) < 6.0)
