"""The seeded input generators (synth/): shapes and the initial-state
recipes the GPU presets and the oracle both start from."""
import numpy as np

import synth


def test_tube_initial_densities_for_a_list_of_slugs():
    """rho03_of with several slugs (no single x0 / length): oil at rho_hi on
    the fluid nodes of every slug, water elsewhere, solids zero."""
    cfg = synth.config_tube(lam=32, r0=6.0, a=2.0)
    cfg["init"] = dict(kind="slug", slugs=[(4, 20), (50, 20)])
    mask = synth.mask3_of(cfg)
    rho = synth.rho03_of(cfg, mask)
    assert rho.shape == (2,) + mask.shape
    x = np.arange(cfg["nx"])
    oil_x = ((x >= 4) & (x < 24)) | ((x >= 50) & (x < 70))
    fluid = mask.astype(bool)
    oil = fluid & oil_x[None, None, :]
    water = fluid & ~oil_x[None, None, :]
    assert np.all(rho[0][oil] == synth.RHO_HI) and np.all(rho[1][oil] == synth.RHO_LO)
    assert np.all(rho[0][water] == synth.RHO_LO) and np.all(rho[1][water] == synth.RHO_HI)
    assert np.all(rho[:, ~fluid] == 0.0)


def test_slug_fraction_step_and_tanh_forms():
    """width 0: a step on [x0, x0 + length) (periodic); width > 0: tanh
    interfaces at x0 - 1/2 and x0 + length - 1/2, clipped to [0, 1] and
    antisymmetric about them up to the other interface's tail (2 e^(-16) for a
    slug of 16 at width 2)."""
    nx = 64
    phi = synth.slug_fraction(nx, 60, 10)
    assert np.array_equal(np.nonzero(phi)[0], np.r_[0:6, 60:64])
    smooth = synth.slug_fraction(nx, 20, 16, width=2.0)
    assert smooth.min() >= 0.0 and smooth.max() <= 1.0
    np.testing.assert_allclose(smooth[19], 1.0 - smooth[20], atol=1e-6)   # about 19.5
    np.testing.assert_allclose(smooth[35], 1.0 - smooth[36], atol=1e-6)   # about 35.5
