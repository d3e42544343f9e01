"""The 16-bit decode of the D2Q9 step kernel (lbm_kernels.hip, dec16) writes
the scaled population w36 (R + d) as one FMA, d w36 + w36 R, so that the
binary16 operand's conversion folds into the instruction.  For the D2Q9
weights w36 in {1, 4, 16} (powers of two) the FMA's single rounding of the
exact d w36 + w36 R equals the rounded sum scaled, bit for bit: checked here in
binary32 over every finite binary16 deviation d against reference densities R
of the formats' range (binary16 values between 1e-3 and 4).  CPU only."""
import numpy as np


def _fma32(a, b, c):
    """Single-rounding a b + c of binary32 operands: the exact value in binary64
    (the products and sums here need fewer than 53 bits), rounded once."""
    return (a.astype(np.float64) * b.astype(np.float64) + c.astype(np.float64)).astype(np.float32)


def test_fma_form_equals_scaled_sum_for_power_of_two_weights():
    d = np.arange(1 << 16, dtype=np.uint32).astype(np.uint16).view(np.float16)
    d = d[np.isfinite(d)].astype(np.float32)
    rng = np.random.default_rng(5)
    R = (10.0 ** rng.uniform(-3.0, np.log10(4.0), 64)).astype(np.float16).astype(np.float32)
    for w in (1.0, 4.0, 16.0):
        w32 = np.float32(w)
        for r in R:
            want = w32 * (np.float32(r) + d)                  # two roundings in binary32
            got = _fma32(d, np.full_like(d, w32), np.full_like(d, w32 * np.float32(r)))
            assert np.array_equal(want.view(np.uint32), got.view(np.uint32)), (w, r)


def test_a_weight_that_is_not_a_power_of_two_would_differ():
    """The identity needs w36 to be a power of two: with 12 (the D3Q19 rest
    weight) some deviations round differently once R + d itself rounds (R of
    3, where small deviations fall below R's binary32 grid), so that kernel
    keeps its own form."""
    d = np.arange(1 << 16, dtype=np.uint32).astype(np.uint16).view(np.float16)
    d = d[np.isfinite(d)].astype(np.float32)
    r = np.float32(np.float16(3.0))
    w32 = np.float32(12.0)
    want = w32 * (r + d)
    got = _fma32(d, np.full_like(d, w32), np.full_like(d, w32 * r))
    assert not np.array_equal(want.view(np.uint32), got.view(np.uint32))
