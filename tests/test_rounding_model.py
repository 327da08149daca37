"""The test-side rounding model (CPU): it rounds like the storage formats."""
import numpy as np

from rounding_model import round16


def test_round16_is_exact_on_representable_values_and_rounds_to_nearest_even():
    # values already in FP16 (after the power-of-two scaling) are unchanged
    z = np.array([1.0, -0.5 + 0.25j, 3.0 - 7.0j, 2.0 ** -20], dtype=np.complex128)
    np.testing.assert_array_equal(round16(z, "f16"), z)
    np.testing.assert_array_equal(round16(z, "bf16"), z)
    # 1/sqrt(2) rounds to the nearest FP16 / BF16 value below it
    r = 1 / np.sqrt(2.0)
    assert round16(np.array([r]), "f16")[0] == 0.70703125
    assert round16(np.array([r]), "bf16")[0] == 0.70703125
    # a tie rounds to even: 1 + 2^-11 is halfway between 1 and 1 + 2^-10 in FP16
    t = round16(np.array([1 + 2.0 ** -11, 2.0]), "f16")
    assert t[0] == 1.0
    t = round16(np.array([1 + 2.0 ** -8, 2.0]), "bf16")
    assert t[0] == 1.0
    # scaling is by powers of two: the relative error is the same at any scale
    x = np.array([0.1 + 0.3j, -0.7j])
    for k in (-40, 0, 40):
        np.testing.assert_array_equal(round16(x * 2.0 ** k, "f16"), round16(x, "f16") * 2.0 ** k)
    # the relative error is at most half an ulp of the format
    rng = np.random.default_rng(0)
    v = rng.normal(size=1000) + 1j * rng.normal(size=1000)
    m = np.max(np.abs(np.concatenate([v.real, v.imag])))
    for fmt, u in (("f16", 2.0 ** -11), ("bf16", 2.0 ** -8)):
        w = round16(v, fmt)
        big = np.abs(v.real) > m * 2.0 ** -12
        assert np.all(np.abs(w.real - v.real)[big] <= u * np.abs(v.real)[big] * (1 + 1e-12))
