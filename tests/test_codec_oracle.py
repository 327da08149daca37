"""Pins of the oracle's low-precision codec (paper Sec. 3.2, Eq. quantcal,
Table quanttable; Eq. compress) against values worked by hand from the
formulas and against properties any correct implementation has."""
import numpy as np
import pytest

from oracle import codec


def test_hand_worked_int4_group():
    # [0, 1, 2, 3]: max - min = 3, scale = 15 / 3 = 5, zero = (0*3 - 15*0) / 3 = 0
    q, s, z = codec.quantize([0.0, 1.0, 2.0, 3.0], "int4")
    np.testing.assert_array_equal(q, [0, 5, 10, 15])
    assert s[0] == 5.0 and z[0] == 0.0
    np.testing.assert_allclose(codec.dequantize(q, s, z, "int4"), [0, 1, 2, 3], atol=1e-12)


def test_hand_worked_int8_power_one_fifth():
    # y = sign(x)|x|^0.2: [-32, 1, 32] -> [-2, 1, 2]; scale = 255 / 4 = 63.75,
    # zero = (-128*2 - 127*(-2)) / 4 = -0.5; q = [-128, 63.25 -> 63, 127]
    q, s, z = codec.quantize([-32.0, 1.0, 32.0], "int8")
    np.testing.assert_array_equal(q, [-128, 63, 127])
    assert s[0] == 63.75 and z[0] == -0.5
    # decode 63: (63 + 0.5) / 63.75 = 0.99607..., to the fifth power
    np.testing.assert_allclose(codec.dequantize(q, s, z, "int8")[1], (63.5 / 63.75) ** 5, rtol=1e-14)


@pytest.mark.parametrize("kind", ["half", "int8", "int4"])
def test_group_extremes_map_to_range_ends(kind):
    rng = np.random.default_rng(1)
    x = rng.normal(size=1000) * 3.0
    p = codec.KINDS[kind]
    q, s, z = codec.quantize(x, kind)
    for a, b in codec.group_bounds(x.size, kind):
        g = q[a:b].astype(np.float64)
        assert g.min() == p["qmin"] and g.max() == p["qmax"], (a, b)


@pytest.mark.parametrize("kind", ["int8", "int4"])
def test_round_trip_within_half_a_step(kind):
    rng = np.random.default_rng(2)
    x = rng.normal(size=4097)          # a ragged last int4 group
    q, s, z = codec.quantize(x, kind)
    e = codec.KINDS[kind]["exp"]
    xr = codec.dequantize(q, s, z, kind)
    y = np.sign(x) * np.abs(x) ** e
    yr = np.sign(xr) * np.abs(xr) ** e
    for gi, (a, b) in enumerate(codec.group_bounds(x.size, kind)):
        assert np.max(np.abs(y[a:b] - yr[a:b])) <= 0.5 / s[gi] * (1 + 1e-6)


def test_half_round_trip_relative():
    rng = np.random.default_rng(3)
    x = rng.normal(size=2048)
    q, s, z = codec.quantize(x, "half")
    xr = codec.dequantize(q, s, z, "half")
    # the map is affine onto +-65504; FP16 keeps 11 significant bits of q
    step = np.maximum(np.abs(q.astype(np.float64)), 2.0 ** -14) * 2.0 ** -11 / s[0]
    assert np.all(np.abs(x - xr) <= step * 1.01 + 1e-12)


@pytest.mark.parametrize("kind", ["half", "int8", "int4"])
def test_codes_monotone_within_a_group(kind):
    rng = np.random.default_rng(4)
    x = np.sort(rng.normal(size=128))
    q, _s, _z = codec.quantize(x, kind)
    assert np.all(np.diff(q.astype(np.float64)) >= 0)


def test_constant_group_decodes_exactly():
    q, s, z = codec.quantize(np.full(300, 0.75), "int4")
    assert np.all(q == 0)
    np.testing.assert_array_equal(codec.dequantize(q, s, z, "int4"), np.full(300, 0.75))


def test_compression_rates_closed_form():
    n = 1 << 20
    assert codec.compression_rate(n, "half") == pytest.approx(0.5, abs=1e-5)
    assert codec.compression_rate(n, "int8") == pytest.approx(0.25, abs=1e-5)
    # int4, groups of 128: per group 8 bytes of scale+zero and 64 bytes of codes over 512 bytes
    assert codec.compression_rate(n, "int4") == pytest.approx(72 / 512, abs=1e-9)


def test_int4_packing_round_trip():
    c = np.arange(16).repeat(3)[:47]
    np.testing.assert_array_equal(codec.unpack_int4(codec.pack_int4(c), c.size), c)
    assert codec.pack_int4([1, 2])[0] == 0x21    # entry 0 in the low nibble


def test_fp32_decisions_agree_with_definition_away_from_ties():
    rng = np.random.default_rng(5)
    x = rng.normal(size=20000).astype(np.float32)
    for kind in ("int8", "int4"):
        q64, _, _ = codec.quantize(x, kind, precision="fp64")
        q32, _, _ = codec.quantize(x, kind, precision="fp32")
        u = codec.unrounded(x, kind)
        far = np.abs(u - np.floor(u) - 0.5) > 1e-3
        np.testing.assert_array_equal(q64[far], q32[far])
        assert np.max(np.abs(q64 - q32)) <= 1


def test_complex_as_interleaved_reals():
    z = np.array([1 + 2j, 3 - 4j], dtype=np.complex64)
    np.testing.assert_array_equal(codec.as_real(z), [1, 2, 3, -4])
