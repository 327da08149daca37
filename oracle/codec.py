"""Low-precision exchange codec (oracle).  Test infrastructure only.

Paper Sec. 3.2 (customized low-precision communication), Eq. ``quantcal`` and Table
``quanttable``: a group [T]_i of real values is mapped to

    Q([T]_i) = [T]_i^exp * scale + zero,
    scale = (q_max - q_min) / (max [T]_i - min [T]_i),
    zero  = (q_min max [T]_i - q_max min [T]_i) / (max [T]_i - min [T]_i),

where max/min are taken over the group after the power (so the group's
extremes land exactly on q_min and q_max).  The three types of the table:

    kind   range            exp   group           round
    half   +-65504          1     whole tensor    no (stored as FP16)
    int8   -128 .. 127      0.2   whole tensor    yes
    int4   0 .. 15          1     groups of 128   yes (two codes per byte)

A complex tensor is quantized as the real array of its interleaved (re, im)
values.  The compression rate is Eq. ``compress`` (Sec. 4.2): (bytes of scales + zeros +
codes) / bytes of the original float32 data.

Readings where the paper is silent (stated here and in the design notes):
* x^exp for exp != 1 is sign(x) |x|^exp (the power of a negative value is
  otherwise undefined); the inverse is sign(y) |y|^(1/exp).
* "rounding" is round-half-to-even to an integer, then clamping to the range.
* The table's half range "+-6.65e4" is read as the largest FP16 value, 65504.
* A group whose values are all equal gets scale = 1 and zero = q_min - value,
  so every entry maps to q_min and decodes exactly.
* scales and zeros are float32; the int4 codes of entries 2j and 2j+1 share
  byte j (2j in the low nibble); a ragged last group is allowed.

Two arithmetics are provided.  ``precision="fp64"`` is the definition,
evaluated in double precision.  ``precision="fp32"`` takes the integer
decision the way a float32 implementation does -- the power with float32
powf, scale and zero formed in float32, then q = y * scale rounded, plus
zero rounded (no fused multiply-add) -- so that codes produced by another
float32 implementation of the same steps agree, except where two powf
implementations differ in the last place next to a rounding tie.
"""
from __future__ import annotations

import numpy as np

KINDS = {
    "half": dict(qmin=-65504.0, qmax=65504.0, exp=1.0, group=0, round=False),
    "int8": dict(qmin=-128.0, qmax=127.0, exp=0.2, group=0, round=True),
    "int4": dict(qmin=0.0, qmax=15.0, exp=1.0, group=128, round=True),
}


def as_real(t) -> np.ndarray:
    """Interleaved (re, im) float32 view of a complex64/complex128 array, or a
    real array as float32."""
    t = np.asarray(t)
    if np.iscomplexobj(t):
        r = np.empty(2 * t.size, dtype=np.float32)
        r[0::2] = t.real.ravel()
        r[1::2] = t.imag.ravel()
        return r
    return t.astype(np.float32).ravel()


def _power(x: np.ndarray, e: float) -> np.ndarray:
    x = np.asarray(x, np.float64)
    return x if e == 1.0 else np.sign(x) * np.abs(x) ** e


def _power32(x: np.ndarray, e: float) -> np.ndarray:
    """sign(x)|x|^e in float32 (C powf on |x| with the float32 exponent)."""
    x = np.asarray(x, np.float32)
    if e == 1.0:
        return x
    return (np.sign(x) * np.power(np.abs(x), np.float32(e))).astype(np.float32)


def group_bounds(n: int, kind: str, group: int | None = None):
    g = KINDS[kind]["group"] if group is None else group
    if g <= 0 or g >= n:
        return [(0, n)]
    return [(s, min(s + g, n)) for s in range(0, n, g)]


def quantize(x, kind: str, group: int | None = None, precision: str = "fp64"):
    """(codes, scales, zeros) of the real array x.  codes are float64 integers
    (int8/int4) or FP16 values (half, as float16)."""
    p = KINDS[kind]
    x = np.asarray(x, np.float32 if precision == "fp32" else np.float64).ravel()
    y = _power32(x, p["exp"]) if precision == "fp32" else _power(x, p["exp"])
    ft = np.float32 if precision == "fp32" else np.float64
    qmin, qmax = ft(p["qmin"]), ft(p["qmax"])
    bounds = group_bounds(x.size, kind, group)
    codes = np.empty(x.size, np.float16 if kind == "half" else np.float64)
    scales = np.empty(len(bounds), np.float32)
    zeros = np.empty(len(bounds), np.float32)
    for gi, (a, b) in enumerate(bounds):
        yg = y[a:b]
        mx, mn = ft(yg.max()), ft(yg.min())
        if mx == mn:
            scale, zero = ft(1.0), ft(qmin - mn)
        else:
            d = ft(mx - mn)
            scale = ft((qmax - qmin) / d)
            zero = ft((ft(qmin * mx) - ft(qmax * mn)) / d)
        q = (yg * scale).astype(ft) + zero
        q = q.astype(ft)
        if p["round"]:
            q = np.clip(np.rint(q), qmin, qmax)
        codes[a:b] = q.astype(np.float16) if kind == "half" else q.astype(np.float64)
        scales[gi], zeros[gi] = scale, zero
    return codes, scales, zeros


def unrounded(x, kind: str, group: int | None = None) -> np.ndarray:
    """The float32 value each code is rounded from (for telling near-ties)."""
    p = KINDS[kind]
    x = np.asarray(x, np.float32).ravel()
    y = _power32(x, p["exp"])
    _c, sc, ze = quantize(x, kind, group, "fp32")
    out = np.empty(x.size, np.float64)
    for gi, (a, b) in enumerate(group_bounds(x.size, kind, group)):
        out[a:b] = ((y[a:b] * sc[gi]).astype(np.float32) + ze[gi]).astype(np.float32)
    return out


def dequantize(codes, scales, zeros, kind: str, group: int | None = None) -> np.ndarray:
    """float64 values decoded from codes (the inverse map, Eq. quantcal solved
    for [T]_i)."""
    p = KINDS[kind]
    q = np.asarray(codes, np.float64).ravel()
    out = np.empty(q.size, np.float64)
    for gi, (a, b) in enumerate(group_bounds(q.size, kind, group)):
        y = (q[a:b] - float(zeros[gi])) / float(scales[gi])
        out[a:b] = _power(y, 1.0 / p["exp"])
    return out


def pack_int4(codes) -> np.ndarray:
    c = np.asarray(codes, np.int64).ravel()
    if c.size % 2:
        c = np.concatenate([c, [0]])
    return (c[0::2] | (c[1::2] << 4)).astype(np.uint8)


def unpack_int4(packed, n: int) -> np.ndarray:
    p = np.asarray(packed, np.uint8).ravel().astype(np.int64)
    c = np.empty(2 * p.size, np.int64)
    c[0::2] = p & 15
    c[1::2] = p >> 4
    return c[:n]


def compression_rate(n_reals: int, kind: str, group: int | None = None) -> float:
    """Eq. compress: (scales + zeros + codes) / original float32 bytes."""
    ng = len(group_bounds(n_reals, kind, group))
    code_bytes = {"half": 2 * n_reals, "int8": n_reals, "int4": (n_reals + 1) // 2}[kind]
    return (4 * ng + 4 * ng + code_bytes) / (4.0 * n_reals)
