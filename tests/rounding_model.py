"""Expected error of the 16-bit forms: a CPU rounding model run through the
oracle's step hook (test-side expectation, not part of the oracle).

Model: the inputs are exact; the result of every pairwise step of the path is
rounded once to the storage format, after the engine's power-of-two scaling
(largest component moved to [2^13, 2^14), which is exact), by numpy's
round-to-nearest-even float16, or by float32 then round-to-nearest-even
bfloat16.  FP32 accumulation inside a step (relative error about 2^-24 x
sqrt(K)) is left out: it is two orders of magnitude below one 16-bit rounding.
The model rounds every step of the given path, including the steps the
library absorbs on the host in FP64, so it rounds at least as often as the
engine does.

A parity test compares the engine's amplitude error with the model's on the
same inputs: the relative L2 error and the largest per-amplitude error
(relative to the largest reference amplitude) may each exceed the model's by
a stated factor, the margin for the engine's different summation orders and
rounding points.
"""
from __future__ import annotations

import numpy as np

from oracle import einsum


def _bf16(x: np.ndarray) -> np.ndarray:
    """float64 -> float32 -> bfloat16 (round to nearest even), as float64.
    The values are scaled below 2^14, so the 32-bit sum cannot carry out."""
    u = np.ascontiguousarray(x, dtype=np.float32).view(np.uint32)
    u = (u + np.uint32(0x7FFF) + ((u >> np.uint32(16)) & np.uint32(1))) & np.uint32(0xFFFF0000)
    return u.view(np.float32).astype(np.float64)


def round16(z: np.ndarray, fmt: str) -> np.ndarray:
    """Round a complex128 array as the engine stores it (fmt 'f16' or 'bf16')."""
    z = np.asarray(z, dtype=np.complex128)
    m = max(np.max(np.abs(z.real), initial=0.0), np.max(np.abs(z.imag), initial=0.0))
    if not np.isfinite(m) or m == 0.0:
        return z
    e = int(np.floor(np.log2(m))) - 13
    re, im = np.ldexp(z.real, -e), np.ldexp(z.imag, -e)
    if fmt == "f16":
        re, im = re.astype(np.float16).astype(np.float64), im.astype(np.float16).astype(np.float64)
    else:
        re, im = _bf16(re), _bf16(im)
    return np.ldexp(re, e) + 1j * np.ldexp(im, e)


def fmt_of(prec: str) -> str:
    return "f16" if prec.startswith("f16") else "bf16"


def model_amplitudes(circuit, structure, ssa, sliced, open_q, bits, prec, slices=None):
    """Amplitudes of `bits` (which agree on every closed qubit) summed over the
    slices in `slices` (default: all), every step result rounded to the
    storage format of `prec`."""
    fmt = fmt_of(prec)
    tensors = einsum.network_tensors(circuit, structure)
    outl = list(structure.output_labels)
    n = circuit.n_qubits
    open_q = sorted(int(q) for q in open_q)
    b0 = int(bits[0])
    closed = {outl[q]: (b0 >> q) & 1 for q in range(n) if q not in open_q}
    sliced = [int(l) for l in sliced]
    if slices is None:
        slices = range(1 << len(sliced))
    acc = None
    for sigma in slices:
        fixed = dict(closed)
        fixed.update({l: (sigma >> j) & 1 for j, l in enumerate(sliced)})
        r = einsum.contract_path(tensors, outl, ssa, fixed=fixed,
                                 after_step=lambda s, lab, d: round16(d, fmt))
        acc = r if acc is None else acc + r
    idx = tuple(np.array([(int(b) >> q) & 1 for b in bits]) for q in open_q)
    return acc[idx] if open_q else np.full(len(bits), complex(acc))


def check_against_model(out, ref, model, l2_factor=2.0, max_factor=4.0):
    """(ok, stats): the engine's errors against the model's expectation."""
    ref = np.asarray(ref)
    scale = np.max(np.abs(ref))
    e_eng = np.abs(np.asarray(out) - ref)
    e_mod = np.abs(np.asarray(model) - ref)
    l2_eng = float(np.linalg.norm(e_eng) / np.linalg.norm(ref))
    l2_mod = float(np.linalg.norm(e_mod) / np.linalg.norm(ref))
    mx_eng = float(np.max(e_eng) / scale)
    mx_mod = float(np.max(e_mod) / scale)
    stats = dict(rel_l2=l2_eng, rel_l2_model=l2_mod, rel_max=mx_eng, rel_max_model=mx_mod)
    ok = l2_eng <= l2_factor * l2_mod and mx_eng <= max_factor * mx_mod
    return ok, stats
