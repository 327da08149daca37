"""FP64 state-vector amplitudes, paper Sec. 2.2 (the state-vector method).

A(x) = <x| U |0^n>, U the circuit's gates applied in circuit order.  A slice
of the tensor network fixes some wire labels to values; fixing wire segment
(q, s) to v is the same as inserting the projector |v><v| on qubit q right
after its s-th gate, so the amplitude of one slice is the state-vector
amplitude of the circuit with those projectors inserted, and the sum over all
values of a wire is the circuit itself.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

from . import build as _build
from . import gates as _gates

_lib = None


def _load():
    global _lib
    if _lib is None:
        path = _build.build(force=False)
        lib = ctypes.CDLL(path)
        dp = ctypes.POINTER(ctypes.c_double)
        lib.sv_zero_state.argtypes = [dp, ctypes.c_int]
        lib.sv_apply_1q.argtypes = [dp, ctypes.c_int, ctypes.c_int, dp]
        lib.sv_apply_2q.argtypes = [dp, ctypes.c_int, ctypes.c_int, ctypes.c_int, dp]
        lib.sv_gather.argtypes = [dp, ctypes.c_int64, ctypes.POINTER(ctypes.c_int64), dp]
        _lib = lib
    return _lib


def _dptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def sv_index(bitstrings, n: int) -> np.ndarray:
    """State-vector index of each bitstring (bit q of x = qubit q; qubit 0 is
    the most significant bit of the index)."""
    b = np.asarray(bitstrings, dtype=np.uint64)
    idx = np.zeros(b.shape, dtype=np.int64)
    for q in range(n):
        idx |= (((b >> np.uint64(q)) & np.uint64(1)).astype(np.int64)) << (n - 1 - q)
    return idx


def _projector(v: int) -> np.ndarray:
    p = np.zeros((2, 2), dtype=np.complex128)
    p[v, v] = 1.0
    return p


def simulate(circuit, wire_fix=None, stop=None) -> np.ndarray:
    """Final state (complex128, length 2^n).

    wire_fix: {(qubit, segment): value}; segment 0 is the initial wire.
    stop: apply only the first ``stop`` gates (for sampled timing).
    """
    n = circuit.n_qubits
    lib = _load()
    psi = np.empty(1 << n, dtype=np.complex128)
    flat = psi.view(np.float64)
    lib.sv_zero_state(_dptr(flat), n)
    fix = dict(wire_fix or {})
    seg = [0] * n

    def project(q):
        key = (q, seg[q])
        if key in fix:
            m = np.ascontiguousarray(_projector(fix[key])).view(np.float64)
            lib.sv_apply_1q(_dptr(flat), n, q, _dptr(m))

    for q in range(n):
        project(q)
    gates = circuit.gates if stop is None else circuit.gates[:stop]
    for g in gates:
        m = np.ascontiguousarray(_gates.matrix(g)).view(np.float64)
        if len(g.qubits) == 1:
            lib.sv_apply_1q(_dptr(flat), n, g.qubits[0], _dptr(m))
        else:
            lib.sv_apply_2q(_dptr(flat), n, g.qubits[0], g.qubits[1], _dptr(m))
        for q in g.qubits:
            seg[q] += 1
            project(q)
    return psi


def amplitudes(circuit, bitstrings, wire_fix=None, psi=None) -> np.ndarray:
    if psi is None:
        psi = simulate(circuit, wire_fix)
    idx = np.ascontiguousarray(sv_index(bitstrings, circuit.n_qubits))
    out = np.empty(len(idx), dtype=np.complex128)
    _load().sv_gather(_dptr(psi.view(np.float64)), len(idx),
                      idx.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), _dptr(out.view(np.float64)))
    return out


def threads() -> int:
    v = os.environ.get("OMP_NUM_THREADS")
    return int(v) if v else (os.cpu_count() or 1)
