"""Requested output bitstrings.

A bitstring is a uint64 whose bit q is the measured value of qubit q.
Correlated subspaces (paper, Sec. 2.2/2.3 on correlated amplitudes): a set of
bitstrings that share the values of some qubits ("closed") and vary on the
others ("open").
"""
from __future__ import annotations

import numpy as np


def uniform_bitstrings(n_qubits: int, count: int, seed: int) -> np.ndarray:
    rng = np.random.default_rng(seed)
    bits = rng.integers(0, 2, size=(count, n_qubits), dtype=np.uint64)
    w = np.left_shift(np.uint64(1), np.arange(n_qubits, dtype=np.uint64))
    return (bits * w).sum(axis=1).astype(np.uint64)


def prefix_bitstrings(n_qubits: int, open_qubits, count: int, seed: int) -> np.ndarray:
    """``count`` bitstrings (drawn with replacement, order kept) that share a
    seeded random value on every qubit not in ``open_qubits``."""
    rng = np.random.default_rng(seed)
    fixed = rng.integers(0, 2, size=n_qubits, dtype=np.uint64)
    open_q = list(open_qubits)
    var = rng.integers(0, 2, size=(count, len(open_q)), dtype=np.uint64)
    out = np.zeros(count, dtype=np.uint64)
    for q in range(n_qubits):
        if q not in open_q:
            out |= np.uint64(int(fixed[q]) << q)
    for j, q in enumerate(open_q):
        out |= var[:, j] << np.uint64(q)
    return out


def subspace_bitstrings(n_qubits: int, open_qubits, seed: int) -> np.ndarray:
    """All 2^len(open) bitstrings of one correlated subspace, enumerated with
    open_qubits[0] as the least significant counter bit."""
    rng = np.random.default_rng(seed)
    fixed = rng.integers(0, 2, size=n_qubits, dtype=np.uint64)
    open_q = list(open_qubits)
    base = 0
    for q in range(n_qubits):
        if q not in open_q:
            base |= int(fixed[q]) << q
    out = np.empty(1 << len(open_q), dtype=np.uint64)
    for v in range(1 << len(open_q)):
        x = base
        for j, q in enumerate(open_q):
            x |= ((v >> j) & 1) << q
        out[v] = x
    return out


def closed_values(bitstrings: np.ndarray, n_qubits: int, open_qubits) -> dict:
    """{qubit: value} for every qubit outside ``open_qubits``; raises if the
    bitstrings disagree on one of them."""
    b = np.asarray(bitstrings, dtype=np.uint64)
    res = {}
    for q in range(n_qubits):
        if q in open_qubits:
            continue
        v = (b >> np.uint64(q)) & np.uint64(1)
        if len(v) and not np.all(v == v[0]):
            raise ValueError(f"bitstrings disagree on closed qubit {q}")
        res[q] = int(v[0]) if len(v) else 0
    return res
