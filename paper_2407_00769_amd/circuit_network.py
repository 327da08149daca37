"""Circuit -> labelled tensor list for tnc_network_create (input marshalling).

Gate matrices follow paper Sec. 2.1 (sqrtX, sqrtY, sqrtW up to a global
phase; fSim(theta, phi) in the basis |00>,|01>,|10>,|11>); the principal
square roots are used for sqrt(i) and sqrt(-i), and cos/sin values below
1e-15 in magnitude are exact zeros.  Tensor placement follows the structure
of ``workloads.tn``: a one-qubit gate G is stored with labels [out, in] as
G[out, in], a two-qubit gate M as [o1, o2, i1, i2] = M[2 o1 + o2, 2 i1 + i2],
an initial wire as |0>.
"""
from __future__ import annotations

import cmath
import math

import numpy as np

_S = 1.0 / math.sqrt(2.0)


def _z(x: float) -> float:
    return 0.0 if abs(x) < 1e-15 else x


def gate_matrix(gate) -> np.ndarray:
    if gate.name == "sqrtX":
        return _S * np.array([[1, -1j], [-1j, 1]], dtype=np.complex128)
    if gate.name == "sqrtY":
        return _S * np.array([[1, -1], [1, 1]], dtype=np.complex128)
    if gate.name == "sqrtW":
        return _S * np.array([[1, -cmath.exp(1j * math.pi / 4)], [cmath.exp(-1j * math.pi / 4), 1]],
                             dtype=np.complex128)
    if gate.name == "fsim":
        th, ph = gate.params
        c, s = _z(math.cos(th)), _z(math.sin(th))
        return np.array([[1, 0, 0, 0], [0, c, -1j * s, 0], [0, -1j * s, c, 0],
                         [0, 0, 0, complex(_z(math.cos(ph)), _z(-math.sin(ph)))]], dtype=np.complex128)
    raise ValueError(gate.name)


def network_arrays(circuit, structure):
    """(ranks, labels, data as interleaved float64, output_labels)."""
    ranks, labels, chunks = [], [], []
    for t in structure.tensors:
        ranks.append(len(t.labels))
        labels.extend(t.labels)
        if t.kind == "init":
            d = np.array([1.0, 0.0], dtype=np.complex128)
        else:
            d = gate_matrix(circuit.gates[t.ref]).reshape(-1)
        chunks.append(d)
    data = np.concatenate(chunks).view(np.float64)
    return (np.array(ranks, np.int32), np.array(labels, np.int32), data,
            np.array(structure.output_labels, np.int32))
