"""Brute-force unitary of a tiny circuit (oracle pin for the state vector).

U is the ordered product of each gate expanded to the full 2^n space with
Kronecker products (qubit 0 is the leftmost factor, i.e. the most significant
index bit; a two-qubit gate is first brought to the two leading factors by a
qubit permutation); A(x) = U[idx(x), 0].
"""
from __future__ import annotations

import numpy as np

from . import gates as _gates


def _expand_1q(m, q, n):
    out = np.array([[1.0 + 0j]])
    for k in range(n):
        out = np.kron(out, m if k == q else np.eye(2))
    return out


def _qubit_permutation(order, n):
    """Permutation matrix P with (P psi)[i'] = psi[i], where qubit order[k] of
    the old index becomes qubit k of the new index."""
    dim = 1 << n
    p = np.zeros((dim, dim))
    for i in range(dim):
        bits = [(i >> (n - 1 - q)) & 1 for q in range(n)]
        j = 0
        for k in range(n):
            j |= bits[order[k]] << (n - 1 - k)
        p[j, i] = 1.0
    return p


def _expand_2q(m, q1, q2, n):
    """P^T (m (x) I) P with P moving (q1, q2) to the two leading qubits."""
    order = [q1, q2] + [q for q in range(n) if q not in (q1, q2)]
    p = _qubit_permutation(order, n)
    return p.T @ np.kron(m, np.eye(1 << (n - 2))) @ p


def unitary(circuit) -> np.ndarray:
    n = circuit.n_qubits
    u = np.eye(1 << n, dtype=np.complex128)
    for g in circuit.gates:
        m = _gates.matrix(g)
        if len(g.qubits) == 1:
            u = _expand_1q(m, g.qubits[0], n) @ u
        else:
            u = _expand_2q(m, g.qubits[0], g.qubits[1], n) @ u
    return u
