"""One pairwise complex contraction (oracle), paper Eq. ``contraction``.

C[gamma] = sum over the reduced labels delta of A[alpha] * B[beta], with
delta = alpha intersect beta minus gamma (labels kept in C that both operands
hold are batch labels).  ``contract_pair`` is numpy.einsum in complex128
(a matrix product through BLAS where the labels allow);
``entry`` computes a single output element as an explicit FP64 dot product
over the reduced labels (for spot checks of large contractions, where the
operands are available only element by element).
"""
from __future__ import annotations

import itertools
import string

import numpy as np

_L = string.ascii_letters


def contract_pair(a, a_labels, b, b_labels, c_labels):
    uni = list(dict.fromkeys(list(a_labels) + list(b_labels)))
    sym = {l: _L[i] for i, l in enumerate(uni)}
    spec = "".join(sym[l] for l in a_labels) + "," + "".join(sym[l] for l in b_labels) + \
        "->" + "".join(sym[l] for l in c_labels)
    return np.einsum(spec, np.asarray(a, np.complex128), np.asarray(b, np.complex128), optimize=True)


def entry(a_at, a_labels, b_at, b_labels, c_labels, c_values):
    """C at the label values ``c_values`` (one per c label).

    a_at / b_at: callables mapping a dict {label: value} to the complex entry
    of that operand.
    """
    fixed = dict(zip(c_labels, c_values))
    reduced = [l for l in dict.fromkeys(list(a_labels) + list(b_labels)) if l not in fixed]
    acc = 0j
    for vals in itertools.product((0, 1), repeat=len(reduced)):
        v = dict(fixed)
        v.update(zip(reduced, vals))
        acc += complex(a_at(v)) * complex(b_at(v))
    return acc


def entry_dot(a_vals, b_vals):
    """One output entry from the operand entries along the reduced labels
    (already gathered in matching order): sum_k a_k b_k in FP64."""
    return complex(np.dot(np.asarray(a_vals, np.complex128), np.asarray(b_vals, np.complex128)))
