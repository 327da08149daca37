"""Top-k post-selection in a correlated subspace (oracle).  Test infrastructure
only.

Sec. 1 and Sec. 2.3 (post-processing, also called post-selection): the
probabilities of every bitstring of a correlated subspace (bitstrings that
share the values of some qubits) are cheap to get together, and keeping only
the k bitstrings with the largest probabilities out of the N of a subspace
gives uncorrelated samples whose linear XEB is raised by roughly ln(N/k).

Definitions used here:
* probability p_i = re_i * re_i + im_i * im_i in float64, each product and the
  sum rounded on its own (no fused multiply-add);
* order: probability descending, then index ascending, a total order, so the
  top-k list is unique even with ties; if k >= N all N entries are returned;
* linear XEB of selected samples x_1..x_m under the ideal distribution:
  2^n * mean(p_ideal(x_j)) - 1.
Every amplitude must be finite.
"""
from __future__ import annotations

import numpy as np


def probabilities(amps) -> np.ndarray:
    a = np.asarray(amps, dtype=np.complex128).ravel()
    re, im = a.real.copy(), a.imag.copy()
    return re * re + im * im


def topk(amps, k: int):
    """(indices, probabilities) of the k most probable entries, in order."""
    p = probabilities(amps)
    order = np.lexsort((np.arange(p.size), -p))
    sel = order[: min(int(k), p.size)]
    return sel.astype(np.int64), p[sel]


def linear_xeb(p_ideal_selected, n_qubits: int) -> float:
    p = np.asarray(p_ideal_selected, dtype=np.float64)
    return float((2.0 ** n_qubits) * np.mean(p) - 1.0)


def expected_max_porter_thomas(n: int) -> float:
    """E[max of n i.i.d. Exp(1)] = H_n, the harmonic number: the mean of
    2^q p over the top-1 of a Porter-Thomas subspace of n bitstrings."""
    return float(np.sum(1.0 / np.arange(1, n + 1)))
