"""Accuracy and randomness metrics (oracle).

* fidelity: paper Eq. ``fidelity``, whose printed form is garbled; read as
  |<b, r>|^2 / (||b||^2 ||r||^2) with <b, r> = sum conj(b_i) r_i.  It is
  blind to a global scale, so ``rel_l2`` is always reported beside it.
* linear XEB of ideal amplitudes: 2^n sum_x p(x)^2 - 1 (about 1 for a
  Porter-Thomas distribution).
* Porter-Thomas distance: Kolmogorov-Smirnov distance between the empirical
  distribution of 2^n p(x) and Exp(1).
"""
from __future__ import annotations

import numpy as np


def fidelity(bench, result) -> float:
    b = np.asarray(bench, dtype=np.complex128).ravel()
    r = np.asarray(result, dtype=np.complex128).ravel()
    nb = np.vdot(b, b).real
    nr = np.vdot(r, r).real
    if nb == 0.0 or nr == 0.0:
        return 1.0 if nb == nr else 0.0
    return float(abs(np.vdot(b, r)) ** 2 / (nb * nr))


def rel_l2(result, bench) -> float:
    b = np.asarray(bench, dtype=np.complex128).ravel()
    r = np.asarray(result, dtype=np.complex128).ravel()
    nb = np.linalg.norm(b)
    return float(np.linalg.norm(r - b) / nb) if nb else float(np.linalg.norm(r))


def rel_max(result, bench) -> float:
    b = np.asarray(bench, dtype=np.complex128).ravel()
    r = np.asarray(result, dtype=np.complex128).ravel()
    mb = np.max(np.abs(b)) if b.size else 0.0
    return float(np.max(np.abs(r - b)) / mb) if mb else float(np.max(np.abs(r), initial=0.0))


def xeb_ideal(probs, n_qubits: int) -> float:
    p = np.asarray(probs, dtype=np.float64)
    return float((2.0 ** n_qubits) * np.sum(p * p) - 1.0)


def porter_thomas_ks(probs, n_qubits: int) -> float:
    x = np.sort((2.0 ** n_qubits) * np.asarray(probs, dtype=np.float64).ravel())
    m = x.size
    cdf = 1.0 - np.exp(-x)
    hi = np.arange(1, m + 1) / m
    lo = np.arange(0, m) / m
    return float(max(np.max(hi - cdf), np.max(cdf - lo)))
