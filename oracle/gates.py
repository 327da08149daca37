"""Gate matrices (oracle copy), paper Sec. 2.1.

sqrtX, sqrtY, sqrtW are pi/2 rotations about equatorial axes, given up to a
global phase; fSim(theta, phi) acts on |00>, |01>, |10>, |11> (first qubit
most significant).

Readings: sqrt(i) = exp(i pi/4) and sqrt(-i) = exp(-i pi/4) (principal
branch); |x| < 1e-15 in cos/sin is snapped to 0 so fSim(pi/2, .) has exact
zeros on its diagonal middle block.
"""
from __future__ import annotations

import cmath
import math

import numpy as np

_R = 1.0 / math.sqrt(2.0)


def _snap(x: float) -> float:
    return 0.0 if abs(x) < 1e-15 else x


def sqrt_x() -> np.ndarray:
    return _R * np.array([[1, -1j], [-1j, 1]], dtype=np.complex128)


def sqrt_y() -> np.ndarray:
    return _R * np.array([[1, -1], [1, 1]], dtype=np.complex128)


def sqrt_w() -> np.ndarray:
    si = cmath.exp(1j * math.pi / 4)     # sqrt(i)
    smi = cmath.exp(-1j * math.pi / 4)   # sqrt(-i)
    return _R * np.array([[1, -si], [smi, 1]], dtype=np.complex128)


def fsim(theta: float, phi: float) -> np.ndarray:
    c = _snap(math.cos(theta))
    s = _snap(math.sin(theta))
    e = complex(_snap(math.cos(phi)), _snap(-math.sin(phi)))
    return np.array([[1, 0, 0, 0],
                     [0, c, -1j * s, 0],
                     [0, -1j * s, c, 0],
                     [0, 0, 0, e]], dtype=np.complex128)


def matrix(gate) -> np.ndarray:
    if gate.name == "sqrtX":
        return sqrt_x()
    if gate.name == "sqrtY":
        return sqrt_y()
    if gate.name == "sqrtW":
        return sqrt_w()
    if gate.name == "fsim":
        return fsim(*gate.params)
    raise ValueError(f"unknown gate {gate.name}")
