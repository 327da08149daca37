"""Seeded synthetic inputs shared by the product path and the oracle.

This module holds no arithmetic of the method: it only decides *which* gates
act on *which* qubits (names, qubit tuples, fSim angles), how the wires of a
circuit are labelled as tensor-network indices, and which output bitstrings
are requested.  Gate matrices, contraction and amplitudes are computed by the
two sides separately (the engine binding and the oracle each build their own
matrices from the gate names).

Circuit form (paper, Sec. 2.1): m full cycles -- a layer of single-qubit gates
drawn from {sqrtX, sqrtY, sqrtW}, then fSim on the couplers of the cycle's
pattern -- followed by a final layer of single-qubit gates.
"""
from .circuits import (  # noqa: F401
    Gate,
    Circuit,
    rect_grid,
    diag_grid,
    random_circuit,
    config_circuit,
)
from .tn import TensorSpec, TNStructure, tn_structure  # noqa: F401
from .bitstrings import (  # noqa: F401
    uniform_bitstrings,
    prefix_bitstrings,
    subspace_bitstrings,
    closed_values,
)
