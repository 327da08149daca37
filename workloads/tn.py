"""Tensor-network structure of a circuit: which labels each tensor carries.

Paper, Sec. 2.2: the n-qubit state is a rank-n tensor, a single-qubit gate a
rank-2 tensor and a two-qubit gate a rank-4 tensor; contracting the network
yields amplitudes.  Every label has dimension 2.

Conventions (fixed here, implemented independently by each consumer):
* Label ids are dense, in creation order: the initial wire of qubit q is
  label q; each gate then creates one new label per qubit it acts on, in gate
  order and, within a gate, in the order of ``gate.qubits``.
* Tensor order: the n initial-state tensors (qubit order), then one tensor per
  gate in circuit order.
* An initial tensor has labels [wire_q]; its entries are the basis state |0>.
* A one-qubit gate G has labels [out, in] with entry [o, i] = G[o, i].
* A two-qubit gate M on (q1, q2) has labels [out1, out2, in1, in2] with entry
  [o1, o2, i1, i2] = M[2*o1 + o2, 2*i1 + i2].
* Dense data is row-major with the first label slowest.
* ``output_labels[q]`` is the last wire of qubit q; ``label_wire[l]`` is
  (qubit, segment) where segment s is the wire after the s-th gate on the qubit.
"""
from __future__ import annotations

from dataclasses import dataclass


@dataclass(frozen=True)
class TensorSpec:
    kind: str        # 'init' (ref = qubit) or 'gate' (ref = index into circuit.gates)
    ref: int
    labels: tuple


@dataclass
class TNStructure:
    tensors: list
    output_labels: list
    n_labels: int
    label_wire: list   # label -> (qubit, segment)


def tn_structure(circuit) -> TNStructure:
    n = circuit.n_qubits
    cur = list(range(n))
    seg = [0] * n
    label_wire = [(q, 0) for q in range(n)]
    tensors = [TensorSpec("init", q, (q,)) for q in range(n)]
    nxt = n
    for gi, g in enumerate(circuit.gates):
        outs = []
        for q in g.qubits:
            seg[q] += 1
            outs.append(nxt)
            label_wire.append((q, seg[q]))
            nxt += 1
        ins = [cur[q] for q in g.qubits]
        for q, o in zip(g.qubits, outs):
            cur[q] = o
        tensors.append(TensorSpec("gate", gi, tuple(outs) + tuple(ins)))
    return TNStructure(tensors, list(cur), nxt, label_wire)
