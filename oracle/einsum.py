"""Naive FP64 tensor-network contraction (oracle).

Paper Eq. ``contraction``: a pairwise einsum sums the product of the two
operands over the reduced labels; the value of a whole network is the sum,
over all assignments of its internal labels, of the product of its tensor
entries, whatever the pairwise order.  Slicing (paper Sec. 3.1, sub-networks
by fixing the values of chosen labels) fixes a label to a value by indexing
every tensor that holds it; the sum over all values of the sliced labels is
the unsliced network.

``contract`` picks its own pairwise order (smallest result first) and calls
``numpy.einsum`` per pair, in complex128; numpy reduces a pair to a matrix
product (tensordot, BLAS) where the labels allow it.  ``brute_force`` is the definition
written out, for tiny networks.
"""
from __future__ import annotations

import itertools
import string

import numpy as np

from . import gates as _gates

_LETTERS = string.ascii_letters


def network_tensors(circuit, structure):
    """[(labels, complex128 ndarray)] for a circuit's network, with the oracle's
    own gate matrices placed as the structure dictates (first label slowest)."""
    out = []
    for t in structure.tensors:
        if t.kind == "init":
            data = np.array([1.0, 0.0], dtype=np.complex128)
        else:
            g = circuit.gates[t.ref]
            m = _gates.matrix(g)
            data = m.reshape((2,) * (2 * len(g.qubits)))
        out.append((tuple(t.labels), data))
    return out


def fix_labels(tensors, fixed: dict):
    """Index every tensor at the fixed label values (removes those labels)."""
    res = []
    for labels, data in tensors:
        sel = tuple(fixed[l] if l in fixed else slice(None) for l in labels)
        res.append((tuple(l for l in labels if l not in fixed), np.ascontiguousarray(data[sel])))
    return res


def _pair(a, b, keep):
    la, da = a
    lb, db = b
    uni = list(dict.fromkeys(la + lb))
    if len(uni) > len(_LETTERS):
        raise ValueError("pair too wide for the oracle")
    sym = {l: _LETTERS[i] for i, l in enumerate(uni)}
    lc = tuple(l for l in uni if l in keep)
    spec = "".join(sym[l] for l in la) + "," + "".join(sym[l] for l in lb) + "->" + \
        "".join(sym[l] for l in lc)
    # optimize: numpy groups the labels and calls its matrix product (BLAS
    # zgemm) when the pair is a plain contraction; the sum is the same
    return lc, np.einsum(spec, da, db, optimize=True)


def contract(tensors, output_labels, fixed=None, max_rank: int = 40):
    """Contract the whole network; result axes follow ``output_labels``.

    Labels in ``fixed`` are indexed first.  Output labels are kept; any other
    label is summed once no remaining tensor but the pair holds it.
    """
    ts = fix_labels(tensors, fixed or {})
    out = tuple(l for l in output_labels if not (fixed and l in fixed))
    alive = {i: t for i, t in enumerate(ts)}
    nxt = len(ts)
    where = {}
    for i, (labels, _d) in alive.items():
        for l in labels:
            where.setdefault(l, set()).add(i)
    outset = set(out)

    # single-tensor labels that are not outputs: sum them now
    for i in list(alive):
        labels, d = alive[i]
        lonely = [l for l in labels if len(where[l]) == 1 and l not in outset]
        if lonely:
            axes = tuple(labels.index(l) for l in lonely)
            alive[i] = (tuple(l for l in labels if l not in lonely), d.sum(axis=axes))
            for l in lonely:
                del where[l]

    while len(alive) > 1:
        best = None
        for l, holders in where.items():
            if len(holders) < 2:
                continue
            hs = sorted(holders)
            for x in range(len(hs)):
                for y in range(x + 1, len(hs)):
                    i, j = hs[x], hs[y]
                    la, lb = alive[i][0], alive[j][0]
                    keep = set()
                    for m in set(la) | set(lb):
                        if m in outset or (where[m] - {i, j}):
                            keep.add(m)
                    r = len(keep)
                    key = (r, i, j)
                    if best is None or key < best[0]:
                        best = (key, i, j, keep)
        if best is None:   # disconnected: outer product of the two smallest
            ids = sorted(alive, key=lambda k: (len(alive[k][0]), k))[:2]
            i, j = ids
            keep = set(alive[i][0]) | set(alive[j][0])
        else:
            _k, i, j, keep = best
        if len(keep) > max_rank:
            raise ValueError(f"oracle contraction needs rank {len(keep)} > {max_rank}")
        lc, dc = _pair(alive[i], alive[j], keep)
        for l in set(alive[i][0]) | set(alive[j][0]):
            where[l].discard(i)
            where[l].discard(j)
            if l in keep:
                where[l].add(nxt)
            elif not where[l]:
                del where[l]
        del alive[i]
        del alive[j]
        alive[nxt] = (lc, dc)
        nxt += 1
    (labels, data), = alive.values()
    if set(labels) != set(out):
        raise ValueError("network does not reduce to the output labels")
    perm = [labels.index(l) for l in out]
    return np.transpose(data, perm) if perm else data


def brute_force(tensors, output_labels, fixed=None):
    """Sum over every assignment of the internal labels of the product of the
    tensor entries (the definition); tiny networks only."""
    ts = fix_labels(tensors, fixed or {})
    out = [l for l in output_labels if not (fixed and l in fixed)]
    labels = sorted({l for lab, _ in ts for l in lab})
    internal = [l for l in labels if l not in out]
    res = np.zeros((2,) * len(out), dtype=np.complex128)
    for ov in itertools.product((0, 1), repeat=len(out)):
        val = {l: v for l, v in zip(out, ov)}
        acc = 0j
        for iv in itertools.product((0, 1), repeat=len(internal)):
            val.update(zip(internal, iv))
            p = 1 + 0j
            for lab, d in ts:
                p *= d[tuple(val[l] for l in lab)]
            acc += p
        res[ov] = acc
    return res


def contract_path(tensors, output_labels, ssa, fixed=None, after_step=None):
    """Contract along a given pairwise order (SSA pairs: ids >= len(tensors)
    name earlier results).  The network's value does not depend on the order
    in exact arithmetic, so the order only changes FP64 rounding; it is data
    here, not arithmetic.  A label is summed when no other live tensor and no
    output holds it.

    ``after_step(s, labels, data) -> data`` may replace the result of pair s
    (the single-step quantization study of Sec. 4.3.1 passes one step's
    result through the exchange codec of Sec. 3.2)."""
    ts = fix_labels(tensors, fixed or {})
    out = tuple(l for l in output_labels if not (fixed and l in fixed))
    outset = set(out)
    live = {i: t for i, t in enumerate(ts)}
    count = {}
    for labels, _d in ts:
        for l in labels:
            count[l] = count.get(l, 0) + 1
    nxt = len(ts)
    for s in range(len(ssa) // 2):
        i, j = int(ssa[2 * s]), int(ssa[2 * s + 1])
        la, lb = live[i][0], live[j][0]
        keep = set()
        for l in set(la) | set(lb):
            others = count[l] - (l in la) - (l in lb)
            if l in outset or others > 0:
                keep.add(l)
        lc, dc = _pair(live[i], live[j], keep)
        if after_step is not None:
            dc = after_step(s, lc, dc)
        for l in set(la) | set(lb):
            count[l] -= (l in la) + (l in lb)
        for l in lc:
            count[l] = count.get(l, 0) + 1
        del live[i]
        del live[j]
        live[nxt] = (lc, dc)
        nxt += 1
    (labels, data), = live.values()
    if set(labels) != set(out):
        raise ValueError("path does not reduce to the output labels")
    return np.transpose(data, [labels.index(l) for l in out]) if out else data
