"""Seeded pairwise-contraction cases (shapes and label orders only).

Each case draws k in [4, 16] reduced labels, b in [0, 6] batch labels and
m, n in [8, 16] free labels of A and B, and keeps it when
20 <= b+m+k <= 34, 20 <= b+n+k <= 34 and b+m+n <= 34 (operands of rank
20-34), and the working set (A, B, C and one permuted copy of each, at 8
bytes per complex entry) stays within 240 GB.  Label orders of A, B and C
are random permutations.  Entries are drawn separately (complex normal,
A scaled by 1/sqrt(K)).
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np


@dataclass(frozen=True)
class Case:
    seed: int
    b: int
    m: int
    n: int
    k: int
    a_labels: tuple
    b_labels: tuple
    c_labels: tuple

    def elems(self):
        return 2 ** (self.b + self.m + self.k), 2 ** (self.b + self.n + self.k), 2 ** (self.b + self.m + self.n)

    def working_set_bytes(self, elem_bytes=8):
        a, b, c = self.elems()
        return 2 * elem_bytes * (a + b + c)


def draw(seed: int) -> Case:
    rng = np.random.default_rng(seed)
    while True:
        k = int(rng.integers(4, 17))
        b = int(rng.integers(0, 7))
        m = int(rng.integers(8, 17))
        n = int(rng.integers(8, 17))
        if not (20 <= b + m + k <= 34 and 20 <= b + n + k <= 34 and b + m + n <= 34):
            continue
        c = Case(seed, b, m, n, k, (), (), ())
        if c.working_set_bytes() > 240e9:
            continue
        labels = list(range(b + m + n + k))
        rng.shuffle(labels)
        bl, ml, nl, kl = labels[:b], labels[b:b + m], labels[b + m:b + m + n], labels[b + m + n:]
        a_l = bl + ml + kl
        b_l = bl + nl + kl
        c_l = bl + ml + nl
        rng.shuffle(a_l)
        rng.shuffle(b_l)
        rng.shuffle(c_l)
        return Case(seed, b, m, n, k, tuple(a_l), tuple(b_l), tuple(c_l))


def cases(count: int = 200, first_seed: int = 0):
    return [draw(first_seed + i) for i in range(count)]
