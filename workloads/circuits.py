"""Random-quantum-circuit generator (structure only).

Paper, Sec. 2.1 ("Quantum circuits"): a random circuit is m full cycles, each a
layer of single-qubit gates on every qubit followed by two-qubit gates on
qubit pairs that change from cycle to cycle, and then a half cycle of
single-qubit gates only.  The single-qubit gate set is {sqrtX, sqrtY, sqrtW};
the two-qubit gate is fSim(theta, phi).

Readings where the paper is silent:
* "m cycles" means m full cycles plus the final single-qubit layer.
* Single-qubit gates are drawn i.i.d. uniform over the three names from a
  seeded PCG64 stream (numpy ``default_rng``), one row of draws per layer.
* Cycle c uses coupler class ``pattern[c % len(pattern)]``.
* Rectangular grid: A = horizontal pairs starting in an even column,
  B = horizontal pairs starting in an odd column, C = vertical pairs starting
  in an even row, D = vertical pairs starting in an odd row.
* Diagonal ("Sycamore-style") grid: 9 rows of 6 sites, even rows at x = 2c,
  odd rows at x = 2c + 1; a site couples to the sites of the next row at
  x - 1 and x + 1.  A = down-right couplers from even rows, B = down-right
  from odd rows, C = down-left from even rows, D = down-left from odd rows.
  One boundary site is removed (dead), leaving 53 qubits numbered in
  row-major site order.
Each coupler class is a matching, so the two-qubit gates of one cycle commute.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

ONE_QUBIT_NAMES = ("sqrtX", "sqrtY", "sqrtW")


@dataclass(frozen=True)
class Gate:
    name: str                 # 'sqrtX' | 'sqrtY' | 'sqrtW' | 'fsim'
    qubits: tuple             # (q,) or (q1, q2); q1 is the more significant bit of the 4x4 basis
    params: tuple = ()        # fsim: (theta, phi)


@dataclass
class Circuit:
    n_qubits: int
    gates: list
    sites: list               # (row, x) per qubit
    cycles: int
    pattern: str
    couplers: dict = field(default_factory=dict)

    def qubit_gate_counts(self):
        c = [0] * self.n_qubits
        for g in self.gates:
            for q in g.qubits:
                c[q] += 1
        return c


def rect_grid(rows: int, cols: int):
    """Sites and coupler classes A-D of a rows x cols rectangular grid."""
    sites = [(r, c) for r in range(rows) for c in range(cols)]
    idx = {s: i for i, s in enumerate(sites)}
    cp = {k: [] for k in "ABCD"}
    for r in range(rows):
        for c in range(cols - 1):
            cp["A" if c % 2 == 0 else "B"].append((idx[(r, c)], idx[(r, c + 1)]))
    for r in range(rows - 1):
        for c in range(cols):
            cp["C" if r % 2 == 0 else "D"].append((idx[(r, c)], idx[(r + 1, c)]))
    return sites, cp


def diag_grid(rows: int = 9, per_row: int = 6, dead=(0, 3)):
    """Rotated-lattice sites (row, x) and coupler classes A-D.

    ``dead`` is (row, column-in-row) of the removed boundary site.
    """
    all_sites = []
    for r in range(rows):
        for c in range(per_row):
            all_sites.append((r, 2 * c + (r % 2), c))
    alive = [s for s in all_sites if dead is None or (s[0], s[2]) != tuple(dead)]
    sites = [(r, x) for (r, x, _c) in alive]
    idx = {s: i for i, s in enumerate(sites)}
    cp = {k: [] for k in "ABCD"}
    for (r, x) in sites:
        for dx, base in ((+1, "AB"), (-1, "CD")):
            t = (r + 1, x + dx)
            if t in idx:
                cls = base[0] if r % 2 == 0 else base[1]
                cp[cls].append((idx[(r, x)], idx[t]))
    return sites, cp


def random_circuit(sites, couplers, cycles: int, seed: int, theta: float = math.pi / 2,
                   phi: float = math.pi / 6, pattern: str = "ABCD") -> Circuit:
    n = len(sites)
    rng = np.random.default_rng(seed)
    draws = rng.integers(0, 3, size=(cycles + 1, n))
    gates = []
    for cyc in range(cycles):
        for q in range(n):
            gates.append(Gate(ONE_QUBIT_NAMES[int(draws[cyc, q])], (q,)))
        for (a, b) in sorted(couplers[pattern[cyc % len(pattern)]]):
            gates.append(Gate("fsim", (a, b), (theta, phi)))
    for q in range(n):
        gates.append(Gate(ONE_QUBIT_NAMES[int(draws[cycles, q])], (q,)))
    return Circuit(n, gates, list(sites), cycles, pattern, couplers)


# Workload catalogue: the synthetic stand-ins for the paper's Sycamore runs.
CONFIGS = {
    # 12-qubit 3x4 grid, 8 cycles, 64 uniform bitstrings, no slicing.
    0: dict(kind="rect", rows=3, cols=4, cycles=8, seed=0),
    # 30-qubit 5x6 grid, 14 cycles, 8 sliced labels, 1024 bitstrings with a 20-bit prefix.
    2: dict(kind="rect", rows=5, cols=6, cycles=14, seed=2),
    # 53 qubits on the 54-site diagonal grid (one dead site), 20 cycles.
    3: dict(kind="diag", rows=9, per_row=6, dead=(0, 3), cycles=20, seed=4),
}


def make_layout(spec: dict):
    if spec["kind"] == "rect":
        return rect_grid(spec["rows"], spec["cols"])
    return diag_grid(spec.get("rows", 9), spec.get("per_row", 6), spec.get("dead", (0, 3)))


def config_circuit(i: int, cycles: int | None = None, seed: int | None = None) -> Circuit:
    spec = CONFIGS[i]
    sites, cp = make_layout(spec)
    return random_circuit(sites, cp, spec["cycles"] if cycles is None else cycles,
                          spec["seed"] if seed is None else seed)
