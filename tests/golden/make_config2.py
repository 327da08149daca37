"""Write the oracle's amplitudes for the 30-qubit workload (5x6 grid,
14 cycles, circuit seed 2; 1024 bitstrings sharing a seeded 20-bit prefix on
qubits 0-19, qubits 20-29 random, seed 3) to config2_amplitudes.npy.

Calls only the oracle (FP64 state vector of 2^30 amplitudes, 16 GiB of host
memory).  Run from the repository root:  python tests/golden/make_config2.py
"""
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import workloads  # noqa: E402
from oracle import statevector  # noqa: E402

OPEN = list(range(20, 30))


def bitstrings():
    return workloads.prefix_bitstrings(30, OPEN, 1024, 3)


def main():
    c = workloads.config_circuit(2)
    t0 = time.time()
    amp = statevector.amplitudes(c, bitstrings())
    out = os.path.join(os.path.dirname(os.path.abspath(__file__)), "config2_amplitudes.npy")
    np.save(out, amp)
    print(f"wrote {out} in {time.time() - t0:.1f} s, |amp|^2 sum {np.sum(np.abs(amp) ** 2):.6e}")


if __name__ == "__main__":
    main()
