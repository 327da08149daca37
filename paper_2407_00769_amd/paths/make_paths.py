"""Search and store the fixed sliced path of the 53-qubit workload.

53 qubits on the 54-site diagonal grid (one dead site), 20 cycles, circuit
seed 4; qubits 41-52 open, the rest closed; no tensor of one slice above 2^33
complex entries (32 GiB in 16-bit complex storage; the workload allows 64 GiB,
but at 2^34 the live tensors of one slice approach the 288 GB of HBM).  Search: 256 randomized greedy restarts
with subtree reconfiguration, seed 1.  The complex64 form cannot hold 2^34
entries in one slice next to its operands, so it runs the same path with extra
sliced labels down to a cap of 2^32 (four complex64 slices per original slice).

Run from the repository root: python -m paper_2407_00769_amd.paths.make_paths
"""
from __future__ import annotations

import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

OPEN = list(range(41, 53))
CAP, CAP_C64, RESTARTS, SEED, RECONF = 33, 32, 256, 1, 16


def network():
    import workloads
    from paper_2407_00769_amd import _tnc as T
    from paper_2407_00769_amd import circuit_network as cn
    c = workloads.config_circuit(3)
    st = workloads.tn_structure(c)
    r, l, d, o = cn.network_arrays(c, st)
    return c, st, T.tnc_network_create(r, l, d, c.n_qubits, o), len(r)


def main():
    os.environ["TNC_SEARCH_RECONF"] = str(RECONF)
    from paper_2407_00769_amd import _tnc as T
    c, st, net, n = network()
    t0 = time.time()
    ssa, sl, cost = T.tnc_search(net, n, OPEN, CAP, restarts=RESTARTS, seed=SEED)
    t_search = time.time() - t0
    sl64 = T.tnc_slice_path(net, ssa, OPEN, CAP_C64, sl)
    info = T.tnc_plan_analyze(net, ssa, sl, OPEN, "f16_4m")
    info64 = T.tnc_plan_analyze(net, ssa, sl64, OPEN, "c64")
    out = {"workload": "53-qubit diagonal grid, 20 cycles, seed 4, qubits 41-52 open",
           "n_tensors": n, "open_qubits": OPEN, "cap_log2": CAP, "cap_log2_c64": CAP_C64,
           "search": {"restarts": RESTARTS, "seed": SEED, "reconfigure_rounds": RECONF, "seconds": t_search},
           "log2_total_flops": cost, "flops_per_slice": info["flops_per_slice"],
           "peak_bytes_per_slice_f16": info["peak_bytes"], "peak_bytes_per_slice_c64": info64["peak_bytes"],
           "ssa": [int(v) for v in ssa], "sliced": [int(v) for v in sl], "sliced_c64": [int(v) for v in sl64]}
    path = os.path.join(HERE, "config3.json")
    with open(path, "w") as f:
        json.dump(out, f)
    print(f"wrote {path}: {len(sl)} sliced labels (+{len(sl64) - len(sl)} for complex64), "
          f"log2 total flops {cost:.1f}, {info['flops_per_slice']:.3e} flops/slice, "
          f"peak {info['peak_bytes'] / 2**30:.1f} GiB (f16), {info64['peak_bytes'] / 2**30:.1f} GiB (c64)")


if __name__ == "__main__":
    main()
