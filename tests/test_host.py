"""Host-side checks of the C-ABI library (no GPU needed): it loads, exports
every entry point the header declares, validates networks and paths, and its
planner derives the same per-step GEMM shapes a plain einsum implies."""
import os
import re

import numpy as np
import pytest

import workloads

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

T = pytest.importorskip("paper_2407_00769_amd._tnc", reason="libtnc.so not built")
from paper_2407_00769_amd import circuit_network as cn  # noqa: E402


def _declared():
    src = open(os.path.join(ROOT, "include", "tnc.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(tnc_[a-z0-9_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    names = _declared()
    assert len(names) >= 20
    for n in names:
        assert hasattr(T.lib, n), n
    assert set(names) == set(T.EXPORTED)
    assert "gfx950" in T.tnc_version()


def _net(cfg=0, cycles=None):
    c = workloads.config_circuit(cfg, cycles=cycles)
    st = workloads.tn_structure(c)
    r, l, d, o = cn.network_arrays(c, st)
    return c, st, T.tnc_network_create(r, l, d, c.n_qubits, o), len(r)


def test_network_validation_errors():
    # repeated label inside one tensor
    with pytest.raises(T.TncError) as e:
        T.tnc_network_create([2], [3, 3], None, 0, [])
    assert e.value.code == -1
    # an output label that no tensor holds, two qubits on one output label
    with pytest.raises(T.TncError):
        T.tnc_network_create([2, 2], [0, 1, 0, 2], None, 2, [1, 5])
    with pytest.raises(T.TncError):
        T.tnc_network_create([2, 2], [0, 1, 0, 2], None, 2, [1, 1])
    # fine: two tensors sharing a label, an output on each
    h = T.tnc_network_create([2, 2], [0, 1, 0, 2], None, 2, [1, 2])
    T.tnc_network_destroy(h)


def test_hyperedges_are_planned_and_lonely_labels_summed():
    """A label in three tensors is accepted by the plan calls (kept as a batch
    label until its last holder) and refused by the search; a label held by
    one tensor that is not an output is summed at creation."""
    # tensors: X[h, a], Y[h, b], W[h, c]; outputs a, b, c; hyperedge h
    data = np.arange(1, 25, dtype=np.float64)
    h = T.tnc_network_create([2, 2, 2], [0, 1, 0, 2, 0, 3], data, 3, [1, 2, 3])
    with pytest.raises(T.TncError) as e:
        T.tnc_search(h, 3, [0, 1, 2], 30, restarts=1, seed=0)
    assert e.value.code == -5
    st = T.tnc_plan_analyze(h, np.array([0, 1, 3, 2], np.int32), [], [0, 1, 2], "c64")
    assert st["n_steps"] + st["n_host_steps"] == 2 and st["out_rank"] == 3
    T.tnc_network_destroy(h)
    # X[a, d] with d held by X only: X becomes the rank-1 tensor sum_d X[a, d]
    h = T.tnc_network_create([2, 1], [1, 9, 1], np.arange(1, 13, dtype=np.float64), 0, [])
    st = T.tnc_plan_analyze(h, np.array([0, 1], np.int32), [], [], "c64")
    assert st["out_rank"] == 0 and st["max_rank"] == 1
    T.tnc_network_destroy(h)


def test_host_pre_contraction_keeps_the_device_path_small():
    """Steps that absorb rank-1/2 tensors run on the host; the device path
    keeps the rest of the given tree, and every step is accounted for."""
    import os as _os
    c, st, net, n = _net(0)
    ssa, sl, _ = T.tnc_search(net, n, list(range(6, 12)), 8, restarts=2, seed=0)
    full = T.tnc_plan_analyze(net, ssa, sl, list(range(6, 12)), "f16_4m")
    assert full["n_host_steps"] > 0
    assert full["n_steps"] + full["n_host_steps"] == n - 1
    _os.environ["TNC_HOST_RANK"] = "0"
    try:
        plain = T.tnc_plan_analyze(net, ssa, sl, list(range(6, 12)), "f16_4m")
    finally:
        del _os.environ["TNC_HOST_RANK"]
    assert plain["n_host_steps"] == 0 and plain["n_steps"] == n - 1
    # the large steps are the same: the flops differ by the tiny host steps only
    assert abs(full["flops_per_slice"] - plain["flops_per_slice"]) <= 0.01 * plain["flops_per_slice"]
    assert full["out_rank"] == plain["out_rank"] == 6


def test_search_returns_a_valid_tree_and_meets_the_cap():
    c, st, net, n = _net(0)
    ssa, sl, cost = T.tnc_search(net, n, list(range(12)), 30, restarts=3, seed=5)
    assert len(ssa) == 2 * (n - 1)
    seen = set()
    for i in range(n - 1):
        a, b = ssa[2 * i], ssa[2 * i + 1]
        assert a not in seen and b not in seen and a < n + i and b < n + i
        seen.update((a, b))
    assert len(sl) == 0
    # a tight cap forces slicing and is met
    open6 = list(range(6))
    ssa2, sl2, cost2 = T.tnc_search(net, n, open6, 7, restarts=3, seed=5)
    info = T.tnc_plan_analyze(net, ssa2, sl2, open6, "c64")
    assert info["max_rank"] <= 7 and len(sl2) > 0
    assert info["out_rank"] == 6
    # determinism
    assert np.array_equal(ssa2, T.tnc_search(net, n, open6, 7, restarts=3, seed=5)[0])
    # an impossible cap (below the open output) is an error
    with pytest.raises(T.TncError):
        T.tnc_search(net, n, list(range(12)), 10, restarts=1, seed=5)


def test_plan_analyze_rejects_bad_inputs():
    c, st, net, n = _net(0)
    ssa, sl, _ = T.tnc_search(net, n, list(range(12)), 30, restarts=1, seed=0)
    bad = ssa.copy()
    bad[1] = bad[0]
    with pytest.raises(T.TncError):
        T.tnc_plan_analyze(net, bad, [], list(range(12)), "c64")
    with pytest.raises(T.TncError):   # an output label cannot be sliced
        T.tnc_plan_analyze(net, ssa, [st.output_labels[0]], list(range(12)), "c64")
    with pytest.raises(T.TncError):   # 3M needs 16-bit storage
        T.tnc_plan_analyze(net, ssa, [], list(range(12)), 5)


def _einsum_flops(tensors, ssa, open_labels):
    """Per-step 8 * 2^|union| from plain label sets (the algorithmic count)."""
    ts = [set(t) for t in tensors]
    need = {}
    for t in ts:
        for l in t:
            need[l] = need.get(l, 0) + 1
    for l in open_labels:
        need[l] = need.get(l, 0) + 1
    total = 0.0
    for i in range(len(ssa) // 2):
        a, b = ts[ssa[2 * i]], ts[ssa[2 * i + 1]]
        uni = a | b
        total += 8.0 * 2 ** len(uni)
        out = set()
        for l in uni:
            after = need[l] - (l in a) - (l in b)
            if after > 0:
                out.add(l)
            need[l] = after + (1 if after > 0 else 0)
        ts.append(out)
    return total


def test_planner_flops_match_label_count(monkeypatch):
    monkeypatch.setenv("TNC_HOST_RANK", "0")   # every step of the path on the device
    c, st, net, n = _net(0)
    open_q = list(range(12))
    ssa, sl, _ = T.tnc_search(net, n, open_q, 30, restarts=2, seed=3)
    info = T.tnc_plan_analyze(net, ssa, sl, open_q, "f16_4m")
    want = _einsum_flops([t.labels for t in st.tensors], list(ssa), st.output_labels)
    assert info["flops_per_slice"] + info["flops_invariant"] == pytest.approx(want, rel=1e-12)


def test_smoke_case_is_sliced_under_its_cap():
    """The host half of the smoke run finds a sliced path under its cap."""
    import __graft_entry__ as ge
    from paper_2407_00769_amd import _tnc as T
    c, net, ssa, sl, open_q, bits = ge.smoke_case()
    info = T.tnc_plan_analyze(net, ssa, sl, open_q, "c64")
    assert len(sl) > 0 and len(ssa) == 2 * (info["n_steps"] + info["n_host_steps"])
    assert T.tnc_plan_analyze(net, ssa, sl, open_q, "c64")["max_rank"] <= 8
    T.tnc_network_destroy(net)


def test_codec_sizes_and_group_rules():
    """Code and group counts of the exchange codec (Sec. 3.2): half 2 bytes and
    int8 1 byte per value in one group; int4 two values per byte in groups of a
    power of two from 16 to 1024 (128 by default); anything else is refused."""
    n = 1000
    assert T.tnc_quant_sizes("half", n) == (2 * n, 1)
    assert T.tnc_quant_sizes("int8", n) == (n, 1)
    assert T.tnc_quant_sizes("int4", n) == ((n + 1) // 2, (n + 127) // 128)
    assert T.tnc_quant_sizes("int4", n, 16) == ((n + 1) // 2, (n + 15) // 16)
    assert T.tnc_quant_sizes("int4", 0) == (0, 0)
    for kind, group in (("int4", 100), ("int4", 2048), ("int4", 8), ("half", 64), ("int8", 128)):
        with pytest.raises(T.TncError):
            T.tnc_quant_sizes(kind, n, group)
    with pytest.raises(T.TncError):
        T.tnc_quant_sizes(7, n)


def test_search_is_deterministic_per_seed():
    c, st, net, nt = _net(2)
    open_q = list(range(20, 30))
    a = T.tnc_search(net, nt, open_q, 24, restarts=4, seed=5)
    b = T.tnc_search(net, nt, open_q, 24, restarts=4, seed=5)
    np.testing.assert_array_equal(a[0], b[0])
    np.testing.assert_array_equal(a[1], b[1])
    T.tnc_network_destroy(net)


def test_slice_path_meets_a_lower_cap():
    """Slicing a found path further (extra sliced labels) brings its largest
    per-slice tensor under a tighter cap, and keeps labels already sliced."""
    c, st, net, nt = _net(2)
    open_q = list(range(20, 30))
    ssa, sl, _ = T.tnc_search(net, nt, open_q, 24, restarts=4, seed=1)
    before = T.tnc_plan_analyze(net, ssa, sl, open_q, "c64")["max_rank"]
    more = T.tnc_slice_path(net, ssa, open_q, before - 2, sliced_in=list(sl))
    assert set(sl) <= set(more.tolist()) and len(more) > len(sl)
    assert T.tnc_plan_analyze(net, ssa, more, open_q, "c64")["max_rank"] <= before - 2
    T.tnc_network_destroy(net)


def test_stored_53_qubit_path_layouts_keep_permutes_low():
    """The planner reads two-run operand layouts in place and orders each result
    for its consumer (small operands and results' kept operands into the order
    the consumers sum in; one-bit reduced runs where a thin consumer could not
    read it otherwise): on the stored 53-qubit path at most 2e10 permute
    bytes per slice remain (a plain [batch][free][contracted] layout for every
    operand would move about 3.75e11)."""
    import json
    path = json.load(open(os.path.join(ROOT, "paper_2407_00769_amd", "paths", "config3.json")))
    c = workloads.config_circuit(3)
    st = workloads.tn_structure(c)
    r, l, d, o = cn.network_arrays(c, st)
    net = T.tnc_network_create(r, l, d, c.n_qubits, o)
    info = T.tnc_plan_analyze(net, np.array(path["ssa"], np.int32), np.array(path["sliced"], np.int32),
                              path["open_qubits"], "f16_4m")
    assert info["max_rank"] == 33
    assert info["permute_bytes_per_slice"] <= 2.0e10, info["permute_bytes_per_slice"]
    assert 2.3e14 < info["flops_per_slice"] < 2.6e14
    T.tnc_network_destroy(net)


def test_recompute_path_meets_the_cap_and_rejects_bad_labels():
    """Recomputation (Sec. 3.4.1): the chosen labels bring one pass under the
    cap, the prefix is shared (no more work than slicing them as well), and
    invalid labels are refused."""
    c, st, net, n = _net(0)
    open_q = list(range(6, 12))
    ssa, sl, _ = T.tnc_search(net, n, open_q, 9, restarts=2, seed=1)
    base = T.tnc_plan_analyze(net, ssa, sl, open_q, "c64")
    cap = base["max_rank"] - 1
    rec = T.tnc_recompute_path(net, ssa, sl, open_q, cap)
    assert len(rec) >= 1 and not set(rec) & set(sl)
    r = T.tnc_plan_analyze(net, ssa, sl, open_q, "c64", recompute=rec)
    s = T.tnc_plan_analyze(net, ssa, np.concatenate([sl, rec]), open_q, "c64")
    assert r["max_rank"] <= cap and r["n_recompute"] == len(rec)
    assert r["peak_bytes"] < base["peak_bytes"]
    assert r["flops_per_slice"] <= s["flops_per_slice"] * 2 ** len(rec) * (1 + 1e-12)
    for bad in ([st.output_labels[0]], [int(sl[0])] if len(sl) else [st.output_labels[1]], [int(rec[0]), int(rec[0])]):
        with pytest.raises(T.TncError):
            T.tnc_plan_analyze(net, ssa, sl, open_q, "c64", recompute=bad)


def test_costmodel_baseline_is_the_roofline_time():
    """The search's step cost is a roofline baseline plus the MLP's learned
    ratio; the baseline is 4 us plus the larger of flops at the dtype's
    matrix-core peak and bytes (A, B, C, and a read and a write of each
    permuted operand) at 8 TB/s."""
    rows = np.array([[10, 10, 10, 0, 0, 0, 1, 0],     # FP16, compute-bound
                     [10, 10, 10, 0, 1, 1, 0, 0],     # complex64, FP32 peak
                     [20, 2, 2, 4, 2, 0, 2, 0],       # BF16, HBM-bound, A permuted
                     [3, 3, 3, 0, 0, 2, 1, 1]],       # tiny: the launch latency
                    np.float32)
    fp16 = 4.0 + 1e6 * (8 * 2.0 ** 30 / 2516.6e12)
    c64 = 4.0 + 1e6 * (8 * 2.0 ** 30 / 157.3e12)
    a, b, c = 2.0 ** 26, 2.0 ** 10, 2.0 ** 26
    hbm = 4.0 + 1e6 * (4 * (a + b + c) + 2 * 4 * a) / 8e12
    tiny = 4.0 + 1e6 * max(8 * 2.0 ** 9 / 2516.6e12, (4 * 3 * 2.0 ** 6 + 2 * 4 * 2.0 ** 6) / 8e12)
    got = T.tnc_costmodel_base(rows)
    np.testing.assert_allclose(got, np.log2([fp16, c64, hbm, tiny]), rtol=0, atol=1e-5)
    with pytest.raises(T.TncError):
        T.lib and T._check(T.lib.tnc_costmodel_base(-1, None, None))


def test_sparse_work_is_smaller_on_a_path_searched_with_open_outputs():
    """For uncorrelated bitstrings the sparse-state plan shares the work done
    before the output legs join; a path searched with every output leg open
    brings them in late, so the plan needs a fraction of the work it needs on
    the path searched for the closed network (16 qubits: about a fifth)."""
    sites, cp = workloads.rect_grid(4, 4)
    c = workloads.random_circuit(sites, cp, 10, 3)
    st = workloads.tn_structure(c)
    r, l, d, o = cn.network_arrays(c, st)
    net = T.tnc_network_create(r, l, d, c.n_qubits, o)
    bits = workloads.uniform_bitstrings(16, 200, 7)

    def work(ssa, sl):
        a = T.tnc_plan_analyze_sparse(net, ssa, sl, bits, "f16_4m")
        return a["flops_per_slice"] * (1 << len(sl)) + a["flops_invariant"]

    ssa0, sl0, _ = T.tnc_search(net, len(r), [], 8, restarts=4, seed=1)
    ssa1, sl1, _ = T.tnc_search(net, len(r), list(range(16)), 16, restarts=4, seed=1)
    assert work(ssa1, sl1) < work(ssa0, sl0) / 3
    T.tnc_network_destroy(net)



def test_30_qubit_path_layouts_keep_permutes_low():
    """The 30-qubit block's path (5x6 grid, 14 cycles, 8 sliced labels, as the
    benchmark finds it): the planner's ordering rules, the thin-consumer one
    included, leave at most 8e7 permute bytes per slice (1.08e8 without the
    thin-consumer rule)."""
    c = workloads.config_circuit(2)
    st = workloads.tn_structure(c)
    r, l, d, o = cn.network_arrays(c, st)
    net = T.tnc_network_create(r, l, d, c.n_qubits, o)
    open_q = list(range(20, 30))
    for seed in range(1, 20):
        ssa, sl, _ = T.tnc_search(net, len(r), open_q, 22, restarts=64, seed=seed)
        if len(sl) == 8:
            break
    info = T.tnc_plan_analyze(net, ssa, sl, open_q, "f16_4m")
    assert info["permute_bytes_per_slice"] <= 8.0e7, info["permute_bytes_per_slice"]
    T.tnc_network_destroy(net)
