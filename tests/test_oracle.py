"""Pins of the CPU FP64 oracle against facts that do not come from the oracle.

Each test fixes a part of the oracle by mathematics or by the paper: gate
identities (the square of each sqrt-gate is the Pauli it is a root of, up to
phase), unitarity, brute-force Kronecker products, the norm of a state, the
path independence of a network's value, the sum over slices, the paper's
worked example, and Porter-Thomas statistics of ideal amplitudes.
"""
import json
import math
import os

import numpy as np
import pytest

import workloads
from oracle import bruteforce, einsum, gates, metrics, pairwise, statevector

GOLD = os.path.join(os.path.dirname(__file__), "golden")

X = np.array([[0, 1], [1, 0]], dtype=complex)
Y = np.array([[0, -1j], [1j, 0]], dtype=complex)
W = (X + Y) / math.sqrt(2)


def test_single_qubit_gates_square_to_paulis():
    # sqrtP @ sqrtP = -i P for P in {X, Y, W}: a pi/2 rotation squared is the
    # pi rotation about the same equatorial axis (paper Sec. 2.1)
    for m, p in ((gates.sqrt_x(), X), (gates.sqrt_y(), Y), (gates.sqrt_w(), W)):
        np.testing.assert_allclose(m @ m, -1j * p, atol=1e-15)


def test_gates_unitary():
    for m in (gates.sqrt_x(), gates.sqrt_y(), gates.sqrt_w(), gates.fsim(math.pi / 2, math.pi / 6),
              gates.fsim(0.3, 1.1)):
        np.testing.assert_allclose(m.conj().T @ m, np.eye(m.shape[0]), atol=1e-15)


def test_fsim_special_cases():
    f = gates.fsim(math.pi / 2, 0.0)
    e01 = np.array([0, 1, 0, 0], dtype=complex)
    np.testing.assert_array_equal(f @ e01, np.array([0, 0, -1j, 0]))      # |01> -> -i|10>
    np.testing.assert_array_equal(gates.fsim(0.0, 0.0), np.eye(4))
    sw = np.array([[1, 0, 0, 0], [0, 0, 1, 0], [0, 1, 0, 0], [0, 0, 0, 1]], dtype=complex)
    f = gates.fsim(math.pi / 2, math.pi / 6)
    np.testing.assert_array_equal(sw @ f @ sw, f)       # symmetric under qubit swap
    assert f[3, 3] == pytest.approx(complex(math.cos(math.pi / 6), -math.sin(math.pi / 6)))
    assert f[1, 1] == 0 and f[2, 2] == 0                 # cos(pi/2) snapped to an exact zero


def _tiny(rows, cols, cycles, seed):
    sites, cp = workloads.rect_grid(rows, cols)
    return workloads.random_circuit(sites, cp, cycles, seed)


@pytest.mark.parametrize("rows,cols,cycles,seed", [(1, 2, 3, 1), (2, 2, 4, 2), (2, 3, 5, 3), (3, 2, 6, 4)])
def test_statevector_matches_bruteforce_unitary(rows, cols, cycles, seed):
    c = _tiny(rows, cols, cycles, seed)
    u = bruteforce.unitary(c)
    n = c.n_qubits
    xs = np.arange(1 << n, dtype=np.uint64)
    amp = statevector.amplitudes(c, xs)
    ref = u[statevector.sv_index(xs, n), 0]
    np.testing.assert_allclose(amp, ref, atol=1e-12)


def test_statevector_norm_after_every_gate():
    c = _tiny(2, 3, 4, 9)
    for stop in range(len(c.gates) + 1):
        psi = statevector.simulate(c, stop=stop)
        assert abs(np.vdot(psi, psi).real - 1.0) < 1e-12


def test_bitstring_order_single_flip():
    # sqrtY on qubit 0 only: the |1> weight must appear on the bitstring with bit 0 set
    c = workloads.Circuit(3, [workloads.Gate("sqrtY", (0,))], [(0, 0), (0, 1), (0, 2)], 0, "A")
    amp = statevector.amplitudes(c, np.array([0, 1, 2, 4], dtype=np.uint64))
    r = 1 / math.sqrt(2)
    np.testing.assert_allclose(amp, [r, r, 0, 0], atol=1e-15)


def test_einsum_all_open_equals_statevector():
    c = workloads.config_circuit(0)
    st = workloads.tn_structure(c)
    ts = einsum.network_tensors(c, st)
    full = einsum.contract(ts, st.output_labels)   # axes = qubits 0..n-1
    psi = statevector.simulate(c)
    # tensor axis order is qubit 0 slowest, the same as the SV's big-endian index
    np.testing.assert_allclose(full.reshape(-1), psi, atol=1e-12)


def test_einsum_matches_brute_force_sum():
    c = _tiny(1, 2, 2, 5)
    st = workloads.tn_structure(c)
    ts = einsum.network_tensors(c, st)
    assert st.n_labels - c.n_qubits <= 14
    bf = einsum.brute_force(ts, st.output_labels)
    np.testing.assert_allclose(einsum.contract(ts, st.output_labels), bf, atol=1e-14)
    # a fixed internal label too
    lab = st.tensors[-1].labels[-1]
    for v in (0, 1):
        np.testing.assert_allclose(einsum.contract(ts, st.output_labels, {lab: v}),
                                   einsum.brute_force(ts, st.output_labels, {lab: v}), atol=1e-14)


def test_slices_sum_to_unsliced():
    c = _tiny(3, 3, 5, 11)
    st = workloads.tn_structure(c)
    ts = einsum.network_tensors(c, st)
    ref = einsum.contract(ts, st.output_labels)
    inner = [l for l in range(c.n_qubits, st.n_labels) if l not in st.output_labels]
    sliced = inner[5:9]
    acc = np.zeros_like(ref)
    for sigma in range(1 << len(sliced)):
        fix = {l: (sigma >> j) & 1 for j, l in enumerate(sliced)}
        acc += einsum.contract(ts, st.output_labels, fix)
    np.testing.assert_allclose(acc, ref, atol=1e-13)


def test_slice_equals_projected_statevector():
    c = _tiny(2, 3, 5, 12)
    st = workloads.tn_structure(c)
    ts = einsum.network_tensors(c, st)
    inner = [l for l in range(c.n_qubits, st.n_labels) if l not in st.output_labels]
    sliced = inner[3:6]
    xs = np.arange(1 << c.n_qubits, dtype=np.uint64)
    for sigma in (0, 5, 7):
        fix = {l: (sigma >> j) & 1 for j, l in enumerate(sliced)}
        tn = einsum.contract(ts, st.output_labels, fix).reshape(-1)
        wf = {st.label_wire[l]: v for l, v in fix.items()}
        sv = statevector.amplitudes(c, xs, wire_fix=wf)
        np.testing.assert_allclose(tn[statevector.sv_index(xs, c.n_qubits)], sv, atol=1e-13)


def test_worked_example_complex_half_padding():
    g = json.load(open(os.path.join(GOLD, "worked_example.json")))
    a = np.array([complex(*p) for p in g["A"]])
    b = np.array([complex(*p) for p in g["B"]])
    c = pairwise.contract_pair(a, "x", b, "y", "xy")
    want = np.array([[complex(*p)] for p in g["C"]])
    np.testing.assert_array_equal(c, want)
    # the padded real form: C_real[a1][c0] = sum_a2 A_real[a1][a2] * Bp[c0][a2]
    ar = np.array(g["A"], dtype=float)
    bp = np.array(g["B_padded"], dtype=float)
    np.testing.assert_array_equal(ar @ bp.T, np.array(g["C"], dtype=float))


def test_pairwise_entry_matches_einsum_with_batch():
    rng = np.random.default_rng(3)
    al, bl, cl = (0, 1, 2, 3, 4), (3, 2, 5, 6), (6, 0, 2, 1, 5)  # batch 2, reduce 3
    a = rng.normal(size=(2,) * 5) + 1j * rng.normal(size=(2,) * 5)
    b = rng.normal(size=(2,) * 4) + 1j * rng.normal(size=(2,) * 4)
    full = pairwise.contract_pair(a, al, b, bl, cl)
    for idx in [(0, 0, 0, 0, 0), (1, 0, 1, 1, 0), (1, 1, 1, 1, 1)]:
        e = pairwise.entry(lambda v: a[tuple(v[l] for l in al)], al,
                           lambda v: b[tuple(v[l] for l in bl)], bl, cl, idx)
        assert abs(e - full[idx]) < 1e-13


def test_metrics_basic():
    rng = np.random.default_rng(0)
    b = rng.normal(size=64) + 1j * rng.normal(size=64)
    assert metrics.fidelity(b, b) == pytest.approx(1.0, abs=1e-15)
    assert metrics.fidelity(b, 3.0 * np.exp(0.7j) * b) == pytest.approx(1.0, abs=1e-14)
    assert metrics.rel_l2(2 * b, b) == pytest.approx(1.0)
    o = np.zeros(64, complex)
    o[0] = 1
    p = np.zeros(64, complex)
    p[1] = 1
    assert metrics.fidelity(o, p) == 0.0


def test_porter_thomas_and_xeb_of_ideal_amplitudes():
    sites, cp = workloads.rect_grid(4, 4)
    c = workloads.random_circuit(sites, cp, 14, 21)
    psi = statevector.simulate(c)
    p = np.abs(psi) ** 2
    assert abs(p.sum() - 1) < 1e-12
    assert metrics.porter_thomas_ks(p, c.n_qubits) < 0.02
    assert abs(metrics.xeb_ideal(p, c.n_qubits) - 1.0) < 0.1
    # a product state is far from Porter-Thomas: catches a generator that entangles nothing
    c0 = workloads.Circuit(4, [workloads.Gate("sqrtX", (q,)) for q in range(4)], [(0, q) for q in range(4)], 0, "A")
    p0 = np.abs(statevector.simulate(c0)) ** 2
    assert metrics.porter_thomas_ks(p0, 4) > 0.2


def test_contract_path_equals_own_order_and_statevector():
    c = _tiny(2, 3, 5, 13)
    st = workloads.tn_structure(c)
    ts = einsum.network_tensors(c, st)
    ref = einsum.contract(ts, st.output_labels)
    rng = np.random.default_rng(0)
    for trial in range(4):
        # a random order of merges along shared labels
        labels = {i: set(t[0]) for i, t in enumerate(ts)}
        ssa = []
        nxt = len(ts)
        while len(labels) > 1:
            pairs = [(i, j) for i in labels for j in labels if i < j and labels[i] & labels[j]]
            if not pairs:
                pairs = [tuple(sorted(labels))[:2]]
            i, j = pairs[rng.integers(len(pairs))]
            labels[nxt] = labels.pop(i) ^ labels.pop(j)
            ssa += [i, j]
            nxt += 1
        got = einsum.contract_path(ts, st.output_labels, ssa)
        np.testing.assert_allclose(got, ref, atol=1e-12)
    psi = statevector.simulate(c)
    np.testing.assert_allclose(ref.reshape(-1), psi, atol=1e-12)


def test_contract_path_step_hook_is_linear():
    """The network's value is linear in every intermediate result, so scaling
    step s's result by lam scales the value by lam; the identity hook changes
    nothing, and the labels handed to the hook are the pair's kept labels."""
    c = _tiny(2, 3, 5, 17)
    st = workloads.tn_structure(c)
    ts = einsum.network_tensors(c, st)
    ref = einsum.contract(ts, st.output_labels)
    labels = {i: set(t[0]) for i, t in enumerate(ts)}
    ssa, nxt = [], len(ts)
    while len(labels) > 1:
        i, j = next((i, j) for i in sorted(labels) for j in sorted(labels) if i < j and labels[i] & labels[j])
        labels[nxt] = labels.pop(i) ^ labels.pop(j)
        ssa += [i, j]
        nxt += 1
    n_steps = len(ssa) // 2
    seen = []

    def ident(s, lab, d):
        assert d.shape == (2,) * len(lab)
        seen.append(s)
        return d

    np.testing.assert_array_equal(einsum.contract_path(ts, st.output_labels, ssa, after_step=ident),
                                  einsum.contract_path(ts, st.output_labels, ssa))
    assert seen == list(range(n_steps))
    for s in (0, n_steps // 2, n_steps - 1):
        lam = 0.5 - 1.25j
        got = einsum.contract_path(ts, st.output_labels, ssa,
                                   after_step=lambda t, lab, d, s=s: d * lam if t == s else d)
        np.testing.assert_allclose(got, lam * ref, atol=1e-12)
