"""GPU parity of the HIP path against the CPU FP64 oracle (through the C-ABI).

* Single contractions (tnc_contract) against oracle.pairwise on the exact
  stored inputs, for every kernel variant and precision, with an elementwise
  error bound from FP32 accumulation plus one rounding of the output.
* The paper's worked complex-half example, exactly.
* Whole circuits (tnc_execute) against the state-vector oracle: complex64 to
  fidelity >= 1 - 1e-8, 16-bit forms to >= 0.99 (FP16 expected >= 0.999).
* Slicing: the sum over all slices equals the state vector; a partial block
  equals the sum of projected state vectors; disjoint ranges add up; two runs
  are bit-identical; the graph launch equals step-by-step launches.
"""
import itertools
import json
import os

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import workloads  # noqa: E402
from oracle import metrics, pairwise, statevector  # noqa: E402

from gpu_util import empty_storage, from_storage, to_storage  # noqa: E402
from rounding_model import check_against_model, model_amplitudes  # noqa: E402

GOLD = os.path.join(os.path.dirname(__file__), "golden")


@pytest.fixture(scope="module")
def T():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2407_00769_amd import _tnc
    return _tnc


@pytest.fixture(scope="module")
def ctx(T):
    ws = torch.empty(256 << 20, dtype=torch.uint8, device="cuda:0")
    st = torch.cuda.Stream()
    c = T.tnc_create(0, ws, stream=st)
    yield c
    T.tnc_destroy(c)
    torch.cuda.synchronize()
    del ws


PRECS = ["c64", "f16_4m", "f16_3m", "bf16_4m", "bf16_3m"]
U = {"c64": 2.0 ** -24, "f16_4m": 2.0 ** -11, "f16_3m": 2.0 ** -11, "bf16_4m": 2.0 ** -8, "bf16_3m": 2.0 ** -8}


@pytest.mark.parametrize("prec", ["c64", "f16_4m", "bf16_4m", "f16_3m"])
def test_worked_example(T, ctx, prec):
    g = json.load(open(os.path.join(GOLD, "worked_example.json")))
    a = np.array([complex(*p) for p in g["A"]])
    b = np.array([complex(*p) for p in g["B"]]).reshape(())
    A, _ = to_storage(a, prec)
    B, _ = to_storage(b.reshape(1), prec)
    C = empty_storage((2,), prec)
    T.tnc_contract(ctx, prec, A, [7], B, [], C, [7], scale_log2=0)
    got = from_storage(C, prec)
    want = np.array([complex(*p) for p in g["C"]])
    np.testing.assert_array_equal(got, want)


def _random_case(rng, nb, m, n, k):
    labels = list(range(nb + m + n + k))
    rng.shuffle(labels)
    beta, ml, nl, kl = labels[:nb], labels[nb:nb + m], labels[nb + m:nb + m + n], labels[nb + m + n:]
    al = beta + ml + kl
    bl = beta + nl + kl
    cl = beta + ml + nl
    for v in (al, bl, cl):
        rng.shuffle(v)
    a = (rng.normal(size=2 ** len(al)) + 1j * rng.normal(size=2 ** len(al))) / np.sqrt(2 * 2 ** k)
    b = (rng.normal(size=2 ** len(bl)) + 1j * rng.normal(size=2 ** len(bl))) / np.sqrt(2)
    return al, bl, cl, a, b


def _check_contract(T, ctx, prec, nb, m, n, k, seed, scale_log2=0):
    rng = np.random.default_rng(seed)
    al, bl, cl, a, b = _random_case(rng, nb, m, n, k)
    A, av = to_storage(a, prec)
    B, bv = to_storage(b, prec)
    C = empty_storage((2 ** len(cl),), prec)
    T.tnc_contract(ctx, prec, A, al, B, bl, C, cl, scale_log2=scale_log2)
    got = from_storage(C, prec, scale_log2).reshape((2,) * len(cl))
    ref = pairwise.contract_pair(av.reshape((2,) * len(al)), al, bv.reshape((2,) * len(bl)), bl, cl)
    mag = pairwise.contract_pair(np.abs(av).reshape((2,) * len(al)), al, np.abs(bv).reshape((2,) * len(bl)), bl, cl)
    K = 2 ** k
    u = U[prec]
    # FP32 accumulation over 2K real terms, plus one rounding of the stored result;
    # 3M adds the rounding of the operand sums and cancellation (Higham's bound)
    acc_u = 2.0 ** -24
    bound = 4 * K * acc_u * np.abs(mag) + u * np.abs(ref) * 1.01 + 1e-30
    if prec.endswith("3m"):
        bound = bound + 6 * u * np.abs(mag)
    err = np.abs(got - ref)
    assert np.all(err <= bound), (prec, float(np.max(err / bound)))
    return got, ref


KERNELS = {"naive": 0, "skinny": 1, "mfma_s": 2, "mfma_m": 3, "mfma_l": 4, "mfma_w": 5, "mfma_xl": 6,
           "mfma_l2": 7, "dma_4": 8, "dma_8": 9, "dma_8w": 10, "dma_2": 11, "dma_n64": 12, "dma_n32": 13,
           "dma3_n64": 14, "dma3_2": 15, "dmap_2": 16, "dmap_n64": 18,
           "thinm": 17}
SHAPES = [  # nb, m, n, k  (log2)
    (0, 9, 6, 5), (1, 8, 5, 3), (0, 10, 4, 6), (2, 7, 7, 4), (0, 8, 0, 2), (0, 6, 3, 0), (0, 12, 5, 7),
    (0, 9, 8, 6), (1, 8, 7, 5),
    (0, 9, 8, 9),   # few tiles, long k: split-K partial sums
    (1, 8, 7, 6),   # one 256 x 128 tile per batch entry
]


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("kname", list(KERNELS))
def test_contract_kernels(T, ctx, prec, kname, monkeypatch):
    monkeypatch.setenv("TNC_FORCE_KERNEL", str(KERNELS[kname]))
    for i, (nb, m, n, k) in enumerate(SHAPES):
        _check_contract(T, ctx, prec, nb, m, n, k, seed=100 + i)


# shapes with more tiles than the persistent kernel has blocks (256 CUs): each
# block walks two tiles and the ring runs on across their ends; k from one
# 32-wide stage per tile to sixteen, and one batched case (the oracle's einsum
# is slow on batch labels, so that one stays small)
PERSISTENT_SHAPES = {
    "dmap_2": [(0, 14, 9, 5), (0, 13, 10, 6), (0, 15, 8, 7), (0, 12, 9, 9), (2, 11, 8, 5)],
    # 256 x 64 tiles, two blocks per CU: one, two and four tiles per block
    "dmap_n64": [(0, 16, 7, 6), (0, 17, 7, 6), (0, 16, 8, 5), (0, 12, 8, 9), (1, 15, 7, 6)],
}


@pytest.mark.parametrize("prec", ["f16_4m", "bf16_4m"])
@pytest.mark.parametrize("kname", ["dmap_2", "dmap_n64"])
def test_persistent_tile_loop(T, ctx, prec, kname, monkeypatch):
    monkeypatch.setenv("TNC_FORCE_KERNEL", str(KERNELS[kname]))
    for i, (nb, m, n, k) in enumerate(PERSISTENT_SHAPES[kname]):
        _check_contract(T, ctx, prec, nb, m, n, k, seed=300 + i)


# thin steps on the matrix cores: N = 4, 8 or 16 complex columns, K = 8..64,
# one to four 64-row passes per wave and batches of up to four
THIN_SHAPES = [(0, 12, 3, 3), (1, 11, 3, 4), (0, 13, 4, 4), (2, 10, 4, 6), (0, 6, 3, 3), (0, 10, 4, 5),
               (0, 12, 2, 3), (1, 10, 2, 4), (0, 12, 5, 3), (1, 10, 5, 4), (0, 6, 5, 3),
               (0, 12, 3, 1), (0, 12, 2, 2), (1, 10, 4, 1), (0, 11, 5, 2)]   # K = 2, 4: one partial chunk


@pytest.mark.parametrize("prec", ["f16_4m", "bf16_4m"])
def test_thin_matrix_core_kernel(T, ctx, prec, monkeypatch):
    monkeypatch.setenv("TNC_FORCE_KERNEL", str(KERNELS["thinm"]))
    for i, (nb, m, n, k) in enumerate(THIN_SHAPES):
        _check_contract(T, ctx, prec, nb, m, n, k, seed=400 + i)
    # read and written in place: A as [m][k] or [k][m] (the latter through
    # LDS), B as [n][k] or [k][n], C as [m][n] or [n][m]; N = 4, 8, 16, 32;
    # K = 2, 4, 8, 16
    rng = np.random.default_rng(14)
    for n, k, a_kc, b_kc, c_nc in itertools.product((2, 3, 4, 5), (1, 2, 3, 4), (1, 0), (1, 0), (1, 0)):
        al, bl, cl, a, b = _oriented_case(rng, 9, n, k, a_kc, b_kc, c_nc)
        A, av = to_storage(a, prec)
        B, bv = to_storage(b, prec)
        C = empty_storage((2 ** len(cl),), prec)
        times, _ = T.tnc_contract(ctx, prec, A, al, B, bl, C, cl)
        assert times[0] < 0.05 and times[1] < 0.05 and times[3] < 0.05   # no permute ran (ms)
        got = from_storage(C, prec).reshape((2,) * len(cl))
        ref = pairwise.contract_pair(av.reshape((2,) * len(al)), al, bv.reshape((2,) * len(bl)), bl, cl)
        mag = pairwise.contract_pair(np.abs(av).reshape((2,) * len(al)), al,
                                     np.abs(bv).reshape((2,) * len(bl)), bl, cl)
        bound = 4 * 2 ** k * 2.0 ** -24 * np.abs(mag) + U[prec] * np.abs(ref) * 1.01 + 1e-30
        err = np.abs(got - ref)
        assert np.all(err <= bound), (prec, n, k, a_kc, b_kc, c_nc, float(np.max(err / bound)))


@pytest.mark.parametrize("kname", ["dma_2", "dma_8w", "dmap_2"])
def test_large_result(T, ctx, kname, monkeypatch):
    """A 2^14 x 2^12 result (2^26 FP16 complex entries, 256 MB, more than the
    caches hold) through the one-tile and persistent kernels against the
    oracle."""
    monkeypatch.setenv("TNC_FORCE_KERNEL", str(KERNELS[kname]))
    ws = torch.empty(2 << 30, dtype=torch.uint8, device="cuda:0")   # room for permuted copies
    big = T.tnc_create(0, ws, stream=torch.cuda.Stream())
    _check_contract(T, big, "f16_4m", 0, 14, 12, 5, seed=520)
    T.tnc_destroy(big)
    torch.cuda.synchronize()
    del ws


def _oriented_case(rng, m, n, k, a_kc, b_kc, c_nc):
    ml = list(range(0, m))
    nl = list(range(m, m + n))
    kl = list(range(m + n, m + n + k))
    rng.shuffle(kl)
    al = ml + kl if a_kc else kl + ml
    bl = nl + kl if b_kc else kl + nl
    cl = ml + nl if c_nc else nl + ml
    a = (rng.normal(size=2 ** len(al)) + 1j * rng.normal(size=2 ** len(al))) / np.sqrt(2 * 2 ** k)
    b = (rng.normal(size=2 ** len(bl)) + 1j * rng.normal(size=2 ** len(bl))) / np.sqrt(2)
    return al, bl, cl, a, b


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("kname", ["skinny", "mfma_s", "mfma_l", "mfma_xl", "mfma_l2", "mfma_w", "dma_4"])
def test_contract_orientations(T, ctx, prec, kname, monkeypatch):
    # every combination of A [m][k] / [k][m], B [n][k] / [k][n], C [m][n] / [n][m]
    # runs without a permute and matches the oracle
    monkeypatch.setenv("TNC_FORCE_KERNEL", str(KERNELS[kname]))
    rng = np.random.default_rng(11)
    for a_kc in (1, 0):
        for b_kc in (1, 0):
            for c_nc in (1, 0):
                al, bl, cl, a, b = _oriented_case(rng, 9, 8, 5, a_kc, b_kc, c_nc)
                A, av = to_storage(a, prec)
                B, bv = to_storage(b, prec)
                C = empty_storage((2 ** len(cl),), prec)
                times, _ = T.tnc_contract(ctx, prec, A, al, B, bl, C, cl)
                assert times[0] < 0.05 and times[1] < 0.05 and times[3] < 0.05   # no permute ran (ms)
                got = from_storage(C, prec).reshape((2,) * len(cl))
                ref = pairwise.contract_pair(av.reshape((2,) * len(al)), al, bv.reshape((2,) * len(bl)), bl, cl)
                mag = pairwise.contract_pair(np.abs(av).reshape((2,) * len(al)), al,
                                             np.abs(bv).reshape((2,) * len(bl)), bl, cl)
                bound = 4 * 32 * 2.0 ** -24 * np.abs(mag) + U[prec] * np.abs(ref) * 1.01 + 1e-30
                if prec.endswith("3m"):
                    bound = bound + 6 * U[prec] * np.abs(mag)
                err = np.abs(got - ref)
                assert np.all(err <= bound), (prec, kname, a_kc, b_kc, c_nc, float(np.max(err / bound)))


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("kname", ["skinny", "mfma_m", "mfma_xl", "mfma_l2", "dma_4", "dma_8", "dma_8w", "dma_2", "dma_n64", "dma_n32",
                                   "dma3_n64", "dma3_2"])
def test_contract_split_layouts(T, ctx, prec, kname, monkeypatch):
    # operands and result whose GEMM indices lie in two runs each (A as
    # [m_hi][k_hi][m_lo][k_lo], B as [k_hi][n][k_lo], C as [m_hi][n_hi][m_lo][n_lo])
    # are used in place, with no permute, and match the oracle
    monkeypatch.setenv("TNC_FORCE_KERNEL", str(KERNELS[kname]))
    rng = np.random.default_rng(12)
    m, n, k = 9, 8, 6
    ml = list(range(0, m))
    nl = list(range(m, m + n))
    kl = list(range(m + n, m + n + k))
    al = ml[:4] + kl[:3] + ml[4:] + kl[3:]
    bl = kl[:3] + nl + kl[3:]
    cl = ml[:5] + nl[:3] + ml[5:] + nl[3:]
    a = (rng.normal(size=2 ** len(al)) + 1j * rng.normal(size=2 ** len(al))) / np.sqrt(2 * 2 ** k)
    b = (rng.normal(size=2 ** len(bl)) + 1j * rng.normal(size=2 ** len(bl))) / np.sqrt(2)
    A, av = to_storage(a, prec)
    B, bv = to_storage(b, prec)
    C = empty_storage((2 ** len(cl),), prec)
    times, _ = T.tnc_contract(ctx, prec, A, al, B, bl, C, cl)
    assert times[0] < 0.05 and times[1] < 0.05 and times[3] < 0.05   # no permute ran (ms)
    got = from_storage(C, prec).reshape((2,) * len(cl))
    ref = pairwise.contract_pair(av.reshape((2,) * len(al)), al, bv.reshape((2,) * len(bl)), bl, cl)
    mag = pairwise.contract_pair(np.abs(av).reshape((2,) * len(al)), al, np.abs(bv).reshape((2,) * len(bl)), bl, cl)
    bound = 4 * 64 * 2.0 ** -24 * np.abs(mag) + U[prec] * np.abs(ref) * 1.01 + 1e-30
    if prec.endswith("3m"):
        bound = bound + 6 * U[prec] * np.abs(mag)
    err = np.abs(got - ref)
    assert np.all(err <= bound), (prec, kname, float(np.max(err / bound)))


@pytest.mark.parametrize("prec", ["f16_4m", "bf16_4m", "f16_3m"])
def test_power_of_two_scale_is_exact(T, ctx, prec):
    # storing C * 2^-s is exact while the stored value stays a normal number:
    # those entries agree bit for bit after undoing s (subnormals lose bits)
    g0, _ = _check_contract(T, ctx, prec, 0, 9, 5, 5, seed=7, scale_log2=0)
    g1, _ = _check_contract(T, ctx, prec, 0, 9, 5, 5, seed=7, scale_log2=3)
    g2, _ = _check_contract(T, ctx, prec, 0, 9, 5, 5, seed=7, scale_log2=-4)
    def normal(g, shift):
        tiny = 2.0 ** (-14 + shift) if prec.startswith("f16") else 1e-30
        ok = (np.abs(g.real) >= tiny) | (g.real == 0)
        return ok & ((np.abs(g.imag) >= tiny) | (g.imag == 0))
    n1, n0 = normal(g0, 3), normal(g0, 0)
    assert n1.mean() > 0.99
    np.testing.assert_array_equal(g0[n1], g1[n1])
    np.testing.assert_array_equal(g0[n0], g2[n0])


def _circuit_plan(T, ctx, cfg, prec, cap, open_q, cycles=None, seed=0, restarts=4, rect=None):
    if rect:
        sites, cp = workloads.rect_grid(*rect)
        c = workloads.random_circuit(sites, cp, cycles, seed)
    else:
        c = workloads.config_circuit(cfg, cycles=cycles)
    from paper_2407_00769_amd import circuit_network as cn
    st = workloads.tn_structure(c)
    r, l, d, o = cn.network_arrays(c, st)
    net = T.tnc_network_create(r, l, d, c.n_qubits, o)
    ssa, sl, _ = T.tnc_search(net, len(r), open_q, cap, restarts=restarts, seed=seed)
    return c, st, net, ssa, sl


@pytest.mark.parametrize("prec", PRECS)
def test_config0_matches_statevector(T, ctx, prec):
    c, st, net, ssa, sl = _circuit_plan(T, ctx, 0, prec, 30, list(range(12)))
    bits = workloads.uniform_bitstrings(12, 64, 1)
    ref = statevector.amplitudes(c, bits)
    plan = T.tnc_plan_create(ctx, net, ssa, sl, list(range(12)), prec)
    out, rep = T.tnc_execute(plan, bits, 0, 1)
    f = metrics.fidelity(ref, out)
    rl = metrics.rel_l2(out, ref)
    if prec == "c64":
        assert f >= 1 - 1e-8 and rl <= 1e-4, (f, rl)
        assert metrics.rel_max(out, ref) <= 1e-4
    else:
        assert f >= (0.999 if prec.startswith("f16") else 0.99), (f, rl)
        # per amplitude: within the rounding model's errors (stated factors)
        model = model_amplitudes(c, st, ssa, sl, list(range(12)), bits, prec)
        ok, stats = check_against_model(out, ref, model)
        print(prec, stats)
        assert ok, stats
    T.tnc_plan_destroy(plan)
    T.tnc_network_destroy(net)


@pytest.mark.parametrize("prec", ["c64", "f16_4m", "f16_3m"])
def test_sliced_sum_matches_statevector(T, ctx, prec):
    open_q = list(range(10, 16))
    c, st, net, ssa, sl = _circuit_plan(T, ctx, None, prec, 10, open_q, cycles=10, seed=3, rect=(4, 4))
    assert len(sl) >= 3
    bits = workloads.prefix_bitstrings(16, open_q, 200, 9)
    ref = statevector.amplitudes(c, bits)
    plan = T.tnc_plan_create(ctx, net, ssa, sl, open_q, prec)
    n = 1 << len(sl)
    out, rep = T.tnc_execute(plan, bits, 0, n)
    assert rep["slices"] == n
    f = metrics.fidelity(ref, out)
    assert f >= (1 - 1e-8 if prec == "c64" else 0.999), f
    if prec != "c64":
        model = model_amplitudes(c, st, ssa, sl, open_q, bits, prec)
        ok, stats = check_against_model(out, ref, model)
        print(prec, stats)
        assert ok, stats
    # a partial block equals the sum of projected state vectors of its slices
    lo, hi = 1, min(n, 6)
    part, _ = T.tnc_execute(plan, bits, lo, hi)
    acc = np.zeros(len(bits), complex)
    for sigma in range(lo, hi):
        wf = {st.label_wire[l]: (sigma >> j) & 1 for j, l in enumerate(sl)}
        acc += statevector.amplitudes(c, bits, wire_fix=wf)
    assert metrics.fidelity(acc, part) >= (1 - 1e-8 if prec == "c64" else 0.999)
    assert metrics.rel_l2(part, acc) <= (1e-4 if prec == "c64" else 0.05)
    # disjoint ranges add up to the whole
    a, _ = T.tnc_execute(plan, bits, 0, n // 2)
    b, _ = T.tnc_execute(plan, bits, n // 2, n)
    np.testing.assert_allclose(a + b, out, rtol=0, atol=1e-12 * np.max(np.abs(out)))
    # determinism
    again, _ = T.tnc_execute(plan, bits, 0, n)
    np.testing.assert_array_equal(again, out)
    T.tnc_plan_destroy(plan)
    T.tnc_network_destroy(net)


def test_graph_equals_stepwise(T, ctx, monkeypatch):
    open_q = list(range(10, 16))
    c, st, net, ssa, sl = _circuit_plan(T, ctx, None, "f16_4m", 10, open_q, cycles=8, seed=4, rect=(4, 4))
    bits = workloads.prefix_bitstrings(16, open_q, 64, 2)
    p1 = T.tnc_plan_create(ctx, net, ssa, sl, open_q, "f16_4m")
    monkeypatch.setenv("TNC_NO_GRAPH", "1")
    p2 = T.tnc_plan_create(ctx, net, ssa, sl, open_q, "f16_4m")
    n = 1 << len(sl)
    o1, r1 = T.tnc_execute(p1, bits, 0, n)
    o2, r2 = T.tnc_execute(p2, bits, 0, n)
    assert r1["graph_launches"] >= 1 and r2["graph_launches"] == 0
    np.testing.assert_array_equal(o1, o2)
    # one slice in flight gives the same bits as many (each slice's arithmetic is independent)
    p3 = T.tnc_plan_create(ctx, net, ssa, sl, open_q, "f16_4m", max_slices_in_flight=1)
    o3, _ = T.tnc_execute(p3, bits, 0, n)
    np.testing.assert_array_equal(o1, o3)
    for p in (p1, p2, p3):
        T.tnc_plan_destroy(p)
    T.tnc_network_destroy(net)


def test_execute_rejects_bad_calls(T, ctx):
    open_q = list(range(10, 16))
    c, st, net, ssa, sl = _circuit_plan(T, ctx, None, "c64", 10, open_q, cycles=6, seed=5, rect=(4, 4))
    plan = T.tnc_plan_create(ctx, net, ssa, sl, open_q, "c64")
    bits = workloads.prefix_bitstrings(16, open_q, 8, 2)
    with pytest.raises(T.TncError):
        T.tnc_execute(plan, bits, 0, (1 << len(sl)) + 1)
    bad = bits.copy()
    bad[0] ^= np.uint64(1)   # qubit 0 is closed: the request disagrees on it
    with pytest.raises(T.TncError):
        T.tnc_execute(plan, bad, 0, 1)
    # empty range: zeros
    z, _ = T.tnc_execute(plan, bits, 1, 1)
    assert np.all(z == 0)
    T.tnc_plan_destroy(plan)
    # a workspace too small for one slice
    tiny = torch.empty(4096, dtype=torch.uint8, device="cuda:0")
    c2 = T.tnc_create(0, tiny, stream=torch.cuda.Stream())
    with pytest.raises(T.TncError) as e:
        T.tnc_plan_create(c2, net, ssa, sl, open_q, "c64")
    assert e.value.code == -2
    T.tnc_destroy(c2)
    T.tnc_network_destroy(net)


@pytest.mark.parametrize("kname", ["dmap_2"])
def test_config2_block_with_persistent_tiles(T, ctx, kname, monkeypatch):
    """The 30-qubit block with the persistent tile loop forced on every step
    it supports: 256 slices in one launch (the tiles of all slices walked by
    one grid), ragged slice groups, against the stored oracle amplitudes with
    the FP16 bounds of the full-block test."""
    ref = np.load(os.path.join(GOLD, "config2_amplitudes.npy"))
    from paper_2407_00769_amd import circuit_network as cn
    c = workloads.config_circuit(2)
    st = workloads.tn_structure(c)
    r, l, d, o = cn.network_arrays(c, st)
    net = T.tnc_network_create(r, l, d, c.n_qubits, o)
    open_q = list(range(20, 30))
    for seed in range(1, 20):
        ssa, sl, _ = T.tnc_search(net, len(r), open_q, 22, restarts=64, seed=seed)
        if len(sl) == 8:
            break
    bits = workloads.prefix_bitstrings(30, open_q, 1024, 3)
    ws = torch.empty(16 << 30, dtype=torch.uint8, device="cuda:0")
    big = T.tnc_create(0, ws, stream=torch.cuda.Stream())
    monkeypatch.setenv("TNC_FORCE_KERNEL", str(KERNELS[kname]))
    plan = T.tnc_plan_create(big, net, ssa, sl, open_q, "f16_4m")
    info = T.tnc_plan_info(plan)
    steps = T.tnc_plan_steps(plan, info["n_steps"])
    n_forced = int(np.sum(steps["kernel"] == KERNELS[kname]))
    assert n_forced >= 1, n_forced
    out, _ = T.tnc_execute(plan, bits, 0, 256)
    f, rl, rm = metrics.fidelity(ref, out), metrics.rel_l2(out, ref), metrics.rel_max(out, ref)
    print(kname, n_forced, "steps; fidelity", f, "rel_l2", rl, "rel_max", rm)
    assert f >= 0.999 and rl <= 0.03 and rm <= 0.06, (f, rl, rm)
    parts = [T.tnc_execute(plan, bits, a, b)[0] for a, b in ((0, 3), (3, 5), (5, 256))]
    np.testing.assert_allclose(sum(parts), out, rtol=0, atol=1e-12 * np.max(np.abs(out)))
    T.tnc_plan_destroy(plan)
    T.tnc_destroy(big)
    T.tnc_network_destroy(net)
    del ws
    torch.cuda.empty_cache()


@pytest.mark.parametrize("prec", ["c64", "f16_4m", "f16_3m", "bf16_4m"])
def test_config2_full_block_matches_oracle(T, ctx, prec):
    """The benchmark's own workload at full size (30 qubits, 256-slice block in
    one launch, 1024 bitstrings) against the stored oracle amplitudes."""
    gold = os.path.join(GOLD, "config2_amplitudes.npy")
    ref = np.load(gold)
    from paper_2407_00769_amd import circuit_network as cn
    c = workloads.config_circuit(2)
    st = workloads.tn_structure(c)
    r, l, d, o = cn.network_arrays(c, st)
    net = T.tnc_network_create(r, l, d, c.n_qubits, o)
    open_q = list(range(20, 30))
    for seed in range(1, 20):
        ssa, sl, _ = T.tnc_search(net, len(r), open_q, 22, restarts=64, seed=seed)
        if len(sl) == 8:
            break
    assert len(sl) == 8
    bits = workloads.prefix_bitstrings(30, open_q, 1024, 3)
    ws = torch.empty(16 << 30, dtype=torch.uint8, device="cuda:0")
    big = T.tnc_create(0, ws, stream=torch.cuda.Stream())
    plan = T.tnc_plan_create(big, net, ssa, sl, open_q, prec)
    out, rep = T.tnc_execute(plan, bits, 0, 256)
    assert rep["graph_launches"] == 1 and rep["slices"] == 256
    f = metrics.fidelity(ref, out)
    rl = metrics.rel_l2(out, ref)
    rm = metrics.rel_max(out, ref)
    print(prec, "fidelity", f, "rel_l2", rl, "rel_max", rm)
    # 16-bit bounds: the rounding model's errors on slice 0 of this path (see
    # test_config2_slice0_within_rounding_model) scaled by the square root of
    # the 256 slices' independent rounding, times the margin of that test
    if prec == "c64":
        assert f >= 1 - 1e-8 and rl <= 1e-4 and rm <= 1e-4, (f, rl, rm)
    elif prec.startswith("f16"):
        assert f >= 0.999 and rl <= 0.03 and rm <= 0.06, (f, rl, rm)
    else:
        assert f >= 0.99 and rl <= 0.2 and rm <= 0.4, (f, rl, rm)
    # partial blocks: a group of fewer slices than the plan holds in flight
    # keeps the split-K factor its partial-sum buffer was sized for
    parts = [T.tnc_execute(plan, bits, a, b)[0] for a, b in ((0, 16), (16, 20), (20, 21), (21, 256))]
    np.testing.assert_allclose(sum(parts), out, rtol=0, atol=1e-12 * np.max(np.abs(out)))
    T.tnc_plan_destroy(plan)
    T.tnc_destroy(big)
    T.tnc_network_destroy(net)
    del ws
    torch.cuda.empty_cache()


def test_tuning_with_thousands_of_slices_in_flight(T, ctx):
    """Plan-time tuning launches cover every slice in flight; their per-slice
    scale bookkeeping must stay inside the library's own buffers.  Device state
    allocated beside them (the cost model's parameters here) is unchanged, and
    the plan's amplitudes match the state vector."""
    from oracle import mlp as omlp
    canary = omlp.init(11).astype(np.float32)
    T.tnc_mlp_set_params(ctx, canary)
    open_q = list(range(16, 20))
    c, st, net, ssa, sl = _circuit_plan(T, ctx, None, "f16_4m", 8, open_q, cycles=12, seed=21, restarts=2,
                                        rect=(4, 5))
    assert len(sl) >= 12, len(sl)
    plan = T.tnc_plan_create(ctx, net, ssa, sl, open_q, "f16_4m")
    assert T.tnc_plan_info(plan)["slices_in_flight"] >= 1024
    np.testing.assert_array_equal(T.tnc_mlp_get_params(ctx), canary)
    bits = workloads.prefix_bitstrings(20, open_q, 16, 4)
    out, rep = T.tnc_execute(plan, bits, 0, 1 << len(sl))
    ref = statevector.amplitudes(c, bits)
    assert metrics.fidelity(ref, out) >= 0.999
    np.testing.assert_array_equal(T.tnc_mlp_get_params(ctx), canary)
    T.tnc_plan_destroy(plan)
    T.tnc_network_destroy(net)


@pytest.fixture(scope="module")
def config2_slice0(T):
    """Slice 0 of the 30-qubit benchmark path: its exact FP64 value and the
    rounding model's FP16 and BF16 values (oracle contraction along the path)."""
    from oracle import einsum
    from paper_2407_00769_amd import circuit_network as cn
    c = workloads.config_circuit(2)
    st = workloads.tn_structure(c)
    r, l, d, o = cn.network_arrays(c, st)
    net = T.tnc_network_create(r, l, d, c.n_qubits, o)
    open_q = list(range(20, 30))
    for seed in range(1, 20):
        ssa, sl, _ = T.tnc_search(net, len(r), open_q, 22, restarts=64, seed=seed)
        if len(sl) == 8:
            break
    bits = workloads.prefix_bitstrings(30, open_q, 1024, 3)
    ts = einsum.network_tensors(c, st)
    closed = {st.output_labels[q]: int((int(bits[0]) >> q) & 1) for q in range(30) if q not in open_q}
    fixed = dict(closed)
    fixed.update({int(lab): 0 for lab in sl})
    exact = einsum.contract_path(ts, list(st.output_labels), ssa, fixed)
    idx = tuple(((bits >> np.uint64(q)) & np.uint64(1)).astype(np.int64) for q in open_q)
    models = {p: model_amplitudes(c, st, ssa, sl, open_q, bits, p, slices=[0]) for p in ("f16_4m", "bf16_4m")}
    yield dict(net=net, ssa=ssa, sl=sl, open_q=open_q, bits=bits, exact=exact[idx], models=models)
    T.tnc_network_destroy(net)


@pytest.mark.parametrize("prec", ["f16_4m", "f16_3m", "bf16_4m"])
def test_config2_slice0_within_rounding_model(T, config2_slice0, prec):
    """Per-amplitude parity of one slice of the 30-qubit path against the exact
    FP64 value, within the rounding model's errors."""
    w = config2_slice0
    ws = torch.empty(4 << 30, dtype=torch.uint8, device="cuda:0")
    ctx = T.tnc_create(0, ws, stream=torch.cuda.Stream())
    plan = T.tnc_plan_create(ctx, w["net"], w["ssa"], w["sl"], w["open_q"], prec)
    out, _ = T.tnc_execute(plan, w["bits"], 0, 1)
    model = w["models"]["f16_4m" if prec.startswith("f16") else "bf16_4m"]
    ok, stats = check_against_model(out, w["exact"], model)
    print(prec, stats)
    assert ok, stats
    T.tnc_plan_destroy(plan)
    T.tnc_destroy(ctx)
    del ws
