"""Sparse-state contraction of uncorrelated bitstrings (paper Sec. 3.4.2)
through the C-ABI.

The bitstrings share no fixed bits, so no correlated subspace covers them;
the sparse-state plan keeps, for every tensor, one dense block per distinct
value of the bitstrings on the qubits whose output labels it holds, and forms
each result block from the matching operand blocks (a gathered multi-pair
GEMM).  Its amplitudes must match the state vector, and, for a set that does
form a correlated subspace, the dense plan's amplitudes.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import workloads  # noqa: E402
from oracle import metrics, statevector  # noqa: E402


@pytest.fixture(scope="module")
def T():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2407_00769_amd import _tnc
    return _tnc


@pytest.fixture(scope="module")
def ctx(T):
    ws = torch.empty(1 << 30, dtype=torch.uint8, device="cuda:0")
    c = T.tnc_create(0, ws, stream=torch.cuda.Stream())
    yield c
    T.tnc_destroy(c)
    torch.cuda.synchronize()
    del ws


@pytest.fixture(scope="module")
def case(T):
    from paper_2407_00769_amd import circuit_network as cn
    sites, cp = workloads.rect_grid(4, 4)
    c = workloads.random_circuit(sites, cp, 10, 3)
    st = workloads.tn_structure(c)
    r, l, d, o = cn.network_arrays(c, st)
    net = T.tnc_network_create(r, l, d, c.n_qubits, o)
    # a path for the network with every output label closed; the sparse plan
    # keeps them as blocks instead
    ssa, sl, _ = T.tnc_search(net, len(r), [], 8, restarts=4, seed=1)
    bits = workloads.uniform_bitstrings(16, 200, 7)
    bits = np.concatenate([bits, bits[:5]])   # duplicates are allowed
    ref = statevector.amplitudes(c, bits)
    yield dict(c=c, st=st, net=net, ssa=ssa, sl=sl, bits=bits, ref=ref)
    T.tnc_network_destroy(net)


@pytest.mark.parametrize("prec", ["c64", "f16_4m", "f16_3m", "bf16_4m"])
def test_sparse_state_matches_state_vector(T, ctx, case, prec):
    assert len(case["sl"]) >= 1
    plan = T.tnc_plan_create_sparse(ctx, case["net"], case["ssa"], case["sl"], case["bits"], prec)
    n = 1 << len(case["sl"])
    out, rep = T.tnc_execute(plan, case["bits"], 0, n)
    assert rep["slices"] == n
    f = metrics.fidelity(case["ref"], out)
    rl = metrics.rel_l2(out, case["ref"])
    rm = metrics.rel_max(out, case["ref"])
    print(prec, "fidelity", f, "rel_l2", rl, "rel_max", rm)
    if prec == "c64":
        assert f >= 1 - 1e-8 and rl <= 1e-5 and rm <= 1e-5, (f, rl, rm)
    elif prec.startswith("f16"):
        assert f >= 0.999 and rl <= 0.02 and rm <= 0.03, (f, rl, rm)
    else:
        assert f >= 0.99 and rl <= 0.1 and rm <= 0.15, (f, rl, rm)
    # duplicates get the same amplitude
    np.testing.assert_array_equal(out[-5:], out[:5])
    # ranges of slices add up
    a, _ = T.tnc_execute(plan, case["bits"], 0, n // 2)
    b, _ = T.tnc_execute(plan, case["bits"], n // 2, n)
    np.testing.assert_allclose(a + b, out, rtol=0, atol=1e-12 * np.max(np.abs(out)))
    # the plan takes only its own bitstrings
    with pytest.raises(T.TncError):
        T.tnc_execute(plan, case["bits"][:-1], 0, n)
    T.tnc_plan_destroy(plan)


@pytest.mark.parametrize("prec", ["c64", "f16_4m"])
def test_sparse_state_on_a_path_searched_with_open_outputs(T, ctx, case, prec):
    """The path the sparse study uses: searched with every output leg open,
    so the output legs enter late (here with two sliced labels); the sparse
    plan keeps those legs as blocks, and its amplitudes match the state
    vector."""
    r_len = len(case["ssa"]) // 2 + 1
    ssa, sl, _ = T.tnc_search(case["net"], r_len, list(range(16)), 16, restarts=4, seed=1)
    assert len(sl) >= 1
    plan = T.tnc_plan_create_sparse(ctx, case["net"], ssa, sl, case["bits"], prec)
    n = 1 << len(sl)
    out, _ = T.tnc_execute(plan, case["bits"], 0, n)
    f = metrics.fidelity(case["ref"], out)
    rl = metrics.rel_l2(out, case["ref"])
    rm = metrics.rel_max(out, case["ref"])
    print(prec, "fidelity", f, "rel_l2", rl, "rel_max", rm)
    if prec == "c64":
        assert f >= 1 - 1e-8 and rl <= 1e-5 and rm <= 1e-5, (f, rl, rm)
    else:
        assert f >= 0.999 and rl <= 0.02 and rm <= 0.03, (f, rl, rm)
    np.testing.assert_array_equal(out[-5:], out[:5])
    T.tnc_plan_destroy(plan)


def test_sparse_state_equals_dense_plan_on_a_subspace(T, ctx, case):
    """Bitstrings that do share a prefix: the sparse plan (which is not told so)
    and the dense correlated-subspace plan give the same amplitudes."""
    open_q = list(range(10, 16))
    bits = workloads.prefix_bitstrings(16, open_q, 64, 5)
    ssa, sl, _ = T.tnc_search(case["net"], len(case["ssa"]) // 2 + 1, open_q, 9, restarts=4, seed=2)
    dense = T.tnc_plan_create(ctx, case["net"], ssa, sl, open_q, "c64")
    sparse = T.tnc_plan_create_sparse(ctx, case["net"], ssa, sl, bits, "c64")
    n = 1 << len(sl)
    od, _ = T.tnc_execute(dense, bits, 0, n)
    osp, _ = T.tnc_execute(sparse, bits, 0, n)
    assert metrics.rel_l2(osp, od) <= 1e-6
    ref = statevector.amplitudes(case["c"], bits)
    assert metrics.fidelity(ref, osp) >= 1 - 1e-8
    T.tnc_plan_destroy(dense)
    T.tnc_plan_destroy(sparse)


@pytest.mark.parametrize("prec", ["c64", "f16_4m"])
def test_second_scheme_with_chunks_equals_first(T, ctx, case, prec, monkeypatch):
    """The padded two-dimensional index (B_P with -1 fill, C taken out of C_P),
    a few A blocks per chunk, against the in-GEMM gathered index."""
    n = 1 << len(case["sl"])
    outs = {}
    for scheme, chunk in (("1", None), ("2", "3")):
        monkeypatch.setenv("TNC_SPARSE_SCHEME", scheme)
        if chunk:
            monkeypatch.setenv("TNC_SPARSE_CHUNK", chunk)
        plan = T.tnc_plan_create_sparse(ctx, case["net"], case["ssa"], case["sl"], case["bits"], prec)
        padded = T.tnc_plan_info(plan)["n_padded_steps"]
        assert (padded > 0) == (scheme == "2"), padded
        outs[scheme], _ = T.tnc_execute(plan, case["bits"], 0, n)
        T.tnc_plan_destroy(plan)
    tol = 1e-6 if prec == "c64" else 2e-2
    assert metrics.rel_l2(outs["2"], outs["1"]) <= tol
    assert metrics.fidelity(case["ref"], outs["2"]) >= (1 - 1e-8 if prec == "c64" else 0.999)
