"""The scale epilogue's overflow path (16-bit forms) through the C-ABI.

Every 16-bit step stores C * 2^-t with t chosen from its operands' stored
maxima and a growth estimate g; a stored maximum above half the FP16 range (or
a non-finite value) flags the step, and the block is replayed with the flagged
steps' g raised by 4, at most 3 times.  Here g is forced low from the host:
  * a few bits low: the block is replayed, the amplitudes still match the
    state vector, and the estimates settle back where the plan had them;
  * far too low: three replays cannot recover, and the call fails with
    TNC_EOVERFLOW; the plan then runs again once g is restored.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import workloads  # noqa: E402
from oracle import metrics, statevector  # noqa: E402

OPEN = list(range(10, 16))


@pytest.fixture(scope="module")
def T():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2407_00769_amd import _tnc
    return _tnc


@pytest.fixture(scope="module")
def ctx(T):
    ws = torch.empty(256 << 20, dtype=torch.uint8, device="cuda:0")
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
    ssa, sl, _ = T.tnc_search(net, len(r), OPEN, 10, restarts=4, seed=3)
    bits = workloads.prefix_bitstrings(16, OPEN, 64, 9)
    ref = statevector.amplitudes(c, bits)
    yield dict(net=net, ssa=ssa, sl=sl, bits=bits, ref=ref)
    T.tnc_network_destroy(net)


@pytest.mark.parametrize("prec", ["f16_4m", "f16_3m"])
def test_low_growth_is_replayed_and_parity_kept(T, ctx, case, prec):
    plan = T.tnc_plan_create(ctx, case["net"], case["ssa"], case["sl"], OPEN, prec)
    n = 1 << len(case["sl"])
    out0, rep0 = T.tnc_execute(plan, case["bits"], 0, n)
    assert rep0["replays"] == 0
    g_adapted = T.tnc_plan_get_growth(plan)
    # a second call with the adapted estimates gives the same amplitudes
    out1, rep1 = T.tnc_execute(plan, case["bits"], 0, n)
    assert rep1["replays"] == 0
    assert metrics.fidelity(case["ref"], out1) >= 0.999
    assert np.max(np.abs(T.tnc_plan_get_growth(plan) - g_adapted)) <= 1
    # six bits too low everywhere: stored maxima near 2^19 overflow FP16
    T.tnc_plan_set_growth(plan, g_adapted - 6)
    out2, rep2 = T.tnc_execute(plan, case["bits"], 0, n)
    assert 1 <= rep2["replays"] <= 3, rep2
    f = metrics.fidelity(case["ref"], out2)
    rl = metrics.rel_l2(out2, case["ref"])
    assert f >= 0.999 and rl <= 0.05, (f, rl)
    # the estimates settle back to what the values realize
    g_after = T.tnc_plan_get_growth(plan)
    assert np.max(np.abs(g_after - g_adapted)) <= 1, (g_after - g_adapted)
    out3, rep3 = T.tnc_execute(plan, case["bits"], 0, n)
    assert rep3["replays"] == 0
    assert metrics.fidelity(case["ref"], out3) >= 0.999
    T.tnc_plan_destroy(plan)


def test_growth_far_too_low_fails_with_eoverflow(T, ctx, case):
    plan = T.tnc_plan_create(ctx, case["net"], case["ssa"], case["sl"], OPEN, "f16_4m")
    n = 1 << len(case["sl"])
    T.tnc_execute(plan, case["bits"], 0, n)
    g = T.tnc_plan_get_growth(plan)
    T.tnc_plan_set_growth(plan, np.full_like(g, -60))
    with pytest.raises(T.TncError) as e:
        T.tnc_execute(plan, case["bits"], 0, n)
    assert e.value.code == -4, e.value
    T.tnc_plan_set_growth(plan, g)
    out, rep = T.tnc_execute(plan, case["bits"], 0, n)
    assert rep["replays"] == 0
    assert metrics.fidelity(case["ref"], out) >= 0.999
    # argument checks
    with pytest.raises(T.TncError):
        T.tnc_plan_set_growth(plan, g[:-1])
    with pytest.raises(T.TncError):
        T.tnc_plan_set_growth(plan, np.full_like(g, 100))
    T.tnc_plan_destroy(plan)
    pc = T.tnc_plan_create(ctx, case["net"], case["ssa"], case["sl"], OPEN, "c64")
    with pytest.raises(T.TncError):
        T.tnc_plan_set_growth(pc, np.zeros(T.tnc_plan_info(pc)["n_steps"], np.int32))
    T.tnc_plan_destroy(pc)
