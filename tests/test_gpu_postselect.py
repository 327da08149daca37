"""Top-k post-selection on the GPU (tnc_topk) against the oracle.

Indices and probabilities are compared bit for bit (the probability is
re*re + im*im with each FP64 operation rounded on its own on both sides, and
the order is a total order), on random amplitudes with planted ties, sizes
from one entry to several candidate rounds, and on the amplitudes a plan
returns for whole correlated subspaces of a 16-qubit circuit, where the kept
samples also raise the linear XEB under the ideal distribution.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import workloads  # noqa: E402
from oracle import postselect, statevector  # noqa: E402


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


def _amps(n, seed):
    rng = np.random.default_rng(seed)
    a = (rng.normal(size=n) + 1j * rng.normal(size=n)) * 2.0 ** -8
    if n > 20:
        a[7:19] = a[3]                     # ties, broken by position
        a[-5:] = a[1]
    return a


@pytest.mark.parametrize("n,k", [(1, 1), (7, 3), (7, 50), (2048, 1), (2048, 1024), (2049, 16), (100003, 64),
                                 (1 << 20, 1024), (1 << 20, 1)])
def test_topk_matches_oracle(T, ctx, n, k):
    a = _amps(n, n + k)
    dev = torch.from_numpy(a).to("cuda:0")
    idx, prob, _ms = T.tnc_topk(ctx, dev, k)
    want_i, want_p = postselect.topk(a, k)
    np.testing.assert_array_equal(idx.cpu().numpy(), want_i)
    np.testing.assert_array_equal(prob.cpu().numpy(), want_p)


def test_topk_rejects_bad_calls(T, ctx):
    dev = torch.from_numpy(_amps(100, 1)).to("cuda:0")
    for k in (0, 1025):
        with pytest.raises(T.TncError):
            T.tnc_topk(ctx, dev, k)
    idx, prob, _ = T.tnc_topk(ctx, dev[:0], 5)
    assert idx.numel() == 0 and prob.numel() == 0


def test_post_selection_of_plan_subspaces_raises_xeb(T, ctx):
    from paper_2407_00769_amd import circuit_network as cn
    sites, cp = workloads.rect_grid(4, 4)
    c = workloads.random_circuit(sites, cp, 12, 31)
    st = workloads.tn_structure(c)
    r, l, d, o = cn.network_arrays(c, st)
    net = T.tnc_network_create(r, l, d, c.n_qubits, o)
    open_q = list(range(8, 16))
    ssa, sl, _ = T.tnc_search(net, len(r), open_q, 12, restarts=4, seed=0)
    plan = T.tnc_plan_create(ctx, net, ssa, sl, open_q, "c64")
    kept, first = [], []
    for seed in range(12):
        bits = workloads.subspace_bitstrings(16, open_q, seed)
        amps, _ = T.tnc_execute(plan, bits, 0, 1 << len(sl))
        idx, prob, _ = T.tnc_topk(ctx, torch.from_numpy(np.ascontiguousarray(amps)).to("cuda:0"), 4)
        want_i, want_p = postselect.topk(amps, 4)
        np.testing.assert_array_equal(idx.cpu().numpy(), want_i)
        np.testing.assert_array_equal(prob.cpu().numpy(), want_p)
        ideal = np.abs(statevector.amplitudes(c, bits)) ** 2
        kept.append(ideal[want_i[0]])
        first.append(ideal[0])
    T.tnc_plan_destroy(plan)
    T.tnc_network_destroy(net)
    # top-1 of 256 Porter-Thomas probabilities: E[2^n p] = H_256 = 6.12; a fixed pick: 1
    xeb_kept = postselect.linear_xeb(kept, 16)
    xeb_first = postselect.linear_xeb(first, 16)
    assert xeb_kept > 3.0, xeb_kept
    assert xeb_kept > xeb_first + 2.0, (xeb_kept, xeb_first)
