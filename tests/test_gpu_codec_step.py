"""Single-step quantization of a complex64 plan against the oracle.

The result of one path step passes through the exchange codec (paper Sec. 3.2)
on every slice, as in the single-step quantization study of Sec. 4.3.1; the
oracle applies its own codec to the same step of its own FP64 contraction.

Whole-tensor kinds (half, int8) code each entry on its own from the tensor's
min and max, so they do not depend on the order in which the plan stores the
step's result: the amplitudes are compared with the oracle's.  The two sides
differ only where an entry's code flips because the complex64 intermediate
differs from the FP64 one in the last bits; the tolerance is a fraction of the
codec's own error (int8 flips are rare: the power 0.2 shrinks the relative
difference fivefold and a code step is wide; half flips more often, each one
ulp of FP16).  int4 groups of consecutive entries do depend on that order, so
there the fidelity loss is compared, within a factor of two.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import workloads  # noqa: E402
from oracle import codec, einsum, metrics  # noqa: E402

N_Q = 16
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
    st = torch.cuda.Stream()
    c = T.tnc_create(0, ws, stream=st)
    yield c
    T.tnc_destroy(c)
    torch.cuda.synchronize()
    del ws


@pytest.fixture(scope="module")
def case(T, ctx):
    from paper_2407_00769_amd import circuit_network as cn
    sites, cp = workloads.rect_grid(4, 4)
    c = workloads.random_circuit(sites, cp, 8, 11)
    st = workloads.tn_structure(c)
    r, l, d, o = cn.network_arrays(c, st)
    net = T.tnc_network_create(r, l, d, c.n_qubits, o)
    ssa, sl, _ = T.tnc_search(net, len(r), OPEN, 9, restarts=4, seed=1)
    bits = workloads.prefix_bitstrings(N_Q, OPEN, 128, 5)
    ts = einsum.network_tensors(c, st)
    closed = workloads.closed_values(bits, N_Q, OPEN)
    fixed0 = {st.output_labels[q]: v for q, v in closed.items()}
    ranks = {}
    einsum.contract_path(ts, st.output_labels, ssa, {**fixed0, **{l: 0 for l in sl}},
                         after_step=lambda s, lab, dd: ranks.__setitem__(s, len(lab)) or dd)
    yield dict(c=c, st=st, net=net, ssa=ssa, sl=list(sl), bits=bits, ts=ts, fixed0=fixed0, ranks=ranks)
    T.tnc_network_destroy(net)


def _oracle(case, step=-1, kind="half", group=None):
    """Sum over all slices of the oracle's path contraction, with the codec
    round trip (float32 in, as the plan holds complex64) after ``step``."""
    st, sl = case["st"], case["sl"]

    def hook(s, lab, d):
        if s != step:
            return d
        r = codec.as_real(d.astype(np.complex64))
        q, sc, ze = codec.quantize(r, kind, group, precision="fp32")
        y = codec.dequantize(q, sc, ze, kind, group)
        return (y[0::2] + 1j * y[1::2]).reshape(d.shape)

    acc = 0
    for sigma in range(1 << len(sl)):
        fixed = {**case["fixed0"], **{l: (sigma >> j) & 1 for j, l in enumerate(sl)}}
        acc = acc + einsum.contract_path(case["ts"], st.output_labels, case["ssa"], fixed, after_step=hook)
    b = case["bits"]
    idx = tuple(((b >> np.uint64(q)) & np.uint64(1)).astype(np.int64) for q in OPEN)
    return acc[idx]


def _steps(case):
    """A late step and the widest step whose result has at least 2^6 entries."""
    r = case["ranks"]
    wide = [s for s in sorted(r) if r[s] >= 6]
    assert wide, r
    return sorted({wide[-1], max(wide, key=lambda s: (r[s], s))})


def test_codec_step_whole_tensor_kinds(T, ctx, case):
    plan = T.tnc_plan_create(ctx, case["net"], case["ssa"], case["sl"], OPEN, "c64")
    n = 1 << len(case["sl"])
    base, _ = T.tnc_execute(plan, case["bits"], 0, n)
    ref = _oracle(case)
    e64 = metrics.rel_l2(base, ref)
    assert e64 <= 1e-4, e64
    for step in _steps(case):
        for kind, frac in (("int8", 0.1), ("half", 0.4)):
            T.tnc_plan_set_codec(plan, step, kind, 0)
            got, _ = T.tnc_execute(plan, case["bits"], 0, n)
            want = _oracle(case, step, kind)
            e_codec = metrics.rel_l2(want, ref)
            err = metrics.rel_l2(got, want)
            print(f"step {step} rank {case['ranks'][step]} {kind}: codec error {e_codec:.3e}, "
                  f"plan vs oracle {err:.3e}, relative fidelity {metrics.fidelity(ref, got):.8f}", flush=True)
            assert e_codec > 10 * e64, (step, kind, e_codec, e64)
            assert err <= frac * e_codec + 3 * e64, (step, kind, err, e_codec, e64)
    # switching it off gives back the plain plan's bits
    T.tnc_plan_set_codec(plan, -1, "half", 0)
    again, _ = T.tnc_execute(plan, case["bits"], 0, n)
    np.testing.assert_array_equal(again, base)
    T.tnc_plan_destroy(plan)


@pytest.mark.parametrize("group", [16, 128, 1024])
def test_codec_step_int4_fidelity(T, ctx, case, group):
    plan = T.tnc_plan_create(ctx, case["net"], case["ssa"], case["sl"], OPEN, "c64")
    n = 1 << len(case["sl"])
    ref = _oracle(case)
    step = _steps(case)[-1]
    T.tnc_plan_set_codec(plan, step, "int4", group)
    got, _ = T.tnc_execute(plan, case["bits"], 0, n)
    want = _oracle(case, step, "int4", group)
    loss_plan = 1 - metrics.fidelity(ref, got)
    loss_oracle = 1 - metrics.fidelity(ref, want)
    print(f"int4 group {group} step {step}: fidelity loss plan {loss_plan:.3e}, oracle {loss_oracle:.3e}",
          flush=True)
    assert loss_oracle > 0
    assert 0.5 * loss_oracle <= loss_plan <= 2 * loss_oracle, (loss_plan, loss_oracle)
    T.tnc_plan_destroy(plan)


def test_codec_step_rejects_bad_calls(T, ctx, case):
    plan = T.tnc_plan_create(ctx, case["net"], case["ssa"], case["sl"], OPEN, "c64")
    n_steps = len(case["ssa"]) // 2
    with pytest.raises(T.TncError):
        T.tnc_plan_set_codec(plan, n_steps, "half", 0)
    with pytest.raises(T.TncError):
        T.tnc_plan_set_codec(plan, _steps(case)[-1], "int4", 100)
    with pytest.raises(T.TncError):
        T.tnc_plan_set_codec(plan, _steps(case)[-1], "int8", 64)
    T.tnc_plan_destroy(plan)
    p16 = T.tnc_plan_create(ctx, case["net"], case["ssa"], case["sl"], OPEN, "f16_4m")
    with pytest.raises(T.TncError):
        T.tnc_plan_set_codec(p16, _steps(case)[-1], "half", 0)
    T.tnc_plan_set_codec(p16, -1, "half", 0)
    T.tnc_plan_destroy(p16)
