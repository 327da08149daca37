"""The step microbenchmark's 200 seeded pairwise contractions (operands of
rank 20-34, 4-16 reduced labels, 0-6 batch labels, random label orders) at
full size through tnc_contract, checked on sampled output entries that the
oracle recomputes as FP64 dot products over the reduced labels of the
stored (rounded) inputs."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from workloads import contractions as wc  # noqa: E402
from oracle import pairwise  # noqa: E402

U = {"c64": 2.0 ** -24, "f16_4m": 2.0 ** -11, "f16_3m": 2.0 ** -11, "bf16_4m": 2.0 ** -8}


@pytest.fixture(scope="module")
def T():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2407_00769_amd import _tnc
    return _tnc


@pytest.fixture(scope="module")
def ctx(T):
    ws = torch.empty(120 << 30, dtype=torch.uint8, device="cuda:0")
    c = T.tnc_create(0, ws, stream=torch.cuda.Stream())
    yield c
    T.tnc_destroy(c)
    torch.cuda.synchronize()
    del ws


def _make(n, scale, prec, gen):
    """Seeded complex normal entries in the engine's storage, on the device
    (generated in chunks so the FP32 temporaries stay small)."""
    out = torch.empty(n, dtype=torch.complex64 if prec == "c64" else torch.int32, device="cuda:0")
    step = 1 << 27
    for o in range(0, n, step):
        m = min(step, n - o)
        ri = torch.randn(m, 2, generator=gen, device="cuda:0", dtype=torch.float32) * scale
        if prec == "c64":
            out[o:o + m] = torch.view_as_complex(ri)
        else:
            dt = torch.float16 if prec.startswith("f16") else torch.bfloat16
            out[o:o + m] = ri.to(dt).contiguous().view(torch.int32).view(m)
        del ri
    return out


def _values(t, idx, prec):
    """Entries at flat indices (a gather on the device, then FP64 on the host)."""
    g = t[torch.from_numpy(idx).to(t.device)]
    if prec == "c64":
        return g.cpu().numpy().astype(np.complex128)
    dt = torch.float16 if prec.startswith("f16") else torch.bfloat16
    ri = g.contiguous().view(dt).view(-1, 2).to(torch.float64).cpu().numpy()
    return (ri[:, 0] + 1j * ri[:, 1]).reshape(idx.shape)


def _flat(labels, values):
    """Flat index (first label slowest) of label assignments; values: dict label -> int array."""
    r = len(labels)
    out = 0
    for pos, l in enumerate(labels):
        out = out + (values[l].astype(np.int64) << (r - 1 - pos))
    return out


def _check_case(T, ctx, case, prec, n_samples, max_gather=1 << 22):
    gen = torch.Generator(device="cuda:0")
    gen.manual_seed(1000 + case.seed)
    na, nb, nc = case.elems()
    K = 2 ** case.k
    A = _make(na, (2.0 * K) ** -0.5, prec, gen)
    B = _make(nb, 0.5 ** 0.5, prec, gen)
    C = torch.empty(nc, dtype=A.dtype, device="cuda:0")
    torch.cuda.synchronize()
    times, _ = T.tnc_contract(ctx, prec, A, list(case.a_labels), B, list(case.b_labels), C, list(case.c_labels))
    rng = np.random.default_rng(case.seed)
    cl = list(case.c_labels)
    red = [l for l in case.a_labels if l in case.b_labels and l not in cl]
    ns = min(n_samples, max(8, max_gather // K))
    cvals = {l: rng.integers(0, 2, ns) for l in cl}
    kk = np.arange(K, dtype=np.int64)
    kvals = {l: (kk >> (len(red) - 1 - i)) & 1 for i, l in enumerate(red)}
    full = {}
    for l in cl:
        full[l] = np.repeat(cvals[l][:, None], K, axis=1)
    for l in red:
        full[l] = np.repeat(kvals[l][None, :], ns, axis=0)
    ia = _flat(list(case.a_labels), full)
    ib = _flat(list(case.b_labels), full)
    av = _values(A, ia, prec)
    bv = _values(B, ib, prec)
    got = _values(C, _flat(cl, cvals), prec)
    for s in range(ns):
        ref = pairwise.entry_dot(av[s], bv[s])
        mag = float(np.dot(np.abs(av[s]), np.abs(bv[s])))
        bound = 4 * K * 2.0 ** -24 * mag + U[prec] * abs(ref) * 1.01 + 1e-30
        if prec.endswith("3m"):
            bound += 6 * U[prec] * mag
        assert abs(got[s] - ref) <= bound, (case, prec, s, abs(got[s] - ref), bound)
    del A, B, C
    return times


@pytest.mark.parametrize("prec", ["f16_4m"])
def test_all_200_cases_sampled(T, ctx, prec):
    for case in wc.cases(200):
        _check_case(T, ctx, case, prec, 64)
    torch.cuda.empty_cache()


@pytest.mark.parametrize("prec", ["c64", "f16_3m", "bf16_4m"])
def test_other_forms_on_a_subset(T, ctx, prec):
    cs = [c for c in wc.cases(200) if c.working_set_bytes(8) <= 48e9][:24]
    for case in cs:
        _check_case(T, ctx, case, prec, 64)
    torch.cuda.empty_cache()


def test_largest_case_4096_entries(T, ctx):
    big = max(wc.cases(200), key=lambda c: c.working_set_bytes())
    _check_case(T, ctx, big, "f16_4m", 4096, max_gather=1 << 26)
    torch.cuda.empty_cache()
