"""tnc_quantize_noalloc (for callers that cannot allocate) against tnc_quantize.

The allocation-free entry point runs the same kernels with the min/max
partials in the library's static device array instead of the context's
buffer, so its codes, scales and zeros must be bit-identical.  Two calls in a
row, the second with a smaller input, check that the array's leftover
contents from the first call do not leak into the second.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def T():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2407_00769_amd import _tnc
    return _tnc


@pytest.fixture(scope="module")
def ctx(T):
    ws = torch.empty(1 << 20, dtype=torch.uint8, device="cuda:0")
    c = T.tnc_create(0, ws, stream=torch.cuda.Stream())
    yield c
    T.tnc_destroy(c)
    torch.cuda.synchronize()
    del ws


def _values(n, seed, scale):
    g = torch.Generator().manual_seed(seed)
    x = (torch.randn(n, generator=g, dtype=torch.float32) * scale).to("cuda:0")
    torch.cuda.synchronize()
    return x


def _noalloc(T, kind, x, group, stream):
    k = T.QKINDS.get(kind, kind)
    cb, ng = T.tnc_quant_sizes(k, x.numel(), group)
    codes = torch.full((max(cb, 16),), 0xA5, dtype=torch.uint8, device="cuda:0")
    scales = torch.full((max(ng, 1),), float("nan"), dtype=torch.float32, device="cuda:0")
    zeros = torch.full((max(ng, 1),), float("nan"), dtype=torch.float32, device="cuda:0")
    torch.cuda.synchronize()
    T.tnc_quantize_noalloc(kind, x, codes, scales, zeros, group=group, stream=stream)
    stream.synchronize()
    return codes[:cb], scales[:ng], zeros[:ng]


@pytest.mark.parametrize("kind,group", [("half", 0), ("int8", 0), ("int4", 128), ("int4", 16)])
def test_noalloc_matches_quantize_twice(T, ctx, kind, group):
    stream = torch.cuda.Stream()
    # first a large input (many min/max partials), then a smaller one whose
    # extremes are far smaller: a stale partial of the first call would show
    for n, seed, scale in ((3_000_003, 1, 100.0), (1_001, 2, 0.01)):
        x = _values(n, seed, scale)
        want = T.tnc_quantize(ctx, kind, x, group)[:3]
        got = _noalloc(T, kind, x, group, stream)
        for w, g in zip(want, got):
            assert torch.equal(w.cpu(), g.cpu()), (kind, n)
    # the null stream works too
    x = _values(4096, 3, 1.0)
    want = T.tnc_quantize(ctx, kind, x, group)[:3]
    k = T.QKINDS.get(kind, kind)
    cb, ng = T.tnc_quant_sizes(k, x.numel(), group)
    codes = torch.empty(max(cb, 16), dtype=torch.uint8, device="cuda:0")
    scales = torch.empty(max(ng, 1), dtype=torch.float32, device="cuda:0")
    zeros = torch.empty(max(ng, 1), dtype=torch.float32, device="cuda:0")
    torch.cuda.synchronize()
    T.tnc_quantize_noalloc(kind, x, codes, scales, zeros, group=group, stream=None)
    torch.cuda.synchronize()
    for w, g in zip(want, (codes[:cb], scales[:ng], zeros[:ng])):
        assert torch.equal(w.cpu(), g.cpu())


def test_noalloc_rejects_bad_calls(T):
    x = _values(1024, 4, 1.0)
    codes = torch.empty(2048, dtype=torch.uint8, device="cuda:0")
    sz = torch.empty(8, dtype=torch.float32, device="cuda:0")
    with pytest.raises(T.TncError):   # unknown kind
        T._check(T.lib.tnc_quantize_noalloc(7, 1024, T._dptr(x), 0, T._dptr(codes), T._dptr(sz), T._dptr(sz), None))
    with pytest.raises(T.TncError):   # bad int4 group
        T.tnc_quantize_noalloc("int4", x, codes, sz, sz, group=100)
    with pytest.raises(T.TncError):   # misaligned values
        T._check(T.lib.tnc_quantize_noalloc(0, 1000, T._dptr(x.data_ptr() + 4), 0, T._dptr(codes), T._dptr(sz),
                                            T._dptr(sz), None))
    with pytest.raises(T.TncError):   # NULL buffer
        T._check(T.lib.tnc_quantize_noalloc(1, 1024, T._dptr(x), 0, None, T._dptr(sz), T._dptr(sz), None))
    # n = 0 is a no-op
    T._check(T.lib.tnc_quantize_noalloc(0, 0, None, 0, None, None, None, None))
