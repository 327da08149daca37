"""The learned step-cost model on the GPU.

* Device gradients (the library's forward and backward kernels, FP32) match
  the FP64 oracle's analytic gradients (themselves pinned by finite
  differences) within 1e-4 relative.
* Training is deterministic for a seed and reduces the loss.
* Trained on the engine's own step timings, the MLP predicts held-out step
  times better than the FLOP model with a fitted scale.
* Outside the trained size range a prediction is the value at the range's
  edge plus the excess (log2 time in proportion to the work).
* Steering the path search with it (three seeds) gives paths whose measured
  block times are at least as fast as the FLOP-steered ones, up to a 3% margin
  for run-to-run timing spread (geometric-mean gain >= 0.97); the gains are
  printed.
"""
import time

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import workloads  # noqa: E402
from oracle import mlp as omlp  # noqa: E402


@pytest.fixture(scope="module")
def T():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2407_00769_amd import _tnc
    return _tnc


@pytest.fixture(scope="module")
def ctx(T):
    ws = torch.empty(16 << 30, dtype=torch.uint8, device="cuda:0")
    c = T.tnc_create(0, ws, stream=torch.cuda.Stream())
    yield c
    T.tnc_destroy(c)
    torch.cuda.synchronize()
    del ws


def _rows(n, seed):
    rng = np.random.default_rng(seed)
    x = np.column_stack([rng.integers(0, 17, n), rng.integers(0, 17, n), rng.integers(0, 17, n),
                         rng.integers(0, 9, n), rng.integers(0, 3, n), rng.integers(0, 3, n),
                         rng.integers(0, 3, n), rng.integers(0, 2, n)]).astype(np.float32)
    y = (0.5 * x[:, 0] + 0.4 * x[:, 1] + 0.3 * x[:, 2] - 8 + 0.2 * x[:, 4]).astype(np.float32)
    return x, y


def test_device_gradients_match_fp64_oracle(T, ctx):
    x, y = _rows(256, 1)
    p = omlp.init(3).astype(np.float32)
    p[omlp.SIZES[0]:omlp.SIZES[0] + omlp.H] = 0.1
    assert T.tnc_mlp_param_count() == omlp.N_PARAMS
    T.tnc_mlp_set_params(ctx, p)
    loss, g = T.tnc_mlp_grad(ctx, x, y)
    l64, g64 = omlp.loss_and_grad(p.astype(np.float64), x.astype(np.float64), y.astype(np.float64))
    assert abs(loss - l64) <= 1e-5 * abs(l64)
    off = 0
    for s in omlp.SIZES:
        a, b = g[off:off + s].astype(np.float64), g64[off:off + s]
        assert np.linalg.norm(a - b) <= 1e-4 * np.linalg.norm(b) + 1e-7, (off, s)
        off += s
    # predictions equal the oracle's forward pass
    pred = T.tnc_mlp_predict(ctx, x)
    ref, _ = omlp.forward(p.astype(np.float64), x.astype(np.float64))
    np.testing.assert_allclose(pred, ref, rtol=1e-5, atol=1e-4)


def test_adam_steps_match_fp64_oracle(T, ctx):
    """A few full-batch Adam steps of the device trainer (FP32) against the
    oracle's Adam (FP64, pinned by closed forms) from the same weights: the
    per-parameter updates agree, which a wrong beta, bias correction or eps
    would break (the first step alone is lr * sign(g) only with the bias
    correction)."""
    x, y = _rows(256, 5)
    p0 = omlp.init(13).astype(np.float32)
    p0[omlp.SIZES[0]:omlp.SIZES[0] + omlp.H] = 0.1
    x64, y64, q0 = x.astype(np.float64), y.astype(np.float64), p0.astype(np.float64)
    _, g0 = omlp.loss_and_grad(q0, x64, y64)
    for steps, lr in ((1, 1e-3), (4, 1e-3), (4, 3e-2)):
        T.tnc_mlp_set_params(ctx, p0)
        loss = T.tnc_mlp_adam(ctx, x, y, steps, lr)
        d_gpu = T.tnc_mlp_get_params(ctx).astype(np.float64) - q0
        p_or, l_or = omlp.adam_full_batch(q0, x64, y64, steps, lr)
        d_or = p_or - q0
        big = np.abs(g0) > 1e-2 * np.max(np.abs(g0))
        assert big.sum() > 1000
        np.testing.assert_allclose(d_gpu[big], d_or[big], rtol=1e-2, atol=1e-3 * lr)
        assert np.linalg.norm(d_gpu - d_or) <= 2e-2 * np.linalg.norm(d_or), steps
        assert abs(loss - l_or) <= 1e-3 * abs(l_or) + 1e-6, (loss, l_or)
        if steps == 1:   # bias-corrected first step: lr * g / (|g| + eps)
            np.testing.assert_allclose(d_gpu[big], -lr * np.sign(g0[big]), rtol=1e-3)


def test_training_is_deterministic_and_learns(T, ctx):
    x, y = _rows(2048, 2)
    l1 = T.tnc_mlp_train(ctx, x, y, epochs=20, batch=128, lr=3e-3, seed=7)
    p1 = T.tnc_mlp_get_params(ctx)
    l2 = T.tnc_mlp_train(ctx, x, y, epochs=20, batch=128, lr=3e-3, seed=7)
    p2 = T.tnc_mlp_get_params(ctx)
    np.testing.assert_array_equal(p1, p2)
    assert l1 == l2
    assert l1 < 0.02 * float(np.var(y)), (l1, float(np.var(y)))


def test_prediction_outside_training_range(T, ctx):
    x, y = _rows(1024, 4)   # size features log2 M, N, K in [0, 16], batch in [0, 8]
    T.tnc_mlp_train(ctx, x, y, epochs=5, batch=128, lr=3e-3, seed=3)
    base = x[:8].copy()
    base[:, 3] = 8.0                      # at the top of the batch range
    above = base.copy()
    above[:, 3] = 11.0                    # 3 above it
    above[:, 0] = 19.0                    # and M 3 above its top (16)
    edge = base.copy()
    edge[:, 0] = 16.0
    below = edge.copy()
    below[:, 2] = -4.0                    # K below its bottom (0): evaluated at 0
    at0 = edge.copy()
    at0[:, 2] = 0.0
    p_edge, p_above = T.tnc_mlp_predict(ctx, edge), T.tnc_mlp_predict(ctx, above)
    np.testing.assert_array_equal(p_above, p_edge)   # clamped to the edge of the range
    np.testing.assert_array_equal(T.tnc_mlp_predict(ctx, below), T.tnc_mlp_predict(ctx, at0))
    # weights set from outside carry no range: evaluated as given
    T.tnc_mlp_set_params(ctx, T.tnc_mlp_get_params(ctx))
    p_raw = T.tnc_mlp_predict(ctx, above)
    ref, _ = omlp.forward(T.tnc_mlp_get_params(ctx).astype(np.float64), above.astype(np.float64))
    np.testing.assert_allclose(p_raw, ref, rtol=1e-5, atol=1e-4)


def _timing_data(T, ctx):
    from paper_2407_00769_amd import costmodel
    circs = []
    for (rows, cols, cyc, seed) in [(4, 4, 10, 101), (4, 5, 10, 102), (5, 5, 12, 103), (4, 6, 12, 104),
                                    (5, 6, 10, 105), (3, 4, 8, 106), (5, 6, 14, 107)]:
        sites, cp = workloads.rect_grid(rows, cols)
        circs.append(workloads.random_circuit(sites, cp, cyc, seed))
    return costmodel.collect(ctx, circs, ["c64", "f16_4m", "f16_3m", "bf16_4m"], caps=[14, 18, 22],
                             open_counts=[4, 8], restarts=2, seed=1)


def test_mlp_beats_flop_model_and_steers_search(T, ctx):
    from paper_2407_00769_amd import circuit_network as cn
    from paper_2407_00769_amd import costmodel
    t0 = time.perf_counter()
    X, y, fl = _timing_data(T, ctx)
    t_collect = time.perf_counter() - t0
    n = len(y)
    assert n > 2000, n
    rng = np.random.default_rng(0)
    perm = rng.permutation(n)
    tr, te = perm[: int(0.8 * n)], perm[int(0.8 * n):]
    t0 = time.perf_counter()
    Xw, yw = costmodel.training_rows(X[tr], y[tr])
    loss = T.tnc_mlp_train(ctx, Xw, yw, epochs=40, batch=256, lr=2e-3, seed=7)
    t_train = time.perf_counter() - t0
    pred = costmodel.predict(ctx, X[te])
    c = costmodel.flop_model_fit(fl[tr], y[tr])
    base = costmodel.flop_model_predict(fl[te], c)
    err_mlp = float(np.median(np.abs(pred - y[te])))
    err_flop = float(np.median(np.abs(base - y[te])))
    print(f"\nrows {n} (collect {t_collect:.1f} s, train {t_train:.1f} s, loss {loss:.4f}); held-out median "
          f"|log2 error|: MLP {err_mlp:.3f}, FLOP model {err_flop:.3f}")
    assert err_mlp < err_flop
    # steer the search for the 30-qubit circuit under each model (three seeds)
    # and time both choices: best of 3 executes each
    T.tnc_costmodel_use(ctx)
    c30 = workloads.config_circuit(2)
    st = workloads.tn_structure(c30)
    r, l, d, o = cn.network_arrays(c30, st)
    net = T.tnc_network_create(r, l, d, c30.n_qubits, o)
    open_q = list(range(20, 30))
    bits = workloads.prefix_bitstrings(30, open_q, 1024, 3)
    gains = []
    for seed in (1, 2, 3):
        times = {}
        for model in (0, 1):
            ssa, sl, _ = T.tnc_search(net, len(r), open_q, 22, cost_model=model, restarts=32, seed=seed)
            plan = T.tnc_plan_create(ctx, net, ssa, sl, open_q, "f16_4m")
            nsl = 1 << len(sl)
            T.tnc_execute(plan, bits, 0, nsl)
            times[model] = min(T.tnc_execute(plan, bits, 0, nsl)[1]["seconds"] for _ in range(3))
            T.tnc_plan_destroy(plan)
        gains.append(times[0] / times[1])
        print(f"seed {seed}: FLOP-steered {times[0] * 1e3:.2f} ms, MLP-steered {times[1] * 1e3:.2f} ms, "
              f"gain x{gains[-1]:.3f}")
    T.tnc_costmodel_use(None)
    T.tnc_network_destroy(net)
    geo = float(np.exp(np.mean(np.log(gains))))
    print(f"geometric-mean gain x{geo:.3f}")
    # the learned model must not lose to the FLOP model: a 3% margin covers
    # the run-to-run spread of the block times
    assert geo >= 0.97, gains
