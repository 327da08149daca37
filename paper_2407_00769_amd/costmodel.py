"""Step-time data for the learned cost model (host-side orchestration).

Rows come from the engine's own measurements: plans of random circuits are
executed with step timing on (HIP events around each step's permutes and
GEMM), and every launch becomes one row

    features = (log2 M, log2 N, log2 K, log2 batch, stride class A,
                stride class B, dtype, algorithm)
    target   = log2(device microseconds of the launch, permutes included)

where batch counts the inner batch times the slices the launch carries,
stride class is 0 (operand read in place as [free][k]), 1 (in place as
[k][free]) or 2 (permuted first), dtype is 0 complex64, 1 FP16, 2 BF16 and
algorithm is 0 for 4M, 1 for 3M.

The model the search uses is the library's roofline baseline of a row
(tnc_costmodel_base: launch latency plus the larger of flops at peak and
bytes at 8 TB/s) plus the MLP's output, so the MLP is trained on the log2
ratio of measured to baseline time (training_rows) and predictions add the
baseline back (predict).
"""
from __future__ import annotations

import math

import numpy as np

from . import _tnc as T
from . import circuit_network as cn

DTYPE_CODE = {"c64": 0, "f16_4m": 1, "f16_3m": 1, "bf16_4m": 2, "bf16_3m": 2}
ALGO_CODE = {"c64": 0, "f16_4m": 0, "f16_3m": 1, "bf16_4m": 0, "bf16_3m": 1}


def step_rows(plan, n_slices, prec, reps=1):
    """(X, y, flops) rows of one timed execute per rep (bitstrings: all zeros on
    closed qubits)."""
    info = T.tnc_plan_info(plan)
    n_steps = info["n_steps"]
    steps = T.tnc_plan_steps(plan, n_steps)
    T.tnc_plan_set_timing(plan, True)
    X, y, fl = [], [], []
    bits = np.zeros(1, dtype=np.uint64)
    for _ in range(reps):
        T.tnc_execute(plan, bits, 0, n_slices)
        g, p, launches = T.tnc_plan_step_times(plan, n_steps)
        for i in range(n_steps):
            if launches[i] == 0:
                continue
            per_launch_slices = n_slices / launches[i] if steps["dep"][i] else 1.0
            m, n, k, b = steps["log2_mnkb"][i]
            sa, sb = steps["perm_ab"][i]
            us = (g[i] + p[i]) * 1e3 / launches[i]
            if us <= 0:
                continue
            X.append([m, n, k, b + math.log2(per_launch_slices), sa, sb, DTYPE_CODE[prec], ALGO_CODE[prec]])
            y.append(math.log2(us))
            fl.append(steps["flops"][i] * per_launch_slices)
    T.tnc_plan_set_timing(plan, False)
    return X, y, fl


def collect(ctx, circuits, precisions, caps, open_counts, restarts=4, seed=0, reps=1, max_slices=256):
    """Timing rows from every (circuit, precision, cap, open count) plan.

    circuits: iterable of workloads.Circuit.  Returns (X float32 [n, 8],
    y float32 [n], flops float64 [n])."""
    import workloads

    X, y, fl = [], [], []
    for c in circuits:
        st = workloads.tn_structure(c)
        r, l, d, o = cn.network_arrays(c, st)
        net = T.tnc_network_create(r, l, d, c.n_qubits, o)
        for cap in caps:
            for n_open in open_counts:
                open_q = list(range(c.n_qubits - n_open, c.n_qubits))
                try:
                    ssa, sl, _ = T.tnc_search(net, len(r), open_q, cap, restarts=restarts, seed=seed)
                except T.TncError:
                    continue
                n_sl = min(1 << len(sl), max_slices)
                for prec in precisions:
                    try:
                        plan = T.tnc_plan_create(ctx, net, ssa, sl, open_q, prec)
                    except T.TncError:
                        continue
                    a, b, f = step_rows(plan, n_sl, prec, reps)
                    X += a
                    y += b
                    fl += f
                    T.tnc_plan_destroy(plan)
        T.tnc_network_destroy(net)
    return np.array(X, np.float32), np.array(y, np.float32), np.array(fl, np.float64)


def weighted_rows(X, y, base_us=16.0, cap=16):
    """Training rows repeated in proportion to the square root of their time
    (at least once, at most cap times).  A path's time is a sum over its
    launches, which the long launches decide, while most rows are short
    launches; the repeats move the fit's attention towards the long ones."""
    X = np.asarray(X, np.float32)
    y = np.asarray(y, np.float32)
    r = np.clip(np.rint(np.sqrt(np.exp2(y.astype(np.float64)) / base_us)), 1, cap).astype(np.int64)
    idx = np.repeat(np.arange(len(y)), r)
    return X[idx], y[idx]


def training_rows(X, y):
    """Weighted rows with the MLP's target: log2 of measured over baseline time."""
    Xw, yw = weighted_rows(X, y)
    return Xw, (yw - T.tnc_costmodel_base(Xw)).astype(np.float32)


def predict(ctx, X):
    """The cost model's log2 step time (us): baseline plus the trained MLP."""
    X = np.asarray(X, np.float32)
    return T.tnc_mlp_predict(ctx, X) + T.tnc_costmodel_base(X)


def flop_model_fit(flops, y):
    """The FLOP cost model with its one scale fitted: log2 t = log2 flops + c."""
    return float(np.median(np.asarray(y, np.float64) - np.log2(np.maximum(flops, 1.0))))


def flop_model_predict(flops, c):
    return np.log2(np.maximum(flops, 1.0)) + c


def path_prediction(ctx, plan, bits, n_slices, prec):
    """Measured and MLP-predicted device time (ms) of one execute of
    [0, n_slices): every launch's features go through the trained model and
    the predicted per-launch times are summed, so the model is judged at the
    level of whole paths as well as single steps."""
    info = T.tnc_plan_info(plan)
    n_steps = info["n_steps"]
    steps = T.tnc_plan_steps(plan, n_steps)
    T.tnc_plan_set_timing(plan, True)
    T.tnc_execute(plan, bits, 0, n_slices)
    g, p, launches = T.tnc_plan_step_times(plan, n_steps)
    T.tnc_plan_set_timing(plan, False)
    X, mult, measured = [], [], 0.0
    for i in range(n_steps):
        if launches[i] == 0:
            continue
        per_launch_slices = n_slices / launches[i] if steps["dep"][i] else 1.0
        m, n, k, b = steps["log2_mnkb"][i]
        sa, sb = steps["perm_ab"][i]
        X.append([m, n, k, b + math.log2(per_launch_slices), sa, sb, DTYPE_CODE[prec], ALGO_CODE[prec]])
        mult.append(float(launches[i]))
        measured += float(g[i] + p[i])
    pred = predict(ctx, np.array(X, np.float32))
    return measured, float(np.sum(np.exp2(pred.astype(np.float64)) * np.array(mult)) * 1e-3)


def search_estimate(ctx, net, ssa, sliced, open_q, slices_per_launch, prec="f16_4m"):
    """The model's cost of a path as the path search forms it (ms): each
    step's features with the plan's slices per launch, times the launches the
    slices need; the same sum the search minimises."""
    a = T.tnc_plan_analyze_steps(net, ssa, sliced, open_q, prec)
    total = 1 << len(sliced)
    S = min(total, slices_per_launch)
    X, mult = [], []
    for i in range(len(a["flops"])):
        if a["flops"][i] <= 0:   # entries past the device steps (host-absorbed pairs run no launch)
            continue
        m, n, k, b = a["log2_mnkb"][i]
        dep = bool(a["dep"][i])
        sa, sb = a["perm_ab"][i]
        X.append([m, n, k, b + (math.log2(S) if dep else 0.0), sa, sb, DTYPE_CODE[prec], ALGO_CODE[prec]])
        mult.append(total / S if dep else 1.0)
    pred = predict(ctx, np.array(X, np.float32))
    return float(np.sum(np.exp2(pred.astype(np.float64)) * np.array(mult)) * 1e-3)
