#!/usr/bin/env python3
"""Throughput of the sliced tensor-network amplitude path on one MI355X.

One step = one tnc_execute over the whole slice block of the workload (every
slice through every contraction step and the FP64 cross-slice sum), launched
as one HIP graph, with the inputs resident on the device.

Workload (default): 30-qubit 5x6 grid random circuit, 14 cycles + final
layer, fSim(pi/2, pi/6), ABCD couplers; 8 sliced labels (256 slices, the
whole block); 1024 bitstrings sharing a 20-bit prefix (qubits 0-19) with
qubits 20-29 open.  The primary form is FP16 storage with FP32-accumulated
matrix-core GEMMs; complex64 runs the same path for the speedup.

Prints one JSON line.  Extra keys: s_per_slice, forms (every precision run),
fidelity against the oracle, roofline of the dominant kernel (HIP events in
a timed pass), cpu_baseline (the FP64 state-vector oracle on a bounded
sample of gates, scaled to the whole circuit).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK = {"f16": 2516.6, "bf16": 2516.6, "c64": 157.3}     # dense MFMA TFLOP/s (fp32 MFMA for c64)
HBM_GBS = 8000.0
RIDGE = {k: v * 1e12 / (HBM_GBS * 1e9) for k, v in PEAK.items()}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def setup_workload(args, T, cn, workloads):
    c = workloads.config_circuit(2)
    st = workloads.tn_structure(c)
    r, l, d, o = cn.network_arrays(c, st)
    net = T.tnc_network_create(r, l, d, c.n_qubits, o)
    open_q = list(range(20, 30))
    t0 = time.perf_counter()
    ssa = sl = None
    for seed in range(1, 20):
        ssa, sl, cost = T.tnc_search(net, len(r), open_q, args.cap, restarts=args.restarts, seed=seed)
        if len(sl) == args.sliced:
            break
    t_search = time.perf_counter() - t0
    bits = workloads.prefix_bitstrings(30, open_q, 1024, 3)
    return c, st, net, open_q, ssa, sl, bits, t_search


def kernel_family(kid):
    return {0: "gemm_naive", 1: "gemm_skinny", 2: "gemm_mfma_64x16", 3: "gemm_mfma_128x32",
            4: "gemm_mfma_128x64", 5: "gemm_mfma_256x16"}.get(int(kid), f"gemm_{kid}")


def run_form(T, ctx, net, ssa, sl, open_q, bits, prec, args, torch):
    plan = T.tnc_plan_create(ctx, net, ssa, sl, open_q, prec)
    pinfo = T.tnc_plan_info(plan)
    n = 1 << len(sl)
    out = np.zeros(len(bits), dtype=np.complex128)
    for _ in range(args.warmup):
        T.tnc_execute(plan, bits, 0, n, out)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    rep = None
    for _ in range(args.steps):
        _, rep = T.tnc_execute(plan, bits, 0, n, out)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / args.steps
    res = {"plan": plan, "out": out.copy(), "sec_per_block": dt, "flops": rep["flops"], "replays": rep["replays"],
           "graph_launches": rep["graph_launches"], "device_sec": rep["seconds"], "info": pinfo, "slices": n}
    return res


def timed_kernels(T, plan, bits, n, n_steps, dtype_key, reps=3):
    """Per kernel family: launches, total ms, algorithmic flops and bytes, from
    HIP events around every launch of a step-by-step execute."""
    T.tnc_plan_set_timing(plan, True)
    steps = T.tnc_plan_steps(plan, n_steps)
    S = T.tnc_plan_info(plan)["slices_in_flight"]
    fam = {}
    es = 8 if dtype_key == "c64" else 4
    for _ in range(reps):
        T.tnc_execute(plan, bits, 0, n)
        g, p, launches = T.tnc_plan_step_times(plan, n_steps)
        for i in range(n_steps):
            if launches[i] == 0:
                continue
            sl_per_launch = (n / launches[i]) if steps["dep"][i] else 1.0
            k = kernel_family(steps["kernel"][i])
            d = fam.setdefault(k, {"ms": 0.0, "launches": 0, "flops": 0.0, "bytes": 0.0})
            d["ms"] += g[i]
            d["launches"] += int(launches[i])
            d["flops"] += steps["flops"][i] * sl_per_launch * launches[i]
            d["bytes"] += steps["bytes"][i] * sl_per_launch * launches[i]
            if p[i] > 0:
                m, nn, kk, b = steps["log2_mnkb"][i]
                pa, pb = (int(v == 2) for v in steps["perm_ab"][i])
                pbytes = 0.0
                if pa:
                    pbytes += 2.0 * es * 2.0 ** (b + m + kk)
                if pb:
                    pbytes += 2.0 * es * 2.0 ** (b + nn + kk)
                d2 = fam.setdefault("permute", {"ms": 0.0, "launches": 0, "flops": 0.0, "bytes": 0.0})
                d2["ms"] += p[i]
                d2["launches"] += int(launches[i]) * (int(pa) + int(pb))
                d2["bytes"] += pbytes * sl_per_launch * launches[i]
    T.tnc_plan_set_timing(plan, False)
    for d in fam.values():
        d["ms"] /= reps
        d["launches"] //= reps
        d["flops"] /= reps
        d["bytes"] /= reps
    return fam


def roofline_entry(fam, dtype_key):
    name, d = max(fam.items(), key=lambda kv: kv[1]["ms"])
    sec = d["ms"] * 1e-3
    per_launch_ms = d["ms"] / max(1, d["launches"])
    if name == "permute":
        bound = "hbm"
    else:
        inten = d["flops"] / max(d["bytes"], 1.0)
        bound = "mfma" if inten >= RIDGE[dtype_key] else "hbm"
    if bound == "mfma":
        ach = d["flops"] / sec / 1e12
        peak = PEAK[dtype_key]
        unit = "TFLOP/s"
    else:
        ach = d["bytes"] / sec / 1e9
        peak = HBM_GBS
        unit = "GB/s"
    return {"kernel": name, "bound": bound, "achieved": round(ach, 3), "peak": peak, "unit": unit,
            "frac": round(ach / peak, 4), "traffic": None, "launches": d["launches"],
            "avg_launch_us": round(per_launch_ms * 1e3, 3),
            "share_of_device_time": round(d["ms"] / sum(v["ms"] for v in fam.values()), 4)}


def cpu_baseline(c, block_flops, n_slices, seconds_target):
    """FP64 state-vector oracle on the host: time a bounded prefix of gates
    and scale to the whole circuit."""
    from oracle import statevector
    threads = statevector.threads()
    n_g = len(c.gates)
    t0 = time.perf_counter()
    statevector.simulate(c, stop=2)
    t_probe = time.perf_counter() - t0
    per_gate_guess = max(t_probe / 2.0, 1e-3)
    g = int(min(n_g, max(4, seconds_target / per_gate_guess)))
    t0 = time.perf_counter()
    statevector.simulate(c, stop=g)
    t_s = time.perf_counter() - t0
    t_full = t_s * n_g / g
    return {"value": round(block_flops / t_full / 1e12, 6), "unit": "TFLOP/s", "cores": threads, "kind": "oracle",
            "sample": f"FP64 state vector (2^{c.n_qubits} amplitudes) over the first {g} of {n_g} gates "
                      f"in {t_s:.1f} s, scaled to all gates: {t_full:.1f} s per block of {n_slices} slices; "
                      f"value = the block's algorithmic contraction flops / that time",
            "seconds_per_block": round(t_full, 3)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--prec", default="f16_4m")
    ap.add_argument("--compare", default="c64,f16_3m,bf16_4m")
    ap.add_argument("--cap", type=float, default=23)
    ap.add_argument("--sliced", type=int, default=8)
    ap.add_argument("--restarts", type=int, default=64)
    ap.add_argument("--workspace-gb", type=float, default=64)
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the slice blocks of several GPUs "
              f"would be independent and are not launched here", file=sys.stderr)
        sys.exit(2)

    import torch
    import workloads
    from paper_2407_00769_amd import _tnc as T
    from paper_2407_00769_amd import circuit_network as cn

    assert torch.cuda.is_available(), "no GPU"
    dev = torch.device("cuda:0")
    c, st, net, open_q, ssa, sl, bits, t_search = setup_workload(args, T, cn, workloads)
    log(f"search: {len(sl)} sliced labels, {t_search:.2f} s")
    ws = torch.empty(int(args.workspace_gb * (1 << 30)), dtype=torch.uint8, device=dev)
    stream = torch.cuda.Stream()
    ctx = T.tnc_create(0, ws, stream=stream)
    forms = [args.prec] + [p for p in args.compare.split(",") if p and p != args.prec]
    results = {}
    for prec in forms:
        results[prec] = run_form(T, ctx, net, ssa, sl, open_q, bits, prec, args, torch)
        r = results[prec]
        log(f"{prec}: {r['sec_per_block'] * 1e3:.2f} ms/block, {r['flops'] / r['sec_per_block'] / 1e12:.2f} TFLOP/s")

    gold_path = os.path.join(ROOT, "tests", "golden", "config2_amplitudes.npy")
    ref = np.load(gold_path) if os.path.exists(gold_path) else None
    ref_kind = "oracle (FP64 state vector)" if ref is not None else "complex64 GPU run"
    if ref is None:
        ref = results["c64"]["out"] if "c64" in results else None

    def fid(out):
        if ref is None:
            return None
        b = ref.ravel()
        r = out.ravel()
        f = abs(np.vdot(b, r)) ** 2 / (np.vdot(b, b).real * np.vdot(r, r).real)
        return float(f), float(np.linalg.norm(r - b) / np.linalg.norm(b))

    main_r = results[args.prec]
    n = main_r["slices"]
    dkey = "c64" if args.prec == "c64" else args.prec.split("_")[0]
    fam = timed_kernels(T, main_r["plan"], bits, n, len(ssa) // 2, dkey)
    roof = roofline_entry(fam, dkey)

    forms_out = {}
    for prec, r in results.items():
        f = fid(r["out"])
        forms_out[prec] = {"tflops": round(r["flops"] / r["sec_per_block"] / 1e12, 3),
                           "s_per_slice": r["sec_per_block"] / n,
                           "ms_per_block": round(r["sec_per_block"] * 1e3, 3),
                           "fidelity": None if f is None else round(f[0], 9),
                           "rel_l2": None if f is None else f[1], "replays": r["replays"]}
    if "c64" in results and args.prec != "c64":
        forms_out[args.prec]["speedup_vs_c64"] = round(results["c64"]["sec_per_block"] / main_r["sec_per_block"], 3)

    cpu = None
    if not args.no_cpu:
        cpu = cpu_baseline(c, main_r["flops"], n, args.cpu_seconds)

    value = main_r["flops"] / main_r["sec_per_block"] / 1e12
    line = {
        "metric": "complex-contraction TFLOPS + s/slice, fp16-MFMA vs c64, at stated fidelity",
        "value": round(value, 3),
        "unit": "TFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(main_r["sec_per_block"] * 1e3, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"f16_4m": "f16", "f16_3m": "f16", "bf16_4m": "bf16", "bf16_3m": "bf16", "c64": "f32"}[args.prec],
        "data": "synthetic",
        "config": {"workload": "30-qubit 5x6 grid random circuit, 14 cycles, 256-slice block (8 sliced labels), "
                               "1024 bitstrings with a 20-bit shared prefix",
                   "precision": args.prec, "slices": n, "bitstrings": int(len(bits)),
                   "slices_in_flight": main_r["info"]["slices_in_flight"],
                   "flops_per_block": main_r["flops"], "max_rank": main_r["info"]["max_rank"],
                   "search_seconds": round(t_search, 3)},
        "s_per_slice": main_r["sec_per_block"] / n,
        "fidelity": forms_out[args.prec]["fidelity"],
        "fidelity_reference": ref_kind,
        "forms": forms_out,
        "roofline": roof,
        "cpu_baseline": cpu,
    }
    for r in results.values():
        T.tnc_plan_destroy(r["plan"])
    T.tnc_network_destroy(net)
    T.tnc_destroy(ctx)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
