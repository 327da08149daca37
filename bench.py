#!/usr/bin/env python3
"""Throughput of the sliced tensor-network amplitude path on one MI355X.

A step is one tnc_execute over one batch of slices of a fixed sliced path
(every slice of the batch through every contraction step, then the FP64
cross-slice sum), launched as one HIP graph with the inputs resident on the
device; consecutive steps take consecutive slice ranges.

Workloads:
  53q (default) -- one GPU's share of a 53-qubit, 20-cycle random circuit on
     the 54-site diagonal grid (one site dead): the stored sliced path
     (paper_2407_00769_amd/paths/config3.json, largest tensor of a slice
     2^33 entries), 4096 correlated amplitudes (qubits 41-52 open), batches of
     8 slices; the default 8 steps cover the 64-slice block [0, 64).
  30q -- 5x6 grid, 14 cycles, 8 sliced labels; one step is the whole
     256-slice block; 1024 bitstrings sharing a 20-bit prefix.
The primary form is FP16 storage with FP32-accumulated matrix-core GEMMs
(4M); FP16-3M, BF16-4M and complex64 run the same path (complex64 with one
slice in flight, recomputing labels per pass if one slice would not fit).

Prints one JSON line.  Extra keys: s_per_slice, forms, fidelity, roofline
(dominant kernel family, HIP events around every launch of a step-timed
pass), cpu_baseline (the oracle on the host, bounded sample).
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

PEAK = {"f16": 2516.6, "bf16": 2516.6, "c64": 157.3}     # dense MFMA TFLOP/s (FP32 MFMA for complex64)
HBM_GBS = 8000.0
RIDGE = {k: v * 1e12 / (HBM_GBS * 1e9) for k, v in PEAK.items()}
DKEY = {"c64": "c64", "f16_4m": "f16", "f16_3m": "f16", "bf16_4m": "bf16", "bf16_3m": "bf16"}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_family(kid):
    return {0: "gemm_naive", 1: "gemm_skinny", 2: "gemm_mfma_s", 3: "gemm_mfma_m", 4: "gemm_mfma_l",
            5: "gemm_mfma_w", 6: "gemm_mfma_xl", 7: "gemm_mfma_l2", 8: "gemm_dma_4",
            9: "gemm_dma_8", 10: "gemm_dma_8w", 11: "gemm_dma_2", 12: "gemm_dma_n64", 13: "gemm_dma_n32", 14: "gemm_dma3_n64", 15: "gemm_dma3_2",
            16: "gemm_dmap_2", 17: "gemm_thinm", 18: "gemm_dmap_n64"}.get(int(kid), f"gemm_{kid}")


# ------------------------------------------------------------------ workloads

def setup_53q(args, T, cn, workloads):
    path = json.load(open(os.path.join(ROOT, "paper_2407_00769_amd", "paths", "config3.json")))
    c = workloads.config_circuit(3)
    st = workloads.tn_structure(c)
    r, l, d, o = cn.network_arrays(c, st)
    assert len(r) == path["n_tensors"], "stored path does not match the network"
    net = T.tnc_network_create(r, l, d, c.n_qubits, o)
    open_q = path["open_qubits"]
    bits = workloads.subspace_bitstrings(53, open_q, 5)
    return dict(name="53q", circuit=c, net=net, open_q=open_q, ssa=np.array(path["ssa"], np.int32),
                sliced=np.array(path["sliced"], np.int32), sliced_c64=np.array(path["sliced_c64"], np.int32),
                bits=bits, per_step=8, steps_default=8, search_seconds=path["search"]["seconds"],
                label="53-qubit, 20-cycle diagonal-grid random circuit (one GPU's share): 8-slice batches of the "
                      "stored sliced path (largest slice tensor 2^33 entries), 4096 correlated amplitudes")


def setup_30q(args, T, cn, workloads):
    c = workloads.config_circuit(2)
    st = workloads.tn_structure(c)
    r, l, d, o = cn.network_arrays(c, st)
    net = T.tnc_network_create(r, l, d, c.n_qubits, o)
    open_q = list(range(20, 30))
    t0 = time.perf_counter()
    for seed in range(1, 20):
        ssa, sl, _ = T.tnc_search(net, len(r), open_q, 22, restarts=64, seed=seed)
        if len(sl) == 8:
            break
    t_search = time.perf_counter() - t0
    bits = workloads.prefix_bitstrings(30, open_q, 1024, 3)
    return dict(name="30q", circuit=c, net=net, open_q=open_q, ssa=ssa, sliced=sl, sliced_c64=sl, bits=bits,
                per_step=256, steps_default=10, search_seconds=t_search,
                label="30-qubit 5x6 grid random circuit, 14 cycles, 256-slice block (8 sliced labels), "
                      "1024 bitstrings with a 20-bit shared prefix")


# ------------------------------------------------------------------ runs

def run_form(T, ctx, w, prec, sliced, per_step, steps, warmup, torch, recompute=None):
    plan = T.tnc_plan_create(ctx, w["net"], w["ssa"], sliced, w["open_q"], prec, recompute=recompute)
    info = T.tnc_plan_info(plan)
    total = 1 << len(sliced)
    out = np.zeros(len(w["bits"]), dtype=np.complex128)

    def rng(k):
        b = (k * per_step) % total
        return b, min(b + per_step, total)

    for k in range(warmup):
        T.tnc_execute(plan, w["bits"], *rng(k), out)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    flops = 0.0
    slices = 0
    rep = None
    for k in range(steps):
        b, e = rng(k)
        _, rep = T.tnc_execute(plan, w["bits"], b, e, out)
        flops += rep["flops"]
        slices += e - b
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    return {"plan": plan, "info": info, "seconds": dt, "flops": flops, "slices": slices,
            "replays": rep["replays"] if rep else 0}


def timed_kernels(T, plan, bits, begin, end, dtype_key):
    """Per kernel family: launches, total ms, algorithmic flops and bytes, from
    HIP events around every launch of one step-timed execute."""
    n_steps = T.tnc_plan_info(plan)["n_steps"]
    steps = T.tnc_plan_steps(plan, n_steps)
    es = 8 if dtype_key == "c64" else 4
    T.tnc_plan_set_timing(plan, True)
    T.tnc_execute(plan, bits, begin, end)
    g, p, launches = T.tnc_plan_step_times(plan, n_steps)
    T.tnc_plan_set_timing(plan, False)
    n = end - begin
    fam = {}
    for i in range(n_steps):
        if launches[i] == 0:
            continue
        per = (n / launches[i]) if steps["dep"][i] else 1.0
        k = kernel_family(steps["kernel"][i])
        d = fam.setdefault(k, {"ms": 0.0, "launches": 0, "flops": 0.0, "bytes": 0.0})
        d["ms"] += g[i]
        d["launches"] += int(launches[i])
        d["flops"] += steps["flops"][i] * per * launches[i]
        d["bytes"] += steps["bytes"][i] * per * launches[i]
        if p[i] > 0:
            m, nn, kk, b = steps["log2_mnkb"][i]
            pa, pb = (int(v == 2) for v in steps["perm_ab"][i])
            pbytes = (2.0 * es * 2.0 ** (b + m + kk) if pa else 0.0) + (2.0 * es * 2.0 ** (b + nn + kk) if pb else 0.0)
            d2 = fam.setdefault("permute", {"ms": 0.0, "launches": 0, "flops": 0.0, "bytes": 0.0})
            d2["ms"] += p[i]
            d2["launches"] += int(launches[i]) * (pa + pb)
            d2["bytes"] += pbytes * per * launches[i]
    return fam


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic.json")


def gemm_source_digest():
    import hashlib
    h = hashlib.sha256()
    for f in ("gemm.hip", "common.h", "device_util.h"):
        with open(os.path.join(ROOT, "paper_2407_00769_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(kernel, workload):
    """HBM bytes per launch of `kernel` from the committed counter summary
    (FETCH_SIZE + WRITE_SIZE, copy-calibrated), or None if there is none for
    this kernel and workload or the GEMM sources changed since it was taken."""
    try:
        with open(TRAFFIC_FILE) as fh:
            t = json.load(fh)
    except (OSError, ValueError):
        return None
    e = t.get(workload, {}).get(kernel)
    if not e or e.get("sources_sha256") != gemm_source_digest():
        return None
    return e["bytes_per_launch"]


def calibrate_copy(torch, gib=1, reps=4):
    """A plain device copy of a known size (for scaling the HBM byte counters)."""
    n = gib << 30
    src = torch.ones(n, dtype=torch.uint8, device="cuda:0")
    dst = torch.empty_like(src)
    for _ in range(reps):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_read": n, "copy_bytes_written": n, "launches": reps}), flush=True)


def codec_bench(torch, T, n_entries=1 << 27, reps=5, cpu_seconds=10.0):
    """Throughput of the exchange codec (quantize, dequantize) on a complex64
    tensor of n_entries (2 n_entries float32 values), against HBM bandwidth;
    the oracle's numpy codec timed on a bounded sample beside it."""
    n = 2 * n_entries
    ws = torch.empty(1 << 20, dtype=torch.uint8, device="cuda:0")
    ctx = T.tnc_create(0, ws, stream=torch.cuda.Stream())
    g = torch.Generator(device="cuda:0").manual_seed(11)
    x = torch.randn(n, dtype=torch.float32, device="cuda:0", generator=g)
    out = {}
    for kind in ("half", "int8", "int4"):
        cb, ng = T.tnc_quant_sizes(kind, n)
        qms, dms = [], []
        for _ in range(reps):
            codes, sc, ze, ms = T.tnc_quantize(ctx, kind, x)
            qms.append(ms)
            _xr, ms2 = T.tnc_dequantize(ctx, kind, n, codes, sc, ze)
            dms.append(ms2)
        q, d = min(qms), min(dms)
        # algorithmic bytes: whole-tensor kinds read the values twice (extremes, then codes)
        q_bytes = (8 if kind != "int4" else 4) * n + cb + 8 * ng
        d_bytes = cb + 8 * ng + 4 * n
        out[kind] = {"quantize_ms": round(q, 3), "quantize_gbs": round(q_bytes / q / 1e6, 1),
                     "dequantize_ms": round(d, 3), "dequantize_gbs": round(d_bytes / d / 1e6, 1),
                     "compression_rate": round(compression_rate(T, kind, n), 5)}
    T.tnc_destroy(ctx)
    cpu = cpu_baseline_codec(cpu_seconds)
    best = max(out.values(), key=lambda v: v["quantize_gbs"])
    return {"metric": "exchange codec throughput (quantize + dequantize of a complex64 tensor)",
            "value": round(min(v["quantize_gbs"] for v in out.values()), 1), "unit": "GB/s",
            "n_gpus": 1, "higher_is_better": True, "data": "synthetic",
            "config": {"workload": f"2^{n_entries.bit_length() - 1}-entry complex64 tensor (2^{n.bit_length() - 1} "
                                   f"float32 values), N(0,1) values"},
            "kinds": out,
            "roofline": {"bound": "hbm", "peak": HBM_GBS, "unit": "GB/s",
                         "frac_best": round(best["quantize_gbs"] / HBM_GBS, 4)},
            "cpu_baseline": cpu}


def compression_rate(T, kind, n_reals, group=0):
    """Eq. compress from the library's own code and group sizes: (scales +
    zeros + codes) / the float32 bytes of the tensor."""
    cb, ng = T.tnc_quant_sizes(kind, n_reals, group)
    return (8.0 * ng + cb) / (4.0 * n_reals)


def codec_study(torch, T, cn, workloads, n_steps=8):
    """Single-step quantization (Sec. 4.3.1) on the 30-qubit path: the result of
    one of its largest steps goes through the codec on every slice, and the
    complex64 amplitudes are compared with the stored oracle amplitudes; the
    relative fidelity is the quantized run's fidelity over the plain run's."""
    w = setup_30q(None, T, cn, workloads)
    ws = torch.empty(64 << 30, dtype=torch.uint8, device="cuda:0")
    ctx = T.tnc_create(0, ws, stream=torch.cuda.Stream())
    plan = T.tnc_plan_create(ctx, w["net"], w["ssa"], w["sliced"], w["open_q"], "c64")
    n = T.tnc_plan_info(plan)["n_steps"]
    steps = T.tnc_plan_steps(plan, n)
    ref = np.load(os.path.join(ROOT, "tests", "golden", "config2_amplitudes.npy"))
    total = 1 << len(w["sliced"])

    def fid(o):
        return float(abs(np.vdot(ref, o)) ** 2 / (np.vdot(ref, ref).real * np.vdot(o, o).real))

    base, _ = T.tnc_execute(plan, w["bits"], 0, total)
    f_c64 = fid(base)
    mnkb = steps["log2_mnkb"]
    rank = [int(mnkb[i][3] + mnkb[i][0] + mnkb[i][1]) for i in range(n)]   # log2 entries of the result
    pick = sorted(sorted(range(n), key=lambda i: (rank[i], i))[-n_steps:])
    rows = []
    for i in pick:
        row = {"step": i, "log2_entries": rank[i], "slice_dependent": bool(steps["dep"][i])}
        for kind in ("half", "int8", "int4"):
            T.tnc_plan_set_codec(plan, i, kind, 0)
            o, _ = T.tnc_execute(plan, w["bits"], 0, total)
            row[kind] = {"relative_fidelity": round(fid(o) / f_c64, 9),
                         "compression_rate": round(compression_rate(T, kind, 2 << rank[i]), 5)}
        rows.append(row)
        log(f"step {i}: 2^{rank[i]} entries, " + ", ".join(f"{k} {row[k]['relative_fidelity']:.6f}"
                                                        for k in ("half", "int8", "int4")))
    T.tnc_plan_set_codec(plan, -1, "half", 0)
    T.tnc_plan_destroy(plan)
    T.tnc_network_destroy(w["net"])
    T.tnc_destroy(ctx)
    return {"study": "single-step quantization, relative fidelity (quantized / complex64, both against the "
                     "stored FP64 oracle amplitudes)",
            "workload": w["label"], "complex64_fidelity": f_c64, "steps": rows}


def postselect_study(torch, T, cn, workloads, n_sub=16, fractions=(1 / 64, 1 / 16, 1 / 4, 1.0)):
    """Top-1 post-selection per correlated subspace (Sec. 1 and 2.3) on the
    30-qubit path: the FP16-4M plan contracts a fraction of the 256 slices of
    each subspace (1024 bitstrings, open qubits 20-29, a seeded 20-bit prefix),
    tnc_topk keeps its most probable bitstring, and the linear XEB of the kept
    samples is taken under the complex64 run of all slices."""
    w = setup_30q(None, T, cn, workloads)
    ws = torch.empty(64 << 30, dtype=torch.uint8, device="cuda:0")
    ctx = T.tnc_create(0, ws, stream=torch.cuda.Stream())
    p64 = T.tnc_plan_create(ctx, w["net"], w["ssa"], w["sliced"], w["open_q"], "c64")
    p16 = T.tnc_plan_create(ctx, w["net"], w["ssa"], w["sliced"], w["open_q"], "f16_4m")
    total = 1 << len(w["sliced"])
    kept = {f: [] for f in fractions}
    fids = {f: [] for f in fractions}
    secs = {f: 0.0 for f in fractions}
    first, topk_ms = [], []
    for seed in range(n_sub):
        bits = workloads.subspace_bitstrings(30, w["open_q"], 100 + seed)
        ideal, _ = T.tnc_execute(p64, bits, 0, total)
        pi = ideal.real ** 2 + ideal.imag ** 2
        first.append(pi[0])
        for f in fractions:
            ns = max(1, int(round(total * f)))
            t0 = time.perf_counter()
            approx, _ = T.tnc_execute(p16, bits, 0, ns)
            secs[f] += time.perf_counter() - t0
            idx, _prob, ms = T.tnc_topk(ctx, torch.from_numpy(np.ascontiguousarray(approx)).to("cuda:0"), 1)
            topk_ms.append(ms)
            kept[f].append(pi[int(idx[0])])
            fids[f].append(float(abs(np.vdot(ideal, approx)) ** 2 / (np.vdot(ideal, ideal).real *
                                                                     np.vdot(approx, approx).real)))
    T.tnc_plan_destroy(p64)
    T.tnc_plan_destroy(p16)
    T.tnc_network_destroy(w["net"])
    T.tnc_destroy(ctx)
    n_bits = 1 << len(w["open_q"])
    harmonic = float(np.sum(1.0 / np.arange(1, n_bits + 1)))
    rows = [{"slice_fraction": f, "slices": max(1, int(round(total * f))),
             "mean_fidelity": round(float(np.mean(fids[f])), 6),
             "xeb_top1": round(float(2.0 ** 30 * np.mean(kept[f]) - 1.0), 4),
             "seconds_per_subspace": round(secs[f] / n_sub, 5)} for f in fractions]
    return {"study": "top-1 post-selection per correlated subspace, linear XEB of the kept samples",
            "workload": w["label"], "subspaces": n_sub, "bitstrings_per_subspace": n_bits,
            "xeb_fixed_pick": round(float(2.0 ** 30 * np.mean(first) - 1.0), 4),
            "xeb_top1_expected_exact": round(harmonic - 1.0, 4),
            "topk_ms_mean": round(float(np.mean(topk_ms)), 4), "rows": rows}


def cpu_baseline_codec(cpu_seconds):
    """The oracle's numpy codec on a bounded sample (float32 decisions)."""
    from oracle import codec as ocodec
    xs = np.random.default_rng(0).normal(size=1 << 22).astype(np.float32)
    t0 = time.perf_counter()
    reps_cpu = 0
    while time.perf_counter() - t0 < cpu_seconds:
        for kind in ("half", "int8", "int4"):
            c, s_, z_ = ocodec.quantize(xs, kind, precision="fp32")
            ocodec.dequantize(c, s_, z_, kind)
        reps_cpu += 1
    dt = time.perf_counter() - t0
    cpu_rate = 3 * reps_cpu * xs.size * 4 / dt / 1e9
    return {"value": round(cpu_rate, 4), "unit": "GB/s of float32 input (quantize + dequantize)",
            "cores": 1, "kind": "oracle",
            "sample": f"oracle codec (numpy, float32 decisions) on 2^22 values, all three kinds, "
                      f"{reps_cpu} rounds in {dt:.1f} s"}


def path_roofline(T, plan, dtype_key, seconds_per_slice):
    """Path-level roofline time per slice, T_roof = sum over the slice's steps
    of max(F_t / P_mfma, B_t / 8 TB/s) with the permutes HBM-bound beside
    them, against the measured time per slice."""
    info = T.tnc_plan_info(plan)
    n = info["n_steps"]
    st = T.tnc_plan_steps(plan, n)
    peak = PEAK[dtype_key] * 1e12
    bw = HBM_GBS * 1e9
    t = 0.0
    for i in range(n):
        if st["dep"][i]:
            t += max(st["flops"][i] / peak, st["bytes"][i] / bw)
    t += info["permute_bytes_per_slice"] / bw
    return {"t_roof_s_per_slice": t, "t_measured_s_per_slice": seconds_per_slice,
            "frac": round(t / seconds_per_slice, 4),
            "note": "slice-dependent steps; GEMM bytes = A + B + C at the storage size, permutes at 8 TB/s"}


def roofline_entry(fam, dtype_key):
    name, d = max(fam.items(), key=lambda kv: kv[1]["ms"])
    sec = d["ms"] * 1e-3
    if name == "permute":
        bound = "hbm"
    else:
        bound = "mfma" if d["flops"] / max(d["bytes"], 1.0) >= RIDGE[dtype_key] else "hbm"
    if bound == "mfma":
        ach, peak, unit = d["flops"] / sec / 1e12, PEAK[dtype_key], "TFLOP/s"
    else:
        ach, peak, unit = d["bytes"] / sec / 1e9, HBM_GBS, "GB/s"
    total_ms = sum(v["ms"] for v in fam.values())
    return {"kernel": name, "bound": bound, "achieved": round(ach, 3), "peak": peak, "unit": unit,
            "frac": round(ach / peak, 4), "traffic": None, "launches": d["launches"],
            "avg_launch_us": round(d["ms"] / max(1, d["launches"]) * 1e3, 3),
            "share_of_device_time": round(d["ms"] / total_ms, 4),
            "families": {k: {"ms": round(v["ms"], 3), "launches": v["launches"],
                             "tflops": round(v["flops"] / max(v["ms"], 1e-9) / 1e9, 2)} for k, v in fam.items()}}


# ------------------------------------------------------------------ step microbenchmark

def microbench(torch, T, forms=("f16_4m", "c64"), count=200, cpu_seconds=10.0):
    """The 200 seeded pairwise contractions (rank 20-34 operands, 4-16 reduced
    labels, 0-6 batch labels, random label orders) through tnc_contract, one
    launch each after a warm launch: GEMM TFLOP/s (algorithmic 8 B M N K) and
    permute GB/s (2 x the permuted tensor's bytes) per case, summarised per
    form.  Cases whose working set does not fit the workspace at a form's
    entry size are skipped for that form (reported)."""
    from workloads import contractions as wc
    cs = wc.cases(count)
    free, _ = torch.cuda.mem_get_info()
    ws_bytes = int(min(free - (24 << 30), 120 << 30))
    ws = torch.empty(ws_bytes, dtype=torch.uint8, device="cuda:0")
    ctx = T.tnc_create(0, ws, stream=torch.cuda.Stream())
    gen = torch.Generator(device="cuda:0").manual_seed(5)
    out = {}
    for prec in forms:
        es = 8 if prec == "c64" else 4
        dk = DKEY[prec]
        rows, skipped = [], 0
        t_start = time.perf_counter()
        for c in cs:
            na, nb, nc = c.elems()
            # operands + result on the device; permuted copies in the workspace
            if es * (na + nb + nc) > free - ws_bytes - (16 << 30) or 2 * es * (na + nb + nc) > ws_bytes:
                skipped += 1
                continue
            dt = torch.complex64 if prec == "c64" else torch.int32
            A = torch.empty(na, dtype=dt, device="cuda:0")
            B = torch.empty(nb, dtype=dt, device="cuda:0")
            C = torch.empty(nc, dtype=dt, device="cuda:0")
            for X, sc in ((A, 2.0 ** (-c.k / 2)), (B, 1.0)):
                ri = torch.view_as_real(X) if prec == "c64" else X.view(torch.float16 if dk == "f16" else torch.bfloat16)
                ri.normal_(0.0, sc * 0.7071, generator=gen)
            torch.cuda.synchronize()
            T.tnc_contract(ctx, prec, A, c.a_labels, B, c.b_labels, C, c.c_labels, scale_log2=0)
            times, _ = T.tnc_contract(ctx, prec, A, c.a_labels, B, c.b_labels, C, c.c_labels, scale_log2=0)
            fl = 8.0 * 2.0 ** (c.b + c.m + c.n + c.k)
            pa, pb, gm, pc = times
            rows.append({"seed": c.seed, "mnkb": [c.m, c.n, c.k, c.b], "gemm_ms": gm, "tflops": fl / (gm * 1e9),
                         "perm_ms": [pa, pb, pc], "perm_bytes": [2.0 * es * na, 2.0 * es * nb, 2.0 * es * nc],
                         "flops": fl})
            del A, B, C
        torch.cuda.empty_cache()
        tf = np.array([r["tflops"] for r in rows])
        g_ms = sum(r["gemm_ms"] for r in rows)
        g_fl = sum(r["flops"] for r in rows)
        # a permute that ran: more than 20 us (the events around a skipped permute read a few us)
        pm = [(b, t) for r in rows for b, t in zip(r["perm_bytes"], r["perm_ms"]) if t > 0.02]
        p_gbs = sum(b for b, _ in pm) / max(sum(t for _, t in pm) * 1e-3, 1e-12) / 1e9
        big = [r for r in rows if r["flops"] >= 1e13]
        out[prec] = {"cases": len(rows), "skipped": skipped,
                     "gemm_tflops_aggregate": round(g_fl / (g_ms * 1e9), 2),
                     "gemm_frac_of_peak_aggregate": round(g_fl / (g_ms * 1e9) / PEAK[dk], 4),
                     "gemm_tflops_median": round(float(np.median(tf)), 2),
                     "gemm_tflops_max": round(float(tf.max()), 2),
                     "gemm_tflops_median_cases_over_1e13_flops": round(float(np.median([r["tflops"] for r in big])), 2)
                     if big else None,
                     "permutes": len(pm), "permute_gbs_aggregate": round(p_gbs, 1),
                     "permute_frac_of_hbm": round(p_gbs / HBM_GBS, 4),
                     "seconds": round(time.perf_counter() - t_start, 1)}
        log(f"microbench {prec}: {out[prec]}")
    T.tnc_destroy(ctx)
    del ws
    # the oracle beside it: one mid-size case through numpy (BLAS), bounded
    from oracle import pairwise
    model, threads = host_cpu()
    c = min((c for c in cs if c.b == 0), key=lambda c: abs(8.0 * 2.0 ** (c.m + c.n + c.k) - 2e10))
    rng = np.random.default_rng(0)
    a = rng.normal(size=(2,) * len(c.a_labels)) + 1j * rng.normal(size=(2,) * len(c.a_labels))
    b = rng.normal(size=(2,) * len(c.b_labels)) + 1j * rng.normal(size=(2,) * len(c.b_labels))
    fl = 8.0 * 2.0 ** (c.b + c.m + c.n + c.k)
    t0, reps = time.perf_counter(), 0
    while time.perf_counter() - t0 < cpu_seconds:
        pairwise.contract_pair(a, c.a_labels, b, c.b_labels, c.c_labels)
        reps += 1
    dt = time.perf_counter() - t0
    cpu = {"value": round(fl * reps / dt / 1e12, 6), "unit": "TFLOP/s", "cores": threads, "kind": "oracle", "cpu": model,
           "sample": f"oracle pairwise contraction of case {c.seed} (2^{c.m} x 2^{c.n} x 2^{c.k}, random label "
                     f"orders), {reps} runs in {dt:.1f} s"}
    return {"metric": "pairwise contraction microbenchmark (200 seeded cases)", "unit": "TFLOP/s",
            "forms": out, "cpu_baseline": cpu}


# ------------------------------------------------------------------ sparse state

def sparse_study(torch, T, cn, workloads, n_bits=1024, cap=20, forms=("f16_4m", "c64"), sv=True):
    """Uncorrelated bitstrings of the 30-qubit, 14-cycle circuit through a
    sparse-state plan (Sec. 3.4.2): n_bits uniform random bitstrings share no
    fixed bits, and each tensor keeps one block per distinct value of the
    bitstrings on its qubits.  The path is searched with every output leg
    open (a leg then costs its full dimension, an upper bound on its block
    count, so the search brings the output legs in late and the blocks stay
    few for most of the contraction), at caps of n and n + 1 bits with
    several seeds, and the library's sparse analysis of the requested
    bitstrings picks the path with the least work; the path for the network
    with every output closed is priced beside it.  Reported: time and
    TFLOP/s per form, the work against one closed contraction per bitstring,
    and parity against the oracle's FP64 state vector (all 2^30 amplitudes,
    on the host)."""
    c = workloads.config_circuit(2)
    st = workloads.tn_structure(c)
    r, l, d, o = cn.network_arrays(c, st)
    net = T.tnc_network_create(r, l, d, c.n_qubits, o)
    bits = workloads.uniform_bitstrings(30, n_bits, 7)

    def sparse_flops(ssa_, sl_):
        a = T.tnc_plan_analyze_sparse(net, ssa_, sl_, bits, "f16_4m")
        return a["flops_per_slice"] * (1 << len(sl_)) + a["flops_invariant"]

    t0 = time.perf_counter()
    cands = []
    for cap_open in (c.n_qubits, c.n_qubits + 1):
        for seed in (1, 2, 3, 4):
            try:
                ssa_c, sl_c, _ = T.tnc_search(net, len(r), list(range(c.n_qubits)), cap_open, restarts=16, seed=seed)
            except T.TncError:
                continue
            cands.append((sparse_flops(ssa_c, sl_c), cap_open, seed, ssa_c, sl_c))
    flops_sparse, cap_used, seed_used, ssa, sl = min(cands, key=lambda x: x[0])
    t_search = time.perf_counter() - t0
    # the path for the network with every output closed: one contraction per
    # bitstring, and the sparse scheme on that path
    ssa0, sl0, _ = T.tnc_search(net, len(r), [], cap, restarts=16, seed=1)
    a_one = T.tnc_plan_analyze(net, ssa0, sl0, [], "f16_4m")
    flops_each = (a_one["flops_per_slice"] * (1 << len(sl0)) + a_one["flops_invariant"]) * n_bits
    flops_sparse_closed = sparse_flops(ssa0, sl0)
    n_sl = 1 << len(sl)
    free, _ = torch.cuda.mem_get_info()
    ws = torch.empty(int(min(free - (16 << 30), 96 << 30)), dtype=torch.uint8, device="cuda:0")
    ctx = T.tnc_create(0, ws, stream=torch.cuda.Stream())
    res = {}
    outs = {}
    for prec in forms:
        plan = T.tnc_plan_create_sparse(ctx, net, ssa, sl, bits, prec)
        info = T.tnc_plan_info(plan)
        T.tnc_execute(plan, bits, 0, min(n_sl, info["slices_in_flight"]))   # warm
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        out, rep = T.tnc_execute(plan, bits, 0, n_sl)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        outs[prec] = out
        res[prec] = {"seconds": round(dt, 4), "tflops": round(rep["flops"] / dt / 1e12, 2),
                     "s_per_bitstring": dt / n_bits, "slices_in_flight": info["slices_in_flight"],
                     "peak_bytes": info["peak_bytes"], "tune_seconds": round(info["tune_seconds"], 2)}
        T.tnc_plan_destroy(plan)
        log(f"sparse {prec}: {res[prec]}")
    T.tnc_destroy(ctx)
    del ws
    ref, ref_kind, t_sv = None, None, None
    if sv:
        from oracle import statevector
        t0 = time.perf_counter()
        ref = statevector.amplitudes(c, bits)
        t_sv = time.perf_counter() - t0
        ref_kind = "oracle FP64 state vector (2^30 amplitudes, host)"
    elif "c64" in outs:
        ref, ref_kind = outs["c64"], "complex64 sparse-state run"
    for prec, out in outs.items():
        if ref is not None and not (ref_kind.startswith("complex64") and prec == "c64"):
            b = ref.ravel()
            res[prec]["fidelity"] = round(float(abs(np.vdot(b, out)) ** 2 / (np.vdot(b, b).real * np.vdot(out, out).real)), 9)
            res[prec]["rel_l2"] = float(np.linalg.norm(out - b) / np.linalg.norm(b))
            res[prec]["rel_max"] = float(np.max(np.abs(out - b)) / np.max(np.abs(b)))
    T.tnc_network_destroy(net)
    model, threads = host_cpu()
    return {"metric": "sparse-state amplitudes of uncorrelated bitstrings", "unit": "s",
            "workload": f"30-qubit 5x6 grid, 14 cycles; {n_bits} uniform random bitstrings (no shared bits); "
                        f"path searched with every output open (cap 2^{cap_used}, seed {seed_used}, least sparse "
                        f"work of {len(cands)} candidates), {len(sl)} sliced labels",
            "search_seconds": round(t_search, 1), "flops_sparse": flops_sparse,
            "flops_sparse_on_closed_path": flops_sparse_closed,
            "flops_one_contraction_per_bitstring": flops_each, "work_ratio": round(flops_each / flops_sparse, 2),
            "forms": res, "reference": ref_kind,
            "cpu_baseline": None if t_sv is None else
            {"value": round(t_sv, 1), "unit": "s", "cores": threads, "kind": "oracle", "cpu": model,
             "sample": "oracle FP64 state vector of the whole 30-qubit circuit (every amplitude)"}}


# ------------------------------------------------------------------ learned cost model study

def costmodel_study(torch, T, cn, workloads, restarts=32, seeds=(1, 2, 3, 4, 5)):
    """Step timings measured by the engine on random 12- to 30-qubit circuits
    under every form train the step-time MLP on the GPU; its held-out error is
    compared with the FLOP model's (one fitted scale), and the path search for
    the 30-qubit circuit is run under each model: the chosen paths' measured
    block times decide what the learned model gains."""
    from oracle import mlp as omlp
    from paper_2407_00769_amd import costmodel
    free, _ = torch.cuda.mem_get_info()
    ws = torch.empty(int(min(free - (16 << 30), 32 << 30)), dtype=torch.uint8, device="cuda:0")
    ctx = T.tnc_create(0, ws, stream=torch.cuda.Stream())
    circs = []
    for i, (r, c, cyc) in enumerate([(3, 4, 8), (4, 4, 10), (4, 5, 10), (5, 5, 12), (4, 6, 12), (5, 6, 10),
                                     (5, 6, 14), (4, 5, 14), (5, 5, 8), (3, 6, 12), (4, 4, 14), (5, 6, 12)]):
        sites, cp = workloads.rect_grid(r, c)
        circs.append(workloads.random_circuit(sites, cp, cyc, 100 + i))
    t0 = time.perf_counter()
    X, y, fl = costmodel.collect(ctx, circs, ["c64", "f16_4m", "f16_3m", "bf16_4m", "bf16_3m"], caps=[14, 18, 22],
                                 open_counts=[4, 8], restarts=2, seed=1)
    t_collect = time.perf_counter() - t0
    n = len(y)
    rng = np.random.default_rng(0)
    perm = rng.permutation(n)
    tr, te = perm[: int(0.8 * n)], perm[int(0.8 * n):]
    t0 = time.perf_counter()
    Xw, yw = costmodel.training_rows(X[tr], y[tr])
    loss = T.tnc_mlp_train(ctx, Xw, yw, epochs=40, batch=256, lr=2e-3, seed=7)
    t_train = time.perf_counter() - t0
    pred = costmodel.predict(ctx, X[te])
    cfit = costmodel.flop_model_fit(fl[tr], y[tr])
    base = costmodel.flop_model_predict(fl[te], cfit)
    err_mlp = np.abs(pred - y[te])
    err_flop = np.abs(base - y[te])
    # the oracle's FP64 trainer on one epoch of the same rows (CPU, timed)
    t0 = time.perf_counter()
    omlp.adam_train(X[tr].astype(np.float64), y[tr].astype(np.float64), 1, 256, 2e-3, 7)
    t_cpu_epoch = time.perf_counter() - t0
    # search the 30-qubit circuit under each model and time the chosen paths
    T.tnc_costmodel_use(ctx)
    c30 = workloads.config_circuit(2)
    st = workloads.tn_structure(c30)
    r, l, d, o = cn.network_arrays(c30, st)
    net = T.tnc_network_create(r, l, d, c30.n_qubits, o)
    open_q = list(range(20, 30))
    bits = workloads.prefix_bitstrings(30, open_q, 1024, 3)
    runs = []
    for seed in seeds:
        rec = {"seed": seed}
        for model, name in ((0, "flop"), (1, "mlp")):
            ts = time.perf_counter()
            ssa, sl, lc = T.tnc_search(net, len(r), open_q, 22, cost_model=model, restarts=restarts, seed=seed)
            t_search = time.perf_counter() - ts
            plan = T.tnc_plan_create(ctx, net, ssa, sl, open_q, "f16_4m")
            nsl = 1 << len(sl)
            T.tnc_execute(plan, bits, 0, nsl)
            best = min(T.tnc_execute(plan, bits, 0, nsl)[1]["seconds"] for _ in range(5))
            steps_ms, pred_ms = costmodel.path_prediction(ctx, plan, bits, nsl, "f16_4m")
            search_ms = costmodel.search_estimate(ctx, net, ssa, sl, open_q,
                                                  T.tnc_plan_info(plan)["slices_in_flight"])
            rec[name] = {"block_ms": round(best * 1e3, 3), "sliced": len(sl), "log2_flops": round(lc, 3),
                         "search_s": round(t_search, 2), "steps_ms": round(steps_ms, 3),
                         "mlp_predicted_ms": round(pred_ms, 3),
                         "mlp_search_estimate_ms": round(search_ms, 3)}
            T.tnc_plan_destroy(plan)
        rec["gain"] = round(rec["flop"]["block_ms"] / rec["mlp"]["block_ms"], 4)
        runs.append(rec)
        log(f"costmodel seed {seed}: {rec}")
    T.tnc_costmodel_use(None)
    T.tnc_network_destroy(net)
    T.tnc_destroy(ctx)
    gains = [x["gain"] for x in runs]
    return {"metric": "learned step-cost model: held-out error and measured gain of MLP-steered paths",
            "rows": int(n), "training_rows_weighted": int(len(yw)), "collect_s": round(t_collect, 1),
            "train_s": round(t_train, 2), "train_loss": loss,
            "heldout_median_abs_log2_err": {"mlp": round(float(np.median(err_mlp)), 4),
                                            "flop": round(float(np.median(err_flop)), 4)},
            "heldout_mape": {"mlp": round(float(np.mean(np.abs(2.0 ** err_mlp - 1))), 4),
                             "flop": round(float(np.mean(np.abs(2.0 ** err_flop - 1))), 4)},
            "search_30q": runs, "gain_geomean": round(float(np.exp(np.mean(np.log(gains)))), 4),
            "cpu_baseline": {"value": round(t_cpu_epoch, 2), "unit": "s per epoch", "cores": host_cpu()[1],
                             "kind": "oracle", "sample": f"oracle FP64 MLP training, one epoch of {len(tr)} rows"}}


# ------------------------------------------------------------------ CPU baselines (the oracle)

def cpu_baseline_sv(c, block_flops, n_slices, seconds_target):
    """FP64 state-vector oracle over a bounded prefix of the gates, scaled to
    the whole circuit (it produces every amplitude of the block)."""
    from oracle import statevector
    threads = statevector.threads()
    model, _ = host_cpu()
    n_g = len(c.gates)
    t0 = time.perf_counter()
    statevector.simulate(c, stop=2)
    per_gate = max((time.perf_counter() - t0) / 2.0, 1e-3)
    g = int(min(n_g, max(4, seconds_target / per_gate)))
    t0 = time.perf_counter()
    statevector.simulate(c, stop=g)
    t_s = time.perf_counter() - t0
    t_full = t_s * n_g / g
    return {"value": round(block_flops / t_full / 1e12, 6), "unit": "TFLOP/s", "cores": threads, "kind": "oracle",
            "cpu": model,
            "sample": f"FP64 state vector (2^{c.n_qubits} amplitudes) over the first {g} of {n_g} gates in "
                      f"{t_s:.1f} s, scaled to all gates: {t_full:.1f} s for the {n_slices}-slice block; value = "
                      f"the block's algorithmic contraction flops / that time",
            "seconds_per_slice": t_full / n_slices}


def host_cpu():
    """(CPU model, BLAS threads numpy uses) of this host."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    threads = os.cpu_count() or 1
    try:
        from threadpoolctl import threadpool_info
        blas = [d["num_threads"] for d in threadpool_info() if d.get("user_api") == "blas"]
        if blas:
            threads = max(blas)
    except Exception:
        pass
    return model, threads


def cpu_baseline_einsum(flops_per_slice, seconds_target):
    """FP64 pairwise contraction of the oracle (numpy complex128 einsum, which
    reduces a plain pair to a BLAS matrix product on all host cores) timed on
    a representative step shape; the per-slice time is an estimate."""
    from oracle import pairwise
    model, threads = host_cpu()
    rng = np.random.default_rng(0)
    # a stem-like step: C has 2^13 x 2^9 entries, 2^10 reduced (3.4e10 flops)
    la, lb, lc = list(range(0, 23)), list(range(13, 32)), list(range(0, 13)) + list(range(23, 32))
    a = rng.normal(size=(2,) * 23) + 1j * rng.normal(size=(2,) * 23)
    b = rng.normal(size=(2,) * 19) + 1j * rng.normal(size=(2,) * 19)
    fl = 8.0 * 2 ** 32
    t0 = time.perf_counter()
    reps = 0
    while time.perf_counter() - t0 < seconds_target:
        pairwise.contract_pair(a, la, b, lb, lc)
        reps += 1
    dt = time.perf_counter() - t0
    rate = fl * reps / dt
    return {"value": round(rate / 1e12, 6), "unit": "TFLOP/s", "cores": threads, "kind": "oracle",
            "cpu": model,
            "sample": f"oracle pairwise contraction (numpy complex128, BLAS zgemm on {threads} threads, {model}) "
                      f"of a 2^13 x 2^9 x 2^10 step, {reps} runs in {dt:.1f} s = {rate / 1e9:.1f} GFLOP/s; "
                      f"estimated {flops_per_slice / rate:.0f} s per slice (no full oracle exists for 53 qubits)",
            "seconds_per_slice": flops_per_slice / rate}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="53q", choices=["53q", "30q"])
    ap.add_argument("--prec", default="f16_4m")
    ap.add_argument("--compare", default="c64,f16_3m,bf16_4m")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run a 1 GiB device copy 4 times (reference for the HBM byte counters)")
    ap.add_argument("--codec", action="store_true",
                    help="only measure the low-precision exchange codec (its own JSON line)")
    ap.add_argument("--codec-study", action="store_true",
                    help="only run the single-step quantization study on the 30-qubit path (its own JSON line)")
    ap.add_argument("--microbench", action="store_true",
                    help="only run the 200-case pairwise contraction microbenchmark (its own JSON line)")
    ap.add_argument("--sparse", action="store_true",
                    help="only run the sparse-state study of uncorrelated bitstrings (its own JSON line)")
    ap.add_argument("--costmodel", action="store_true",
                    help="only run the learned cost-model study (its own JSON line)")
    ap.add_argument("--postselect", action="store_true",
                    help="only run the top-1 post-selection study on the 30-qubit path (its own JSON line)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}): slice blocks on several GPUs "
              f"would be independent ranges summed by one all-reduce, which this program does not launch",
              file=sys.stderr)
        sys.exit(2)

    import torch
    if args.calibrate_copy:
        calibrate_copy(torch)
        return
    import workloads
    from paper_2407_00769_amd import _tnc as T
    if args.codec:
        print(json.dumps(codec_bench(torch, T)), flush=True)
        return
    if args.microbench:
        print(json.dumps(microbench(torch, T)), flush=True)
        return
    if args.sparse:
        from paper_2407_00769_amd import circuit_network as cn
        print(json.dumps(sparse_study(torch, T, cn, workloads)), flush=True)
        return
    if args.costmodel:
        from paper_2407_00769_amd import circuit_network as cn
        print(json.dumps(costmodel_study(torch, T, cn, workloads)), flush=True)
        return
    if args.postselect:
        from paper_2407_00769_amd import circuit_network as cn
        print(json.dumps(postselect_study(torch, T, cn, workloads)), flush=True)
        return
    if args.codec_study:
        from paper_2407_00769_amd import circuit_network as cn
        print(json.dumps(codec_study(torch, T, cn, workloads)), flush=True)
        return
    from paper_2407_00769_amd import circuit_network as cn

    assert torch.cuda.is_available(), "no GPU"
    dev = torch.device("cuda:0")
    w = (setup_53q if args.workload == "53q" else setup_30q)(args, T, cn, workloads)
    steps = args.steps if args.steps is not None else w["steps_default"]
    free, _total = torch.cuda.mem_get_info()
    ws_bytes = int(min(free - (12 << 30), 200 << 30))
    ws = torch.empty(ws_bytes, dtype=torch.uint8, device=dev)
    ctx = T.tnc_create(0, ws, stream=torch.cuda.Stream())
    log(f"workload {w['name']}: {len(w['sliced'])} sliced labels, workspace {ws_bytes / 2**30:.0f} GiB")

    forms = [args.prec] + [p for p in args.compare.split(",") if p and p != args.prec]
    res = {}
    for prec in forms:
        if prec == "c64" and w["name"] == "53q":
            # complex64 runs the same sliced path (one slice in flight); if one
            # slice does not fit the workspace, labels are recomputed per pass
            # (Sec. 3.4.1) until it does; time 2 slices after 2 warm ones
            rec = None
            try:
                r = run_form(T, ctx, w, prec, w["sliced"], 2, 1, 1, torch)
            except T.TncError as e:
                if e.code != -2:
                    raise
                rec = T.tnc_recompute_path(w["net"], w["ssa"], w["sliced"], w["open_q"], 32)
                r = run_form(T, ctx, w, prec, w["sliced"], 2, 1, 1, torch, recompute=rec)
            r["recompute"] = None if rec is None else [int(x) for x in rec]
            r["per_original_slice"] = r["seconds"] / r["slices"]
        else:
            r = run_form(T, ctx, w, prec, w["sliced"], w["per_step"], steps if prec == args.prec else 1,
                         args.warmup if prec == args.prec else 1, torch)
            r["per_original_slice"] = r["seconds"] / r["slices"]
        res[prec] = r
        log(f"{prec}: {r['seconds'] / r['slices'] * 1e3:.2f} ms per slice run, "
            f"{r['flops'] / r['seconds'] / 1e12:.2f} TFLOP/s, tune {r['info']['tune_seconds']:.1f} s")
    main_r = res[args.prec]

    # fidelity: the stored oracle amplitudes (30q) or the complex64 run of slice 0 (53q)
    bits = w["bits"]
    ref, ref_kind = None, None
    if w["name"] == "30q":
        gold = os.path.join(ROOT, "tests", "golden", "config2_amplitudes.npy")
        if os.path.exists(gold):
            ref = np.load(gold)
            ref_kind = "oracle (FP64 state vector, stored)"
    if ref is None and "c64" in res:
        if w["name"] == "53q":
            ref, _ = T.tnc_execute(res["c64"]["plan"], bits, 0, 1)
            ref_kind = "complex64 GPU run of slice 0; no full oracle for 53 qubits"
        else:
            ref, _ = T.tnc_execute(res["c64"]["plan"], bits, 0, main_r["slices"])
            ref_kind = "complex64 GPU run"

    def fid(prec):
        if ref is None or prec == "c64":
            return None, None
        n = 1 if w["name"] == "53q" else 1 << len(w["sliced"])
        o, _ = T.tnc_execute(res[prec]["plan"], bits, 0, n)
        b = ref.ravel()
        f = abs(np.vdot(b, o)) ** 2 / (np.vdot(b, b).real * np.vdot(o, o).real)
        return float(f), float(np.linalg.norm(o - b) / np.linalg.norm(b))

    forms_out = {}
    for prec, r in res.items():
        f, rl = fid(prec)
        forms_out[prec] = {"tflops": round(r["flops"] / r["seconds"] / 1e12, 3),
                           "s_per_slice": r["per_original_slice"], "slices_timed": r["slices"],
                           "fidelity": None if f is None else round(f, 9), "rel_l2": rl, "replays": r["replays"],
                           "slices_in_flight": r["info"]["slices_in_flight"],
                           "tune_seconds": round(r["info"]["tune_seconds"], 2),
                           "peak_bytes": r["info"]["peak_bytes"]}
        if r.get("recompute"):
            forms_out[prec]["recompute_labels"] = r["recompute"]
    if "c64" in res and args.prec != "c64":
        forms_out[args.prec]["speedup_vs_c64"] = round(res["c64"]["per_original_slice"] / main_r["per_original_slice"], 3)

    dkey = DKEY[args.prec]
    fam = timed_kernels(T, main_r["plan"], bits, 0, min(w["per_step"], 1 << len(w["sliced"])), dkey)
    roof = roofline_entry(fam, dkey)
    roof["traffic"] = measured_traffic(roof["kernel"], f"{w['name']}_{args.prec}")
    roof["path"] = path_roofline(T, main_r["plan"], dkey, main_r["seconds"] / main_r["slices"])

    cpu = None
    if not args.no_cpu:
        if w["name"] == "30q":
            cpu = cpu_baseline_sv(w["circuit"], main_r["flops"] / steps, main_r["slices"] // steps, args.cpu_seconds)
        else:
            cpu = cpu_baseline_einsum(main_r["info"]["flops_per_slice"], args.cpu_seconds)

    value = main_r["flops"] / main_r["seconds"] / 1e12
    line = {
        "metric": "complex-contraction TFLOPS + s/slice, fp16-MFMA vs c64, at stated fidelity",
        "value": round(value, 3),
        "unit": "TFLOP/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": args.warmup,
        "ms_per_step": round(main_r["seconds"] / steps * 1e3, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"f16_4m": "f16", "f16_3m": "f16", "bf16_4m": "bf16", "bf16_3m": "bf16", "c64": "f32"}[args.prec],
        "data": "synthetic",
        "config": {"workload": w["label"], "precision": args.prec, "slices_per_step": w["per_step"],
                   "slices_timed": main_r["slices"], "bitstrings": int(len(bits)),
                   "sliced_labels": int(len(w["sliced"])),
                   "slices_in_flight": main_r["info"]["slices_in_flight"],
                   "flops_per_slice": main_r["info"]["flops_per_slice"],
                   "peak_bytes": main_r["info"]["peak_bytes"], "max_rank": main_r["info"]["max_rank"],
                   "search_seconds": round(w["search_seconds"], 2)},
        "s_per_slice": main_r["seconds"] / main_r["slices"],
        "fidelity": forms_out[args.prec]["fidelity"],
        "fidelity_reference": ref_kind,
        "forms": forms_out,
        "roofline": roof,
        "cpu_baseline": cpu,
    }
    for r in res.values():
        T.tnc_plan_destroy(r["plan"])
    T.tnc_network_destroy(w["net"])
    T.tnc_destroy(ctx)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
