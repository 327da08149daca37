"""ctypes binding of libtnc (argument marshalling only).

Every function here has the name of the C entry point it wraps and does no
arithmetic of its own: it converts numpy arrays and torch tensors to
pointers, calls the library, raises ``TncError`` on a nonzero return code and
returns the outputs.  The library is loaded from this package directory;
importing this module fails loudly when it has not been built.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
# TNC_LIB names another build of the library (the host-code sanitizer build
# that the CPU tests load); the default is the in-tree libtnc.so
LIB_PATH = os.environ.get("TNC_LIB") or os.path.join(HERE, "libtnc.so")

TNC_C64, TNC_F16_4M, TNC_F16_3M, TNC_BF16_4M, TNC_BF16_3M = 0, 1, 2, 3, 4
PRECISIONS = {"c64": TNC_C64, "f16_4m": TNC_F16_4M, "f16_3m": TNC_F16_3M, "bf16_4m": TNC_BF16_4M,
              "bf16_3m": TNC_BF16_3M}
ERRORS = {-1: "EINVAL", -2: "ENOMEM", -3: "EDEVICE", -4: "EOVERFLOW", -5: "EUNSUPPORTED"}
MLP_FEATURES = 8
MLP_HIDDEN = 128

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is not built: run __graft_entry__.build() (hipcc, gfx950)")

# libtnc.so needs the HIP runtime by its soname, libamdhip64.so.7.  torch ships
# its own copy of that runtime (same soname, different file) and loads it by
# path.  Loading torch first lets the dynamic loader satisfy libtnc.so's need
# with torch's copy, so the process holds one HIP runtime and one ROCr, and
# device memory and streams that torch hands over are valid in the library.
# Loading libtnc.so first would map /opt/rocm's copies beside torch's, and the
# library's runtime would then see no device.
import torch  # noqa: E402,F401

lib = ctypes.CDLL(LIB_PATH)

c_int32_p = ctypes.POINTER(ctypes.c_int32)
c_double_p = ctypes.POINTER(ctypes.c_double)
c_float_p = ctypes.POINTER(ctypes.c_float)
c_u64_p = ctypes.POINTER(ctypes.c_uint64)
vp = ctypes.c_void_p


class tnc_plan_stats(ctypes.Structure):
    _fields_ = [("n_steps", ctypes.c_int32), ("n_dep_steps", ctypes.c_int32), ("n_sliced", ctypes.c_int32),
                ("max_rank", ctypes.c_int32), ("slices_in_flight", ctypes.c_int32), ("out_rank", ctypes.c_int32),
                ("flops_per_slice", ctypes.c_double), ("flops_invariant", ctypes.c_double),
                ("bytes_per_slice", ctypes.c_double), ("permute_bytes_per_slice", ctypes.c_double),
                ("peak_bytes", ctypes.c_double), ("peak_elems_per_slice", ctypes.c_double),
                ("tune_seconds", ctypes.c_double), ("n_host_steps", ctypes.c_int32),
                ("n_recompute", ctypes.c_int32), ("n_padded_steps", ctypes.c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class tnc_report(ctypes.Structure):
    _fields_ = [("seconds", ctypes.c_double), ("flops", ctypes.c_double), ("slices", ctypes.c_int64),
                ("replays", ctypes.c_int32), ("graph_launches", ctypes.c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_SIGS = {
    "tnc_last_error": (ctypes.c_char_p, []),
    "tnc_version": (ctypes.c_char_p, []),
    "tnc_create": (ctypes.c_int, [ctypes.POINTER(vp), ctypes.c_int, vp, ctypes.c_size_t, vp]),
    "tnc_destroy": (ctypes.c_int, [vp]),
    "tnc_network_create": (ctypes.c_int, [ctypes.c_int32, c_int32_p, c_int32_p, c_double_p, ctypes.c_int32,
                                          c_int32_p, ctypes.POINTER(vp)]),
    "tnc_network_destroy": (ctypes.c_int, [vp]),
    "tnc_search": (ctypes.c_int, [vp, ctypes.c_int32, c_int32_p, ctypes.c_double, ctypes.c_int32, ctypes.c_int32,
                                  ctypes.c_uint64, c_int32_p, ctypes.c_int32, c_int32_p, c_int32_p, c_double_p]),
    "tnc_slice_path": (ctypes.c_int, [vp, ctypes.c_int32, c_int32_p, ctypes.c_int32, c_int32_p, ctypes.c_double,
                                      ctypes.c_int32, c_int32_p, ctypes.c_int32, c_int32_p, c_int32_p]),
    "tnc_plan_create": (ctypes.c_int, [vp, vp, ctypes.c_int32, c_int32_p, ctypes.c_int32, c_int32_p,
                                       ctypes.c_int32, c_int32_p, ctypes.c_int, ctypes.c_int32,
                                       ctypes.POINTER(vp)]),
    "tnc_plan_create_recompute": (ctypes.c_int, [vp, vp, ctypes.c_int32, c_int32_p, ctypes.c_int32, c_int32_p,
                                                 ctypes.c_int32, c_int32_p, ctypes.c_int32, c_int32_p, ctypes.c_int,
                                                 ctypes.c_int32, ctypes.POINTER(vp)]),
    "tnc_plan_analyze_recompute": (ctypes.c_int, [vp, ctypes.c_int32, c_int32_p, ctypes.c_int32, c_int32_p,
                                                  ctypes.c_int32, c_int32_p, ctypes.c_int32, c_int32_p, ctypes.c_int,
                                                  ctypes.POINTER(tnc_plan_stats)]),
    "tnc_recompute_path": (ctypes.c_int, [vp, ctypes.c_int32, c_int32_p, ctypes.c_int32, c_int32_p, ctypes.c_int32,
                                          c_int32_p, ctypes.c_double, ctypes.c_int32, c_int32_p, c_int32_p]),
    "tnc_plan_create_sparse": (ctypes.c_int, [vp, vp, ctypes.c_int32, c_int32_p, ctypes.c_int32, c_int32_p,
                                              ctypes.c_int64, c_u64_p, ctypes.c_int, ctypes.c_int32,
                                              ctypes.POINTER(vp)]),
    "tnc_plan_analyze_sparse": (ctypes.c_int, [vp, ctypes.c_int32, c_int32_p, ctypes.c_int32, c_int32_p,
                                               ctypes.c_int64, c_u64_p, ctypes.c_int, ctypes.POINTER(tnc_plan_stats)]),
    "tnc_plan_destroy": (ctypes.c_int, [vp]),
    "tnc_plan_info": (ctypes.c_int, [vp, ctypes.POINTER(tnc_plan_stats)]),
    "tnc_plan_analyze": (ctypes.c_int, [vp, ctypes.c_int32, c_int32_p, ctypes.c_int32, c_int32_p, ctypes.c_int32,
                                        c_int32_p, ctypes.c_int, ctypes.POINTER(tnc_plan_stats)]),
    "tnc_execute": (ctypes.c_int, [vp, ctypes.c_int64, c_u64_p, ctypes.c_int64, ctypes.c_int64, vp,
                                   ctypes.POINTER(tnc_report)]),
    "tnc_quant_sizes": (ctypes.c_int, [ctypes.c_int32, ctypes.c_int64, ctypes.c_int32,
                                       ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int64)]),
    "tnc_quantize": (ctypes.c_int, [vp, ctypes.c_int32, ctypes.c_int64, vp, ctypes.c_int32, vp, vp, vp, c_double_p]),
    "tnc_quantize_noalloc": (ctypes.c_int, [ctypes.c_int32, ctypes.c_int64, vp, ctypes.c_int32, vp, vp, vp, vp]),
    "tnc_dequantize": (ctypes.c_int, [vp, ctypes.c_int32, ctypes.c_int64, vp, vp, vp, ctypes.c_int32, vp,
                                      c_double_p]),
    "tnc_plan_set_codec": (ctypes.c_int, [vp, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32]),
    "tnc_topk": (ctypes.c_int, [vp, ctypes.c_int64, vp, ctypes.c_int32, vp, vp, c_double_p]),
    "tnc_plan_set_timing": (ctypes.c_int, [vp, ctypes.c_int32]),
    "tnc_plan_get_growth": (ctypes.c_int, [vp, ctypes.c_int32, c_int32_p]),
    "tnc_plan_set_growth": (ctypes.c_int, [vp, ctypes.c_int32, c_int32_p]),
    "tnc_plan_step_times": (ctypes.c_int, [vp, ctypes.c_int32, c_double_p, c_double_p, c_int32_p]),
    "tnc_plan_steps": (ctypes.c_int, [vp, ctypes.c_int32, c_int32_p, c_int32_p, c_int32_p, c_int32_p, c_double_p,
                                      c_double_p]),
    "tnc_plan_analyze_steps": (ctypes.c_int, [vp, ctypes.c_int32, c_int32_p, ctypes.c_int32, c_int32_p,
                                              ctypes.c_int32, c_int32_p, ctypes.c_int, c_int32_p, c_int32_p,
                                              c_int32_p, c_int32_p, c_double_p, c_double_p]),
    "tnc_contract": (ctypes.c_int, [vp, ctypes.c_int, vp, ctypes.c_int32, c_int32_p, vp, ctypes.c_int32, c_int32_p,
                                    vp, ctypes.c_int32, c_int32_p, ctypes.c_int32, c_double_p, c_float_p]),
    "tnc_mlp_train": (ctypes.c_int, [vp, ctypes.c_int64, c_float_p, c_float_p, ctypes.c_int32, ctypes.c_int32,
                                     ctypes.c_float, ctypes.c_uint64, c_float_p]),
    "tnc_mlp_adam": (ctypes.c_int, [vp, ctypes.c_int64, c_float_p, c_float_p, ctypes.c_int32, ctypes.c_float,
                                    c_float_p]),
    "tnc_mlp_predict": (ctypes.c_int, [vp, ctypes.c_int64, c_float_p, c_float_p]),
    "tnc_costmodel_base": (ctypes.c_int, [ctypes.c_int64, c_float_p, c_float_p]),
    "tnc_mlp_grad": (ctypes.c_int, [vp, ctypes.c_int64, c_float_p, c_float_p, c_float_p, c_float_p]),
    "tnc_mlp_param_count": (ctypes.c_int64, []),
    "tnc_mlp_get_params": (ctypes.c_int, [vp, c_float_p]),
    "tnc_mlp_set_params": (ctypes.c_int, [vp, c_float_p]),
    "tnc_costmodel_use": (ctypes.c_int, [vp]),
}
for _name, (_res, _args) in _SIGS.items():
    _f = getattr(lib, _name)
    _f.restype = _res
    _f.argtypes = _args

EXPORTED = tuple(_SIGS)


class TncError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{ERRORS.get(code, code)}: {msg}")
        self.code = code


def _check(rc):
    if rc != 0:
        raise TncError(rc, lib.tnc_last_error().decode())


def _i32(a):
    a = np.ascontiguousarray(a, dtype=np.int32)
    return a, a.ctypes.data_as(c_int32_p)


def _dptr(t):
    """Device pointer of a torch tensor, or an int address."""
    return ctypes.c_void_p(t if isinstance(t, int) else t.data_ptr())


def tnc_last_error() -> str:
    return lib.tnc_last_error().decode()


def tnc_version() -> str:
    return lib.tnc_version().decode()


def tnc_create(device: int, workspace=None, workspace_bytes: int = 0, stream=None):
    """workspace: torch uint8 tensor on the device (caller keeps it alive);
    stream: torch.cuda.Stream, an int hipStream_t, or None."""
    h = vp()
    ws = vp(0) if workspace is None else _dptr(workspace)
    nbytes = workspace_bytes if workspace is None else workspace.numel() * workspace.element_size()
    if stream is None:
        sp = vp(0)
    elif isinstance(stream, int):
        sp = vp(stream)
    else:
        sp = vp(stream.cuda_stream)
    _check(lib.tnc_create(ctypes.byref(h), int(device), ws, ctypes.c_size_t(nbytes), sp))
    return h


def tnc_destroy(ctx):
    _check(lib.tnc_destroy(ctx))


def tnc_network_create(ranks, labels, data_c128, n_qubits, output_labels):
    r, rp = _i32(ranks)
    lab, lp = _i32(labels)
    d = None
    dp = None
    if data_c128 is not None:
        d = np.ascontiguousarray(data_c128, dtype=np.float64)
        need = 2 * sum(1 << int(x) for x in r if 0 <= int(x) <= 30)
        if d.size != need:
            raise ValueError(f"data_c128 holds {d.size} doubles, the ranks need {need}")
        dp = d.ctypes.data_as(c_double_p)
    if int(np.sum(r)) != len(lab):
        raise ValueError("labels must hold sum(ranks) entries")
    o, op = _i32(output_labels)
    h = vp()
    _check(lib.tnc_network_create(len(r), rp, lp, dp, int(n_qubits), op, ctypes.byref(h)))
    return h


def tnc_network_destroy(net):
    _check(lib.tnc_network_destroy(net))


def tnc_search(net, n_tensors, open_qubits, log2_cap, cost_model=0, restarts=8, seed=0, max_sliced=62):
    oq, op = _i32(open_qubits)
    ssa = np.zeros(2 * (n_tensors - 1), dtype=np.int32)
    sl = np.zeros(max(max_sliced, 1), dtype=np.int32)
    ns = ctypes.c_int32(0)
    cost = ctypes.c_double(0)
    _check(lib.tnc_search(net, len(oq), op, float(log2_cap), int(cost_model), int(restarts), ctypes.c_uint64(seed),
                          ssa.ctypes.data_as(c_int32_p), int(max_sliced), sl.ctypes.data_as(c_int32_p),
                          ctypes.byref(ns), ctypes.byref(cost)))
    return ssa, sl[:ns.value].copy(), cost.value


def tnc_slice_path(net, ssa, open_qubits, log2_cap, sliced_in=(), max_sliced=62):
    s, sp = _i32(ssa)
    oq, op = _i32(open_qubits)
    si, sip = _i32(list(sliced_in))
    out = np.zeros(max_sliced, dtype=np.int32)
    n = ctypes.c_int32(0)
    _check(lib.tnc_slice_path(net, len(s) // 2, sp, len(oq), op, float(log2_cap), len(si), sip, int(max_sliced),
                              out.ctypes.data_as(c_int32_p), ctypes.byref(n)))
    return out[:n.value].copy()


def tnc_plan_create(ctx, net, ssa, sliced, open_qubits, precision, max_slices_in_flight=0, recompute=None):
    """recompute: labels recomputed per pass (tnc_plan_create_recompute)."""
    s, sp = _i32(ssa)
    sl, slp = _i32(sliced)
    oq, op = _i32(open_qubits)
    prec = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
    h = vp()
    if recompute is not None and len(recompute):
        rc, rp = _i32(recompute)
        _check(lib.tnc_plan_create_recompute(ctx, net, len(s) // 2, sp, len(sl), slp, len(rc), rp, len(oq), op, prec,
                                             int(max_slices_in_flight), ctypes.byref(h)))
    else:
        _check(lib.tnc_plan_create(ctx, net, len(s) // 2, sp, len(sl), slp, len(oq), op, prec,
                                   int(max_slices_in_flight), ctypes.byref(h)))
    return h


def tnc_recompute_path(net, ssa, sliced, open_qubits, log2_cap, max_recompute=8):
    s, sp = _i32(ssa)
    sl, slp = _i32(sliced)
    oq, op = _i32(open_qubits)
    out = np.zeros(max(max_recompute, 1), dtype=np.int32)
    n = ctypes.c_int32(0)
    _check(lib.tnc_recompute_path(net, len(s) // 2, sp, len(sl), slp, len(oq), op, float(log2_cap), int(max_recompute),
                                  out.ctypes.data_as(c_int32_p), ctypes.byref(n)))
    return out[:n.value].copy()


def tnc_plan_create_sparse(ctx, net, ssa, sliced, bitstrings, precision, max_slices_in_flight=0):
    s, sp = _i32(ssa)
    sl, slp = _i32(sliced)
    b = np.ascontiguousarray(bitstrings, dtype=np.uint64)
    prec = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
    h = vp()
    _check(lib.tnc_plan_create_sparse(ctx, net, len(s) // 2, sp, len(sl), slp, len(b), b.ctypes.data_as(c_u64_p),
                                      prec, int(max_slices_in_flight), ctypes.byref(h)))
    return h


def tnc_plan_analyze_sparse(net, ssa, sliced, bitstrings, precision) -> dict:
    s, sp = _i32(ssa)
    sl, slp = _i32(sliced)
    b = np.ascontiguousarray(bitstrings, dtype=np.uint64)
    prec = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
    st = tnc_plan_stats()
    _check(lib.tnc_plan_analyze_sparse(net, len(s) // 2, sp, len(sl), slp, len(b), b.ctypes.data_as(c_u64_p), prec,
                                       ctypes.byref(st)))
    return st.as_dict()


def tnc_plan_destroy(plan):
    _check(lib.tnc_plan_destroy(plan))


def tnc_plan_info(plan) -> dict:
    st = tnc_plan_stats()
    _check(lib.tnc_plan_info(plan, ctypes.byref(st)))
    return st.as_dict()


def tnc_plan_analyze(net, ssa, sliced, open_qubits, precision, recompute=None) -> dict:
    s, sp = _i32(ssa)
    sl, slp = _i32(sliced)
    oq, op = _i32(open_qubits)
    prec = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
    st = tnc_plan_stats()
    if recompute is not None and len(recompute):
        rc, rp = _i32(recompute)
        _check(lib.tnc_plan_analyze_recompute(net, len(s) // 2, sp, len(sl), slp, len(rc), rp, len(oq), op, prec,
                                              ctypes.byref(st)))
    else:
        _check(lib.tnc_plan_analyze(net, len(s) // 2, sp, len(sl), slp, len(oq), op, prec, ctypes.byref(st)))
    return st.as_dict()


def tnc_execute(plan, bitstrings, slice_begin, slice_end, out=None):
    """out: None (a new host complex128 array is returned), a host complex128
    array, or a torch float64/complex128 device tensor of 2*n doubles."""
    b = np.ascontiguousarray(bitstrings, dtype=np.uint64)
    rep = tnc_report()
    if out is None:
        host = np.zeros(len(b), dtype=np.complex128)
        optr = vp(host.ctypes.data)
    elif isinstance(out, np.ndarray):
        assert out.dtype == np.complex128 and out.flags.c_contiguous and len(out) == len(b)
        host = out
        optr = vp(out.ctypes.data)
    else:
        host = None
        optr = _dptr(out)
    _check(lib.tnc_execute(plan, len(b), b.ctypes.data_as(c_u64_p), int(slice_begin), int(slice_end), optr,
                           ctypes.byref(rep)))
    return (host if host is not None else out), rep.as_dict()


def tnc_plan_set_timing(plan, on: bool):
    _check(lib.tnc_plan_set_timing(plan, int(bool(on))))


def tnc_plan_get_growth(plan) -> np.ndarray:
    n = tnc_plan_info(plan)["n_steps"]
    g = np.zeros(n, dtype=np.int32)
    _check(lib.tnc_plan_get_growth(plan, n, g.ctypes.data_as(c_int32_p)))
    return g


def tnc_plan_set_growth(plan, growth):
    g = np.ascontiguousarray(growth, dtype=np.int32)
    _check(lib.tnc_plan_set_growth(plan, len(g), g.ctypes.data_as(c_int32_p)))


def tnc_plan_step_times(plan, n_steps):
    """(gemm_ms, permute_ms, launches) per step of the last timed execute."""
    g = np.zeros(n_steps, dtype=np.float64)
    p = np.zeros(n_steps, dtype=np.float64)
    n = np.zeros(n_steps, dtype=np.int32)
    _check(lib.tnc_plan_step_times(plan, n_steps, g.ctypes.data_as(c_double_p), p.ctypes.data_as(c_double_p),
                                   n.ctypes.data_as(c_int32_p)))
    return g, p, n


def _step_arrays(n_steps):
    return (np.zeros(4 * n_steps, dtype=np.int32), np.zeros(n_steps, dtype=np.int32),
            np.zeros(n_steps, dtype=np.int32), np.zeros(2 * n_steps, dtype=np.int32),
            np.zeros(n_steps, dtype=np.float64), np.zeros(n_steps, dtype=np.float64))


def _step_ptrs(arrs):
    mnkb, kern, dep, pab, fl, by = arrs
    return (mnkb.ctypes.data_as(c_int32_p), kern.ctypes.data_as(c_int32_p), dep.ctypes.data_as(c_int32_p),
            pab.ctypes.data_as(c_int32_p), fl.ctypes.data_as(c_double_p), by.ctypes.data_as(c_double_p))


def _step_dict(arrs):
    mnkb, kern, dep, pab, fl, by = arrs
    return {"log2_mnkb": mnkb.reshape(-1, 4), "kernel": kern, "dep": dep, "perm_ab": pab.reshape(-1, 2),
            "flops": fl, "bytes": by}


def tnc_plan_steps(plan, n_steps) -> dict:
    """Static per-step shapes, kernels and algorithmic work."""
    arrs = _step_arrays(n_steps)
    _check(lib.tnc_plan_steps(plan, n_steps, *_step_ptrs(arrs)))
    return _step_dict(arrs)


def tnc_plan_analyze_steps(net, ssa, sliced, open_qubits, precision) -> dict:
    s, sp = _i32(ssa)
    sl, slp = _i32(sliced)
    oq, op = _i32(open_qubits)
    prec = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
    n_steps = len(s) // 2
    arrs = _step_arrays(n_steps)
    _check(lib.tnc_plan_analyze_steps(net, n_steps, sp, len(sl), slp, len(oq), op, prec, *_step_ptrs(arrs)))
    return _step_dict(arrs)


def tnc_contract(ctx, precision, A, a_labels, B, b_labels, C, c_labels, scale_log2=0):
    al, ap = _i32(a_labels)
    bl, bp = _i32(b_labels)
    cl, cp = _i32(c_labels)
    prec = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
    times = np.zeros(4, dtype=np.float64)
    mx = ctypes.c_float(0)
    _check(lib.tnc_contract(ctx, prec, _dptr(A), len(al), ap, _dptr(B), len(bl), bp, _dptr(C), len(cl), cp,
                            int(scale_log2), times.ctypes.data_as(c_double_p), ctypes.byref(mx)))
    return times, mx.value


def tnc_mlp_param_count() -> int:
    return int(lib.tnc_mlp_param_count())


def _f32(a):
    a = np.ascontiguousarray(a, dtype=np.float32)
    return a, a.ctypes.data_as(c_float_p)


def tnc_mlp_train(ctx, x, y, epochs, batch, lr, seed):
    xa, xp = _f32(x)
    ya, yp = _f32(y)
    loss = ctypes.c_float(0)
    _check(lib.tnc_mlp_train(ctx, len(ya), xp, yp, int(epochs), int(batch), float(lr), ctypes.c_uint64(seed),
                             ctypes.byref(loss)))
    return loss.value


def tnc_mlp_adam(ctx, x, y, steps, lr):
    xa, xp = _f32(x)
    ya, yp = _f32(y)
    loss = ctypes.c_float(0)
    _check(lib.tnc_mlp_adam(ctx, len(ya), xp, yp, int(steps), float(lr), ctypes.byref(loss)))
    return loss.value


def tnc_mlp_predict(ctx, x):
    xa, xp = _f32(x)
    n = xa.shape[0]
    y = np.zeros(n, dtype=np.float32)
    _check(lib.tnc_mlp_predict(ctx, n, xp, y.ctypes.data_as(c_float_p)))
    return y


def tnc_costmodel_base(x):
    """Roofline baseline (log2 us) of feature rows: the part of the search's
    step cost that the MLP does not learn."""
    xa, xp = _f32(x)
    n = xa.shape[0]
    y = np.zeros(n, dtype=np.float32)
    _check(lib.tnc_costmodel_base(n, xp, y.ctypes.data_as(c_float_p)))
    return y


def tnc_mlp_grad(ctx, x, y):
    xa, xp = _f32(x)
    ya, yp = _f32(y)
    g = np.zeros(tnc_mlp_param_count(), dtype=np.float32)
    loss = ctypes.c_float(0)
    _check(lib.tnc_mlp_grad(ctx, len(ya), xp, yp, ctypes.byref(loss), g.ctypes.data_as(c_float_p)))
    return loss.value, g


def tnc_mlp_get_params(ctx):
    p = np.zeros(tnc_mlp_param_count(), dtype=np.float32)
    _check(lib.tnc_mlp_get_params(ctx, p.ctypes.data_as(c_float_p)))
    return p


def tnc_mlp_set_params(ctx, params):
    pa, pp = _f32(params)
    assert len(pa) == tnc_mlp_param_count()
    _check(lib.tnc_mlp_set_params(ctx, pp))


def tnc_costmodel_use(ctx):
    _check(lib.tnc_costmodel_use(ctx))


QKINDS = {"half": 0, "int8": 1, "int4": 2}


def tnc_quant_sizes(kind, n, group=0):
    cb, ng = ctypes.c_int64(0), ctypes.c_int64(0)
    _check(lib.tnc_quant_sizes(QKINDS.get(kind, kind), int(n), int(group), ctypes.byref(cb), ctypes.byref(ng)))
    return cb.value, ng.value


def tnc_quantize(ctx, kind, x, group=0):
    """x: contiguous float32 device tensor.  Returns (codes uint8 tensor,
    scales, zeros (float32 tensors), device ms)."""
    import torch
    k = QKINDS.get(kind, kind)
    n = x.numel()
    cb, ng = tnc_quant_sizes(k, n, group)
    codes = torch.empty(max(cb, 16), dtype=torch.uint8, device=x.device)
    scales = torch.empty(max(ng, 1), dtype=torch.float32, device=x.device)
    zeros = torch.empty(max(ng, 1), dtype=torch.float32, device=x.device)
    torch.cuda.synchronize(x.device)
    ms = ctypes.c_double(0)
    _check(lib.tnc_quantize(ctx, k, n, _dptr(x), int(group), _dptr(codes), _dptr(scales), _dptr(zeros),
                            ctypes.byref(ms)))
    return codes[:cb], scales[:ng], zeros[:ng], ms.value


def tnc_quantize_noalloc(kind, x, codes, scales, zeros, group=0, stream=None):
    """The allocation-free quantize: x, codes, scales, zeros are caller-owned
    device tensors (sizes from tnc_quant_sizes); the work is enqueued on
    `stream` (a torch stream, None = the null stream) without waiting."""
    k = QKINDS.get(kind, kind)
    sp = ctypes.c_void_p(stream.cuda_stream) if stream is not None else None
    _check(lib.tnc_quantize_noalloc(k, x.numel(), _dptr(x), int(group), _dptr(codes), _dptr(scales), _dptr(zeros),
                                    sp))


def tnc_dequantize(ctx, kind, n, codes, scales, zeros, group=0):
    """Returns (float32 device tensor of n values, device ms)."""
    import torch
    k = QKINDS.get(kind, kind)
    x = torch.empty(max(n, 4), dtype=torch.float32, device=codes.device)
    torch.cuda.synchronize(codes.device)
    ms = ctypes.c_double(0)
    _check(lib.tnc_dequantize(ctx, k, int(n), _dptr(codes), _dptr(scales), _dptr(zeros), int(group), _dptr(x),
                              ctypes.byref(ms)))
    return x[:n], ms.value


def tnc_plan_set_codec(plan, step, kind="int4", group=0):
    _check(lib.tnc_plan_set_codec(plan, int(step), QKINDS.get(kind, kind), int(group)))


def tnc_topk(ctx, amps, k):
    """Top-k post-selection of device complex128 amplitudes (a torch tensor on
    the context's device); returns (indices, probabilities, ms) as torch
    tensors on that device."""
    import torch
    assert amps.dtype == torch.complex128 and amps.is_contiguous()
    n = amps.numel()
    kk = min(int(k), n)
    idx = torch.empty(max(kk, 1), dtype=torch.int64, device=amps.device)
    prob = torch.empty(max(kk, 1), dtype=torch.float64, device=amps.device)
    ms = ctypes.c_double(0.0)
    torch.cuda.synchronize(amps.device)
    _check(lib.tnc_topk(ctx, n, ctypes.c_void_p(amps.data_ptr()), int(k), ctypes.c_void_p(idx.data_ptr()),
                        ctypes.c_void_p(prob.data_ptr()), ctypes.byref(ms)))
    return idx[:kk], prob[:kk], ms.value
