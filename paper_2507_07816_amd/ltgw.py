"""ctypes binding of the ltgw C ABI (include/ltgw.h), names as in the header.

Argument marshalling only: every step of the search runs in the HIP library
``libltgw.so`` built next to this file.  Arrays may be numpy arrays or torch
tensors (host or device); device tensors are passed by address.  If the
library is missing the import of this module fails loudly: there is no
fallback implementation.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libltgw.so")

LTGW_OK = 0
LTGW_E_INVALID_ARG = -1
LTGW_E_STATE = -2
LTGW_E_NOMEM = -3
LTGW_E_DEVICE = -4
LTGW_E_UNSUPPORTED = -5
LTGW_E_IO = -6

LTGW_STORE_F32 = 0
LTGW_STORE_BF16 = 1
LTGW_STORE_FP8 = 2
STORES = {"f32": LTGW_STORE_F32, "bf16": LTGW_STORE_BF16, "fp8": LTGW_STORE_FP8}

LTGW_STAT_POWER = 1
LTGW_STAT_COUNT = 2
STATS = {"power": LTGW_STAT_POWER, "count": LTGW_STAT_COUNT}

LTGW_MAX_DET = 256
LTGW_MAX_SEARCH_DET = 4
LTGW_MAX_TOPK = 256
LTGW_NOALLOC_SCRATCH_BYTES = 256 << 20
LTGW_NOALLOC_MAX_AXIS = 4096
TILE_SHAPES = {0: (1, 8), 1: (1, 16), 2: (2, 8), 3: (2, 16)}  # (templates per lane, segments per batch)

# every symbol include/ltgw.h declares
EXPORTS = ("ltgw_create", "ltgw_destroy", "ltgw_last_error", "ltgw_load_spectrogram",
           "ltgw_set_velocity_table", "ltgw_set_antenna", "ltgw_sft_normalise", "ltgw_eval_templates", "ltgw_psi",
           "ltgw_topk_candidates", "ltgw_diagnostics", "ltgw_inject_track", "ltgw_read_store", "ltgw_read_tables",
           "ltgw_eval_batch", "ltgw_batch_results", "ltgw_batch_latency", "ltgw_autotune",
           "ltgw_set_tile_shape", "ltgw_tune_save", "ltgw_tune_load",
           "ltgw_generate_noise", "ltgw_inject_stack", "ltgw_load_stack", "ltgw_stack_psi",
           "ltgw_stack_psi_list", "ltgw_cnn_param_count", "ltgw_cnn_work_floats", "ltgw_cnn_forward",
           "ltgw_cnn_backward", "ltgw_softmax_xent", "ltgw_adam_step", "ltgw_select_top",
           "ltgw_propose", "ltgw_stack_features", "ltgw_stack_best", "ltgw_cells_from_templates",
           "ltgw_eval_list", "ltgw_eval_templates_noalloc", "ltgw_proposer_save", "ltgw_proposer_load")


class ltgw_spec_desc(C.Structure):
    _fields_ = [("n_seg", C.c_int32), ("n_bins", C.c_int32), ("k_lo", C.c_int64),
                ("t_sft", C.c_double), ("t_seg", C.c_void_p), ("weights", C.c_void_p),
                ("rho_th", C.c_float), ("store", C.c_int32)]


class ltgw_template(C.Structure):
    _fields_ = [("f0", C.c_double), ("tau", C.c_double), ("brake", C.c_double), ("sky", C.c_double * 3)]


class ltgw_grid(C.Structure):
    _fields_ = [("f0_min", C.c_double), ("f0_step", C.c_double), ("n_f0", C.c_int32),
                ("tau", C.c_void_p), ("n_tau", C.c_int32), ("brake", C.c_void_p),
                ("n_brake", C.c_int32), ("sky", C.c_void_p), ("n_sky", C.c_int32),
                ("t0", C.c_double), ("det_mask", C.c_uint32)]


class ltgw_candidate(C.Structure):
    _fields_ = [("index", C.c_int64), ("f0", C.c_double), ("tau", C.c_double),
                ("brake", C.c_double), ("sky", C.c_int32), ("n_valid", C.c_int32),
                ("stat", C.c_double), ("psi", C.c_double)]


class ltgw_diag(C.Structure):
    _fields_ = [("pow_undecided", C.c_int64), ("templates", C.c_int64), ("evals", C.c_int64),
                ("in_band", C.c_int64), ("eval_kernel_ms", C.c_double), ("tables_ms", C.c_double),
                ("tile_shape", C.c_int32), ("eval_launches", C.c_int32), ("ingest_ms", C.c_double),
                ("pow_slow", C.c_int64), ("pow_exact", C.c_int64)]


class ltgw_search(C.Structure):
    _fields_ = [("grid", ltgw_grid), ("dets", C.c_int32 * 4), ("n_dets", C.c_int32)]


class ltgw_batch_stats(C.Structure):
    _fields_ = [("graph_replayed", C.c_int32), ("variant", C.c_int32),
                ("templates_per_lane", C.c_int32), ("segments_per_batch", C.c_int32),
                ("workgroups", C.c_int32), ("tiles", C.c_int32), ("templates", C.c_int64),
                ("evals", C.c_int64), ("in_band", C.c_int64), ("kernel_ms", C.c_double),
                ("total_ms", C.c_double)]


class ltgw_proposer(C.Structure):
    _fields_ = [("params", C.c_void_p), ("c_in", C.c_int32), ("c_out", C.c_int32), ("L", C.c_int32),
                ("n_select", C.c_int32), ("block", C.c_int32), ("n_select2", C.c_int32),
                ("psi_threshold", C.c_double), ("coarse_threshold", C.c_double), ("tier2_threshold", C.c_double),
                ("blocks", C.c_void_p), ("coarse_map", C.c_void_p)]


class LtgwError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"ltgw error {code}: {msg}")
        self.code = code


_lib = None


def library():
    """The loaded libltgw.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with "
                              "`python -c 'import __graft_entry__ as g; g.build()'`")
        L = C.CDLL(LIB_PATH)
        P, i32, u32, d, f = C.c_void_p, C.c_int32, C.c_uint32, C.c_double, C.c_float
        sig = {
            "ltgw_create": (i32, [i32, P, C.POINTER(P)]),
            "ltgw_destroy": (None, [P]),
            "ltgw_last_error": (C.c_char_p, [P]),
            "ltgw_load_spectrogram": (i32, [P, i32, C.POINTER(ltgw_spec_desc), P]),
            "ltgw_set_velocity_table": (i32, [P, i32, P, i32]),
            "ltgw_set_antenna": (i32, [P, i32, P, P, i32]),
            "ltgw_sft_normalise": (i32, [P, P, i32, i32, C.c_int64, i32, i32, P]),
            "ltgw_eval_templates": (i32, [P, C.POINTER(ltgw_grid), u32, P, P, P]),
            "ltgw_eval_templates_noalloc": (i32, [P, C.POINTER(ltgw_grid), u32, P, P, P]),
            "ltgw_proposer_save": (i32, [P, C.c_char_p, P, i32, i32]),
            "ltgw_proposer_load": (i32, [P, C.c_char_p, C.POINTER(i32), C.POINTER(i32), P, C.c_int64]),
            "ltgw_eval_list": (i32, [P, P, C.c_int64, d, u32, P, P, P]),
            "ltgw_psi": (i32, [P, u32, P]),
            "ltgw_topk_candidates": (i32, [P, u32, i32, C.POINTER(ltgw_candidate), C.POINTER(i32)]),
            "ltgw_diagnostics": (i32, [P, C.POINTER(ltgw_diag)]),
            "ltgw_inject_track": (i32, [P, i32, P, d, d, d, P, d, f]),
            "ltgw_read_store": (i32, [P, i32, P, P]),
            "ltgw_read_tables": (i32, [P, i32, P, P, P]),
            "ltgw_eval_batch": (i32, [P, P, i32, i32, P, P, P, P, C.POINTER(ltgw_batch_stats)]),
            "ltgw_batch_results": (i32, [P, i32, P, P, P, P, P]),
            "ltgw_batch_latency": (i32, [P, P]),
            "ltgw_autotune": (i32, [P, C.POINTER(ltgw_grid), C.POINTER(i32)]),
            "ltgw_set_tile_shape": (i32, [P, i32]),
            "ltgw_tune_save": (i32, [P, C.c_char_p]),
            "ltgw_tune_load": (i32, [P, C.c_char_p]),
            "ltgw_generate_noise": (i32, [P, C.c_uint64, u32, i32, i32, C.c_int64, P]),
            "ltgw_inject_stack": (i32, [P, i32, P, i32, P, P, d]),
            "ltgw_load_stack": (i32, [P, i32, i32, P, i32, i32]),
            "ltgw_stack_psi": (i32, [P, C.POINTER(ltgw_grid), i32, i32, P]),
            "ltgw_stack_psi_list": (i32, [P, C.POINTER(ltgw_grid), u32, P, i32, P]),
            "ltgw_cnn_param_count": (C.c_int64, [i32, i32]),
            "ltgw_cnn_work_floats": (C.c_int64, [i32, i32, i32, i32]),
            "ltgw_cnn_forward": (i32, [P, P, P, i32, i32, i32, i32, P, P]),
            "ltgw_cnn_backward": (i32, [P, P, P, i32, i32, i32, i32, P, P, P, C.c_int64, P]),
            "ltgw_softmax_xent": (i32, [P, P, i32, i32, P, i32, P, P]),
            "ltgw_adam_step": (i32, [P, P, P, P, P, C.c_int64, f, f, f, f, i32]),
            "ltgw_select_top": (i32, [P, P, i32, i32, i32, P]),
            "ltgw_stack_features": (i32, [P, C.POINTER(ltgw_grid), i32, P]),
            "ltgw_stack_best": (i32, [P, C.POINTER(ltgw_grid), u32, P, P]),
            "ltgw_cells_from_templates": (i32, [P, P, i32, i32, P, P, d, P]),
            "ltgw_propose": (i32, [P, C.POINTER(ltgw_grid), C.POINTER(ltgw_grid), C.POINTER(ltgw_proposer),
                                   P, P, P]),
        }
        for name, (res, args) in sig.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


# ---------------------------------------------------------------------------
def _addr(x):
    """(address, keep-alive) of a numpy array / torch tensor / None."""
    if x is None:
        return None, None
    if hasattr(x, "data_ptr"):
        if not x.is_contiguous():
            raise ValueError("tensor must be contiguous")
        return x.data_ptr(), x
    a = np.ascontiguousarray(x)
    return a.ctypes.data, a


def _check(ctx, rc):
    if rc != LTGW_OK:
        msg = library().ltgw_last_error(ctx)
        raise LtgwError(rc, msg.decode() if msg else "")


def ltgw_create(device=0, stream=None):
    """Context handle on `device`; `stream` is a hipStream_t address (int) or None."""
    h = C.c_void_p()
    rc = library().ltgw_create(int(device), C.c_void_p(stream) if stream else None, C.byref(h))
    _check(None, rc)
    return h


def ltgw_destroy(ctx):
    library().ltgw_destroy(ctx)


def ltgw_last_error(ctx):
    m = library().ltgw_last_error(ctx)
    return m.decode() if m else ""


def ltgw_load_spectrogram(ctx, det, power, k_lo, t_sft, t_seg, weights=None, rho_th=1.6,
                          store="f32"):
    if hasattr(power, "dtype") and str(power.dtype) not in ("float32", "torch.float32"):
        raise TypeError("power must be float32")
    n_seg, n_bins = (int(power.shape[0]), int(power.shape[1]))
    t_seg = np.ascontiguousarray(t_seg, dtype=np.float64) if not hasattr(t_seg, "data_ptr") else t_seg
    if weights is not None and not hasattr(weights, "data_ptr"):
        weights = np.ascontiguousarray(weights, dtype=np.float32)
    pp, kp = _addr(power)
    tp, kt = _addr(t_seg)
    wp, kw = _addr(weights)
    d = ltgw_spec_desc(n_seg, n_bins, int(k_lo), float(t_sft), tp, wp, float(np.float32(rho_th)),
                       STORES[store] if isinstance(store, str) else int(store))
    _check(ctx, library().ltgw_load_spectrogram(ctx, int(det), C.byref(d), pp))


def ltgw_set_velocity_table(ctx, det, v):
    if not hasattr(v, "data_ptr"):
        v = np.ascontiguousarray(v, dtype=np.float64)
    vp, kv = _addr(v)
    _check(ctx, library().ltgw_set_velocity_table(ctx, int(det), vp, int(v.shape[0])))


def ltgw_set_antenna(ctx, det, arms, era):
    """arms: [2][3] Earth-fixed unit arm vectors (host), or None to clear;
    era: [n_seg] Earth rotation angles (host array or device tensor)."""
    if arms is None:
        _check(ctx, library().ltgw_set_antenna(ctx, int(det), None, None, 0))
        return
    a = np.ascontiguousarray(arms, dtype=np.float64).reshape(6)
    if not hasattr(era, "data_ptr"):
        era = np.ascontiguousarray(era, dtype=np.float64)
    ep, ke = _addr(era)
    _check(ctx, library().ltgw_set_antenna(ctx, int(det), a.ctypes.data, ep, int(era.shape[0])))


def ltgw_sft_normalise(ctx, strain, n_seg, n_fft, k_lo, n_bins, window, out):
    """strain: device FP32 [n_seg * n_fft]; out: device FP32 [n_seg][n_bins]."""
    sp, _a = _addr(strain)
    op, _b = _addr(out)
    _check(ctx, library().ltgw_sft_normalise(ctx, sp, int(n_seg), int(n_fft), int(k_lo), int(n_bins), int(window), op))


def make_grid(f0_min, f0_step, n_f0, tau, brake, sky, t0=0.0, det_mask=0):
    """(ltgw_grid, keep-alive arrays) for the cubic lattice bank."""
    tau = np.ascontiguousarray(tau, dtype=np.float64)
    brake = np.ascontiguousarray(brake, dtype=np.float64)
    sky = np.ascontiguousarray(sky, dtype=np.float64).reshape(-1, 3)
    g = ltgw_grid(float(f0_min), float(f0_step), int(n_f0), tau.ctypes.data, len(tau),
                  brake.ctypes.data, len(brake), sky.ctypes.data, len(sky), float(t0),
                  int(det_mask))
    return g, (tau, brake, sky)


def ltgw_eval_templates(ctx, grid, stats=LTGW_STAT_POWER | LTGW_STAT_COUNT, out_s=None,
                        out_c=None, out_n=None):
    sp, _a = _addr(out_s)
    cp, _b = _addr(out_c)
    np_, _c = _addr(out_n)
    _check(ctx, library().ltgw_eval_templates(ctx, C.byref(grid), int(stats), sp, cp, np_))


def ltgw_eval_templates_noalloc(ctx, grid, stats=LTGW_STAT_POWER | LTGW_STAT_COUNT, out_s=None,
                                out_c=None, out_n=None):
    sp, _a = _addr(out_s)
    cp, _b = _addr(out_c)
    np_, _c = _addr(out_n)
    _check(ctx, library().ltgw_eval_templates_noalloc(ctx, C.byref(grid), int(stats), sp, cp, np_))


def ltgw_proposer_save(ctx, path, params, c_in, c_out):
    """Write the network parameters (device tensor, or host float32 array with
    ctx None) to `path`."""
    if not hasattr(params, "data_ptr"):
        params = np.ascontiguousarray(params, dtype=np.float32)
    pp, params = _addr(params)
    _check(ctx, library().ltgw_proposer_save(ctx, os.fsencode(path), pp, int(c_in), int(c_out)))


def ltgw_proposer_load(ctx, path, params=None):
    """(c_in, c_out) of the network in `path`; with params (device tensor, or
    host float32 array with ctx None) the parameters are read into it."""
    ci, co = C.c_int32(0), C.c_int32(0)
    lib = library()
    if params is None:
        _check(ctx, lib.ltgw_proposer_load(ctx, os.fsencode(path), C.byref(ci), C.byref(co), None, 0))
        return ci.value, co.value
    if hasattr(params, "data_ptr"):
        if not params.is_contiguous():
            raise ValueError("tensor must be contiguous")
        pp, n = params.data_ptr(), params.numel()
    else:
        if not (isinstance(params, np.ndarray) and params.dtype == np.float32 and params.flags.c_contiguous):
            raise ValueError("params must be a contiguous float32 array or tensor")
        pp, n = params.ctypes.data, params.size
    _check(ctx, lib.ltgw_proposer_load(ctx, os.fsencode(path), C.byref(ci), C.byref(co), pp, int(n)))
    return ci.value, co.value


def ltgw_eval_list(ctx, params, t0=0.0, det_mask=0, out_s=None, out_c=None, out_n=None):
    """params: [n][6] host array of (f0, tau, n, sky x, y, z) (ltgw_template records)."""
    p = np.ascontiguousarray(params, dtype=np.float64).reshape(-1, 6)
    assert C.sizeof(ltgw_template) == 48
    sp, _a = _addr(out_s)
    cp, _b = _addr(out_c)
    np_, _c = _addr(out_n)
    _check(ctx, library().ltgw_eval_list(ctx, p.ctypes.data, p.shape[0], float(t0), int(det_mask), sp, cp, np_))


def ltgw_psi(ctx, stat, out_psi):
    pp, _k = _addr(out_psi)
    _check(ctx, library().ltgw_psi(ctx, STATS.get(stat, stat), pp))


def ltgw_topk_candidates(ctx, stat, k):
    """List of dicts (index, f0, tau, brake, sky, n_valid, stat, psi)."""
    arr = (ltgw_candidate * int(k))()
    n = C.c_int32()
    _check(ctx, library().ltgw_topk_candidates(ctx, STATS.get(stat, stat), int(k), arr, C.byref(n)))
    return [{f: getattr(arr[i], f) for f, _ in ltgw_candidate._fields_} for i in range(n.value)]


def ltgw_diagnostics(ctx):
    d = ltgw_diag()
    _check(ctx, library().ltgw_diagnostics(ctx, C.byref(d)))
    return {f: getattr(d, f) for f, _ in ltgw_diag._fields_}


def ltgw_inject_track(ctx, det, power, f0, tau, brake, sky, t0, amp):
    pp, _k = _addr(power)
    sky = np.ascontiguousarray(sky, dtype=np.float64)
    _check(ctx, library().ltgw_inject_track(ctx, int(det), pp, float(f0), float(tau), float(brake),
                                            sky.ctypes.data, float(t0), float(np.float32(amp))))


def ltgw_read_store(ctx, det, n_seg, n_bins, store):
    """(codes, scales) of a detector's device store as numpy arrays."""
    dt = {"f32": np.uint32, "bf16": np.uint16, "fp8": np.uint8}[store]
    out = np.empty((n_seg, n_bins), dt)
    sc = np.empty(n_seg, np.float32)
    _check(ctx, library().ltgw_read_store(ctx, int(det), out.ctypes.data, sc.ctypes.data))
    return out, sc


def ltgw_read_tables(ctx, det, n_seg):
    """(g, H) tables of the last eval on detector slot `det` as FP64 numpy
    arrays [rows][n_seg]."""
    rows = (C.c_int32 * 2)()
    _check(ctx, library().ltgw_read_tables(ctx, int(det), None, None, rows))
    g = np.empty((rows[0], int(n_seg)), np.float64)
    h = np.empty((rows[1], int(n_seg)), np.float64)
    _check(ctx, library().ltgw_read_tables(ctx, int(det), g.ctypes.data, h.ctypes.data, None))
    return g, h


def ltgw_eval_batch(ctx, searches, k):
    """searches: list of (make_grid(...) result, detector slot list).  Returns
    (top_power, top_count, stats): per-search lists of candidate dicts and a dict."""
    n = len(searches)
    arr = (ltgw_search * n)()
    keep = []
    for i, ((g, kg), dets) in enumerate(searches):
        keep.append(kg)
        arr[i].grid = g
        if not 1 <= len(dets) <= LTGW_MAX_SEARCH_DET:
            raise ValueError("a search sums 1..4 detectors")
        for q, d in enumerate(dets):
            arr[i].dets[q] = int(d)
        arr[i].n_dets = len(dets)
    tp = (ltgw_candidate * (n * k))()
    tc = (ltgw_candidate * (n * k))()
    npw = (C.c_int32 * n)()
    nct = (C.c_int32 * n)()
    st = ltgw_batch_stats()
    _check(ctx, library().ltgw_eval_batch(ctx, C.cast(arr, C.c_void_p), n, int(k), C.cast(tp, C.c_void_p),
                                          C.cast(tc, C.c_void_p), C.cast(npw, C.c_void_p),
                                          C.cast(nct, C.c_void_p), C.byref(st)))
    rec = lambda a, j: {f: getattr(a[j], f) for f, _ in ltgw_candidate._fields_}
    top_p = [[rec(tp, i * k + r) for r in range(npw[i])] for i in range(n)]
    top_c = [[rec(tc, i * k + r) for r in range(nct[i])] for i in range(n)]
    return top_p, top_c, {f: getattr(st, f) for f, _ in ltgw_batch_stats._fields_}


def ltgw_batch_results(ctx, i, out_s=None, out_c=None, out_n=None, psi_power=None, psi_count=None):
    a = [_addr(x)[0] for x in (out_s, out_c, out_n, psi_power, psi_count)]
    _check(ctx, library().ltgw_batch_results(ctx, int(i), *a))


def ltgw_batch_latency(ctx, n):
    out = np.empty(n, np.float64)
    _check(ctx, library().ltgw_batch_latency(ctx, out.ctypes.data))
    return out


def ltgw_autotune(ctx, grid):
    v = C.c_int32()
    _check(ctx, library().ltgw_autotune(ctx, C.byref(grid), C.byref(v)))
    return v.value


def ltgw_set_tile_shape(ctx, variant):
    _check(ctx, library().ltgw_set_tile_shape(ctx, int(variant)))


def ltgw_tune_save(ctx, path):
    _check(ctx, library().ltgw_tune_save(ctx, str(path).encode()))


def ltgw_tune_load(ctx, path):
    _check(ctx, library().ltgw_tune_load(ctx, str(path).encode()))


# ---- learned proposer ------------------------------------------------------
def _dev(x, dtype):
    """Address of a contiguous device tensor of the given torch dtype."""
    if not hasattr(x, "data_ptr") or not x.is_cuda:
        raise TypeError("expected a device tensor")
    if x.dtype != dtype:
        raise TypeError(f"expected {dtype}, got {x.dtype}")
    if not x.is_contiguous():
        raise ValueError("tensor must be contiguous")
    return x.data_ptr()


def ltgw_generate_noise(ctx, seed, stream, r0, out):
    """Exp(1) noise into the device float32 tensor out[R][...] (realisations r0..)."""
    import torch
    R = int(out.shape[0])
    n = out.numel() // R
    _check(ctx, library().ltgw_generate_noise(ctx, int(seed), int(stream), int(r0), R, n,
                                              _dev(out, torch.float32)))


def ltgw_inject_stack(ctx, det, stack, params, sky, t0=0.0):
    """Add tracks params[r] = (f0, tau, brake, amp) to the device stack [R][n_seg][n_bins]."""
    import torch
    params = np.ascontiguousarray(params, dtype=np.float64).reshape(-1, 4)
    sky = np.ascontiguousarray(sky, dtype=np.float64).reshape(3)
    _check(ctx, library().ltgw_inject_stack(ctx, int(det), _dev(stack, torch.float32), len(params),
                                            params.ctypes.data, sky.ctypes.data, float(t0)))


def ltgw_load_stack(ctx, det, stack, store="f32", coarse=True):
    """coarse: False (none), True (pairs of segments) or the segments per coarse row (2, 4)."""
    import torch
    cs = int(coarse) if not isinstance(coarse, bool) else (1 if coarse else 0)
    _check(ctx, library().ltgw_load_stack(ctx, int(det), int(stack.shape[0]), _dev(stack, torch.float32),
                                          STORES[store] if isinstance(store, str) else int(store), cs))


def ltgw_stack_psi(ctx, grid, level, out_psi, nan_to_zero=False):
    import torch
    _check(ctx, library().ltgw_stack_psi(ctx, C.byref(grid), int(level), 1 if nan_to_zero else 0,
                                         _dev(out_psi, torch.float64)))


def ltgw_stack_psi_list(ctx, grid, idx, out_psi, stat="power"):
    import torch
    _check(ctx, library().ltgw_stack_psi_list(ctx, C.byref(grid), STATS.get(stat, stat), _dev(idx, torch.int32),
                                              int(idx.shape[1]), _dev(out_psi, torch.float64)))


def ltgw_stack_features(ctx, grid, x, counts=False):
    import torch
    _check(ctx, library().ltgw_stack_features(ctx, C.byref(grid), 1 if counts else 0, _dev(x, torch.float32)))


def ltgw_stack_best(ctx, grid, best_index, best_psi, stat="power"):
    import torch
    _check(ctx, library().ltgw_stack_best(ctx, C.byref(grid), STATS.get(stat, stat), _dev(best_index, torch.int32),
                                          _dev(best_psi, torch.float64)))


def ltgw_cells_from_templates(ctx, tpl, L, cells, mask=None, psi=None, min_psi=0.0):
    import torch
    _check(ctx, library().ltgw_cells_from_templates(ctx, _dev(tpl, torch.int32), tpl.numel(), int(L),
                                                    None if mask is None else _dev(mask, torch.int32),
                                                    None if psi is None else _dev(psi, torch.float64),
                                                    float(min_psi), _dev(cells, torch.int32)))


def ltgw_cnn_param_count(c_in, c_out):
    return int(library().ltgw_cnn_param_count(int(c_in), int(c_out)))


def ltgw_cnn_work_floats(B, c_in, c_out, L):
    return int(library().ltgw_cnn_work_floats(int(B), int(c_in), int(c_out), int(L)))


def ltgw_cnn_forward(ctx, params, x, c_out, act, logits):
    import torch
    B, c_in, L = (int(v) for v in x.shape)
    f = torch.float32
    _check(ctx, library().ltgw_cnn_forward(ctx, _dev(params, f), _dev(x, f), B, c_in, int(c_out), L,
                                           None if act is None else _dev(act, f), _dev(logits, f)))


def ltgw_cnn_backward(ctx, params, x, c_out, act, dlogits, work, grads):
    import torch
    B, c_in, L = (int(v) for v in x.shape)
    f = torch.float32
    _check(ctx, library().ltgw_cnn_backward(ctx, _dev(params, f), _dev(x, f), B, c_in, int(c_out), L,
                                            _dev(act, f), _dev(dlogits, f), _dev(work, f), work.numel(),
                                            _dev(grads, f)))


def ltgw_softmax_xent(ctx, logits, target, n_valid, loss, dlogits):
    import torch
    B = int(logits.shape[0])
    _check(ctx, library().ltgw_softmax_xent(ctx, _dev(logits, torch.float32), B, logits.numel() // B,
                                            _dev(target, torch.int32), int(n_valid),
                                            _dev(loss, torch.float32), _dev(dlogits, torch.float32)))


def ltgw_adam_step(ctx, params, grads, m, v, lr, beta1, beta2, eps, step):
    import torch
    f = torch.float32
    _check(ctx, library().ltgw_adam_step(ctx, _dev(params, f), _dev(grads, f), _dev(m, f), _dev(v, f),
                                         params.numel(), float(lr), float(beta1), float(beta2), float(eps),
                                         int(step)))


def ltgw_select_top(ctx, score, M, out_idx):
    import torch
    R = int(score.shape[0])
    _check(ctx, library().ltgw_select_top(ctx, _dev(score, torch.float32), R, score.numel() // R, int(M),
                                          _dev(out_idx, torch.int32)))


def propose_block_counts(n_select, n_select2, block):
    """(K1, K2): blocks of the first and second tier."""
    return -(-int(n_select) // int(block)), (-(-int(n_select2) // int(block)) if n_select2 > 0 else 0)


def ltgw_propose(ctx, fine, coarse, params, c_in, c_out, L, n_select, psi_threshold, coarse_threshold, R,
                 block=1, n_select2=0, return_blocks=False, tier2_threshold=-1e300, coarse_map=None):
    """(best_index[R], best_psi[R], fallback[R]) numpy arrays, and with
    return_blocks the evaluated blocks [R][K1 + K2] (-1: tier not taken).
    params None: rank by the coarse power ratios through coarse_map
    ([fine groups][2] int32)."""
    import torch
    K1, K2 = propose_block_counts(n_select, n_select2, block)
    blocks = np.empty((R, K1 + K2), np.int32) if return_blocks else None
    cmap = None if coarse_map is None else np.ascontiguousarray(coarse_map, dtype=np.int32)
    p = ltgw_proposer(None if params is None else _dev(params, torch.float32), int(c_in), int(c_out), int(L),
                      int(n_select), int(block), int(n_select2), float(psi_threshold), float(coarse_threshold),
                      float(tier2_threshold), blocks.ctypes.data if return_blocks else None,
                      None if cmap is None else cmap.ctypes.data)
    bi = np.empty(R, np.int32)
    bp = np.empty(R, np.float64)
    fb = np.empty(R, np.int32)
    _check(ctx, library().ltgw_propose(ctx, C.byref(fine), C.byref(coarse), C.byref(p), bi.ctypes.data,
                                       bp.ctypes.data, fb.ctypes.data))
    return (bi, bp, fb, blocks) if return_blocks else (bi, bp, fb)


# ---------------------------------------------------------------------------
class Context:
    """Convenience wrapper: one ltgw context bound to a torch device and stream."""

    def __init__(self, device=0, stream=None):
        import torch

        self.torch = torch
        self.device = torch.device("cuda", device)
        if stream is None:
            stream = torch.cuda.current_stream(self.device).cuda_stream
        self.h = ltgw_create(device, stream)
        self._grid = None
        self.shapes = {}

    def close(self):
        if self.h:
            ltgw_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def load_spectrogram(self, det, power, k_lo, t_sft, t_seg, weights=None, rho_th=1.6,
                         store="f32"):
        ltgw_load_spectrogram(self.h, det, power, k_lo, t_sft, t_seg, weights, rho_th, store)
        self.shapes[det] = (int(power.shape[0]), int(power.shape[1]), store)

    def set_velocity_table(self, det, v):
        ltgw_set_velocity_table(self.h, det, v)

    def set_antenna(self, det, arms, era=None):
        ltgw_set_antenna(self.h, det, arms, era)

    def sft_normalise(self, strain, n_fft, k_lo, n_bins, window=101):
        """Normalised power [n_seg][n_bins] (device FP32) of a device strain series."""
        n_seg = int(strain.numel()) // int(n_fft)
        out = self.torch.empty((n_seg, int(n_bins)), dtype=self.torch.float32, device=self.device)
        ltgw_sft_normalise(self.h, strain, n_seg, n_fft, k_lo, n_bins, window, out)
        return out

    def eval_templates(self, f0_min, f0_step, n_f0, tau, brake, sky, t0=0.0, det_mask=0,
                       stats=LTGW_STAT_POWER | LTGW_STAT_COUNT, outputs=True):
        """Evaluate; with outputs=True returns device tensors (s, c, N)."""
        g, keep = make_grid(f0_min, f0_step, n_f0, tau, brake, sky, t0, det_mask)
        self._grid = (g, keep)
        n = int(n_f0) * len(keep[0]) * len(keep[1]) * len(keep[2])
        if outputs:
            T = self.torch
            s = T.empty(n, dtype=T.float32, device=self.device)
            c = T.empty(n, dtype=T.int32, device=self.device)
            N = T.empty(n, dtype=T.int32, device=self.device)
            ltgw_eval_templates(self.h, g, stats, s, c, N)
            return s, c, N
        ltgw_eval_templates(self.h, g, stats)
        return None

    def eval_list(self, params, t0=0.0, det_mask=0, outputs=True):
        """Explicit templates (f0, tau, n, sky x, y, z) per row; with outputs=True
        returns device tensors (s, c, N) in list order."""
        n = int(np.asarray(params).reshape(-1, 6).shape[0])
        if outputs:
            T = self.torch
            s = T.empty(n, dtype=T.float32, device=self.device)
            c = T.empty(n, dtype=T.int32, device=self.device)
            N = T.empty(n, dtype=T.int32, device=self.device)
            ltgw_eval_list(self.h, params, t0, det_mask, s, c, N)
            return s, c, N
        ltgw_eval_list(self.h, params, t0, det_mask)
        return None

    def psi(self, stat, n):
        out = self.torch.empty(n, dtype=self.torch.float64, device=self.device)
        ltgw_psi(self.h, stat, out)
        return out

    def topk(self, stat, k):
        return ltgw_topk_candidates(self.h, stat, k)

    def diagnostics(self):
        return ltgw_diagnostics(self.h)

    def inject_track(self, det, power, f0, tau, brake, sky, t0, amp):
        ltgw_inject_track(self.h, det, power, f0, tau, brake, sky, t0, amp)

    def read_store(self, det):
        n_seg, n_bins, store = self.shapes[det]
        return ltgw_read_store(self.h, det, n_seg, n_bins, store)

    def read_tables(self, det):
        return ltgw_read_tables(self.h, det, self.shapes[det][0])

    def eval_batch(self, searches, k=10):
        """searches: list of dicts with f0_min, f0_step, n_f0, tau, brake, sky, t0, dets."""
        specs = [(make_grid(s["f0_min"], s["f0_step"], s["n_f0"], s["tau"], s["brake"], s["sky"],
                            s.get("t0", 0.0)), s["dets"]) for s in searches]
        self._batch = specs
        return ltgw_eval_batch(self.h, specs, k)

    def batch_results(self, i, n_templates):
        T = self.torch
        s = T.empty(n_templates, dtype=T.float32, device=self.device)
        c = T.empty(n_templates, dtype=T.int32, device=self.device)
        N = T.empty(n_templates, dtype=T.int32, device=self.device)
        pp = T.empty(n_templates, dtype=T.float64, device=self.device)
        pc = T.empty(n_templates, dtype=T.float64, device=self.device)
        ltgw_batch_results(self.h, i, s, c, N, pp, pc)
        return s, c, N, pp, pc

    def batch_latency(self, n):
        return ltgw_batch_latency(self.h, n)

    def autotune(self, f0_min, f0_step, n_f0, tau, brake, sky, t0=0.0, det_mask=0):
        g, keep = make_grid(f0_min, f0_step, n_f0, tau, brake, sky, t0, det_mask)
        return ltgw_autotune(self.h, g)

    def set_tile_shape(self, variant):
        ltgw_set_tile_shape(self.h, variant)

    def tune_save(self, path):
        ltgw_tune_save(self.h, path)

    def tune_load(self, path):
        ltgw_tune_load(self.h, path)
