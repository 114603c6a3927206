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

LTGW_STORE_F32 = 0
LTGW_STORE_BF16 = 1
LTGW_STORE_FP8 = 2
STORES = {"f32": LTGW_STORE_F32, "bf16": LTGW_STORE_BF16, "fp8": LTGW_STORE_FP8}

LTGW_STAT_POWER = 1
LTGW_STAT_COUNT = 2
STATS = {"power": LTGW_STAT_POWER, "count": LTGW_STAT_COUNT}

LTGW_MAX_DET = 4
LTGW_MAX_TOPK = 256

# every symbol include/ltgw.h declares
EXPORTS = ("ltgw_create", "ltgw_destroy", "ltgw_last_error", "ltgw_load_spectrogram",
           "ltgw_set_velocity_table", "ltgw_eval_templates", "ltgw_psi",
           "ltgw_topk_candidates", "ltgw_diagnostics", "ltgw_inject_track", "ltgw_read_store")


class ltgw_spec_desc(C.Structure):
    _fields_ = [("n_seg", C.c_int32), ("n_bins", C.c_int32), ("k_lo", C.c_int64),
                ("t_sft", C.c_double), ("t_seg", C.c_void_p), ("weights", C.c_void_p),
                ("rho_th", C.c_float), ("store", C.c_int32)]


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
                ("in_band", C.c_int64), ("eval_kernel_ms", C.c_double), ("tables_ms", C.c_double)]


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
            "ltgw_eval_templates": (i32, [P, C.POINTER(ltgw_grid), u32, P, P, P]),
            "ltgw_psi": (i32, [P, u32, P]),
            "ltgw_topk_candidates": (i32, [P, u32, i32, C.POINTER(ltgw_candidate), C.POINTER(i32)]),
            "ltgw_diagnostics": (i32, [P, C.POINTER(ltgw_diag)]),
            "ltgw_inject_track": (i32, [P, i32, P, d, d, d, P, d, f]),
            "ltgw_read_store": (i32, [P, i32, P, P]),
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
