"""CPU oracle for the template-bank detection statistic (FP64, plain C + numpy).

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, the smoke check and the CPU-baseline
leg of the benchmark may import this package.  It shares no code with the HIP
library; the two are compared, never combined.

The arithmetic lives in ``oracle.c`` (every FP64 operation correctly rounded,
in the order written, no fused multiply-add).  This module marshals numpy
arrays into it and adds the two steps that are plain library calls: the
ranking of critical ratios (a sort) and nothing else.

Paper references (Merou, Tenorio, Sintes, long-transient GW search):
Eq. 1 (frequency track), Eq. 2 (Doppler factor), Sec. 2 (statistic summed
over the bins the track selects), Eq. 4 (critical ratio), Sec. 3 (detection
by the largest critical ratios).
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

from . import build as _build

C_LIGHT = 299792458.0

_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_build.LIB):
            _build.build()
        L = C.CDLL(_build.LIB)
        d, i32, i64, f32 = C.c_double, C.c_int32, C.c_int64, C.c_float
        P = C.c_void_p
        L.oracle_spin_factor.restype = d
        L.oracle_spin_factor.argtypes = [d, d, d, d]
        L.oracle_doppler.restype = d
        L.oracle_doppler.argtypes = [P, P]
        L.oracle_bin.restype = i64
        L.oracle_bin.argtypes = [d, d, d, d, i64]
        L.oracle_lattice_f0.restype = d
        L.oracle_lattice_f0.argtypes = [d, d, i64]
        L.oracle_eval.restype = None
        L.oracle_eval.argtypes = [P, i32, P, i64, i64, P, P, P, P, P]
        L.oracle_eval_list.restype = None
        L.oracle_eval_list.argtypes = [P, i32, P, P, i64, P, P, P, P, P]
        L.oracle_eval_params.restype = None
        L.oracle_eval_params.argtypes = [P, i32, P, i64, d, P, P, P, P, P]
        L.oracle_philox4x32_10.restype = None
        L.oracle_philox4x32_10.argtypes = [P, P, P]
        L.oracle_exp_noise.restype = None
        L.oracle_exp_noise.argtypes = [C.c_uint64, C.c_uint32, i32, i64, P]
        L.oracle_threads.restype = i32
        L.oracle_threads.argtypes = []
        L.oracle_track_bins.restype = None
        L.oracle_track_bins.argtypes = [P, d, d, d, P, d, P]
        L.oracle_count_q.restype = d
        L.oracle_count_q.argtypes = [f32]
        L.oracle_psi_power.restype = None
        L.oracle_psi_power.argtypes = [i64, P, P, P, P, P]
        L.oracle_psi_count.restype = None
        L.oracle_psi_count.argtypes = [i64, P, P, f32, P]
        L.oracle_bf16_rne.restype = C.c_uint16
        L.oracle_bf16_rne.argtypes = [f32]
        L.oracle_bf16_decode.restype = f32
        L.oracle_bf16_decode.argtypes = [C.c_uint16]
        L.oracle_e4m3_rne_sat.restype = C.c_uint8
        L.oracle_e4m3_rne_sat.argtypes = [f32]
        L.oracle_e4m3_decode.restype = f32
        L.oracle_e4m3_decode.argtypes = [C.c_uint8]
        L.oracle_fp8_row_scale.restype = f32
        L.oracle_fp8_row_scale.argtypes = [P, i32]
        L.oracle_dequantised.restype = None
        L.oracle_dequantised.argtypes = [P, i32, i32, i32, P, P]
        L.oracle_bf16_rne_array.restype = None
        L.oracle_bf16_rne_array.argtypes = [P, i64, P]
        L.oracle_e4m3_rne_sat_array.restype = None
        L.oracle_e4m3_rne_sat_array.argtypes = [P, i64, P]
        L.oracle_antenna.restype = d
        L.oracle_antenna.argtypes = [P, d, P]
        L.oracle_spin_factor_array.restype = None
        L.oracle_spin_factor_array.argtypes = [P, i64, d, d, d, P]
        _lib = L
    return _lib


def _p(a):
    return a.ctypes.data_as(C.c_void_p) if a is not None else None


class _Det(C.Structure):
    _fields_ = [("n_seg", C.c_int32), ("n_bins", C.c_int32), ("k_lo", C.c_int64),
                ("t_sft", C.c_double), ("t_seg", C.c_void_p), ("w", C.c_void_p),
                ("v", C.c_void_p), ("P", C.c_void_p), ("rho", C.c_void_p),
                ("rho_th", C.c_float), ("arms", C.c_void_p), ("era", C.c_void_p)]


class _Grid(C.Structure):
    _fields_ = [("f0_min", C.c_double), ("f0_step", C.c_double), ("n_f0", C.c_int32),
                ("tau", C.c_void_p), ("n_tau", C.c_int32),
                ("brake", C.c_void_p), ("n_brake", C.c_int32),
                ("sky", C.c_void_p), ("n_sky", C.c_int32), ("t0", C.c_double)]


class Detector:
    """One detector's data as the oracle sees it.

    rho: FP32 [n_seg, n_bins] normalised power (the count compares it with
    rho_th in FP32).  values: FP64 [n_seg, n_bins] that the power sum adds up;
    by default the FP32 powers themselves, or the dequantised values of a
    BF16/FP8 store (see ``dequantised``)."""

    def __init__(self, rho, t_seg, v, k_lo, t_sft, weights=None, rho_th=1.6, values=None,
                 arms=None, era=None):
        self.rho = np.ascontiguousarray(rho, dtype=np.float32)
        self.n_seg, self.n_bins = self.rho.shape
        self.t_seg = np.ascontiguousarray(t_seg, dtype=np.float64)
        self.v = np.ascontiguousarray(v, dtype=np.float64).reshape(self.n_seg, 3)
        self.k_lo = int(k_lo)
        self.t_sft = float(t_sft)
        self.w = None if weights is None else np.ascontiguousarray(weights, dtype=np.float32)
        self.rho_th = np.float32(rho_th)
        self.values = (self.rho.astype(np.float64) if values is None
                       else np.ascontiguousarray(values, dtype=np.float64))
        assert self.values.shape == self.rho.shape
        # antenna response (Sec. 2 weighting): arms [2][3] Earth-fixed unit
        # vectors and the Earth rotation angle at each segment; the weight of
        # segment j for sky n is then w_j * (F+^2 + Fx^2)(n, j)
        self.arms = None if arms is None else np.ascontiguousarray(arms, dtype=np.float64).reshape(2, 3)
        self.era = None if era is None else np.ascontiguousarray(era, dtype=np.float64).reshape(self.n_seg)
        assert (self.arms is None) == (self.era is None)

    def _struct(self):
        return _Det(self.n_seg, self.n_bins, self.k_lo, self.t_sft, _p(self.t_seg), _p(self.w),
                    _p(self.v), _p(self.values), _p(self.rho), float(self.rho_th), _p(self.arms),
                    _p(self.era))


class Grid:
    """Cubic lattice bank (Sec. 2): f0 = f0_min + i*step, tau list, n list, sky list."""

    def __init__(self, f0_min, f0_step, n_f0, tau, brake, sky, t0=0.0):
        self.f0_min, self.f0_step, self.n_f0 = float(f0_min), float(f0_step), int(n_f0)
        self.tau = np.ascontiguousarray(tau, dtype=np.float64)
        self.brake = np.ascontiguousarray(brake, dtype=np.float64)
        self.sky = np.ascontiguousarray(sky, dtype=np.float64).reshape(-1, 3)
        self.t0 = float(t0)

    @property
    def n_templates(self):
        return self.n_f0 * len(self.tau) * len(self.brake) * len(self.sky)

    def _struct(self):
        return _Grid(self.f0_min, self.f0_step, self.n_f0, _p(self.tau), len(self.tau),
                     _p(self.brake), len(self.brake), _p(self.sky), len(self.sky), self.t0)

    def params(self, index):
        """(f0, tau, n, sky) of template index (order: sky, n, tau, f0 fastest)."""
        index = np.asarray(index, dtype=np.int64)
        i_f0 = index % self.n_f0
        grp = index // self.n_f0
        i_tau = grp % len(self.tau)
        r = grp // len(self.tau)
        i_n = r % len(self.brake)
        i_sky = r // len(self.brake)
        f0 = np.array([lattice_f0(self.f0_min, self.f0_step, int(i)) for i in np.ravel(i_f0)])
        return f0.reshape(i_f0.shape), self.tau[i_tau], self.brake[i_n], i_sky


def spin_factor(t, t0, tau, brake):
    return lib().oracle_spin_factor(float(t), float(t0), float(tau), float(brake))


def spin_factor_array(t, t0, tau, brake):
    t = np.ascontiguousarray(t, dtype=np.float64)
    out = np.empty_like(t)
    lib().oracle_spin_factor_array(_p(t), t.size, float(t0), float(tau), float(brake), _p(out))
    return out


def antenna(arms, era, n):
    """F+^2 + Fx^2 of a detector with Earth-fixed arms [2][3] at Earth rotation
    angle era, for a wave from unit direction n (Sec. 2 weighting)."""
    a = np.ascontiguousarray(arms, dtype=np.float64).reshape(6)
    k = np.ascontiguousarray(n, dtype=np.float64).reshape(3)
    return lib().oracle_antenna(_p(a), float(era), _p(k))


def doppler(v, n):
    v = np.ascontiguousarray(v, dtype=np.float64)
    n = np.ascontiguousarray(n, dtype=np.float64)
    return lib().oracle_doppler(_p(v), _p(n))


def bin_index(f0, g, D, t_sft, k_lo):
    return lib().oracle_bin(float(f0), float(g), float(D), float(t_sft), int(k_lo))


def lattice_f0(f0_min, f0_step, i):
    return lib().oracle_lattice_f0(float(f0_min), float(f0_step), int(i))


def track_bins(det: Detector, f0, tau, brake, sky, t0):
    """Columns of the template's track on det, INT64_MIN where t_j < T0."""
    out = np.empty(det.n_seg, dtype=np.int64)
    sky = np.ascontiguousarray(sky, dtype=np.float64)
    s = det._struct()
    lib().oracle_track_bins(C.byref(s), float(f0), float(tau), float(brake), _p(sky),
                            float(t0), _p(out))
    return out


def evaluate(dets, grid: Grid, begin=0, end=None):
    """Statistic for templates [begin, end): dict of s, c, N, W1, W2 arrays."""
    if isinstance(dets, Detector):
        dets = [dets]
    end = grid.n_templates if end is None else int(end)
    n = end - begin
    out = {"s": np.empty(n, np.float64), "c": np.empty(n, np.int32),
           "N": np.empty(n, np.int32), "W1": np.empty(n, np.float64),
           "W2": np.empty(n, np.float64)}
    arr = (_Det * len(dets))(*[d._struct() for d in dets])
    gs = grid._struct()
    lib().oracle_eval(C.cast(arr, C.c_void_p), len(dets), C.byref(gs), int(begin), int(end),
                      _p(out["s"]), _p(out["c"]), _p(out["N"]), _p(out["W1"]), _p(out["W2"]))
    return out


def evaluate_list(dets, grid: Grid, index):
    """Statistic for the template indices in `index` (any order, repeats allowed)."""
    if isinstance(dets, Detector):
        dets = [dets]
    index = np.ascontiguousarray(index, dtype=np.int64)
    n = index.size
    out = {"s": np.empty(n, np.float64), "c": np.empty(n, np.int32),
           "N": np.empty(n, np.int32), "W1": np.empty(n, np.float64),
           "W2": np.empty(n, np.float64)}
    arr = (_Det * len(dets))(*[d._struct() for d in dets])
    gs = grid._struct()
    lib().oracle_eval_list(C.cast(arr, C.c_void_p), len(dets), C.byref(gs), _p(index), n,
                           _p(out["s"]), _p(out["c"]), _p(out["N"]), _p(out["W1"]), _p(out["W2"]))
    return out


def evaluate_params(dets, params, t0=0.0):
    """Statistic of explicit templates, params [n][6] = (f0, tau, n, sky x, y, z)
    (the uniform random bank of Sec. 2): dict of s, c, N, W1, W2 arrays."""
    if isinstance(dets, Detector):
        dets = [dets]
    params = np.ascontiguousarray(params, dtype=np.float64).reshape(-1, 6)
    n = params.shape[0]
    out = {"s": np.empty(n, np.float64), "c": np.empty(n, np.int32),
           "N": np.empty(n, np.int32), "W1": np.empty(n, np.float64),
           "W2": np.empty(n, np.float64)}
    arr = (_Det * len(dets))(*[d._struct() for d in dets])
    lib().oracle_eval_params(C.cast(arr, C.c_void_p), len(dets), _p(params), n, float(t0),
                             _p(out["s"]), _p(out["c"]), _p(out["N"]), _p(out["W1"]), _p(out["W2"]))
    return out


def threads():
    """Threads the oracle's parallel loops use."""
    return lib().oracle_threads()


def count_q(rho_th=1.6):
    return lib().oracle_count_q(float(np.float32(rho_th)))


def psi_power(res):
    n = res["s"].size
    out = np.empty(n, np.float64)
    lib().oracle_psi_power(n, _p(res["s"]), _p(res["N"]), _p(res["W1"]), _p(res["W2"]), _p(out))
    return out


def psi_count(res, rho_th=1.6):
    n = res["c"].size
    out = np.empty(n, np.float64)
    lib().oracle_psi_count(n, _p(res["c"]), _p(res["N"]), float(np.float32(rho_th)), _p(out))
    return out


def topk(psi, k, index_offset=0):
    """Indices of the k largest critical ratios, ordered by (psi desc, index asc);
    NaN (no in-band segment) never ranks.  Detection ranks templates by their
    critical ratio (Sec. 3)."""
    psi = np.asarray(psi, dtype=np.float64)
    idx = np.nonzero(~np.isnan(psi))[0]
    order = np.lexsort((idx, -psi[idx]))
    return idx[order[:k]] + index_offset


# --- storage formats -------------------------------------------------------
def bf16_rne(x):
    x = np.ascontiguousarray(x, dtype=np.float32)
    out = np.empty(x.shape, np.uint16)
    lib().oracle_bf16_rne_array(_p(x), x.size, _p(out))
    return out


def e4m3_rne_sat(x):
    x = np.ascontiguousarray(x, dtype=np.float32)
    out = np.empty(x.shape, np.uint8)
    lib().oracle_e4m3_rne_sat_array(_p(x), x.size, _p(out))
    return out


def e4m3_decode(code):
    return lib().oracle_e4m3_decode(int(code))


def bf16_decode(code):
    return lib().oracle_bf16_decode(int(code))


def dequantised(rho, store):
    """FP64 values a store reproduces (store: 'f32', 'bf16' or 'fp8'), and the
    per-segment FP8 scales (None otherwise)."""
    rho = np.ascontiguousarray(rho, dtype=np.float32)
    code = {"f32": 0, "bf16": 1, "fp8": 2}[store]
    out = np.empty(rho.shape, np.float64)
    sc = np.empty(rho.shape[0], np.float32) if code == 2 else None
    lib().oracle_dequantised(_p(rho), rho.shape[0], rho.shape[1], code, _p(out), _p(sc))
    return out, sc


# --- counter-based noise (proposer training data) --------------------------
def philox4x32_10(ctr, key):
    """Philox4x32-10 block: 4 counter words, 2 key words -> 4 output words."""
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    out = np.empty(4, np.uint32)
    lib().oracle_philox4x32_10(_p(c), _p(k), _p(out))
    return out


def exp_noise(seed, stream, r, n):
    """Exp(1) noise of realisation r (n values), as the proposer's generator defines it."""
    out = np.empty(int(n), np.float32)
    lib().oracle_exp_noise(int(seed), int(stream), int(r), int(n), _p(out))
    return out
