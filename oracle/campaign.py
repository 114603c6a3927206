"""Reference of the synthetic sensitivity campaign (Sec. 3, Figs. 3-4).

TEST INFRASTRUCTURE ONLY: only the tests use this module.  It shares no code
with the library: realisations come from this package's Philox Exp(1)
generator, injections from its own track bins, statistics from its FP64
evaluation, the close neighbourhood from a direct scan of the lattice, and
the fit from a general-purpose minimiser of the binomial likelihood.

- A realisation is Exp(1) noise (Philox4x32-10 stream and counter as the
  library's generator is documented) plus, for an injection (f0, tau, n, A),
  A * w_j added in FP32 at the track's bin of every in-band segment.
- Detection (Sec. 3): a template close to the injection has a critical ratio
  above the largest one of the noise-only realisations.  Close: the lattice
  f0 index within 2 of the injection's nearest, tau (nearest in log) and n
  indices within 1; for a random bank, the box of the same extent in
  parameter units.
- Efficiency vs amplitude: eff(A) = 1/(1 + exp(-(ln A - mu)/sigma)) fitted
  by maximum likelihood; A90 = exp(mu + sigma ln 9).  When no detection
  occurs below a miss the maximum does not exist: the step sits midway in
  ln A between the last amplitude with a miss and the first with a detection.
"""
import math

import numpy as np
from scipy.optimize import minimize

from . import Detector, evaluate, evaluate_params, exp_noise, psi_count, psi_power, track_bins


def realisation(geo, seed, stream, r, inj=None, sky=None, t0=0.0):
    n_seg, n_bins = len(geo["t_seg"]), int(geo["n_bins"])
    P = exp_noise(seed, stream, r, n_seg * n_bins).reshape(n_seg, n_bins).copy()
    if inj is not None and inj[3] != 0:
        det = Detector(P, geo["t_seg"], geo["v"], geo["k_lo"], geo["t_sft"], weights=geo.get("weights"))
        b = track_bins(det, inj[0], inj[1], inj[2], sky, t0)
        w = np.ones(n_seg, np.float32) if geo.get("weights") is None else np.asarray(geo["weights"], np.float32)
        for j in range(n_seg):
            if 0 <= b[j] < n_bins:
                P[j, b[j]] = np.float32(P[j, b[j]] + np.float32(np.float32(inj[3]) * w[j]))
    return Detector(P, geo["t_seg"], geo["v"], geo["k_lo"], geo["t_sft"], weights=geo.get("weights"))


def _best(res):
    out = []
    for psi in (psi_power(res), psi_count(res)):
        out.append(float(np.nanmax(psi)) if np.any(~np.isnan(psi)) else -math.inf)
    return out


def lattice_region(grid, inj):
    """Template rows of the lattice close to inj = (f0, tau, n, ...)."""
    f0, tau, n = inj[:3]
    idx = np.arange(grid.n_templates)
    tf0, ttau, tn, isky = grid.params(idx)
    i_f0 = np.rint((tf0 - grid.f0_min) / grid.f0_step)
    i0 = round((f0 - grid.f0_min) / grid.f0_step)
    lt = np.log(grid.tau)
    j0 = int(np.argmin(np.abs(lt - math.log(tau))))
    k0 = int(np.argmin(np.abs(grid.brake - n)))
    jt = np.array([int(np.nonzero(grid.tau == x)[0][0]) for x in ttau])
    kt = np.array([int(np.nonzero(grid.brake == x)[0][0]) for x in tn])
    ok = (np.abs(i_f0 - i0) <= 2) & (np.abs(jt - j0) <= 1) & (np.abs(kt - k0) <= 1) & (isky == 0)
    sel = idx[ok]
    return np.column_stack([tf0[sel], ttau[sel], tn[sel], grid.sky[isky[sel]]])


def bank_region(bank, grid, inj):
    f0, tau, n = inj[:3]
    lt = np.log(grid.tau)
    dlt = (lt.max() - lt.min()) / max(len(lt) - 1, 1)
    dn = (grid.brake.max() - grid.brake.min()) / max(len(grid.brake) - 1, 1)
    keep = []
    for q, row in enumerate(bank):
        if (abs(row[0] - f0) <= 2 * grid.f0_step + 1e-12 and abs(math.log(row[1]) - math.log(tau)) <= dlt + 1e-12
                and abs(row[2] - n) <= dn + 1e-12):
            keep.append(q)
    return np.asarray(bank)[keep]


def noise_maxima(geo, grid, R, seed, stream=1, bank=None):
    bp, bc = [], []
    for r in range(R):
        det = realisation(geo, seed, stream, r)
        res = evaluate(det, grid) if bank is None else evaluate_params(det, bank, grid.t0)
        p, c = _best(res)
        bp.append(p)
        bc.append(c)
    return np.array(bp), np.array(bc)


def injected_maxima(geo, grid, inj, seed, stream=2, bank=None):
    bp, bc = [], []
    for r, row in enumerate(np.asarray(inj, np.float64)):
        det = realisation(geo, seed, stream, r, row, grid.sky[0], grid.t0)
        rows = lattice_region(grid, row) if bank is None else bank_region(bank, grid, row)
        if len(rows) == 0:
            bp.append(-math.inf)
            bc.append(-math.inf)
            continue
        p, c = _best(evaluate_params(det, rows, grid.t0))
        bp.append(p)
        bc.append(c)
    return np.array(bp), np.array(bc)


def fit_logistic(amp, k, n):
    """Maximum-likelihood (mu, sigma) of eff(A) = 1/(1 + exp(-(ln A - mu)/sigma)),
    by a general-purpose minimiser of the binomial negative log-likelihood."""
    x = np.log(np.asarray(amp, np.float64))
    k = np.asarray(k, np.float64)
    n = np.asarray(n, np.float64)
    # no finite maximum unless a detection occurs below a miss: then a step
    # midway (in ln A) between the last amplitude with a miss and the first
    # with a detection, sigma = 0
    has_miss = [i for i in range(len(x)) if k[i] < n[i]]
    has_hit = [i for i in range(len(x)) if k[i] > 0]
    overlap = any(x[h] < x[m] for h in has_hit for m in has_miss)
    if not overlap:
        lo = max(x[i] for i in has_miss) if has_miss else min(x[i] for i in has_hit)
        hi = min(x[i] for i in has_hit) if has_hit else max(x[i] for i in has_miss)
        mu = (lo + hi) / 2.0
        return {"mu": mu, "sigma": 0.0, "a90": math.exp(mu), "separable": True, "rising": True}

    def nll(th):
        z = th[0] + th[1] * x
        # log p = -log(1 + e^-z), log(1 - p) = -log(1 + e^z)
        return float(np.sum(k * np.logaddexp(0.0, -z) + (n - k) * np.logaddexp(0.0, z)))

    sd = max(float(np.std(x)), 1e-3)
    start = np.array([-float(np.mean(x)) / sd, 1.0 / sd])
    r = minimize(nll, start, method="Nelder-Mead",
                 options={"xatol": 1e-12, "fatol": 1e-14, "maxiter": 40000, "maxfev": 80000})
    a, b = float(r.x[0]), float(r.x[1])
    if not b > 0.0:
        return {"mu": math.nan, "sigma": math.inf, "a90": math.inf, "separable": False, "rising": False}
    mu, sigma = -a / b, 1.0 / b
    return {"mu": mu, "sigma": sigma, "a90": math.exp(min(mu + sigma * math.log(9.0), 700.0)),
            "separable": False, "rising": True}
