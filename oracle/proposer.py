"""Reference definitions of the learned proposer's data path (test
infrastructure only: the product never imports this module).

- coarse_power: the coarsened map over S consecutive segments and 2 bins
  (S = 2 by default).  Pixel (j', m) is the FP32 sum, segment by segment in
  order, of the segments' bin-pair sums P[S j' + s][2m] + P[S j' + s][2m+1],
  rounded to bfloat16; under noise alone it is a sum of 2 S Exp(1) values
  (mean 2 S, variance 2 S).
- coarse_psi: the power critical ratio (Eq. 4 with that mean and variance)
  of a template on the coarse map.  The template's column in segment group
  j' is its fine column (Eqs. 1-2 and the bin rule of Sec. 2) at the group's
  first segment, halved (floor); the group's weight is the FP32 sum of its S
  weights (in order) times 1/S.
- coarse_count / coarse_psi_count: the number count on the same blocks.
  Pixel (j', m) counts the 2 S fine pixels of the block whose normalised
  power exceeds rho_th (compared in FP32, strictly, as the fine count of
  Sec. 2); under noise alone it is Binomial(2 S, q) with q = exp(-rho_th).
  The count ratio of a template (Eq. 4 for the count) sums the counts of its
  coarse pixels (same columns as coarse_psi) against N 2 S q, N the in-band
  coarse segments, with variance N 2 S q (1 - q); the count is unweighted.
- cells and templates: network output cell (channel ch, position l) is fine
  template (group ch // 2, f0 index 2 l + ch % 2).
- best_template: the largest Psi of a list (ties: lowest template index),
  the quantity the proposer reports per realisation.
"""
import numpy as np

import oracle


def coarse_power(P, S=2):
    """P: FP32 [n_seg][n_bins] (n_seg a multiple of S, n_bins even) -> FP64
    values of the BF16 coarse map [n_seg / S][n_bins / 2]."""
    P = np.asarray(P, dtype=np.float32)
    s = P[0::S, 0::2] + P[0::S, 1::2]
    for k in range(1, S):
        s = (s + (P[k::S, 0::2] + P[k::S, 1::2])).astype(np.float32)
    codes = oracle.bf16_rne(s.astype(np.float32)).astype(np.uint32) << 16
    return codes.view(np.float32).astype(np.float64)


def coarse_weights(w, n_seg, S=2):
    w = np.ones(n_seg, np.float32) if w is None else np.asarray(w, np.float32)
    s = w[0::S].copy()
    for k in range(1, S):
        s = (s + w[k::S]).astype(np.float32)
    return (s * np.float32(1.0 / S)).astype(np.float32)


def coarse_psi(det: "oracle.Detector", grid: "oracle.Grid", P, nan_to_zero=False, S=2):
    """Coarse power critical ratio of every template of grid on det's geometry
    with fine power P (FP32 [n_seg][n_bins]); FP64 [n_templates]."""
    C = coarse_power(P, S)
    w2 = coarse_weights(det.w, det.n_seg, S).astype(np.float64)
    nb2 = det.n_bins // 2
    mu = 2.0 * S
    out = np.empty(grid.n_templates)
    for t in range(grid.n_templates):
        f0, tau, brake, i_sky = grid.params(t)
        b = oracle.track_bins(det, float(f0), float(tau), float(brake), grid.sky[int(i_sky)], grid.t0)
        b = b[0::S]
        m = np.where(b == np.iinfo(np.int64).min, -1, b // 2)
        inb = (m >= 0) & (m < nb2)
        j = np.nonzero(inb)[0]
        if j.size == 0:
            out[t] = 0.0 if nan_to_zero else np.nan
            continue
        s = np.sum(w2[j] * C[j, m[j]])
        W1 = np.sum(w2[j])
        W2 = np.sum(w2[j] ** 2)
        out[t] = (s - mu * W1) / np.sqrt(mu * W2)
    return out


def coarse_count(P, S=2, rho_th=1.6):
    """P: FP32 [n_seg][n_bins] -> int [n_seg / S][n_bins / 2]: pixels above
    rho_th (FP32, strict) in each S x 2 block."""
    above = (np.asarray(P, dtype=np.float32) > np.float32(rho_th)).astype(np.int64)
    c = above[0::S, 0::2] + above[0::S, 1::2]
    for k in range(1, S):
        c = c + above[k::S, 0::2] + above[k::S, 1::2]
    return c


def coarse_psi_count(det: "oracle.Detector", grid: "oracle.Grid", P, nan_to_zero=False, S=2):
    """Coarse count critical ratio of every template (columns as coarse_psi);
    FP64 [n_templates]."""
    C = coarse_count(P, S, float(det.rho_th))
    nb2 = det.n_bins // 2
    q = oracle.count_q(float(det.rho_th))
    m = 2.0 * S
    out = np.empty(grid.n_templates)
    for t in range(grid.n_templates):
        f0, tau, brake, i_sky = grid.params(t)
        b = oracle.track_bins(det, float(f0), float(tau), float(brake), grid.sky[int(i_sky)], grid.t0)
        b = b[0::S]
        col = np.where(b == np.iinfo(np.int64).min, -1, b // 2)
        j = np.nonzero((col >= 0) & (col < nb2))[0]
        if j.size == 0:
            out[t] = 0.0 if nan_to_zero else np.nan
            continue
        c = float(np.sum(C[j, col[j]]))
        n = float(j.size)
        out[t] = (c - n * m * q) / np.sqrt(n * m * q * (1.0 - q))
    return out


def cell_to_template(cell, L):
    """Network cell (ch * L + l) -> fine template index (fine n_f0 = 2 L)."""
    cell = np.asarray(cell, dtype=np.int64)
    ch, l = cell // L, cell % L
    return (ch // 2) * (2 * L) + 2 * l + (ch % 2)


def template_to_cell(tpl, L):
    tpl = np.asarray(tpl, dtype=np.int64)
    grp, i = tpl // (2 * L), tpl % (2 * L)
    return (2 * grp + i % 2) * L + i // 2


def best_template(psi, index):
    """(index, psi) of the largest finite psi (ties: lowest index); (-1, -inf) if none."""
    psi = np.asarray(psi, dtype=np.float64)
    index = np.asarray(index, dtype=np.int64)
    ok = np.isfinite(psi)
    if not ok.any():
        return -1, -np.inf
    p, i = psi[ok], index[ok]
    top = p.max()
    return int(i[p == top].min()), float(top)
